// Host runtime behind include/mm.h: the context (all device memory reserved
// at creation), argument validation, the enqueue order of one step and the
// single status readback per call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "../../include/mm.h"
#include "mm_internal.h"

using namespace mm;

struct mm_ctx {
  mm_params p{};
  int64_t ncap = 0, fcap = 0, nbcap = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  // Sort and tessellation.
  int32_t *key = nullptr, *perm = nullptr, *deferred = nullptr;
  double *spos = nullptr, *geo = nullptr, *rmax2 = nullptr, *minv = nullptr;
  unsigned long long *bcount = nullptr, *boff = nullptr, *scan_tmp = nullptr, *counts = nullptr, *off = nullptr;
  StageNbr* stage_nb = nullptr;
  StageGeo* stage_geo = nullptr;
  Face* faces = nullptr;
  int32_t* csr = nullptr;
  NbrEntry* nbr = nullptr;
  // State in internal order.
  void *U = nullptr, *G = nullptr, *Uh = nullptr, *Gh = nullptr, *phi = nullptr;
  double *w = nullptr, *Qs = nullptr, *dQs = nullptr;
  DevStatus* st = nullptr;
  DevStatus* st_host = nullptr;   // pinned mirror
  // Mesh held by the context.
  bool have_mesh = false;
  int64_t n_mesh = 0, n_faces = 0;
  GridParams grid{};
  double rfac = 2.0;   // first-pass candidate radius in mean spacings (adapted per call)
  // Stage timing.
  bool timing = false;
  hipEvent_t ev[9] = {};
  double stage_ms[8] = {};
  std::string err;
};

namespace {

const char* kVersion = "mm-mi355x 0.1 (gfx950)";

// Message of the last failed mm_create on this thread (there is no context
// to hold it).
thread_local std::string g_create_err;

mm_status fail(mm_ctx* c, mm_status code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

mm_status create_fail(mm_status code, const std::string& msg) {
  g_create_err = msg;
  return code;
}

#define HIPCHECK(ctx, call)                                                                  \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail(ctx, MM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));          \
  } while (0)

bool params_ok(const mm_params* p, std::string& why) {
  for (int a = 0; a < 3; ++a)
    if (!(std::isfinite(p->box[a]) && p->box[a] > 0)) { why = "box lengths must be finite and positive"; return false; }
  if (!(p->gamma > 1.0 && std::isfinite(p->gamma))) { why = "gamma must exceed 1"; return false; }
  if (!(p->cfl > 0.0)) { why = "cfl must be positive"; return false; }
  if (!(p->zeta > 0.0)) { why = "zeta must be positive"; return false; }
  if (!(p->rho_floor > 0.0 && p->p_floor > 0.0)) { why = "floors must be positive"; return false; }
  if (p->precision != MM_FP64 && p->precision != MM_MIXED) { why = "precision must be MM_FP64 or MM_MIXED"; return false; }
  if (p->riemann != MM_HLLC) { why = "riemann must be MM_HLLC"; return false; }
  if (p->limit_mask < 0 || p->limit_mask > 3) { why = "limit_mask must be in 0..3"; return false; }
  if (p->predictor_frame != 0 && p->predictor_frame != 1) { why = "predictor_frame must be 0 or 1"; return false; }
  return true;
}

HydroParams hydro_params(const mm_params& p) {
  HydroParams h;
  for (int a = 0; a < 3; ++a) h.L[a] = p.box[a];
  h.gamma = p.gamma;
  h.cfl = p.cfl;
  h.eta = p.eta;
  h.chi = p.chi;
  h.zeta = p.zeta;
  h.theta = p.theta;
  h.rho_floor = p.rho_floor;
  h.p_floor = p.p_floor;
  h.limit_mask = p.limit_mask;
  h.predictor_frame = p.predictor_frame;
  return h;
}

// Bucket grid for n points.  Buckets are about one mean spacing wide
// whatever the candidate radius, so the cell order (bucket, then caller
// index) and with it every result do not depend on the radius.  First-pass
// candidates are the images within r_filter = rfac mean spacings (twice the
// farthest vertex of a cell of a jittered lattice is about 1.75 spacings);
// the stencil half-width is the number of buckets that covers r_filter.
GridParams make_grid(const mm_params& p, int64_t n, int64_t nbcap, double rfac) {
  GridParams g;
  const double vol = p.box[0] * p.box[1] * p.box[2];
  const double spacing = std::cbrt(vol / (double)n);
  g.r_filter = rfac * spacing;
  double h = spacing;
  for (;;) {
    int64_t nbt = 1;
    for (int a = 0; a < 3; ++a) {
      g.nb[a] = std::max(1, (int)std::floor(p.box[a] / h));
      nbt *= g.nb[a];
    }
    if (nbt <= nbcap) {
      g.nbt = (int)nbt;
      break;
    }
    h *= 1.1;
  }
  for (int a = 0; a < 3; ++a) {
    g.hb[a] = p.box[a] / g.nb[a];
    g.inv_hb[a] = 1.0 / g.hb[a];
    g.L[a] = p.box[a];
  }
  const double hmin = std::min(g.hb[0], std::min(g.hb[1], g.hb[2]));
  g.ring = std::max(1, (int)std::ceil(g.r_filter / hmin * (1.0 - 1e-12)));
  // Few buckets along an axis: the stencil may not exceed the axis' buckets
  // (images beyond one box length are outside the scheme's premise).
  g.ring = std::min(g.ring, std::min(g.nb[0], std::min(g.nb[1], g.nb[2])));
  return g;
}

size_t rsize(const mm_ctx* c) { return c->p.precision == MM_MIXED ? sizeof(float) : sizeof(double); }

template <typename T>
hipError_t dalloc(T** p, size_t count) {
  return hipMalloc((void**)p, std::max<size_t>(count, 1) * sizeof(T));
}

void free_all(mm_ctx* c) {
  void* ptrs[] = {c->key, c->perm, c->deferred, c->spos, c->geo, c->rmax2, c->minv, c->bcount, c->boff,
                  c->scan_tmp, c->counts, c->off, c->stage_nb, c->stage_geo, c->faces, c->csr, c->nbr, c->U, c->G, c->Uh,
                  c->Gh, c->phi, c->w, c->Qs, c->dQs, c->st};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  if (c->st_host) (void)hipHostFree(c->st_host);
  for (hipEvent_t& e : c->ev)
    if (e) (void)hipEventDestroy(e);
}

// Maps the device failure bits to a status code and a message.
mm_status check_status(mm_ctx* c, const DevStatus& s) {
  if (!s.flags) return MM_OK;
  char buf[256];
  std::snprintf(buf, sizeof buf, "device flags 0x%x (first internal cell %d)", s.flags, s.bad_cell);
  const std::string at(buf);
  if (s.flags & F_BADPOS) return fail(c, MM_EINVAL, "a position is not finite or lies outside [0, L): " + at);
  if (s.flags & F_PLANES) return fail(c, MM_ECAPACITY, "a cell has more than 64 live faces: " + at);
  if (s.flags & F_VERTS) return fail(c, MM_ECAPACITY, "a cell has more than 128 vertices: " + at);
  if (s.flags & F_CANDS) return fail(c, MM_ECAPACITY, "more than 128 neighbour candidates in a cell's stencil: " + at);
  if (s.flags & F_FACECAP) return fail(c, MM_ECAPACITY, "more unique faces than the face capacity: " + at);
  if (s.flags & F_BOX)
    return fail(c, MM_EDEGENERATE, "a cell is too large for the periodic box (needs 2 R_max < L): " + at);
  if (s.flags & F_INCOMPLETE) return fail(c, MM_EDEGENERATE, "a cell could not be completed: " + at);
  if (s.flags & F_ASYM) {
    // Name the two points of one unmatched face in the caller's numbering.
    int32_t pi = -1, pj = -1;
    if (s.asym_cell >= 0 && s.asym_nbr >= 0) {
      (void)hipMemcpy(&pi, c->perm + s.asym_cell, sizeof pi, hipMemcpyDeviceToHost);
      (void)hipMemcpy(&pj, c->perm + s.asym_nbr, sizeof pj, hipMemcpyDeviceToHost);
    }
    char pair[96];
    std::snprintf(pair, sizeof pair, "; points %d and %d", pi, pj);
    return fail(c, MM_EDEGENERATE, "asymmetric face topology (degenerate input?): " + at + pair);
  }
  if (s.flags & (F_WALK | F_VOLUME)) return fail(c, MM_EDEGENERATE, "corrupted or empty cell: " + at);
  if (s.flags & F_NONFINITE) return fail(c, MM_ENONFINITE, "a state became NaN or infinite: " + at);
  return fail(c, MM_EDEGENERATE, at);
}

mm_status readback(mm_ctx* c) {
  HIPCHECK(c, hipMemcpyAsync(c->st_host, c->st, sizeof(DevStatus), hipMemcpyDeviceToHost, c->stream));
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  return MM_OK;
}

// The first-pass radius only changes how much work goes to the shell pass,
// never the cells (clipping is always in order of distance): widen it when
// many cells were deferred, narrow it slowly when none were.
void adapt_filter(mm_ctx* c, int deferred, int64_t n) {
  if (deferred > 0.02 * (double)n) c->rfac = std::min(c->rfac * 1.15, 3.0);
  else if (deferred < 0.002 * (double)n) c->rfac = std::max(c->rfac * 0.98, 1.9);
}

void mark(mm_ctx* c, int k) {
  if (c->timing) (void)hipEventRecord(c->ev[k], c->stream);
}

// Enqueues sort, cell construction and mesh assembly for n positions.
void enqueue_tessellation(mm_ctx* c, int64_t n, const double* pos) {
  c->grid = make_grid(c->p, n, c->nbcap, c->rfac);
  mark(c, 0);
  launch_sort(pos, n, c->grid, c->bcount, c->boff, c->scan_tmp, c->key, c->perm, c->spos, c->st, c->stream);
  mark(c, 1);
  launch_tessellate(c->spos, n, c->grid, c->boff, c->stage_nb, c->stage_geo, c->counts, c->geo, c->rmax2, c->deferred, c->st,
                    c->stream);
  mark(c, 2);
  scan_u64(c->counts, c->off, n, c->scan_tmp, c->stream);
  launch_build_mesh(c->spos, c->geo, n, c->grid, c->stage_nb, c->stage_geo, c->counts, c->off, c->fcap, c->faces, c->csr, c->nbr,
                    c->minv, c->st, c->stream);
}

void fill_info(const mm_ctx* c, const DevStatus& s, mm_step_info* info, double dt_max) {
  if (!info) return;
  const double dcfl = s.dt_bits == 0x7ff0000000000000ull ? INFINITY : [&] {
    double d;
    std::memcpy(&d, &s.dt_bits, sizeof d);
    return d;
  }();
  info->dt_cfl = dcfl;
  info->dt = std::min(dcfl, dt_max);
  info->n_faces = (int64_t)s.n_faces;
  info->max_faces_cell = s.max_faces;
  info->deferred_cells = s.n_deferred;
  for (int k = 0; k < 4; ++k) info->floor_hits[k] = (int64_t)s.floor_hits[k];
  info->flags = s.flags;
  info->reserved = 0;
}

mm_status check_n(mm_ctx* c, int64_t n) {
  if (n < 1 || n > c->ncap) return fail(c, MM_EINVAL, "n must be in [1, n_capacity]");
  if (n > (1ll << 26)) return fail(c, MM_EINVAL, "n exceeds 2^26");
  return MM_OK;
}

mm_status need_mesh(mm_ctx* c) {
  if (!c->have_mesh) return fail(c, MM_ESTATE, "no tessellation: call mm_tessellate first");
  return MM_OK;
}

}  // namespace

extern "C" {

void mm_default_params(mm_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->box[0] = p->box[1] = p->box[2] = 1.0;
  p->gamma = 5.0 / 3.0;
  p->cfl = 0.3;
  p->eta = 1.0;
  p->chi = 1.0;
  p->zeta = 0.25;
  p->theta = 0.49;
  p->rho_floor = 1e-12;
  p->p_floor = 1e-14;
  p->precision = MM_FP64;
  p->riemann = MM_HLLC;
  p->limit_mask = 3;
  p->predictor_frame = 0;
}

const char* mm_version(void) { return kVersion; }

const char* mm_last_error(const mm_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_err.c_str(); }

mm_status mm_create(mm_ctx** out, const mm_params* p, int64_t n_capacity, int64_t face_capacity, void* hip_stream) {
  if (!out || !p) return create_fail(MM_EINVAL, "out or p is NULL");
  *out = nullptr;
  std::string why;
  if (!params_ok(p, why)) return create_fail(MM_EINVAL, why);
  if (n_capacity < 1 || n_capacity > (1ll << 26) || face_capacity < 0)
    return create_fail(MM_EINVAL, "n_capacity must be in [1, 2^26] and face_capacity >= 0");
  mm_ctx* c = new (std::nothrow) mm_ctx();
  if (!c) return create_fail(MM_ENOMEM, "host allocation failed");
  c->p = *p;
  c->ncap = n_capacity;
  c->fcap = face_capacity ? face_capacity : 12 * n_capacity;
  if (c->fcap > 0x7fffffffll) c->fcap = 0x7fffffffll;
  c->nbcap = n_capacity + 8;
  c->stream = (hipStream_t)hip_stream;
  {
    const hipError_t e = hipGetDevice(&c->device);
    if (e != hipSuccess) {
      delete c;
      return create_fail(MM_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    }
  }
  const int64_t N = n_capacity, F = c->fcap;
  const size_t rs = rsize(c);
  bool ok = true;
  ok &= dalloc(&c->key, N) == hipSuccess;
  ok &= dalloc(&c->perm, N) == hipSuccess;
  ok &= dalloc(&c->deferred, N) == hipSuccess;
  ok &= dalloc(&c->spos, 3 * N) == hipSuccess;
  ok &= dalloc(&c->geo, 4 * N) == hipSuccess;
  ok &= dalloc(&c->rmax2, N) == hipSuccess;
  ok &= dalloc(&c->minv, 6 * N) == hipSuccess;
  ok &= dalloc(&c->bcount, c->nbcap) == hipSuccess;
  ok &= dalloc(&c->boff, c->nbcap + 1) == hipSuccess;
  ok &= dalloc(&c->scan_tmp, scan_tmp_elems(std::max(N, c->nbcap))) == hipSuccess;
  ok &= dalloc(&c->counts, N) == hipSuccess;
  ok &= dalloc(&c->off, N + 1) == hipSuccess;
  ok &= dalloc(&c->stage_nb, (size_t)N * kMaxFaces) == hipSuccess;
  ok &= dalloc(&c->stage_geo, (size_t)N * kMaxFaces) == hipSuccess;
  ok &= dalloc(&c->faces, F) == hipSuccess;
  ok &= dalloc(&c->csr, 2 * F) == hipSuccess;
  ok &= dalloc(&c->nbr, 2 * F) == hipSuccess;
  ok &= hipMalloc(&c->U, 5 * N * rs) == hipSuccess;
  ok &= hipMalloc(&c->G, 15 * N * rs) == hipSuccess;
  ok &= hipMalloc(&c->Uh, 5 * N * rs) == hipSuccess;
  ok &= hipMalloc(&c->Gh, 15 * N * rs) == hipSuccess;
  ok &= hipMalloc(&c->phi, 5 * F * rs) == hipSuccess;
  ok &= dalloc(&c->w, 3 * N) == hipSuccess;
  ok &= dalloc(&c->Qs, 5 * N) == hipSuccess;
  ok &= dalloc(&c->dQs, 5 * N) == hipSuccess;
  ok &= dalloc(&c->st, 1) == hipSuccess;
  ok &= hipHostMalloc((void**)&c->st_host, sizeof(DevStatus), hipHostMallocDefault) == hipSuccess;
  for (hipEvent_t& e : c->ev) ok &= hipEventCreate(&e) == hipSuccess;
  if (!ok) {
    const hipError_t e = hipGetLastError();
    free_all(c);
    delete c;
    return create_fail(MM_ENOMEM, std::string("device allocation failed: ") + hipGetErrorString(e));
  }
  *out = c;
  return MM_OK;
}

mm_status mm_destroy(mm_ctx* c) {
  if (!c) return MM_EINVAL;
  (void)hipStreamSynchronize(c->stream);
  free_all(c);
  delete c;
  return MM_OK;
}

mm_status mm_set_params(mm_ctx* c, const mm_params* p) {
  if (!c || !p) return MM_EINVAL;
  std::string why;
  if (!params_ok(p, why)) return fail(c, MM_EINVAL, why);
  if (p->precision != c->p.precision) return fail(c, MM_EINVAL, "precision is fixed at mm_create");
  const bool same_box = p->box[0] == c->p.box[0] && p->box[1] == c->p.box[1] && p->box[2] == c->p.box[2];
  c->p = *p;
  if (!same_box) c->have_mesh = false;
  return MM_OK;
}

mm_status mm_tessellate(mm_ctx* c, int64_t n, const double* pos, mm_step_info* info) {
  if (!c) return MM_EINVAL;
  if (!pos) return fail(c, MM_EINVAL, "pos is NULL");
  if (mm_status r = check_n(c, n)) return r;
  c->have_mesh = false;
  launch_status_reset(c->st, c->stream);
  enqueue_tessellation(c, n, pos);
  if (mm_status r = readback(c)) return r;
  const DevStatus s = *c->st_host;
  fill_info(c, s, info, INFINITY);
  if (mm_status r = check_status(c, s)) return r;
  c->n_mesh = n;
  c->n_faces = (int64_t)s.n_faces;
  adapt_filter(c, s.n_deferred, n);
  c->have_mesh = true;
  return MM_OK;
}

mm_status mm_get_mesh_view(const mm_ctx* c, mm_mesh_view* out) {
  if (!c || !out) return MM_EINVAL;
  if (!c->have_mesh) return MM_ESTATE;
  out->n = c->n_mesh;
  out->n_faces = c->n_faces;
  out->perm = c->perm;
  out->pos = c->spos;
  out->geo = c->geo;
  out->faces = c->faces;
  return MM_OK;
}

mm_status mm_mesh_export(mm_ctx* c, double* V, double* centroid, int64_t face_cap, int32_t* face_i,
                         int32_t* face_j, int32_t* face_code, double* face_A, double* face_f, int64_t* n_faces) {
  if (!c) return MM_EINVAL;
  if (mm_status r = need_mesh(c)) return r;
  if (n_faces) *n_faces = c->n_faces;
  const bool want_faces = face_i || face_j || face_code || face_A || face_f;
  if (want_faces && face_cap < c->n_faces) return fail(c, MM_ECAPACITY, "face_cap is smaller than the face count");
  launch_export_mesh(c->n_mesh, want_faces ? c->n_faces : 0, c->perm, c->spos, c->geo, c->faces, V, centroid,
                     face_i, face_j, face_code, face_A, face_f, c->stream);
  HIPCHECK(c, hipGetLastError());
  return MM_OK;
}

mm_status mm_init_charges(mm_ctx* c, const double* prim, double* Q) {
  if (!c) return MM_EINVAL;
  if (mm_status r = need_mesh(c)) return r;
  if (!prim || !Q) return fail(c, MM_EINVAL, "prim or Q is NULL");
  launch_init_charges(hydro_params(c->p), c->n_mesh, prim, c->perm, c->geo, Q, c->stream);
  HIPCHECK(c, hipGetLastError());
  return MM_OK;
}

mm_status mm_cell_state(mm_ctx* c, const double* Q, void* U, double* w, double* dt_cfl, int64_t* floor_hits) {
  if (!c) return MM_EINVAL;
  if (mm_status r = need_mesh(c)) return r;
  if (!Q) return fail(c, MM_EINVAL, "Q is NULL");
  const int64_t n = c->n_mesh;
  launch_status_reset(c->st, c->stream);
  const HydroParams hp = hydro_params(c->p);
  if (c->p.precision == MM_MIXED) {
    launch_cell_state<float>(hp, n, Q, c->perm, c->geo, c->Qs, (float*)c->U, c->w, c->st, c->stream);
    if (U) launch_scatter_rows<float>((const float*)c->U, c->perm, n, 5, (float*)U, c->stream);
  } else {
    launch_cell_state<double>(hp, n, Q, c->perm, c->geo, c->Qs, (double*)c->U, c->w, c->st, c->stream);
    if (U) launch_scatter_rows<double>((const double*)c->U, c->perm, n, 5, (double*)U, c->stream);
  }
  if (w) launch_scatter_rows<double>(c->w, c->perm, n, 3, w, c->stream);
  if (mm_status r = readback(c)) return r;
  const DevStatus s = *c->st_host;
  mm_step_info info;
  fill_info(c, s, &info, INFINITY);
  if (dt_cfl) *dt_cfl = info.dt_cfl;
  if (floor_hits) *floor_hits = info.floor_hits[0];
  return check_status(c, s);
}

mm_status mm_gradients(mm_ctx* c, const void* U, void* grad, int32_t limit) {
  if (!c) return MM_EINVAL;
  if (mm_status r = need_mesh(c)) return r;
  if (!U || !grad) return fail(c, MM_EINVAL, "U or grad is NULL");
  const int64_t n = c->n_mesh;
  const HydroParams hp = hydro_params(c->p);
  if (c->p.precision == MM_MIXED) {
    launch_gather_rows<float>((const float*)U, c->perm, n, 5, (float*)c->U, c->stream);
    launch_gradient<float>(hp, n, (const float*)c->U, c->off, c->nbr, c->minv, limit ? 1 : 0, (float*)c->G, nullptr,
                           nullptr, 0.0, nullptr, c->st, c->stream);
    launch_scatter_rows<float>((const float*)c->G, c->perm, n, 15, (float*)grad, c->stream);
  } else {
    launch_gather_rows<double>((const double*)U, c->perm, n, 5, (double*)c->U, c->stream);
    launch_gradient<double>(hp, n, (const double*)c->U, c->off, c->nbr, c->minv, limit ? 1 : 0, (double*)c->G,
                            nullptr, nullptr, 0.0, nullptr, c->st, c->stream);
    launch_scatter_rows<double>((const double*)c->G, c->perm, n, 15, (double*)grad, c->stream);
  }
  HIPCHECK(c, hipGetLastError());
  return MM_OK;
}

mm_status mm_predict(mm_ctx* c, const void* U, const void* grad, const double* w, double dt, void* U_half) {
  if (!c) return MM_EINVAL;
  if (mm_status r = need_mesh(c)) return r;
  if (!U || !grad || !w || !U_half) return fail(c, MM_EINVAL, "NULL argument");
  if (!(dt >= 0.0 && std::isfinite(dt))) return fail(c, MM_EINVAL, "dt must be finite and >= 0");
  const int64_t n = c->n_mesh;
  const HydroParams hp = hydro_params(c->p);
  launch_gather_rows<double>(w, c->perm, n, 3, c->w, c->stream);
  if (c->p.precision == MM_MIXED) {
    launch_gather_rows<float>((const float*)U, c->perm, n, 5, (float*)c->U, c->stream);
    launch_gather_rows<float>((const float*)grad, c->perm, n, 15, (float*)c->G, c->stream);
    launch_predict<float>(hp, n, (const float*)c->U, (const float*)c->G, c->w, nullptr, dt, (float*)c->Uh, c->st,
                          c->stream);
    launch_scatter_rows<float>((const float*)c->Uh, c->perm, n, 5, (float*)U_half, c->stream);
  } else {
    launch_gather_rows<double>((const double*)U, c->perm, n, 5, (double*)c->U, c->stream);
    launch_gather_rows<double>((const double*)grad, c->perm, n, 15, (double*)c->G, c->stream);
    launch_predict<double>(hp, n, (const double*)c->U, (const double*)c->G, c->w, nullptr, dt, (double*)c->Uh,
                           c->st, c->stream);
    launch_scatter_rows<double>((const double*)c->Uh, c->perm, n, 5, (double*)U_half, c->stream);
  }
  HIPCHECK(c, hipGetLastError());
  return MM_OK;
}

mm_status mm_fluxes(mm_ctx* c, const void* U_half, const void* grad_half, const double* w, double dt, double* dQ) {
  if (!c) return MM_EINVAL;
  if (mm_status r = need_mesh(c)) return r;
  if (!U_half || !grad_half || !w || !dQ) return fail(c, MM_EINVAL, "NULL argument");
  if (!(dt >= 0.0 && std::isfinite(dt))) return fail(c, MM_EINVAL, "dt must be finite and >= 0");
  const int64_t n = c->n_mesh;
  const HydroParams hp = hydro_params(c->p);
  launch_gather_rows<double>(w, c->perm, n, 3, c->w, c->stream);
  if (c->p.precision == MM_MIXED) {
    launch_gather_rows<float>((const float*)U_half, c->perm, n, 5, (float*)c->Uh, c->stream);
    launch_gather_rows<float>((const float*)grad_half, c->perm, n, 15, (float*)c->Gh, c->stream);
    launch_flux<float>(hp, c->n_faces, nullptr, c->faces, c->spos, c->geo, (const float*)c->Uh, (const float*)c->Gh,
                       c->w, nullptr, dt, (float*)c->phi, c->st, c->stream);
    launch_accumulate<float>(n, c->off, c->csr, (const float*)c->phi, c->perm, dQ, c->stream);
  } else {
    launch_gather_rows<double>((const double*)U_half, c->perm, n, 5, (double*)c->Uh, c->stream);
    launch_gather_rows<double>((const double*)grad_half, c->perm, n, 15, (double*)c->Gh, c->stream);
    launch_flux<double>(hp, c->n_faces, nullptr, c->faces, c->spos, c->geo, (const double*)c->Uh,
                        (const double*)c->Gh, c->w, nullptr, dt, (double*)c->phi, c->st, c->stream);
    launch_accumulate<double>(n, c->off, c->csr, (const double*)c->phi, c->perm, dQ, c->stream);
  }
  HIPCHECK(c, hipGetLastError());
  return MM_OK;
}

mm_status mm_step(mm_ctx* c, int64_t n, double* pos, double* w, double* Q, double dt_max, mm_step_info* info) {
  if (!c) return MM_EINVAL;
  if (!pos || !w || !Q) return fail(c, MM_EINVAL, "pos, w or Q is NULL");
  if (mm_status r = check_n(c, n)) return r;
  if (!(dt_max > 0.0)) return fail(c, MM_EINVAL, "dt_max must be positive");
  c->have_mesh = false;
  const HydroParams hp = hydro_params(c->p);
  launch_status_reset(c->st, c->stream);
  enqueue_tessellation(c, n, pos);
  mark(c, 3);
  // Upper bound of the face count for the flux launch; the kernel reads the
  // exact count on the device.
  const int64_t fbound = c->fcap;
  const unsigned long long* nf_dev = &c->st->n_faces;
  const int lim0 = hp.limit_mask & 1, lim1 = (hp.limit_mask >> 1) & 1;
  if (c->p.precision == MM_MIXED) {
    float *U = (float*)c->U, *Uh = (float*)c->Uh, *Gh = (float*)c->Gh, *phi = (float*)c->phi;
    launch_cell_state<float>(hp, n, Q, c->perm, c->geo, c->Qs, U, c->w, c->st, c->stream);
    mark(c, 4);
    launch_gradient<float>(hp, n, U, c->off, c->nbr, c->minv, lim0, nullptr, c->w, c->st, dt_max, Uh, c->st,
                           c->stream);
    mark(c, 5);
    launch_gradient<float>(hp, n, Uh, c->off, c->nbr, c->minv, lim1, Gh, nullptr, nullptr, 0.0, nullptr, c->st,
                           c->stream);
    mark(c, 6);
    launch_flux<float>(hp, fbound, nf_dev, c->faces, c->spos, c->geo, Uh, Gh, c->w, c->st, dt_max, phi, c->st,
                       c->stream);
    mark(c, 7);
    launch_update<float>(hp, n, c->off, c->csr, phi, c->geo, c->perm, c->Qs, Q, c->spos, c->w, pos, w, c->st, dt_max,
                         c->st, c->stream);
  } else {
    double *U = (double*)c->U, *Uh = (double*)c->Uh, *Gh = (double*)c->Gh, *phi = (double*)c->phi;
    launch_cell_state<double>(hp, n, Q, c->perm, c->geo, c->Qs, U, c->w, c->st, c->stream);
    mark(c, 4);
    launch_gradient<double>(hp, n, U, c->off, c->nbr, c->minv, lim0, nullptr, c->w, c->st, dt_max, Uh, c->st,
                            c->stream);
    mark(c, 5);
    launch_gradient<double>(hp, n, Uh, c->off, c->nbr, c->minv, lim1, Gh, nullptr, nullptr, 0.0, nullptr, c->st,
                            c->stream);
    mark(c, 6);
    launch_flux<double>(hp, fbound, nf_dev, c->faces, c->spos, c->geo, Uh, Gh, c->w, c->st, dt_max, phi, c->st,
                        c->stream);
    mark(c, 7);
    launch_update<double>(hp, n, c->off, c->csr, phi, c->geo, c->perm, c->Qs, Q, c->spos, c->w, pos, w, c->st,
                          dt_max, c->st, c->stream);
  }
  mark(c, 8);
  HIPCHECK(c, hipGetLastError());
  if (mm_status r = readback(c)) return r;
  const DevStatus s = *c->st_host;
  fill_info(c, s, info, dt_max);
  if (c->timing) {
    for (int k = 0; k < 8; ++k) {
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, c->ev[k], c->ev[k + 1]);
      c->stage_ms[k] = ms;
    }
  }
  if (mm_status r = check_status(c, s)) return r;
  c->n_mesh = n;
  c->n_faces = (int64_t)s.n_faces;
  adapt_filter(c, s.n_deferred, n);
  c->have_mesh = true;
  return MM_OK;
}

mm_status mm_set_stage_timing(mm_ctx* c, int32_t enable) {
  if (!c) return MM_EINVAL;
  c->timing = enable != 0;
  return MM_OK;
}

mm_status mm_get_stage_ms(const mm_ctx* c, double* ms, int32_t n_stages) {
  if (!c || !ms || n_stages < 0) return MM_EINVAL;
  for (int k = 0; k < std::min(n_stages, 8); ++k) ms[k] = c->stage_ms[k];
  return MM_OK;
}

}  // extern "C"
