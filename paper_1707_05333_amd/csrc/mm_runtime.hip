// Host runtime of the one-simulation interface of include/mm.h: a context
// owns one engine (all device memory reserved at creation) whose segment
// table holds a single segment; this file validates arguments, enqueues the
// work of each call and reads the status back once per call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "../../include/mm.h"
#include "mm_engine.h"
#include "mm_internal.h"

using namespace mm;

struct mm_ctx {
  mm_params p{};
  Engine E;
  bool have_mesh = false;
  GridParams grid{};
  std::string err;
};

namespace {

const char* kVersion = "mm-mi355x 0.2 (gfx950)";

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

// Writes the single segment descriptor (grid of the last sort, parameters,
// dt cap) and uploads it.
mm_status put_segment(mm_ctx* c, double dt_max) {
  SegDesc* d = c->E.staging();
  d[0].g = c->grid;
  d[0].hp = hydro_params(c->p);
  d[0].dt_max = dt_max;
  d[0].fresh = 0;
  d[0].pad = 0;
  if (mm_status r = c->E.upload(1)) return fail(c, r, c->E.err);
  return MM_OK;
}

mm_status readback(mm_ctx* c) {
  if (mm_status r = c->E.readback()) return fail(c, r, c->E.err);
  return MM_OK;
}

mm_status check_status(mm_ctx* c) {
  std::string msg;
  const DevStatus& s = *c->E.st_host;
  const mm_status r = c->E.check_flags(s.flags, s.bad_cell, msg);
  return r ? fail(c, r, msg) : MM_OK;
}

void fill_info(const mm_ctx* c, mm_step_info* info, double dt_max) {
  if (!info) return;
  const DevStatus& s = *c->E.st_host;
  const SegStatus& g = c->E.segst_host[0];
  const double dcfl = dt_from_bits(g.dt_bits);
  info->dt_cfl = dcfl;
  info->dt = std::min(dcfl, dt_max);
  info->n_faces = (int64_t)s.n_faces;
  info->max_faces_cell = s.max_faces;
  info->deferred_cells = s.n_deferred;
  for (int k = 0; k < 4; ++k) info->floor_hits[k] = (int64_t)g.floor_hits[k];
  info->flags = s.flags;
  info->rebuilt_cells = s.n_redo + s.n_dredo;
}

mm_status check_n(mm_ctx* c, int64_t n) {
  if (n < 1 || n > c->E.ncap) return fail(c, MM_EINVAL, "n must be in [1, n_capacity]");
  return MM_OK;
}

mm_status need_mesh(mm_ctx* c) {
  if (!c->have_mesh) return fail(c, MM_ESTATE, "no tessellation: call mm_tessellate first");
  return MM_OK;
}

// Grid, segment upload, status reset and the tessellation of n positions.
mm_status start_tessellation(mm_ctx* c, int64_t n, const double* pos, double dt_max) {
  c->grid = make_grid(c->p, n, c->E.rfac, 0);
  if (mm_status r = put_segment(c, dt_max)) return r;
  c->E.n = n;
  c->E.reset_status();
  return MM_OK;
}

void finish_mesh(mm_ctx* c, int64_t n) {
  c->E.n = n;
  c->E.n_faces = (int64_t)c->E.st_host->n_faces;
  c->have_mesh = true;
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
  const int64_t fcap = face_capacity ? face_capacity : kFacesPerCell * n_capacity;
  if (mm_status r = c->E.init(p->precision, n_capacity, n_capacity, fcap, 1, (hipStream_t)hip_stream, true)) {
    const std::string msg = c->E.err;
    delete c;
    return create_fail(r, msg);
  }
  *out = c;
  return MM_OK;
}

mm_status mm_destroy(mm_ctx* c) {
  if (!c) return MM_EINVAL;
  (void)hipStreamSynchronize(c->E.stream);
  c->E.release();
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
  if (c->have_mesh) return put_segment(c, INFINITY);
  return MM_OK;
}

mm_status mm_tessellate(mm_ctx* c, int64_t n, const double* pos, mm_step_info* info) {
  if (!c) return MM_EINVAL;
  if (!pos) return fail(c, MM_EINVAL, "pos is NULL");
  if (mm_status r = check_n(c, n)) return r;
  c->have_mesh = false;
  if (mm_status r = start_tessellation(c, n, pos, INFINITY)) return r;
  c->E.enqueue_tessellation(pos, n, nullptr, n, c->grid.nbt);
  if (mm_status r = readback(c)) return r;
  fill_info(c, info, INFINITY);
  if (mm_status r = check_status(c)) return r;
  finish_mesh(c, n);
  return MM_OK;
}

mm_status mm_get_mesh_view(const mm_ctx* c, mm_mesh_view* out) {
  if (!c || !out) return MM_EINVAL;
  if (!c->have_mesh) return MM_ESTATE;
  out->n = c->E.n;
  out->n_faces = c->E.n_faces;
  out->perm = c->E.perm;
  out->pos = c->E.spos;
  out->geo = c->E.geo;
  out->faces = c->E.faces;
  return MM_OK;
}

mm_status mm_mesh_export(mm_ctx* c, double* V, double* centroid, int64_t face_cap, int32_t* face_i,
                         int32_t* face_j, int32_t* face_code, double* face_A, double* face_f, int64_t* n_faces) {
  if (!c) return MM_EINVAL;
  if (mm_status r = need_mesh(c)) return r;
  if (n_faces) *n_faces = c->E.n_faces;
  const bool want_faces = face_i || face_j || face_code || face_A || face_f;
  if (want_faces && face_cap < c->E.n_faces) return fail(c, MM_ECAPACITY, "face_cap is smaller than the face count");
  launch_export_mesh(c->E.n, want_faces ? c->E.n_faces : 0, c->E.perm, c->E.spos, c->E.geo, c->E.faces, V, centroid,
                     face_i, face_j, face_code, face_A, face_f, c->E.stream);
  HIPCHECK(c, hipGetLastError());
  return MM_OK;
}

mm_status mm_init_charges(mm_ctx* c, const double* prim, double* Q) {
  if (!c) return MM_EINVAL;
  if (mm_status r = need_mesh(c)) return r;
  if (!prim || !Q) return fail(c, MM_EINVAL, "prim or Q is NULL");
  launch_init_charges(c->E.segs, c->E.sseg, c->E.n, prim, c->E.perm, c->E.geo, Q, 0, c->E.stream);
  HIPCHECK(c, hipGetLastError());
  return MM_OK;
}

mm_status mm_cell_state(mm_ctx* c, const double* Q, void* U, double* w, double* dt_cfl, int64_t* floor_hits) {
  if (!c) return MM_EINVAL;
  if (mm_status r = need_mesh(c)) return r;
  if (!Q) return fail(c, MM_EINVAL, "Q is NULL");
  Engine& E = c->E;
  const int64_t n = E.n;
  E.reset_status();
  if (c->p.precision == MM_MIXED) {
    launch_cell_state<float>(E.segs, E.sseg, n, Q, E.perm, E.geo, E.Qs, (float*)E.U, E.w, E.st, E.segst, E.stream);
    if (U) launch_scatter_rows<float>((const float*)E.U, E.perm, n, 5, (float*)U, E.stream);
  } else {
    launch_cell_state<double>(E.segs, E.sseg, n, Q, E.perm, E.geo, E.Qs, (double*)E.U, E.w, E.st, E.segst,
                              E.stream);
    if (U) launch_scatter_rows<double>((const double*)E.U, E.perm, n, 5, (double*)U, E.stream);
  }
  if (w) launch_scatter_rows<double>(E.w, E.perm, n, 3, w, E.stream);
  if (mm_status r = readback(c)) return r;
  mm_step_info info;
  fill_info(c, &info, INFINITY);
  if (dt_cfl) *dt_cfl = info.dt_cfl;
  if (floor_hits) *floor_hits = info.floor_hits[0];
  return check_status(c);
}

mm_status mm_gradients(mm_ctx* c, const void* U, void* grad, int32_t limit) {
  if (!c) return MM_EINVAL;
  if (mm_status r = need_mesh(c)) return r;
  if (!U || !grad) return fail(c, MM_EINVAL, "U or grad is NULL");
  Engine& E = c->E;
  const int64_t n = E.n;
  const int lim = limit ? kLimitOn : kLimitOff;
  if (c->p.precision == MM_MIXED) {
    launch_gather_rows<float>((const float*)U, E.perm, n, 5, (float*)E.U, E.stream);
    launch_gradient<float>(E.segs, E.sseg, n, (const float*)E.U, E.counts, E.soff, (const NbrEntry<float>*)E.nbr, E.minv, lim, (float*)E.G, nullptr,
                           nullptr, 0.0, nullptr, nullptr, nullptr, nullptr, E.segst, E.stream);
    launch_scatter_rows<float>((const float*)E.G, E.perm, n, 15, (float*)grad, E.stream);
  } else {
    launch_gather_rows<double>((const double*)U, E.perm, n, 5, (double*)E.U, E.stream);
    launch_gradient<double>(E.segs, E.sseg, n, (const double*)E.U, E.counts, E.soff, (const NbrEntry<double>*)E.nbr, E.minv, lim, (double*)E.G,
                            nullptr, nullptr, 0.0, nullptr, nullptr, nullptr, nullptr, E.segst, E.stream);
    launch_scatter_rows<double>((const double*)E.G, E.perm, n, 15, (double*)grad, E.stream);
  }
  HIPCHECK(c, hipGetLastError());
  return MM_OK;
}

mm_status mm_predict(mm_ctx* c, const void* U, const void* grad, const double* w, double dt, void* U_half) {
  if (!c) return MM_EINVAL;
  if (mm_status r = need_mesh(c)) return r;
  if (!U || !grad || !w || !U_half) return fail(c, MM_EINVAL, "NULL argument");
  if (!(dt >= 0.0 && std::isfinite(dt))) return fail(c, MM_EINVAL, "dt must be finite and >= 0");
  Engine& E = c->E;
  const int64_t n = E.n;
  launch_gather_rows<double>(w, E.perm, n, 3, E.w, E.stream);
  if (c->p.precision == MM_MIXED) {
    launch_gather_rows<float>((const float*)U, E.perm, n, 5, (float*)E.U, E.stream);
    launch_gather_rows<float>((const float*)grad, E.perm, n, 15, (float*)E.G, E.stream);
    launch_predict<float>(E.segs, E.sseg, n, (const float*)E.U, (const float*)E.G, E.w, nullptr, dt, (float*)E.Uh,
                          E.segst, E.stream);
    launch_scatter_rows<float>((const float*)E.Uh, E.perm, n, 5, (float*)U_half, E.stream);
  } else {
    launch_gather_rows<double>((const double*)U, E.perm, n, 5, (double*)E.U, E.stream);
    launch_gather_rows<double>((const double*)grad, E.perm, n, 15, (double*)E.G, E.stream);
    launch_predict<double>(E.segs, E.sseg, n, (const double*)E.U, (const double*)E.G, E.w, nullptr, dt,
                           (double*)E.Uh, E.segst, E.stream);
    launch_scatter_rows<double>((const double*)E.Uh, E.perm, n, 5, (double*)U_half, E.stream);
  }
  HIPCHECK(c, hipGetLastError());
  return MM_OK;
}

mm_status mm_fluxes(mm_ctx* c, const void* U_half, const void* grad_half, const double* w, double dt, double* dQ) {
  if (!c) return MM_EINVAL;
  if (mm_status r = need_mesh(c)) return r;
  if (!U_half || !grad_half || !w || !dQ) return fail(c, MM_EINVAL, "NULL argument");
  if (!(dt >= 0.0 && std::isfinite(dt))) return fail(c, MM_EINVAL, "dt must be finite and >= 0");
  Engine& E = c->E;
  const int64_t n = E.n;
  launch_gather_rows<double>(w, E.perm, n, 3, E.w, E.stream);
  if (c->p.precision == MM_MIXED) {
    launch_gather_rows<float>((const float*)U_half, E.perm, n, 5, (float*)E.Uh, E.stream);
    launch_gather_rows<float>((const float*)grad_half, E.perm, n, 15, (float*)E.G, E.stream);
    launch_pack_flux_cells<float>(n, (const float*)E.Uh, (const float*)E.G, E.w, E.geo, E.spos,
                                  (FluxCell<float>*)E.rec, E.stream);
    launch_flux<float>(E.segs, E.n_faces, nullptr, E.faces, (const FluxCell<float>*)E.rec, nullptr, dt,
                       (float*)E.phi, E.segst, E.stream);
    launch_accumulate<float>(n, E.counts, E.soff, E.csr, (const float*)E.phi, E.perm, dQ, E.stream);
  } else {
    launch_gather_rows<double>((const double*)U_half, E.perm, n, 5, (double*)E.Uh, E.stream);
    launch_gather_rows<double>((const double*)grad_half, E.perm, n, 15, (double*)E.G, E.stream);
    launch_pack_flux_cells<double>(n, (const double*)E.Uh, (const double*)E.G, E.w, E.geo, E.spos,
                                   (FluxCell<double>*)E.rec, E.stream);
    launch_flux<double>(E.segs, E.n_faces, nullptr, E.faces, (const FluxCell<double>*)E.rec, nullptr, dt,
                        (double*)E.phi, E.segst, E.stream);
    launch_accumulate<double>(n, E.counts, E.soff, E.csr, (const double*)E.phi, E.perm, dQ, E.stream);
  }
  HIPCHECK(c, hipGetLastError());
  return MM_OK;
}

static mm_status step_common(mm_ctx* c, int64_t n, double* pos, double* w, double* Q, double* S, float* mach,
                             double dt_max, mm_step_info* info) {
  if (!pos || !w || !Q) return fail(c, MM_EINVAL, "pos, w or Q is NULL");
  if (mm_status r = check_n(c, n)) return r;
  if (!(dt_max > 0.0)) return fail(c, MM_EINVAL, "dt_max must be positive");
  c->have_mesh = false;
  c->grid = make_grid(c->p, n, c->E.rfac, 0);
  if (mm_status r = put_segment(c, dt_max)) return r;
  c->E.n = n;
  c->E.enqueue_step(pos, w, Q, n, nullptr, n, c->grid.nbt, false, c->p.half_step_mesh != 0, S, mach);
  if (mm_status r = readback(c)) return r;
  fill_info(c, info, dt_max);
  c->E.finish_timing();
  if (mm_status r = check_status(c)) return r;
  finish_mesh(c, n);
  return MM_OK;
}

mm_status mm_step(mm_ctx* c, int64_t n, double* pos, double* w, double* Q, double dt_max, mm_step_info* info) {
  if (!c) return MM_EINVAL;
  if (c->p.mach_threshold > 0.0) return fail(c, MM_EINVAL, "mach_threshold > 0 needs mm_step_entropy");
  return step_common(c, n, pos, w, Q, nullptr, nullptr, dt_max, info);
}

mm_status mm_step_entropy(mm_ctx* c, int64_t n, double* pos, double* w, double* Q, double* S, float* mach,
                          double dt_max, mm_step_info* info) {
  if (!c) return MM_EINVAL;
  if (!S) return fail(c, MM_EINVAL, "S is NULL");
  if (c->p.half_step_mesh) return fail(c, MM_EINVAL, "the entropy column is not combined with half_step_mesh");
  return step_common(c, n, pos, w, Q, S, mach, dt_max, info);
}

mm_status mm_init_entropy(mm_ctx* c, const double* prim, double* S) {
  if (!c) return MM_EINVAL;
  if (mm_status r = need_mesh(c)) return r;
  if (!prim || !S) return fail(c, MM_EINVAL, "prim or S is NULL");
  launch_init_entropy(c->E.segs, c->E.sseg, c->E.n, prim, c->E.perm, c->E.geo, S, c->E.stream);
  HIPCHECK(c, hipGetLastError());
  return MM_OK;
}

// ---------------------------------------------------------------------------
// The allocation-free step.  Its buffers live in one file-scope device array
// per GPU, of fixed size; host code reaches that array only through the
// device address hipGetSymbolAddress gives for the current device (the
// array's name is a host-side stand-in, not a device address).
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {

constexpr int64_t kStaticPoints = MM_STATIC_MAX_POINTS;
constexpr int64_t kStaticFaces = kFacesPerCell * kStaticPoints;
constexpr size_t kScratchBytes = 64ull << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_static_mu;
void* g_scratch_dev[kMaxDevices];          // device address of scratch, per device (set once)
mm_ctx g_static_ctx[kMaxDevices];          // one context per device, carved from its scratch
SegDesc g_static_seg[kMaxDevices];         // host mirrors of the one segment and its status
SegStatus g_static_segst[kMaxDevices];
DevStatus g_static_st[kMaxDevices];

mm_status static_fail(mm_status code, const std::string& msg) {
  g_create_err = msg;
  return code;
}

}  // namespace

extern "C" {

mm_status mm_step_static(const mm_params* p, int64_t n, double* pos, double* w, double* Q, double dt_max,
                         mm_step_info* info, void* hip_stream) {
  if (!p) return static_fail(MM_EINVAL, "p is NULL");
  std::string why;
  if (!params_ok(p, why)) return static_fail(MM_EINVAL, why);
  if (p->half_step_mesh) return static_fail(MM_EINVAL, "mm_step_static does not take half_step_mesh = 1");
  if (p->mach_threshold > 0.0) return static_fail(MM_EINVAL, "mm_step_static does not take the entropy switch");
  if (n < 1 || n > kStaticPoints)
    return static_fail(MM_EINVAL, "n must be in [1, MM_STATIC_MAX_POINTS = " + std::to_string(kStaticPoints) + "]");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return static_fail(MM_EHIP, "no usable current device");
  {
    // Once per device, with that device current: the device address of its
    // copy of the scratch array.
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_scratch_dev[dev]) {
      void* ptr = nullptr;
      const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr)
        return static_fail(MM_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      const size_t need = std::max(Engine::arena_bytes(MM_FP64, kStaticPoints, kStaticFaces),
                                   Engine::arena_bytes(MM_MIXED, kStaticPoints, kStaticFaces));
      if (need > kScratchBytes) return static_fail(MM_ECAPACITY, "scratch array smaller than its buffers");
      g_scratch_dev[dev] = ptr;
    }
  }
  // The context is carved anew each call (pointer arithmetic only), so each
  // call may bring its own parameters, precision and stream.
  mm_ctx* c = &g_static_ctx[dev];
  c->p = *p;
  c->have_mesh = false;
  if (mm_status r = c->E.init_arena(p->precision, kStaticPoints, kStaticFaces, g_scratch_dev[dev], kScratchBytes,
                                    &g_static_seg[dev], &g_static_segst[dev], &g_static_st[dev],
                                    (hipStream_t)hip_stream))
    return static_fail(r, c->E.err);
  const mm_status r = step_common(c, n, pos, w, Q, nullptr, nullptr, dt_max, info);
  if (r != MM_OK) g_create_err = c->err;
  return r;
}

mm_status mm_set_stage_timing(mm_ctx* c, int32_t enable) {
  if (!c) return MM_EINVAL;
  c->E.timing = enable != 0;
  return MM_OK;
}

mm_status mm_get_stage_ms(const mm_ctx* c, double* ms, int32_t n_stages) {
  if (!c || !ms || n_stages < 0) return MM_EINVAL;
  for (int k = 0; k < std::min(n_stages, 9); ++k) ms[k] = c->E.stage_ms[k];
  return MM_OK;
}

}  // extern "C"
