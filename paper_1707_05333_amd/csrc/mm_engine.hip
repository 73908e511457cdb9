// Engine: device memory of the internal cell space, segment table, enqueue
// order of a tessellation and of a step, status readback.
#include "mm_engine.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

namespace mm {

namespace {

// Hands out the engine's device buffers: from hipMalloc, or carved from one
// arena by a bump pointer (256-byte aligned, no allocation), or only counted
// (no base: the bytes an arena must hold).
struct Reserver {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  bool arena = false, ok = true;
  template <typename T>
  void operator()(T** p, size_t count) {
    bytes((void**)p, std::max<size_t>(count, 1) * sizeof(T));
  }
  void bytes(void** p, size_t b) {
    b = std::max<size_t>(b, 1);
    if (!arena) {
      ok &= hipMalloc(p, b) == hipSuccess;
      return;
    }
    const size_t at = (used + 255) & ~size_t(255);
    used = at + b;
    if (!base || used > cap) {
      *p = nullptr;
      ok &= base == nullptr;   // counting only
      return;
    }
    *p = base + at;
  }
};

__global__ void k_put_segment(SegDesc d, SegDesc* dst) {
  if (threadIdx.x == 0) *dst = d;
}

}  // namespace

int64_t engine_bytes_per_cell(int precision) {
  const int64_t r = precision == MM_MIXED ? 4 : 8;
  const int64_t per_cell = 4 * 6                                       // key, perm, sseg, deferred, dcells, redo
                           + 8 * (3 + 4 + 1 + 6 + 1 + 1)               // spos, geo, rmax2, minv, counts, off
                           + 16 + 8 + 4                                // bucket count, offset, sub-table base; sub-offsets
                           + (int64_t)kMaxFaces * (sizeof(StageNbr) + sizeof(StageGeo))
                           + kListPerCell * (4 + (r == 4 ? sizeof(NbrEntry<float>) : sizeof(NbrEntry<double>)))
                           + r * (5 + 15 + 5) + 8 * (3 + 5 + 3)        // U, G, Uh, w, Qs, pn
                           + (r == 4 ? sizeof(FluxCell<float>) : sizeof(FluxCell<double>));
  const int64_t per_face = sizeof(Face) + 5 * r;                       // face, phi
  return per_cell + kFacesPerCell * per_face;
}

GridParams make_grid(const mm_params& p, int64_t n, double rfac, int64_t base) {
  GridParams g{};
  const double vol = p.box[0] * p.box[1] * p.box[2];
  const double spacing = std::cbrt(vol / (double)n);
  g.r_filter = rfac * spacing;
  // At most n + 8 buckets per segment (the shared table is sized for it).
  double h = spacing;
  for (;;) {
    int64_t nbt = 1;
    for (int a = 0; a < 3; ++a) {
      g.nb[a] = std::max(1, (int)std::floor(p.box[a] / h));
      nbt *= g.nb[a];
    }
    if (nbt <= n + 8) {
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
  g.pad = 0;
  g.ppb = (double)n / (double)g.nbt;
  g.base = base;
  return g;
}

static_assert(MM_HLLC == kRiemannHllc && MM_HLL == kRiemannHll, "solver codes of the interface and the kernels");

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
  h.riemann = p.riemann;
  h.pad = 0;
  h.mach_threshold = p.mach_threshold;
  return h;
}

bool params_ok(const mm_params* p, std::string& why) {
  for (int a = 0; a < 3; ++a)
    if (!(std::isfinite(p->box[a]) && p->box[a] > 0)) { why = "box lengths must be finite and positive"; return false; }
  if (!(p->gamma > 1.0 && std::isfinite(p->gamma))) { why = "gamma must exceed 1"; return false; }
  if (!(p->cfl > 0.0)) { why = "cfl must be positive"; return false; }
  if (!(p->zeta > 0.0)) { why = "zeta must be positive"; return false; }
  if (!(p->rho_floor > 0.0 && p->p_floor > 0.0)) { why = "floors must be positive"; return false; }
  if (p->precision != MM_FP64 && p->precision != MM_MIXED) { why = "precision must be MM_FP64 or MM_MIXED"; return false; }
  if (p->riemann != MM_HLLC && p->riemann != MM_HLL) { why = "riemann must be MM_HLLC or MM_HLL"; return false; }
  if (p->limit_mask < 0 || p->limit_mask > 3) { why = "limit_mask must be in 0..3"; return false; }
  if (p->predictor_frame != 0 && p->predictor_frame != 1) { why = "predictor_frame must be 0 or 1"; return false; }
  if (p->half_step_mesh != 0 && p->half_step_mesh != 1) { why = "half_step_mesh must be 0 or 1"; return false; }
  if (p->reserved != 0) { why = "reserved must be 0"; return false; }
  if (!(p->mach_threshold >= 0.0 && std::isfinite(p->mach_threshold))) {
    why = "mach_threshold must be finite and non-negative";
    return false;
  }
  return true;
}

double dt_from_bits(unsigned long long bits) {
  if (bits == 0x7ff0000000000000ull) return INFINITY;
  double d;
  std::memcpy(&d, &bits, sizeof d);
  return d;
}

// Every device buffer of the engine, in one list for both ways of
// reserving them.
template <typename Res>
void reserve_buffers(Engine& E, Res& R, bool single) {
  const int64_t N = E.ncap, F = E.fcap, slot_cap = E.slot_cap, nbcap = E.nbcap, sell_cap = E.sell_cap;
  const int precision = E.precision, segcap = E.segcap;
  const size_t rs = precision == MM_MIXED ? sizeof(float) : sizeof(double);
  R(&E.key, slot_cap);
  R(&E.perm, N);
  R(&E.sseg, N);
  R(&E.deferred, N);
  R(&E.dcells, N);
  R(&E.redo, N);
  R(&E.spos, 3 * N);
  R(&E.geo, 4 * N);
  R(&E.rmax2, N);
  R(&E.minv, 6 * N);
  R(&E.bcount, nbcap);
  R(&E.boff, nbcap + 1);
  R(&E.sbase, nbcap + 1);
  R(&E.soffs, N);
  R(&E.scan_tmp, scan_tmp_elems(std::max(N, nbcap)));
  R(&E.counts, N);
  R(&E.off, N + 1);
  R(&E.sw, (N + 63) / 64 + 1);
  R(&E.soff, (N + 63) / 64 + 2);
  R(&E.stage_nb, (size_t)N * kMaxFaces);
  R(&E.stage_geo, (size_t)N * kMaxFaces);
  R(&E.faces, F);
  R(&E.csr, sell_cap);
  R.bytes(&E.nbr, sell_cap * (precision == MM_MIXED ? sizeof(NbrEntry<float>)
                                                                            : sizeof(NbrEntry<double>)));
  R.bytes(&E.U, 5 * N * rs);
  R.bytes(&E.G, 15 * N * rs);
  R.bytes(&E.Uh, 5 * N * rs);
  R.bytes(&E.rec, N * (precision == MM_MIXED ? sizeof(FluxCell<float>)
                                                                       : sizeof(FluxCell<double>)));
  R.bytes(&E.phi, 5 * F * rs);
  R(&E.w, 3 * N);
  R(&E.Qs, 5 * N);
  R(&E.pn, 3 * N);
  if (single) {
    R(&E.pos_half, 3 * slot_cap);
    R.bytes(&E.Uh_slots, 5 * slot_cap * rs);
    R.bytes(&E.Xe, N * rs);
    R.bytes(&E.Xh, N * rs);
    R.bytes(&E.recx, N * 4 * rs);
    R.bytes(&E.phiX, F * rs);
    R(&E.machF, F);
    R(&E.machs, N);
    R(&E.Ss, N);
  }
  R(&E.segs, segcap);
  R(&E.segst, segcap);
  R(&E.st, 1);
}

void Engine::set_capacity(int prec, int64_t n_cap, int64_t s_cap, int64_t f_cap, int seg_cap) {
  precision = prec;
  ncap = n_cap;
  slot_cap = s_cap;
  fcap = std::min<int64_t>(f_cap, 0x7fffffffll);
  segcap = seg_cap;
  nbcap = ncap + 8ll * segcap;
  sell_cap = kListPerCell * ((ncap + 63) / 64) * 64;   // whole slices of 64 cells
}

size_t Engine::arena_bytes(int prec, int64_t n_cap, int64_t f_cap) {
  Engine E;
  E.set_capacity(prec, n_cap, n_cap, f_cap, 1);
  Reserver R;
  R.arena = true;   // no base: counts the bytes
  reserve_buffers(E, R, false);
  return R.used;
}

mm_status Engine::init_arena(int prec, int64_t n_cap, int64_t f_cap, void* arena, size_t bytes, SegDesc* seg_host,
                             SegStatus* seg_status_host, DevStatus* status_host, hipStream_t s) {
  *this = Engine();
  set_capacity(prec, n_cap, n_cap, f_cap, 1);
  stream = s;
  arena_mode = true;
  if (hipGetDevice(&device) != hipSuccess) return fail(MM_EHIP, "hipGetDevice failed");
  Reserver R;
  R.arena = true;
  R.base = (char*)arena;
  R.cap = bytes;
  reserve_buffers(*this, R, false);
  if (!R.ok || !arena) return fail(MM_ECAPACITY, "the buffers do not fit the arena");
  segs_host = seg_host;
  segst_host = seg_status_host;
  st_host = status_host;
  return MM_OK;
}

mm_status Engine::init(int prec, int64_t n_cap, int64_t s_cap, int64_t f_cap, int seg_cap, hipStream_t s,
                       bool single) {
  set_capacity(prec, n_cap, s_cap, f_cap, seg_cap);
  stream = s;
  if (hipGetDevice(&device) != hipSuccess) return fail(MM_EHIP, "hipGetDevice failed");
  Reserver R;
  reserve_buffers(*this, R, single);
  bool ok = R.ok;
  ok &= hipHostMalloc((void**)&segs_host, sizeof(SegDesc) * segcap, hipHostMallocDefault) == hipSuccess;
  ok &= hipHostMalloc((void**)&segst_host, sizeof(SegStatus) * segcap, hipHostMallocDefault) == hipSuccess;
  ok &= hipHostMalloc((void**)&st_host, sizeof(DevStatus), hipHostMallocDefault) == hipSuccess;
  ok &= hipEventCreateWithFlags(&upload_done, hipEventDisableTiming) == hipSuccess;
  for (hipEvent_t& e : ev) ok &= hipEventCreate(&e) == hipSuccess;
  if (!ok) {
    const hipError_t e = hipGetLastError();
    release();
    return fail(MM_ENOMEM, std::string("device allocation failed: ") + hipGetErrorString(e));
  }
  std::memset(segs_host, 0, sizeof(SegDesc) * segcap);
  std::memset(segst_host, 0, sizeof(SegStatus) * segcap);
  std::memset(st_host, 0, sizeof(DevStatus));
  return MM_OK;
}

void Engine::release() {
  if (arena_mode) {   // nothing of its own: the arena and the host mirrors belong to the caller
    *this = Engine();
    return;
  }
  void* ptrs[] = {key, perm, sseg, deferred, dcells, redo, spos, geo, rmax2, minv, bcount, boff, sbase, soffs, scan_tmp, counts, off, sw, soff,
                  stage_nb, stage_geo, faces, csr, nbr, U, G, Uh, rec, phi, w, Qs, pn, pos_half, Uh_slots,
                  Xe, Xh, recx, phiX, machF, machs, Ss, segs, segst, st};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  void* hptrs[] = {segs_host, segst_host, st_host};
  for (void* q : hptrs)
    if (q) (void)hipHostFree(q);
  if (upload_done) (void)hipEventDestroy(upload_done);
  for (hipEvent_t& e : ev)
    if (e) (void)hipEventDestroy(e);
  *this = Engine();
}

mm_status Engine::upload(int k) {
  if (k < 0 || k > segcap) return fail(MM_EINVAL, "segment count beyond capacity");
  nseg = k;
  if (k == 0) return MM_OK;
  if (arena_mode) {
    // Each descriptor travels as a kernel argument (copied at the launch):
    // no staging memory, and the host copy is free again at once.
    for (int q = 0; q < k; ++q) hipLaunchKernelGGL(k_put_segment, dim3(1), dim3(64), 0, stream, segs_host[q], segs + q);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(MM_EHIP, std::string("segment upload: ") + hipGetErrorString(e));
    return MM_OK;
  }
  const hipError_t e = hipMemcpyAsync(segs, segs_host, sizeof(SegDesc) * k, hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return fail(MM_EHIP, std::string("segment upload: ") + hipGetErrorString(e));
  (void)hipEventRecord(upload_done, stream);
  return MM_OK;
}

SegDesc* Engine::staging() {
  // The staging buffer may be rewritten only once the last upload has run.
  if (!arena_mode) (void)hipEventSynchronize(upload_done);
  return segs_host;
}

void Engine::reset_status() { launch_status_reset(st, segst, nseg, stream); }

void Engine::enqueue_tessellation(const double* pos, int64_t n_slots, const int32_t* slot_seg, int64_t n_cells,
                                  int64_t n_buckets) {
  nbt = n_buckets;
  mark(0);
  launch_sort(pos, n_slots, slot_seg, n_cells, segs, n_buckets, bcount, boff, scan_tmp, sbase, soffs, key, perm,
              sseg, spos, dcells, st, segst, stream);
  mark(1);
  // One segment: its grid (the descriptor uploaded last) travels with the
  // pair passes' arguments.
  last_dense_cap = launch_tessellate(spos, n_cells, segs, sseg, boff, sbase, soffs, stage_nb, stage_geo, counts, geo,
                                     rmax2, deferred, dcells, redo, hints, nseg == 1 ? &segs_host[0].g : nullptr, st,
                                     segst, stream);
  mark(2);
  scan_u64(counts, off, n_cells, scan_tmp, stream);
  launch_build_mesh(spos, geo, n_cells, segs, sseg, stage_nb, stage_geo, counts, off, sw, soff, scan_tmp, fcap,
                    sell_cap, faces, csr, nbr, precision, minv, st, segst, stream);
}

namespace {

template <typename R>
void enqueue_hydro(Engine& E, double* pos, double* w_slots, double* Q, int64_t n, bool any_fresh, bool half,
                   int64_t nbt, double* S_slots, float* mach_slots) {
  static_assert(sizeof(XCell<R>) == 4 * sizeof(R), "entropy records are four values");
  const bool ent = S_slots != nullptr;
  R *Xe = (R*)E.Xe, *Xh = (R*)E.Xh;
  XCell<R>* recx = (XCell<R>*)E.recx;
  const unsigned long long* nf_dev = &E.st->n_faces;
  R *U = (R*)E.U, *Uh = (R*)E.Uh, *phi = (R*)E.phi;
  FluxCell<R>* rec = (FluxCell<R>*)E.rec;
  if (any_fresh) launch_init_charges(E.segs, E.sseg, n, Q, E.perm, E.geo, Q, 1, E.stream);
  launch_cell_state<R>(E.segs, E.sseg, n, Q, E.perm, E.geo, E.Qs, U, E.w, E.st, E.segst, E.stream);
  if (ent) launch_entropy_state<R>(n, E.perm, E.geo, S_slots, E.Ss, Xe, E.stream);
  E.mark(4);
  launch_gradient<R>(E.segs, E.sseg, n, U, E.counts, E.soff, (const NbrEntry<R>*)E.nbr, E.minv, kLimitMaskBit0,
                     ent ? (R*)E.G : nullptr, E.w, E.segst, 0.0, Uh, nullptr, nullptr, nullptr, E.segst, E.stream);
  if (ent)
    launch_entropy_gradient<R>(E.segs, E.sseg, n, Xe, E.counts, E.soff, (const NbrEntry<R>*)E.nbr, E.minv,
                               kLimitMaskBit0, U, (const R*)E.G, E.w, E.segst, Xh, nullptr, E.stream);
  if (half) {
    // Half-step geometry: park U_half and w in slot order, move the
    // generators by w dt/2, rebuild the mesh there and bring the parked
    // values (and the charges) into its cell order.
    if (E.timing) (void)hipEventRecord(E.ev[9], E.stream);
    launch_half_park<R>(E.segs, E.sseg, n, E.perm, Uh, E.w, E.segst, pos, E.pos_half, (R*)E.Uh_slots, w_slots,
                        E.stream);
    launch_remesh_reset(E.st, E.stream);
    E.enqueue_tessellation(E.pos_half, n, nullptr, n, nbt);
    launch_half_unpark<R>(n, E.perm, (const R*)E.Uh_slots, w_slots, Q, Uh, E.w, E.Qs, E.stream);
    if (E.timing) (void)hipEventRecord(E.ev[10], E.stream);
  }
  E.mark(5);
  launch_gradient<R>(E.segs, E.sseg, n, Uh, E.counts, E.soff, (const NbrEntry<R>*)E.nbr, E.minv, kLimitMaskBit1, nullptr, E.w, nullptr,
                     0.0, nullptr, rec, E.geo, E.spos, E.segst, E.stream);
  if (ent)
    launch_entropy_gradient<R>(E.segs, E.sseg, n, Xh, E.counts, E.soff, (const NbrEntry<R>*)E.nbr, E.minv,
                               kLimitMaskBit1, nullptr, nullptr, nullptr, E.segst, nullptr, recx, E.stream);
  E.mark(6);
  launch_flux<R>(E.segs, E.fcap, nf_dev, E.faces, rec, E.segst, 0.0, phi, E.segst, E.stream, ent ? recx : nullptr,
                 (R*)E.phiX, E.machF);
  E.mark(7);
  launch_update<R>(E.segs, E.sseg, n, E.counts, E.soff, E.csr, phi, E.geo, E.perm, E.Qs, E.spos, E.w, pos, E.pn,
                   E.segst, E.st, E.segst, E.stream, half, ent ? E.Ss : nullptr, (const R*)E.phiX, E.machF, E.machs);
  // Results reach the caller's arrays only for segments without a failure,
  // so a failed step leaves the state it started from.
  launch_commit(E.sseg, n, E.perm, E.st, E.segst, E.Qs, E.pn, E.w, ent ? E.Ss : nullptr, E.machs, Q, pos, w_slots,
                ent ? S_slots : nullptr, mach_slots, E.stream);
}

}  // namespace

void Engine::enqueue_step(double* pos, double* w_slots, double* Q, int64_t n_slots, const int32_t* slot_seg,
                          int64_t n_cells, int64_t n_buckets, bool any_fresh, bool half_step, double* S,
                          float* mach) {
  const bool half = half_step && pos_half && Uh_slots && n_slots == n_cells && !slot_seg && !S;
  if (!(Ss && n_slots == n_cells && !slot_seg)) S = nullptr, mach = nullptr;
  remeshed = half;
  reset_status();
  enqueue_tessellation(pos, n_slots, slot_seg, n_cells, n_buckets);
  mark(3);
  if (precision == MM_MIXED) enqueue_hydro<float>(*this, pos, w_slots, Q, n_cells, any_fresh, half, n_buckets, S, mach);
  else enqueue_hydro<double>(*this, pos, w_slots, Q, n_cells, any_fresh, half, n_buckets, S, mach);
  mark(8);
}

mm_status Engine::readback() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(MM_EHIP, std::string("launch: ") + hipGetErrorString(e));
  e = hipMemcpyAsync(st_host, st, sizeof(DevStatus), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess && nseg > 0)
    e = hipMemcpyAsync(segst_host, segst, sizeof(SegStatus) * nseg, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return fail(MM_EHIP, std::string("status readback: ") + hipGetErrorString(e));
  const DevStatus& s = *st_host;
  hints.dense_cells = s.n_dense_cells;
  hints.redo = s.n_redo;
  hints.dense_redo = s.n_dredo + std::max<int64_t>(0, (int64_t)s.n_dense_cells - last_dense_cap);
  hints.deferred = s.n_deferred;
  return MM_OK;
}

void Engine::finish_timing() {
  if (!timing) return;
  for (int k = 0; k < 8; ++k) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ev[k], ev[k + 1]);
    stage_ms[k] = ms;
  }
  stage_ms[8] = 0.0;
  if (remeshed) {
    // The remesh runs inside the predictor stage's events: report it apart.
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ev[9], ev[10]);
    stage_ms[8] = ms;
    stage_ms[4] -= ms;
  }
}

mm_status Engine::check_flags(int flags, int bad_cell, std::string& msg) const {
  if (!flags) return MM_OK;
  char buf[256];
  std::snprintf(buf, sizeof buf, "device flags 0x%x (first internal cell %d)", flags, bad_cell);
  const std::string at(buf);
  if (flags & F_BADPOS) { msg = "a position is not finite or lies outside [0, L): " + at; return MM_EINVAL; }
  if (flags & F_PLANES) { msg = "a cell has more than 64 live faces: " + at; return MM_ECAPACITY; }
  if (flags & F_VERTS) { msg = "a cell has more than 128 vertices: " + at; return MM_ECAPACITY; }
  if (flags & F_CANDS) {
    msg = "more than " + std::to_string(kCands) + " neighbour candidates in one distance shell of a cell: " + at;
    return MM_ECAPACITY;
  }
  if (flags & F_DENSE) {
    msg = "a grid bucket holds more than " + std::to_string(kDenseMax) +
          " points (density contrast beyond the neighbour search's range): " + at;
    return MM_ECAPACITY;
  }
  if (flags & F_FACECAP) { msg = "more unique faces than the face capacity: " + at; return MM_ECAPACITY; }
  if (flags & F_BOX) { msg = "a cell is too large for the periodic box (needs 2 R_max < L): " + at; return MM_EDEGENERATE; }
  if (flags & F_INCOMPLETE) { msg = "a cell could not be completed: " + at; return MM_EDEGENERATE; }
  if (flags & F_ASYM) {
    // Name the two points of one unmatched face in the slot numbering.
    int32_t pi = -1, pj = -1;
    if (st_host->asym_cell >= 0 && st_host->asym_nbr >= 0) {
      (void)hipMemcpy(&pi, perm + st_host->asym_cell, sizeof pi, hipMemcpyDeviceToHost);
      (void)hipMemcpy(&pj, perm + st_host->asym_nbr, sizeof pj, hipMemcpyDeviceToHost);
    }
    char pair[96];
    std::snprintf(pair, sizeof pair, "; points %d and %d", pi, pj);
    msg = "asymmetric face topology (degenerate input?): " + at + pair;
    return MM_EDEGENERATE;
  }
  if (flags & (F_WALK | F_VOLUME)) { msg = "corrupted or empty cell: " + at; return MM_EDEGENERATE; }
  if (flags & F_NONFINITE) { msg = "a state became NaN or infinite: " + at; return MM_ENONFINITE; }
  msg = at;
  return MM_EDEGENERATE;
}

}  // namespace mm
