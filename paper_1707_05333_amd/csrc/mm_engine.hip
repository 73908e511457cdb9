// Engine: device memory of the internal cell space, segment table, enqueue
// order of a tessellation and of a step, status readback.
#include "mm_engine.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

namespace mm {

namespace {

template <typename T>
hipError_t dalloc(T** p, size_t count) {
  return hipMalloc((void**)p, std::max<size_t>(count, 1) * sizeof(T));
}

}  // namespace

int64_t engine_bytes_per_cell(int precision) {
  const int64_t r = precision == MM_MIXED ? 4 : 8;
  const int64_t per_cell = 4 * 5                                       // key, perm, sseg, deferred, dcells
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

mm_status Engine::init(int prec, int64_t n_cap, int64_t s_cap, int64_t f_cap, int seg_cap, hipStream_t s,
                       bool single) {
  precision = prec;
  ncap = n_cap;
  slot_cap = s_cap;
  fcap = std::min<int64_t>(f_cap, 0x7fffffffll);
  segcap = seg_cap;
  nbcap = ncap + 8ll * segcap;
  sell_cap = kListPerCell * ((ncap + 63) / 64) * 64;   // whole slices of 64 cells
  stream = s;
  if (hipGetDevice(&device) != hipSuccess) return fail(MM_EHIP, "hipGetDevice failed");
  const int64_t N = ncap, F = fcap;
  const size_t rs = precision == MM_MIXED ? sizeof(float) : sizeof(double);
  bool ok = true;
  ok &= dalloc(&key, slot_cap) == hipSuccess;
  ok &= dalloc(&perm, N) == hipSuccess;
  ok &= dalloc(&sseg, N) == hipSuccess;
  ok &= dalloc(&deferred, N) == hipSuccess;
  ok &= dalloc(&dcells, N) == hipSuccess;
  ok &= dalloc(&spos, 3 * N) == hipSuccess;
  ok &= dalloc(&geo, 4 * N) == hipSuccess;
  ok &= dalloc(&rmax2, N) == hipSuccess;
  ok &= dalloc(&minv, 6 * N) == hipSuccess;
  ok &= dalloc(&bcount, nbcap) == hipSuccess;
  ok &= dalloc(&boff, nbcap + 1) == hipSuccess;
  ok &= dalloc(&sbase, nbcap + 1) == hipSuccess;
  ok &= dalloc(&soffs, N) == hipSuccess;
  ok &= dalloc(&scan_tmp, scan_tmp_elems(std::max(N, nbcap))) == hipSuccess;
  ok &= dalloc(&counts, N) == hipSuccess;
  ok &= dalloc(&off, N + 1) == hipSuccess;
  ok &= dalloc(&sw, (N + 63) / 64 + 1) == hipSuccess;
  ok &= dalloc(&soff, (N + 63) / 64 + 2) == hipSuccess;
  ok &= dalloc(&stage_nb, (size_t)N * kMaxFaces) == hipSuccess;
  ok &= dalloc(&stage_geo, (size_t)N * kMaxFaces) == hipSuccess;
  ok &= dalloc(&faces, F) == hipSuccess;
  ok &= dalloc(&csr, sell_cap) == hipSuccess;
  ok &= hipMalloc(&nbr, std::max<size_t>(sell_cap * (precision == MM_MIXED ? sizeof(NbrEntry<float>)
                                                                            : sizeof(NbrEntry<double>)), 1)) == hipSuccess;
  ok &= hipMalloc(&U, std::max<size_t>(5 * N * rs, 1)) == hipSuccess;
  ok &= hipMalloc(&G, std::max<size_t>(15 * N * rs, 1)) == hipSuccess;
  ok &= hipMalloc(&Uh, std::max<size_t>(5 * N * rs, 1)) == hipSuccess;
  ok &= hipMalloc(&rec, std::max<size_t>(N * (precision == MM_MIXED ? sizeof(FluxCell<float>)
                                                                       : sizeof(FluxCell<double>)), 1)) == hipSuccess;
  ok &= hipMalloc(&phi, std::max<size_t>(5 * F * rs, 1)) == hipSuccess;
  ok &= dalloc(&w, 3 * N) == hipSuccess;
  ok &= dalloc(&Qs, 5 * N) == hipSuccess;
  ok &= dalloc(&pn, 3 * N) == hipSuccess;
  if (single) {
    ok &= dalloc(&pos_half, 3 * slot_cap) == hipSuccess;
    ok &= hipMalloc(&Uh_slots, std::max<size_t>(5 * slot_cap * rs, 1)) == hipSuccess;
    ok &= hipMalloc(&Xe, std::max<size_t>(N * rs, 1)) == hipSuccess;
    ok &= hipMalloc(&Xh, std::max<size_t>(N * rs, 1)) == hipSuccess;
    ok &= hipMalloc(&recx, std::max<size_t>(N * 4 * rs, 1)) == hipSuccess;
    ok &= hipMalloc(&phiX, std::max<size_t>(F * rs, 1)) == hipSuccess;
    ok &= dalloc(&machF, F) == hipSuccess;
    ok &= dalloc(&machs, N) == hipSuccess;
    ok &= dalloc(&Ss, N) == hipSuccess;
  }
  ok &= dalloc(&segs, segcap) == hipSuccess;
  ok &= dalloc(&segst, segcap) == hipSuccess;
  ok &= dalloc(&st, 1) == hipSuccess;
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
  void* ptrs[] = {key, perm, sseg, deferred, dcells, spos, geo, rmax2, minv, bcount, boff, sbase, soffs, scan_tmp, counts, off, sw, soff,
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
  const hipError_t e = hipMemcpyAsync(segs, segs_host, sizeof(SegDesc) * k, hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return fail(MM_EHIP, std::string("segment upload: ") + hipGetErrorString(e));
  (void)hipEventRecord(upload_done, stream);
  return MM_OK;
}

SegDesc* Engine::staging() {
  // The staging buffer may be rewritten only once the last upload has run.
  (void)hipEventSynchronize(upload_done);
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
  launch_tessellate(spos, n_cells, segs, sseg, boff, sbase, soffs, stage_nb, stage_geo, counts, geo, rmax2, deferred,
                    dcells, st, segst, stream);
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
