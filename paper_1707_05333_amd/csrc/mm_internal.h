// Internal declarations shared by the HIP kernels and the host runtime of the
// MI355X moving-mesh step.  Not part of the public interface (include/mm.h).
//
// Every launch works on a set of segments: independent simulations (each
// with its own periodic box, point count, scheme parameters and timestep)
// whose cells share one internal index space.  A single simulation is the
// one-segment case.  Cells of a segment are contiguous in the internal
// (bucket-sorted) order, and nothing a kernel computes for a cell reads
// another segment's data, so a simulation's results do not depend on what
// else shares its launches.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mm {

// ---------------------------------------------------------------------------
// Fixed per-cell capacities of the tessellation kernel (one wavefront per
// cell).  A cell may hold up to kPlanes live faces at once (one 64-bit mask),
// kVerts vertices and kCands candidate neighbours inside its stencil.
// ---------------------------------------------------------------------------
constexpr int kPlanes = 64;
constexpr int kVerts = 128;
constexpr int kCands = 92;
constexpr int kMaxFaces = kPlanes;   // staging slots per cell

// Failure bits collected in DevStatus::flags and SegStatus::flags.
enum : int {
  F_BADPOS = 1 << 0,      // position not finite or outside [0, L)
  F_PLANES = 1 << 1,      // more than kPlanes live faces
  F_VERTS = 1 << 2,       // more than kVerts vertices
  F_CANDS = 1 << 3,       // more than kCands candidates in a stencil
  F_INCOMPLETE = 1 << 4,  // stencil could not cover twice the farthest vertex
  F_ASYM = 1 << 5,        // a face has no partner in the neighbour's list
  F_FACECAP = 1 << 6,     // more unique faces than the face capacity
  F_NONFINITE = 1 << 7,   // NaN or infinite state
  F_WALK = 1 << 8,        // corrupted face cycle
  F_VOLUME = 1 << 9,      // non-positive cell volume
  F_BOX = 1 << 10,        // stencil wider than the periodic box allows
  F_DENSE = 1 << 11,      // a grid bucket holds more than kDenseMax points
};

// Status of the whole launch set, read back once per call.
struct DevStatus {
  int flags;                     // OR of every segment's flags
  int n_deferred;                // cells handed to the wide-stencil pass
  int max_faces;
  int bad_cell;                  // lowest internal cell index with a failure
  int n_overflow;                // of those, cells whose first-pass candidates overflowed
  int n_dense;                   // buckets with a sub-grid (length of the sort's dense-bucket list)
  int n_dense_cells;             // cells for the dense first pass (follows n_dense: cleared together)
  int n_redo;                    // cells the two-cell first pass hands to the one-cell one (cleared with n_dense)
  int n_dredo;                   // cells the two-cell dense pass hands to the one-cell one (cleared with n_dense)
  unsigned long long n_faces;    // unique faces (copy of the scan total)
  unsigned long long n_csr;      // directed faces (copy of the scan total)
  int asym_cell, asym_nbr;       // one face without a partner (internal cells), for diagnostics
};

// Status of one segment.
struct SegStatus {
  unsigned long long dt_bits;    // min over the segment's cells of dt_i as IEEE bits (dt_i > 0)
  int flags;
  int bad_cell;                  // lowest internal cell index with a failure
  unsigned long long floor_hits[4];
};

// Periodic bucket grid of one segment for the neighbour search.
struct GridParams {
  int nb[3];        // buckets per axis
  int nbt;          // total buckets
  double hb[3];     // bucket size per axis
  double inv_hb[3];
  double L[3];      // box
  int ring;         // stencil half-width (in buckets) of the first pass
  int pad;
  double r_filter;  // first-pass candidate radius
  double ppb;       // mean points per bucket
  int64_t base;     // first bucket of this grid in the shared bucket table
};

// Scheme parameters as the kernels need them.
constexpr int kRiemannHllc = 0, kRiemannHll = 1;

struct HydroParams {
  double L[3];
  double gamma, cfl, eta, chi, zeta, theta, rho_floor, p_floor;
  int limit_mask;
  int predictor_frame;
  int riemann;      // kRiemannHllc or kRiemannHll (the MM_HLLC / MM_HLL values)
  int pad;
  double mach_threshold;   // entropy switch (Sec. 4.3); 0: energy equation only
};

// One segment as the kernels see it.
struct SegDesc {
  GridParams g;
  HydroParams hp;
  double dt_max;    // cap of the segment's timestep
  int32_t fresh;    // 1: the charges still hold primitives (first step after admission)
  int32_t pad;
};

// One face of a cell as written by the tessellation kernel (cell-local list),
// split so that a search of a neighbour's list reads 8 bytes per entry.
struct StageNbr {
  int32_t j;        // neighbour cell (internal index)
  int32_t meta;     // bits 0-7 image code, bit 8 owned, bits 16-31 rank among owned faces
};
struct StageGeo {
  double A;         // area
  double f[3];      // area centroid minus the generator
};

// Unique face, stored once by its owner.
struct Face {
  int32_t i, j;     // owner and neighbour (internal)
  int32_t code;     // periodic image of j seen from i
  int32_t seg;      // segment of both cells
  double A;
  double f[3];      // area centroid minus r_i
};

// Everything the face kernel reads of one cell, in one aligned record: the
// half-step state and its gradient, the mesh velocity and the centroid
// minus the generator, all in the precision type, and the generator in
// FP64 (face normals are differences of nearby generators).  240 bytes in
// FP64, 144 in mixed precision.
template <typename R>
struct __align__(16) FluxCell {
  R U[5];
  R G[15];
  R w[3];      // mesh velocity
  R c[3];      // centroid relative to the generator
  double r[3];
  // A record stride of a whole number of cache lines puts the same word of
  // every gathered record in the same cache bank; the mixed record is
  // padded off the 128-byte multiple.
  double pad[sizeof(R) == 4 ? 2 : 0];
};

static_assert(sizeof(StageNbr) == 8, "two staged entries per 16-byte load");
static_assert(sizeof(FluxCell<float>) == 144 && sizeof(FluxCell<double>) == 240, "face kernel record sizes");

// Per-cell neighbour entry used by the gradient kernels: neighbour index,
// centroid displacement d = c_j + s - c_i and LSQ weight A / |d|^2, in the
// precision of the gradient arithmetic (40 bytes in FP64, 20 in mixed).
// NbrEntry is the unit of the list storage; each sliced row of 64 entries
// holds its 64 (index, weight) pairs (NbrW), then its 64 displacements
// (three values each), so the limiter's second pass over a list reads the
// displacements only.
template <typename R>
struct NbrEntry;
template <>
struct NbrEntry<double> {
  int32_t o;
  int32_t pad;
  double d[3];
  double wgt;
};
template <>
struct NbrEntry<float> {
  int32_t o;
  float d[3];
  float wgt;
};
template <typename R>
struct NbrW;
template <>
struct NbrW<double> {
  int32_t o;
  int32_t pad;
  double wgt;
};
template <>
struct NbrW<float> {
  int32_t o;
  float wgt;
};
static_assert(sizeof(NbrW<double>) + 3 * sizeof(double) == sizeof(NbrEntry<double>) &&
                  sizeof(NbrW<float>) + 3 * sizeof(float) == sizeof(NbrEntry<float>),
              "a row of 64 entries splits into its pairs and its displacements");
// The (index, weight) pair and the displacement of list slot `slot`.
template <typename R>
inline __host__ __device__ NbrW<R>* nbr_w(NbrEntry<R>* nbr, int64_t slot) {
  return reinterpret_cast<NbrW<R>*>(nbr + (slot & ~63ll)) + (slot & 63);
}
template <typename R>
inline __host__ __device__ const NbrW<R>* nbr_w(const NbrEntry<R>* nbr, int64_t slot) {
  return reinterpret_cast<const NbrW<R>*>(nbr + (slot & ~63ll)) + (slot & 63);
}
template <typename R>
inline __host__ __device__ R* nbr_d(NbrEntry<R>* nbr, int64_t slot) {
  return reinterpret_cast<R*>(reinterpret_cast<NbrW<R>*>(nbr + (slot & ~63ll)) + 64) + 3 * (slot & 63);
}
template <typename R>
inline __host__ __device__ const R* nbr_d(const NbrEntry<R>* nbr, int64_t slot) {
  return reinterpret_cast<const R*>(reinterpret_cast<const NbrW<R>*>(nbr + (slot & ~63ll)) + 64) + 3 * (slot & 63);
}

// Bucket of one coordinate; the sort and the tessellation must agree on it.
// Not-a-number and out-of-box coordinates land in a valid bucket (the sort
// flags them separately).
inline __device__ int bucket_coord(double x, double inv_h, int nb) {
  const double t = floor(x * inv_h);
  return t >= 0.0 ? (t < (double)nb ? (int)t : nb - 1) : 0;
}

// Two-level grid.  Buckets are sized for the mean spacing; a bucket holding
// more than kDense points (a region several times denser than the mean) is
// split into s^3 sub-buckets, s the largest value in [2, kSubMax] with
// 2 s^3 <= count, its points ordered sub-bucket by sub-bucket (x fastest,
// then by slot).  Its s^3 + 1 sub-bucket offsets, relative to the bucket's
// first point, sit in a shared table at the bucket's sub-table base.  A
// query then reads only the sub-bucket rows that meet its sphere, so the
// work per cell follows the local density.  kDenseMax bounds the points of
// one bucket (they are sorted in LDS).
constexpr int kDense = 8;
constexpr int kSubMax = 16;
constexpr int kDenseMax = 4096;

inline __host__ __device__ int sub_size(unsigned cnt) {
  int s = 2;
  while (s < kSubMax && 2u * (unsigned)((s + 1) * (s + 1) * (s + 1)) <= cnt) ++s;
  return s;
}

// Sub-bucket of a coordinate inside bucket b of an axis (b from
// bucket_coord): monotone in x, clamped to [0, s - 1], so a query interval
// [lo, hi] covers every point in it by the sub-buckets from
// sub_coord(lo) to sub_coord(hi).
inline __device__ int sub_coord(double x, double inv_h, int b, int s) {
  const double t = floor((x * inv_h - (double)b) * (double)s);
  return t >= 0.0 ? (t < (double)s ? (int)t : s - 1) : 0;
}

// Position of bucket (bx, by, bz) in the grid's table (before the grid's
// base), and so in the cell order.  Buckets are numbered tile by tile
// (tiles of kTile^3 buckets, row-major over tiles, x fastest; row-major
// inside a tile, the last tile of an axis as wide as what remains), so the
// neighbours of most cells lie within a few hundred positions: the hydro
// kernels' gathers stay in cache.  A bijection onto [0, nb_x nb_y nb_z).
constexpr int kTile = 8;
inline __host__ __device__ int bucket_key(const int nb[3], int bx, int by, int bz) {
  const int tx = bx / kTile, ty = by / kTile, tz = bz / kTile;
  const int ex = min(kTile, nb[0] - tx * kTile), ey = min(kTile, nb[1] - ty * kTile),
            ez = min(kTile, nb[2] - tz * kTile);
  const int lx = bx - tx * kTile, ly = by - ty * kTile, lz = bz - tz * kTile;
  return nb[0] * nb[1] * (tz * kTile) + nb[0] * (ty * kTile) * ez + (tx * kTile) * ey * ez + lx +
         ex * (ly + ey * lz);
}

inline __host__ __device__ int code_of(int kx, int ky, int kz) { return (kx + 1) + 3 * (ky + 1) + 9 * (kz + 1); }
inline __host__ __device__ void decode(int code, int& kx, int& ky, int& kz) {
  kx = code % 3 - 1;
  ky = (code / 3) % 3 - 1;
  kz = code / 9 - 1;
}

// Workgroups are handed to the eight XCDs in turn (workgroup b runs on XCD
// b mod 8).  This renumbering gives each XCD one contiguous run of logical
// blocks, so the neighbour reuse inside a run stays in that XCD's L2.
constexpr int kXcds = 8;
inline __device__ int64_t xcd_block() {
  const int64_t b = blockIdx.x, nb = gridDim.x;
  const int64_t x = b % kXcds, k = b / kXcds, q = nb / kXcds, r = nb % kXcds;
  return x * q + (x < r ? x : r) + k;
}

// Timestep of segment `seg`: the device CFL minimum capped by the segment's
// dt_max, or dt_fixed when no status is given (component calls).
inline __device__ double seg_dt(const SegDesc* segs, const SegStatus* dt_src, int seg, double dt_fixed) {
  if (!dt_src) return dt_fixed;
  return fmin(__longlong_as_double((long long)dt_src[seg].dt_bits), segs[seg].dt_max);
}

inline __device__ void seg_fail(DevStatus* st, SegStatus* segst, int seg, int bits, int cell) {
  atomicOr(&st->flags, bits);
  atomicMin(&st->bad_cell, cell);
  atomicOr(&segst[seg].flags, bits);
  atomicMin(&segst[seg].bad_cell, cell);
}

// ---------------------------------------------------------------------------
// Host-side launchers (each enqueues on `st`).
// ---------------------------------------------------------------------------

// Exclusive prefix sum of n uint64 values into out[0..n] (out[n] = total).
// tmp must hold scan_tmp_elems(n) elements.
size_t scan_tmp_elems(int64_t n);
void scan_u64(const unsigned long long* in, unsigned long long* out, int64_t n, unsigned long long* tmp,
              hipStream_t st);

void launch_fill_u64(unsigned long long* p, unsigned long long v, int64_t n, hipStream_t st);
void launch_status_reset(DevStatus* s, SegStatus* segst, int nseg, hipStream_t st);
// Clears the per-mesh counters (deferred and overflowing cells, face and
// list totals) before a second tessellation in one step; failure flags, the
// timestep minimum and the floor counts are kept.
void launch_remesh_reset(DevStatus* s, hipStream_t st);

// Bucket sort of the generators of every segment (grid hash, counting sort,
// caller order inside a bucket).  pos covers n_slots slots; slot_seg[q] is
// the segment of slot q (-1: unused slot), or NULL for one segment covering
// every slot.  Writes perm (internal -> slot), the segment of each internal
// cell, the sorted positions and the bucket offsets of all nbt buckets.
void launch_sort(const double* pos, int64_t n_slots, const int32_t* slot_seg, int64_t n, const SegDesc* segs,
                 int64_t nbt, unsigned long long* bcount, unsigned long long* boff, unsigned long long* scan_tmp,
                 unsigned long long* sbase, uint32_t* soffs, int32_t* key, int32_t* perm, int32_t* sseg,
                 double* spos, int32_t* dcells, DevStatus* st_dev, SegStatus* segst, hipStream_t st);

// Lengths of an earlier tessellation's cell lists (-1: none yet).  They size
// the grids of the passes that read the lists, never their results (those
// passes walk their lists with a grid stride; the two-cell dense pass hands
// listed cells beyond its grid to the one-cell dense pass).
struct TessHints {
  int64_t dense_cells = -1;   // cells listed for the dense passes
  int64_t redo = -1;          // cells the lean two-cell pass handed on
  int64_t dense_redo = -1;    // cells of the one-cell dense pass
  int64_t deferred = -1;      // cells of the shell pass
};

// Tessellation: pass 1 over every cell, then the listed and deferred cells.
// Returns the number of listed dense cells the two-cell dense pass takes.
int64_t launch_tessellate(const double* spos, int64_t n, const SegDesc* segs, const int32_t* sseg,
                          const unsigned long long* boff, const unsigned long long* sbase, const uint32_t* soffs,
                          StageNbr* stage_nb, StageGeo* stage_geo, unsigned long long* counts, double* geo,
                          double* rmax2, int32_t* deferred, int32_t* dcells, int32_t* redo, const TessHints& hints,
                          const GridParams* g_one, DevStatus* st_dev, SegStatus* segst, hipStream_t st);

// Per-cell lists (face ids with sign, neighbour entries) use a sliced ELL
// layout: slices of 64 consecutive internal cells, each as wide as its
// longest list; entry e of cell s sits at soff[s / 64] + 64 e + s % 64.
inline __host__ __device__ int64_t sell_slot(const unsigned long long* soff, int64_t s, int e) {
  return (int64_t)soff[s >> 6] + 64ll * e + (s & 63);
}

// Unique faces, per-cell lists (slice offsets soff, from the slice widths sw),
// neighbour entries and inverse LSQ matrices from the staged lists.
void launch_build_mesh(const double* spos, const double* geo, int64_t n, const SegDesc* segs, const int32_t* sseg,
                       const StageNbr* stage_nb, const StageGeo* stage_geo, const unsigned long long* counts,
                       const unsigned long long* off, unsigned long long* sw, unsigned long long* soff,
                       unsigned long long* scan_tmp, int64_t face_cap, int64_t sell_cap, Face* faces, int32_t* csr,
                       void* nbr, int precision, double* minv, DevStatus* st_dev, SegStatus* segst, hipStream_t st);

// Hydro kernels, instantiated for double (MM_FP64) and float (MM_MIXED).
// Slot-space arrays (Q, pos, w, prim) are indexed through perm.  dt_src
// (may be NULL, then dt_fixed applies) holds each segment's CFL minimum.
template <typename R>
void launch_cell_state(const SegDesc* segs, const int32_t* sseg, int64_t n, const double* Q_slots,
                       const int32_t* perm, const double* geo, double* Qs, R* U, double* w, DevStatus* st_dev,
                       SegStatus* segst, hipStream_t st);
// Limiter selection of the gradient kernel: off, on, or the segment's own
// limit_mask bit 0 (first gradient) / bit 1 (second gradient).
enum : int { kLimitOff = 0, kLimitOn = 1, kLimitMaskBit0 = 2, kLimitMaskBit1 = 3 };
// Gradients of U (to G when set); with U_half set, the half-step predictor
// (needs w); with rec set, the face kernel's cell records (needs w, geo and
// spos).
template <typename R>
void launch_gradient(const SegDesc* segs, const int32_t* sseg, int64_t n, const R* U,
                     const unsigned long long* counts, const unsigned long long* soff, const NbrEntry<R>* nbr,
                     const double* minv, int limit, R* G, const double* w, const SegStatus* dt_src, double dt_fixed,
                     R* U_half, FluxCell<R>* rec, const double* geo, const double* spos, SegStatus* segst,
                     hipStream_t st);
template <typename R>
void launch_pack_flux_cells(int64_t n, const R* U, const R* G, const double* w, const double* geo,
                            const double* spos, FluxCell<R>* rec, hipStream_t st);
template <typename R>
void launch_predict(const SegDesc* segs, const int32_t* sseg, int64_t n, const R* U, const R* G, const double* w,
                    const SegStatus* dt_src, double dt_fixed, R* U_half, SegStatus* segst, hipStream_t st);
// nf_dev (device count, may be NULL) overrides nf_host, which then only
// bounds the launch.
// Entropy charges S = m P rho^-gamma of primitive states (slot order).
void launch_init_entropy(const SegDesc* segs, const int32_t* sseg, int64_t n, const double* prim_slots,
                         const int32_t* perm, const double* geo, double* S_slots, hipStream_t st);
// Entropy column X = rho A (Sec. 4.3) of a cell for the face kernel: its
// half-step value and limited gradient.
template <typename R>
struct XCell {
  R X, g[3];
};
// X = S / V in internal order, with S (the caller's entropy charges, slot
// order) gathered into Ss.
template <typename R>
void launch_entropy_state(int64_t n, const int32_t* perm, const double* geo, const double* S_slots, double* Ss,
                          R* X, hipStream_t st);
// Least-squares gradient of X with the S10 limiter (limit as in
// launch_gradient).  With Xh: the half-step X from the predictor rate
// -div(X v) (+ w . grad X), needing the time-n U, its gradient G and w.
// With recx: the face kernel's records.
template <typename R>
void launch_entropy_gradient(const SegDesc* segs, const int32_t* sseg, int64_t n, const R* X,
                             const unsigned long long* counts, const unsigned long long* soff, const NbrEntry<R>* nbr,
                             const double* minv, int limit, const R* U, const R* G, const double* w,
                             const SegStatus* dt_src, R* Xh, XCell<R>* recx, hipStream_t st);
template <typename R>
void launch_flux(const SegDesc* segs, int64_t nf_host, const unsigned long long* nf_dev, const Face* faces,
                 const FluxCell<R>* rec, const SegStatus* dt_src, double dt_fixed, R* phi, SegStatus* segst,
                 hipStream_t st, const XCell<R>* recx = nullptr, R* phiX = nullptr, float* machF = nullptr);
// Update of the charges with the floors after the step, and the drift
// (internal order): Qs is overwritten with the new charges, pn receives the
// new positions, Ss (entropy column, may be NULL) the new entropy charges
// and machs each cell's largest face Mach number.  The caller's arrays are
// untouched; launch_commit copies the results out.
template <typename R>
void launch_update(const SegDesc* segs, const int32_t* sseg, int64_t n, const unsigned long long* counts,
                   const unsigned long long* soff, const int32_t* csr, const R* phi, const double* geo,
                   const int32_t* perm, double* Qs, const double* spos, const double* w, const double* pos_slots,
                   double* pn, const SegStatus* dt_src, DevStatus* st_dev, SegStatus* segst, hipStream_t st,
                   bool drift_from_slots = false, double* Ss = nullptr, const R* phiX = nullptr,
                   const float* machF = nullptr, float* machs = nullptr);
// Copies the results of launch_update into the slot-order arrays of every
// segment whose status holds no failure; a failed segment keeps its state
// (all of them do after an overflow of the shared face capacity).
void launch_commit(const int32_t* sseg, int64_t n, const int32_t* perm, const DevStatus* st_dev,
                   const SegStatus* segst, const double* Qn, const double* pn, const double* w, const double* Ss,
                   const float* machs, double* Q_slots, double* pos_slots, double* w_slots, double* S_slots,
                   float* mach_slots, hipStream_t st);
// Half-step mesh: U_half and w of internal cell s go to slot perm[s], and
// pos_half[slot] = wrap(pos[slot] + w dt/2) (single segment, slots = cells).
template <typename R>
void launch_half_park(const SegDesc* segs, const int32_t* sseg, int64_t n, const int32_t* perm, const R* Uh,
                      const double* w, const SegStatus* dt_src, const double* pos_slots, double* pos_half,
                      R* Uh_slots, double* w_slots, hipStream_t st);
// ... and back into the cell order of the rebuilt mesh, with the charges.
template <typename R>
void launch_half_unpark(int64_t n, const int32_t* perm, const R* Uh_slots, const double* w_slots,
                        const double* Q_slots, R* Uh, double* w, double* Qs, hipStream_t st);
template <typename R>
void launch_accumulate(int64_t n, const unsigned long long* counts, const unsigned long long* soff, const int32_t* csr,
                       const R* phi,
                       const int32_t* perm, double* dQ_slots, hipStream_t st);

// Layout conversions between slot order and internal order.
template <typename R>
void launch_gather_rows(const R* src_slots, const int32_t* perm, int64_t n, int width, R* dst, hipStream_t st);
template <typename R>
void launch_scatter_rows(const R* src, const int32_t* perm, int64_t n, int width, R* dst_slots, hipStream_t st);
// Charges from primitives, Q = U(prim) V; with only_fresh set, only for
// segments flagged fresh, reading and writing the same slot array.
void launch_init_charges(const SegDesc* segs, const int32_t* sseg, int64_t n, const double* prim_slots,
                         const int32_t* perm, const double* geo, double* Q_slots, int only_fresh, hipStream_t st);
void launch_export_mesh(int64_t n, int64_t nf, const int32_t* perm, const double* spos, const double* geo,
                        const Face* faces, double* V, double* centroid, int32_t* fi, int32_t* fj, int32_t* fc,
                        double* fA, double* ff, hipStream_t st);
// Copies n rows of `width` doubles (device to device, may not overlap).
void launch_copy_rows(const double* src, double* dst, int64_t n, int width, hipStream_t st);
void launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st);

}  // namespace mm
