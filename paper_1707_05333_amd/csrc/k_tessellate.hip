// Periodic Voronoi tessellation by half-space clipping (Sec. 3 of the paper:
// start from a box around the generator, cut it by the bisector plane of each
// neighbour in order of distance, and stop once the next neighbour is farther
// than twice the farthest vertex).  The first pass builds two cells per
// wavefront, one per half (the cells of uniform regions, most of them); the
// cells it hands on, and those of the later passes, get a wavefront each.
//
// Cell representation (all in the wavefront's LDS slice).  A convex cell is
// stored by its dual: every face is a plane slot (normal d = r_j + s - r_i
// relative to the generator, offset h = |d|^2/2), and every vertex is a
// triangle of three plane slots, the planes that meet there.  Triangles are
// oriented consistently, so each directed pair of planes (x -> y) belongs to
// exactly one live triangle; the table E[x][y] stores it.  Cutting by a new
// plane p:
//   * each lane tests its two vertex slots against p (d_p . v > h_p, plain
//     FP64, no epsilon) and a ballot gives the removed set;
//   * an edge (x -> y) of a removed triangle whose neighbour E[y][x] survives
//     lies on the boundary of the removed cap, and gets the new triangle
//     (x, y, p) in a free slot: the fan of new vertices around the new face;
//   * new vertices are intersections of three planes (Cramer's rule).
// Vertex tests and triangle creation are lane-parallel; only the walk over
// the distance-ordered candidates is serial.
//
// Epilogue: lane p walks the polygon of face p through E (from its lowest
// triangle slot, so sums are deterministic) and integrates its area and area
// centroid as a fan from that first vertex; the cell volume is the sum of
// the pyramids A |d| / 6 over faces and the centroid the pyramids' weighted
// centroids (3/4 of the way from the generator to each face centroid).
#include <algorithm>

#include "mm_internal.h"

namespace mm {

namespace {

#ifndef MM_TESS_WAVES
#define MM_TESS_WAVES 1
#endif
constexpr int kWaves = MM_TESS_WAVES;   // cells (wavefronts) per workgroup
constexpr int kShells = 512;            // distance shells of the second pass
constexpr int kShells1 = 3;             // extra shells a cell may take in the first pass
constexpr int kFewCands = 8;            // below this many first candidates, a cell's region is thin
constexpr int kThinRing = 8;            // widest stencil of a thin region's first gather
// Live vertices the shell pass keeps for pruning candidates (a cell with
// more, rare, gathers its shells unpruned); 13 KB of LDS per wavefront with
// the cell, so the pass's 12 waves per CU (by registers) fit.
constexpr int kPruneVerts = 96;

// 10 KB per wavefront, so 16 cells fit the 160 KB of LDS of a CU (as many
// as the one-cell first passes' registers allow, 4 waves per SIMD).  The candidate list and the cut's
// scratch are only needed while cutting and the vertex copies only in the
// epilogue (while cutting, vertices and their triangles live in registers),
// so the two share storage.
struct __align__(16) TessLds {
  double4 pl[kPlanes];                 // plane: d.x, d.y, d.z, h
  union {
    struct {                           // while the cell is cut
      double4 cd[kCands];              // candidate image: d, |d|^2 / 2
      int32_t cjk[kCands];             // candidate: j << 5 | image code
      uint8_t order[kCands];
      uint16_t elist[kVerts];          // boundary edges of one cut: x | y << 8
      uint8_t kept[kVerts];            // 1 for a live vertex slot that survives the current cut
    };
    struct {                           // in the epilogue
      double vx[kVerts], vy[kVerts], vz[kVerts];
      int32_t first[kPlanes];
      uint32_t tri[kVerts];            // a | b << 8 | c << 16
    };
  };
  int32_t pcand[kPlanes];              // neighbour of each plane slot (j << 5 | image code); -1 - k for box plane k
  uint8_t E[kPlanes * kPlanes];
};
static_assert(sizeof(TessLds) <= 10240, "16 cells per CU");

struct TessArgs {
  const double* spos;
  int64_t n;
  const SegDesc* segs;
  const int32_t* sseg;
  const unsigned long long* boff;
  const unsigned long long* sbase;   // sub-table base of each dense bucket
  const uint32_t* soffs;             // sub-bucket offsets of the dense buckets
  StageNbr* stage_nb;
  StageGeo* stage_geo;
  unsigned long long* counts;
  double* geo;
  double* rmax2;
  int32_t* deferred;
  int32_t* dcells;                   // cells for the dense first pass
  int32_t* redo;                     // cells the two-cell first pass hands to the one-cell one
  int64_t dense_cap;                 // listed dense cells the two-cell dense pass takes (even)
  DevStatus* st;
  SegStatus* segst;
  GridParams g1;                     // the grid when there is one segment (a kernel argument)
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ unsigned long long lanes_below() { return (1ull << __lane_id()) - 1ull; }

// This lane's bit of a wavefront mask (a select on the mask itself, no shift).
__device__ __forceinline__ bool lane_on(unsigned long long m) { return __builtin_amdgcn_inverse_ballot_w64(m); }

// Exclusive prefix sum over the wave; *total gets the wave's sum.  DPP lane
// moves: row shifts by 1, 2, 4 and 8 inside each row of 16 lanes (lanes
// shifted in from outside the row read 0), then the last lane of row 0
// added to row 1 and of row 2 to row 3, then lane 31 to rows 2 and 3.
// Called by the whole wavefront.
__device__ __forceinline__ int wave_excl_scan(int x, int* total) {
  int v = x;
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, true);
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, true);
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, true);
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, true);
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false);
  *total = __builtin_amdgcn_readlane(v, 63);
  return v - x;
}

// Wave-wide reductions with DPP lane moves (no LDS round trip): within each
// row of 16 lanes by quad permutes and row rotations, then across rows by
// the row broadcasts; lane 63 ends with the result, read as a scalar.
#define MM_DPP_REDUCE(OP, x)                                                        \
  do {                                                                              \
    x = OP(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xF, 0xF, false));  \
    x = OP(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x4E, 0xF, 0xF, false));  \
    x = OP(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x124, 0xF, 0xF, false)); \
    x = OP(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x128, 0xF, 0xF, false)); \
    x = OP(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false)); \
    x = OP(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false)); \
  } while (0)

__device__ __forceinline__ unsigned op_max(unsigned a, unsigned b) { return a > b ? a : b; }
__device__ __forceinline__ unsigned op_or(unsigned a, unsigned b) { return a | b; }

__device__ __forceinline__ unsigned wave_umax32(unsigned x) {
  MM_DPP_REDUCE(op_max, x);
  return (unsigned)__builtin_amdgcn_readlane((int)x, 63);
}

__device__ __forceinline__ unsigned long long wave_or(unsigned long long v) {
  unsigned lo = (unsigned)v, hi = (unsigned)(v >> 32);
  MM_DPP_REDUCE(op_or, lo);
  MM_DPP_REDUCE(op_or, hi);
  return ((unsigned long long)(unsigned)__builtin_amdgcn_readlane((int)hi, 63) << 32) |
         (unsigned)__builtin_amdgcn_readlane((int)lo, 63);
}

// Upper bound of the wave's largest non-negative finite value.  Bit patterns
// of non-negative doubles order like the values, so the high word plus one
// (low word zero) lies above every value with that high word.
__device__ __forceinline__ double wave_max_bound(double x) {
  const unsigned hi = (unsigned)((unsigned long long)__double_as_longlong(x) >> 32) + 1u;
  return __longlong_as_double((long long)((unsigned long long)wave_umax32(hi) << 32));
}

// Butterfly sum: every lane ends with the bitwise-same result.
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

__device__ __forceinline__ unsigned long long plane_bits(uint32_t t) {
  return (1ull << (t & 255u)) | (1ull << ((t >> 8) & 255u)) | (1ull << ((t >> 16) & 255u));
}

// 1/x from the hardware estimate refined by two Newton steps (within an
// ulp of the quotient; the estimate's error squares at each step), with
// correctly rounded division outside the normal range, where the estimate
// would over- or underflow.
__device__ __forceinline__ double rcp_nr(double x) {
  if (fabs(x) > 1e-280 && fabs(x) < 1e280) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(fma(-x, r, 1.0), r, r);
    return fma(fma(-x, r, 1.0), r, r);
  }
  return 1.0 / x;
}

// 1/sqrt(x) for x > 0 likewise: the hardware estimate and two Newton steps
// (y <- y + y (1 - x y^2) / 2), the square root and a division outside the
// normal range.
__device__ __forceinline__ double rsqrt_nr(double x) {
  if (x > 1e-280 && x < 1e280) {
    double y = __builtin_amdgcn_rsq(x);
    y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
    return fma(0.5 * y, fma(-x * y, y, 1.0), y);
  }
  return 1.0 / sqrt(x);
}

// Vertex where planes a, b, c meet: solve [a; b; c] v = (a.w, b.w, c.w).
// By Cramer's rule v = (a.w (b x c) + b.w (c x a) + c.w (a x b)) / det with
// det = a . (b x c) = c . (a x b); the first two terms are one cross
// product, (a.w b - b.w a) x c, so two cross products and one dot product
// do (c is the new plane of a cut, a and b the planes of the edge it cuts).
__device__ __forceinline__ void intersect3(const double4 a, const double4 b, const double4 c, double& x, double& y,
                                           double& z) {
  const double abx = a.y * b.z - a.z * b.y, aby = a.z * b.x - a.x * b.z, abz = a.x * b.y - a.y * b.x;
  const double det = c.x * abx + c.y * aby + c.z * abz;
  const double ux = a.w * b.x - b.w * a.x, uy = a.w * b.y - b.w * a.y, uz = a.w * b.z - b.w * a.z;
  const double inv = rcp_nr(det);
  x = (uy * c.z - uz * c.y + c.w * abx) * inv;
  y = (uz * c.x - ux * c.z + c.w * aby) * inv;
  z = (ux * c.y - uy * c.x + c.w * abz) * inv;
}

__device__ void fail_cell(const TessArgs& A, int s, int seg, int bit) {
  if (__lane_id() == 0) {
    seg_fail(A.st, A.segst, seg, bit, s);
    A.counts[s] = 0ull;
    A.geo[4 * (int64_t)s] = 0.0;
  }
}

// Per-lane view of the cell under construction: lane k holds vertex slots
// k and k + 64 (triangle and position); the live masks and the squared
// farthest-vertex distance are wave-uniform.
struct CellRegs {
  unsigned long long L0, L1;
  uint32_t t0, t1;
  double v0x, v0y, v0z, v1x, v1y, v1z;
  double rmax2;
  int np;   // plane slots handed out so far
};

// Starting cell: the box r +- L/2, bounded by the bisectors of the
// generator's six axis images (the large box each cell is cut from, Sec. 3).
__device__ void init_box(TessLds& S, const GridParams& g, CellRegs& C) {
  const int lane = __lane_id();
  if (lane < 6) {
    const int ax = lane >> 1;
    const double sg = (lane & 1) ? -1.0 : 1.0;
    double d[3] = {0.0, 0.0, 0.0};
    d[ax] = sg * g.L[ax];
    S.pl[lane] = make_double4(d[0], d[1], d[2], 0.5 * (g.L[ax] * g.L[ax]));
    S.pcand[lane] = -1 - lane;
  }
  C.t0 = C.t1 = 0u;
  C.v0x = C.v0y = C.v0z = C.v1x = C.v1y = C.v1z = 0.0;
  if (lane < 8) {
    const int sx = (lane & 1) ? -1 : 1, sy = (lane & 2) ? -1 : 1, sz = (lane & 4) ? -1 : 1;
    const int px = sx > 0 ? 0 : 1, py = sy > 0 ? 2 : 3, pz = sz > 0 ? 4 : 5;
    int a1 = py, a2 = pz;
    if (sx * sy * sz < 0) { a1 = pz; a2 = py; }   // orientation: det(d_a, d_b, d_c) > 0
    C.t0 = (uint32_t)(px | (a1 << 8) | (a2 << 16));
    C.v0x = sx * (0.5 * g.L[0]);
    C.v0y = sy * (0.5 * g.L[1]);
    C.v0z = sz * (0.5 * g.L[2]);
    S.E[px * kPlanes + a1] = (uint8_t)lane;
    S.E[a1 * kPlanes + a2] = (uint8_t)lane;
    S.E[a2 * kPlanes + px] = (uint8_t)lane;
  }
  wave_sync();
  C.L0 = 0xffull;
  C.L1 = 0ull;
  C.np = 6;
  C.rmax2 = wave_max_bound(lane < 8 ? C.v0x * C.v0x + C.v0y * C.v0y + C.v0z * C.v0z : 0.0);
}

// Smallest stencil half-width whose buckets contain every image closer than
// sqrt(r2) to the generator.
__device__ int ring_for(const GridParams& g, const double edge[3], double r2) {
  const double r = sqrt(r2);
  int ring = 1;
#pragma unroll
  for (int a = 0; a < 3; ++a) ring = max(ring, (int)ceil((r - edge[a]) / g.hb[a]));
  return ring;
}

// One stencil bucket of a lane: its first point, its point count and the
// periodic image (code and shift) under which its points are seen.
struct StencilBucket {
  int bst, cnt, code;
  double sx, sy, sz;
};

// Division by the stencil width W: q = umulhi(o, m) with m = 2^32 / W
// rounded up is exact for o * W < 2^32, which holds for every o < W^3 when
// W < 256 (the quotient's error o (m W - 2^32) / 2^32 stays below 1 / W).
struct WidthDiv {
  unsigned W, m;
};
__device__ inline WidthDiv width_div(unsigned W) { return WidthDiv{W, 0xffffffffu / W + 1u}; }
__device__ inline unsigned div_width(unsigned o, const WidthDiv& d) {
  return d.W < 256u ? __umulhi(o, d.m) : o / d.W;
}

__device__ inline StencilBucket stencil_bucket(const TessArgs& A, const GridParams& g, const int b[3], int ring,
                                               int o, int W3, const WidthDiv& D, int* bb_out = nullptr,
                                               int64_t* key_out = nullptr) {
  StencilBucket B{0, 0, 13, 0.0, 0.0, 0.0};
  if (o < W3) {
    const unsigned W = D.W;
    const unsigned q1 = div_width((unsigned)o, D), q2 = div_width(q1, D);
    const int oo[3] = {(int)((unsigned)o - q1 * W) - ring, (int)(q1 - q2 * W) - ring, (int)q2 - ring};
    int kk[3], bb[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int t = b[a] + oo[a];
      kk[a] = t < 0 ? -1 : (t >= g.nb[a] ? 1 : 0);
      bb[a] = t - kk[a] * g.nb[a];
    }
    const int64_t key = g.base + bucket_key(g.nb, bb[0], bb[1], bb[2]);
    const unsigned long long b0 = A.boff[key];
    B.bst = (int)b0;
    B.cnt = (int)(A.boff[key + 1] - b0);
    B.code = code_of(kk[0], kk[1], kk[2]);
    B.sx = kk[0] * g.L[0];
    B.sy = kk[1] * g.L[1];
    B.sz = kk[2] * g.L[2];
    if (bb_out) {
      bb_out[0] = bb[0];
      bb_out[1] = bb[1];
      bb_out[2] = bb[2];
    }
    if (key_out) *key_out = key;
  }
  return B;
}

// Whether any of the nv vertices vl (relative to the generator) lies beyond
// the bisector of image d (|d|^2 = d2) by more than a relative margin: an
// image that fails it cannot cut the cell (nor any part of it the later
// cuts leave), so it need not be gathered.  The margin keeps borderline
// images for the exact test of the cutting loop.
__device__ inline bool may_cut(const double4* vl, int nv, double dx, double dy, double dz, double d2) {
  const double h = 0.5 * d2 * (1.0 - 1e-12);
  bool out = false;
  for (int t = 0; t < nv; ++t) {
    const double4 v = vl[t];
    out |= dx * v.x + dy * v.y + dz * v.z > h;
  }
  return out;
}

// Whether a box (relative to the generator) may hold an image that cuts the
// cell: a point cuts it only if it is closer to some vertex v than the
// generator is, so the box must come within |v| of some v (vl[t].w holds
// |v|^2).  The margins make the test looser than may_cut's, so no image
// that may_cut keeps is lost with its box.
__device__ inline bool box_may_cut(const double4* vl, int nv, const double lo[3], const double hi[3],
                                   double slack) {
  bool out = false;
  for (int t = 0; t < nv; ++t) {
    const double4 v = vl[t];
    const double ex = fmax(0.0, fmax(lo[0] - v.x, v.x - hi[0]));
    const double ey = fmax(0.0, fmax(lo[1] - v.y, v.y - hi[1]));
    const double ez = fmax(0.0, fmax(lo[2] - v.z, v.z - hi[2]));
    out |= ex * ex + ey * ey + ez * ez < v.w * (1.0 + 1e-9) + slack;
  }
  return out;
}

// The same two tests with the roles of lanes turned round, for when few
// lanes ask (the sparse stencils of a thin region): each asking lane's box
// or image is broadcast in turn and every lane tests the vertex it holds
// (vertex k in lane k, vertex k + 64 in the second register).  Each
// (box or image, vertex) pair is the same comparison as above, so the
// answers are the same; only the work follows the number of asking lanes
// instead of the number of vertices.
struct LaneVerts {
  double4 a, b;   // vertices lane and lane + 64 (w = -1: none)
  bool two;       // some lane holds a second vertex
};

__device__ inline LaneVerts lane_verts(const double4* vl, int nv) {
  const int lane = __lane_id();
  LaneVerts V;
  const double4 none = make_double4(0.0, 0.0, 0.0, -1.0);
  V.a = lane < nv ? vl[lane] : none;
  V.b = lane + 64 < nv ? vl[lane + 64] : none;
  V.two = nv > 64;
  return V;
}

__device__ inline double readlane_d(double x, int l) {
  const long long b = __double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ inline bool vert_near_box(const double4 v, const double lo[3], const double hi[3], double slack) {
  const double ex = fmax(0.0, fmax(lo[0] - v.x, v.x - hi[0]));
  const double ey = fmax(0.0, fmax(lo[1] - v.y, v.y - hi[1]));
  const double ez = fmax(0.0, fmax(lo[2] - v.z, v.z - hi[2]));
  return ex * ex + ey * ey + ez * ez < v.w * (1.0 + 1e-9) + slack;
}

// box_may_cut for every lane with `ask` set (false for the others); called
// by the whole wavefront.
__device__ inline bool boxes_may_cut(bool ask, const double4* vl, int nv, const LaneVerts& V, const double lo[3],
                                     const double hi[3], double slack) {
  const unsigned long long m = __ballot(ask);
  if (m == 0ull) return false;
  if (3 * __popcll(m) >= nv) return ask && box_may_cut(vl, nv, lo, hi, slack);
  const int lane = __lane_id();
  bool res = false;
  for (unsigned long long r = m; r; r &= r - 1ull) {
    const int l = __builtin_ctzll(r);
    const double blo[3] = {readlane_d(lo[0], l), readlane_d(lo[1], l), readlane_d(lo[2], l)};
    const double bhi[3] = {readlane_d(hi[0], l), readlane_d(hi[1], l), readlane_d(hi[2], l)};
    bool t = vert_near_box(V.a, blo, bhi, slack);
    if (V.two) t |= vert_near_box(V.b, blo, bhi, slack);
    if (__ballot(t) != 0ull && lane == l) res = true;
  }
  return res;
}

// may_cut for every lane with `ask` set (false for the others); called by
// the whole wavefront.
__device__ inline bool images_may_cut(bool ask, const double4* vl, int nv, const LaneVerts& V, double dx, double dy,
                                      double dz, double d2) {
  const unsigned long long m = __ballot(ask);
  if (m == 0ull) return false;
  if (4 * __popcll(m) >= nv) return ask && may_cut(vl, nv, dx, dy, dz, d2);
  const int lane = __lane_id();
  bool res = false;
  for (unsigned long long r = m; r; r &= r - 1ull) {
    const int l = __builtin_ctzll(r);
    const double x = readlane_d(dx, l), y = readlane_d(dy, l), z = readlane_d(dz, l);
    const double h = 0.5 * readlane_d(d2, l) * (1.0 - 1e-12);
    bool t = x * V.a.x + y * V.a.y + z * V.a.z > h;
    if (V.two) t |= x * V.b.x + y * V.b.y + z * V.b.z > h;
    if (__ballot(t) != 0ull && lane == l) res = true;
  }
  return res;
}

// Gather of one 128-bucket chunk of the stencil that holds dense buckets.
// Each bucket contributes runs of consecutive points: a sparse bucket its
// whole range, a dense one the part of each sub-bucket row (along x) that
// meets the box around the query sphere; buckets that miss the box give
// nothing.  The wave takes the runs 64 at a time, one per lane (the lane
// finds the bucket of its run by a binary search over the buckets' run
// prefix sums), and steps through their points together.  The test on each
// point is the one of the uniform path, so the candidates are the same;
// only the points read are fewer.  Returns the new candidate count.
__device__ int gather_runs(TessLds& S, const TessArgs& A, const GridParams& g, const int s, const double r[3],
                           const int b[3], const int ring, const int chunk, const int W3, const WidthDiv& D,
                           const double lo2, const double hi2, const double4* vl, const int nv, int nc) {
  const int lane = __lane_id();
  // Half-width of the query box, with a margin far above the rounding of
  // the distance test, so that every point the test keeps lies inside.
  const double rq = sqrt(hi2) * (1.0 + 1e-9) + 1e-9 * fmin(g.hb[0], fmin(g.hb[1], g.hb[2]));
  LaneVerts V{};
  if (vl) V = lane_verts(vl, nv);
  for (int half = 0; half < 2; ++half) {
    int bb[3] = {0, 0, 0};
    int64_t key = 0;
    const StencilBucket B = stencil_bucket(A, g, b, ring, chunk + 64 * half + lane, W3, D, bb, &key);
    int nr = 0, pack = 0, base = 0;
    const double sh[3] = {B.sx, B.sy, B.sz};
    double qlo[3] = {0.0, 0.0, 0.0}, qhi[3] = {0.0, 0.0, 0.0};
    bool meet = false;
    // the bucket's box relative to the generator, widened a little
    double blo[3] = {0.0, 0.0, 0.0}, bhi[3] = {0.0, 0.0, 0.0};
    if (B.cnt > 0) {
      meet = true;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        qlo[a] = (r[a] - rq) - sh[a];
        qhi[a] = (r[a] + rq) - sh[a];
        // bucket bb holds the points with floor(x / hb) = bb (the last one
        // also those rounding to nb)
        const double tlo = qlo[a] * g.inv_hb[a], thi = qhi[a] * g.inv_hb[a];
        if (thi < (double)bb[a] || (tlo >= (double)(bb[a] + 1) && bb[a] < g.nb[a] - 1)) meet = false;
      }
      if (meet && vl) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          blo[a] = (bb[a] * g.hb[a] + sh[a]) - r[a] - 1e-9 * g.hb[a];
          bhi[a] = ((bb[a] + 1) * g.hb[a] + sh[a]) - r[a] + 1e-9 * g.hb[a];
        }
      }
    }
    if (vl) meet = boxes_may_cut(meet, vl, nv, V, blo, bhi, 1e-12 * hi2);
    if (B.cnt > 0) {
      if (meet) {
        if (B.cnt <= kDense || B.cnt > kDenseMax) {
          nr = 1;
        } else {
          const int ss = sub_size((unsigned)B.cnt);
          int l[3], m[3];
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            l[a] = sub_coord(qlo[a], g.inv_hb[a], bb[a], ss);
            m[a] = sub_coord(qhi[a], g.inv_hb[a], bb[a], ss) - l[a] + 1;
          }
          nr = m[1] * m[2];
          pack = ss | l[0] << 5 | m[0] << 10 | l[1] << 15 | m[1] << 20 | l[2] << 25;
          base = (int)A.sbase[key];
        }
      }
    }
    int total;
    const int excl = wave_excl_scan(nr, &total);
    for (int t0 = 0; t0 < total; t0 += 64) {
      const int t = t0 + lane;
      // the last bucket whose runs start at or before t
      int ow = 0;
#pragma unroll
      for (int step = 32; step > 0; step >>= 1) {
        const int e = __shfl(excl, ow + step, 64);
        if (e <= t) ow += step;
      }
      const int e_o = __shfl(excl, ow, 64);
      const int bst_o = __shfl(B.bst, ow, 64), cnt_o = __shfl(B.cnt, ow, 64), code_o = __shfl(B.code, ow, 64);
      const int pack_o = __shfl(pack, ow, 64), base_o = __shfl(base, ow, 64);
      // (shuffles stay outside the branches below: a lane reads another's
      // register only while both are active)
      int bx_o = 0, by_o = 0, bz_o = 0;
      if (vl) {
        bx_o = __shfl(bb[0], ow, 64);
        by_o = __shfl(bb[1], ow, 64);
        bz_o = __shfl(bb[2], ow, 64);
      }
      int kx, ky, kz;
      decode(code_o, kx, ky, kz);
      const double sx = kx * g.L[0], sy = ky * g.L[1], sz = kz * g.L[2];
      int start = bst_o, count = t < total ? cnt_o : 0;
      const bool row = pack_o != 0 && t < total;
      const int ss = pack_o & 31, x0 = (pack_o >> 5) & 31, nx = (pack_o >> 10) & 31;
      const int y0 = (pack_o >> 15) & 31, ny = (pack_o >> 20) & 31, z0 = (pack_o >> 25) & 31;
      const int jr = t - e_o;
      const int ry = row ? y0 + jr % ny : 0, rz = row ? z0 + jr / ny : 0;
      bool take = row;
      if (vl) {
        // the row's box: sub-buckets x0 .. x0 + nx - 1 of row (ry, rz)
        double lo[3] = {0.0, 0.0, 0.0}, hi[3] = {0.0, 0.0, 0.0};
        if (row) {
          const double is = 1.0 / ss;
          lo[0] = (bx_o + x0 * is) * g.hb[0] + sx - r[0] - 1e-9 * g.hb[0];
          lo[1] = (by_o + ry * is) * g.hb[1] + sy - r[1] - 1e-9 * g.hb[1];
          lo[2] = (bz_o + rz * is) * g.hb[2] + sz - r[2] - 1e-9 * g.hb[2];
          hi[0] = (bx_o + (x0 + nx) * is) * g.hb[0] + sx - r[0] + 1e-9 * g.hb[0];
          hi[1] = (by_o + (ry + 1) * is) * g.hb[1] + sy - r[1] + 1e-9 * g.hb[1];
          hi[2] = (bz_o + (rz + 1) * is) * g.hb[2] + sz - r[2] + 1e-9 * g.hb[2];
        }
        take = boxes_may_cut(row, vl, nv, V, lo, hi, 1e-12 * hi2);
      }
      if (row) {
        count = 0;
        if (take) {
          const int ri = (rz * ss + ry) * ss + x0;
          const uint32_t* so = A.soffs + base_o;
          const int a0 = (int)so[ri], a1 = (int)so[ri + nx];
          start = bst_o + a0;
          count = a1 - a0;
        }
      }
      const int maxc = (int)wave_umax32((unsigned)count);
      for (int k = 0; k < maxc; ++k) {
        const int j = start + k;
        const bool v = k < count && j != s;
        double x = 0, y = 0, z = 0;
        if (v) {
          x = A.spos[3 * (int64_t)j];
          y = A.spos[3 * (int64_t)j + 1];
          z = A.spos[3 * (int64_t)j + 2];
        }
        const double dx = (x + sx) - r[0], dy = (y + sy) - r[1], dz = (z + sz) - r[2];
        const double d2 = dx * dx + dy * dy + dz * dz;
        bool keep = v && (d2 >= lo2) && (d2 < hi2);
        if (vl) keep = images_may_cut(keep, vl, nv, V, dx, dy, dz, d2);
        const unsigned long long mk = __ballot(keep);
        if (keep) {
          const int idx = nc + __popcll(mk & lanes_below());
          if (idx < kCands) {
            S.cd[idx] = make_double4(dx, dy, dz, 0.5 * d2);
            S.cjk[idx] = (j << 5) | code_o;
          }
        }
        nc += __popcll(mk);
      }
    }
  }
  return nc;
}

// Gathers the neighbour images with lo2 <= |d|^2 < hi2 from the stencil of
// half-width `ring` into LDS (at most kCands of them); returns their number.
// Each lane takes two buckets of the stencil at a time and the wave steps
// through their points together, so the loads of 128 buckets are in flight
// at once (two memory round trips for the usual 125-bucket stencil).  The
// generator's own images are not gathered: the box planes stand for them.
// With a vertex list (vl, nv) of the current cell, images that cannot cut it
// are left out (a cell next to a much denser region then sees only the few
// points that face it).
// Without RUNS (the first pass over all cells) a stencil chunk that holds a
// dense bucket ends the gather with -1: the cell goes to the first pass for
// cells near dense regions.
template <bool RUNS>
__device__ int gather(TessLds& S, const TessArgs& A, const GridParams& g, const int s, const double r[3],
                      const int b[3], const int ring, const double lo2, const double hi2,
                      const double4* vl = nullptr, int nv = 0) {
  const int W = 2 * ring + 1, W3 = W * W * W;
  const WidthDiv D = width_div((unsigned)W);
  const int lane = __lane_id();
  int nc = 0;
  for (int chunk = 0; chunk < W3; chunk += 128) {
    const StencilBucket B0 = stencil_bucket(A, g, b, ring, chunk + lane, W3, D);
    const StencilBucket B1 = stencil_bucket(A, g, b, ring, chunk + 64 + lane, W3, D);
    // With a vertex list every chunk takes the run path, whose boxes prune
    // whole buckets and rows.
    if (__ballot(B0.cnt > kDense || B1.cnt > kDense) || (RUNS && vl)) {
      if constexpr (!RUNS) return -1;
      nc = gather_runs(S, A, g, s, r, b, ring, chunk, W3, D, lo2, hi2, vl, nv, nc);
      continue;
    }
    const int maxc = (int)wave_umax32((unsigned)max(B0.cnt, B1.cnt));
    for (int k = 0; k < maxc; ++k) {
      const int j0 = B0.bst + k, j1 = B1.bst + k;
      const bool v0 = k < B0.cnt && j0 != s, v1 = k < B1.cnt && j1 != s;
      double x0 = 0, y0 = 0, z0 = 0, x1 = 0, y1 = 0, z1 = 0;
      if (v0) {
        x0 = A.spos[3 * (int64_t)j0];
        y0 = A.spos[3 * (int64_t)j0 + 1];
        z0 = A.spos[3 * (int64_t)j0 + 2];
      }
      if (v1) {
        x1 = A.spos[3 * (int64_t)j1];
        y1 = A.spos[3 * (int64_t)j1 + 1];
        z1 = A.spos[3 * (int64_t)j1 + 2];
      }
      const double dx0 = (x0 + B0.sx) - r[0], dy0 = (y0 + B0.sy) - r[1], dz0 = (z0 + B0.sz) - r[2];
      const double dx1 = (x1 + B1.sx) - r[0], dy1 = (y1 + B1.sy) - r[1], dz1 = (z1 + B1.sz) - r[2];
      const double d20 = dx0 * dx0 + dy0 * dy0 + dz0 * dz0;
      const double d21 = dx1 * dx1 + dy1 * dy1 + dz1 * dz1;
      bool keep0 = v0 && (d20 >= lo2) && (d20 < hi2);
      bool keep1 = v1 && (d21 >= lo2) && (d21 < hi2);
      if (vl) {
        if (keep0) keep0 = may_cut(vl, nv, dx0, dy0, dz0, d20);
        if (keep1) keep1 = may_cut(vl, nv, dx1, dy1, dz1, d21);
      }
      const unsigned long long mk0 = __ballot(keep0), mk1 = __ballot(keep1);
      if (keep0) {
        const int idx = nc + __popcll(mk0 & lanes_below());
        if (idx < kCands) {
          S.cd[idx] = make_double4(dx0, dy0, dz0, 0.5 * d20);
          S.cjk[idx] = (j0 << 5) | B0.code;
        }
      }
      const int n0 = __popcll(mk0);
      if (keep1) {
        const int idx = nc + n0 + __popcll(mk1 & lanes_below());
        if (idx < kCands) {
          S.cd[idx] = make_double4(dx1, dy1, dz1, 0.5 * d21);
          S.cjk[idx] = (j1 << 5) | B1.code;
        }
      }
      nc += n0 + __popcll(mk1);
    }
  }
  wave_sync();
  return nc;
}

// Orders the gathered candidates by distance; ties by neighbour and image,
// so the order does not depend on how the stencil was walked.  Exact ties
// are rare (lattice symmetries), so the ranks are first taken by distance
// alone and redone with the identities only when some distance repeats.
__device__ void sort_candidates(TessLds& S, const int nc) {
  // Rank by distance alone; with no repeated distance the ranks are a
  // permutation, and a repeated one makes two candidates write the same
  // slot, which the read-back shows.
  int lt0 = 0, lt1 = 0;
  const int c0 = __lane_id(), c1 = __lane_id() + 64;
  if (nc <= 64) {
    if (c0 < nc) {
      const double k0 = S.cd[c0].w;
      for (int m = 0; m < nc; ++m) lt0 += S.cd[m].w < k0;
      S.order[lt0] = (uint8_t)c0;
    }
  } else {
    const double k0 = S.cd[c0].w, k1 = c1 < nc ? S.cd[c1].w : 0.0;
    for (int m = 0; m < nc; ++m) {
      const double km = S.cd[m].w;
      lt0 += km < k0;
      lt1 += km < k1;
    }
    S.order[lt0] = (uint8_t)c0;
    if (c1 < nc) S.order[lt1] = (uint8_t)c1;
  }
  wave_sync();
  const bool tie = (c0 < nc && S.order[lt0] != c0) || (c1 < nc && S.order[lt1] != c1);
  if (__ballot(tie) == 0ull) return;
  wave_sync();
  for (int c = __lane_id(); c < nc; c += 64) {
    const double key = S.cd[c].w;
    const int id = S.cjk[c];
    int rank = 0;
    for (int m = 0; m < nc; ++m) {
      const double km = S.cd[m].w;
      rank += (km < key) || (km == key && (S.cjk[m] < id || (S.cjk[m] == id && m < c)));
    }
    S.order[rank] = (uint8_t)c;
  }
  wave_sync();
}

// A value every lane holds equally (read from LDS at a uniform address),
// moved to a scalar register so branches on it are uniform.
__device__ inline int uniform_i32(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Squared distance bound of the farthest live vertex (float, rounded up).
__device__ inline double farthest_bound(const CellRegs& C) {
  double m2 = 0.0;
  if (lane_on(C.L0)) m2 = C.v0x * C.v0x + C.v0y * C.v0y + C.v0z * C.v0z;
  if (C.L1 != 0ull && lane_on(C.L1)) m2 = fmax(m2, C.v1x * C.v1x + C.v1y * C.v1y + C.v1z * C.v1z);
  return wave_max_bound(m2);
}

// Cuts the cell by the ordered candidates, stopping at the first one farther
// than twice the farthest vertex (Sec. 3).  Returns 0 or a failure bit.
// A cut only moves vertices inward (new vertices are convex combinations of
// old ones), so the bound of the farthest vertex stays valid after a cut: it
// is recomputed after every fourth cut, when the stop test would fire, and
// at the end.
__device__ int clip_candidates(TessLds& S, const int nc, CellRegs& C) {
  const int lane = __lane_id();
  bool stale = false;
  int since = 0;   // cuts since the bound was last recomputed
  double lim = 2.0 * C.rmax2;   // a candidate with |d|^2 / 2 >= lim cannot cut
  for (int k = 0; k < nc; ++k) {
    // Every lane reads the same candidate (an LDS broadcast); it stays in
    // vector registers, and the stop test is made uniform by a ballot.
    const int c = S.order[k];
    const double4 q = S.cd[c];
    const double h = q.w;                 // |d|^2 / 2: the plane's offset
    if (__ballot(h >= lim)) {   // farther images cannot cut the cell
      if (!stale) break;
      C.rmax2 = farthest_bound(C);
      stale = false;
      since = 0;
      lim = 2.0 * C.rmax2;
      if (__ballot(h >= lim)) break;
    }
    // Most cells keep every vertex in the first register (64 slots); the
    // second register's work is skipped while it holds none (a
    // wavefront-uniform test).
    const bool two = C.L1 != 0ull;
    // The test runs on every slot; the live masks (wavefront-uniform) keep
    // the live ones.
    const unsigned long long M0 = __ballot(q.x * C.v0x + q.y * C.v0y + q.z * C.v0z > h) & C.L0;
    unsigned long long M1 = 0ull;
    if (two) M1 = __ballot(q.x * C.v1x + q.y * C.v1y + q.z * C.v1z > h) & C.L1;
    if ((M0 | M1) == 0ull) continue;
    const bool live0 = lane_on(C.L0), live1 = two && lane_on(C.L1);
    const bool out0 = lane_on(M0), out1 = lane_on(M1);

    // Plane slot for the new face: the next unused slot while there is one,
    // then the lowest slot no surviving vertex uses.
    const bool kept0 = live0 && !out0, kept1 = live1 && !out1;
    int p;
    if (C.np < kPlanes) {
      p = C.np++;
    } else {
      unsigned long long u = 0ull;
      if (kept0) u |= plane_bits(C.t0);
      if (kept1) u |= plane_bits(C.t1);
      const unsigned long long used = wave_or(u);
      if (used == ~0ull) return F_PLANES;
      p = __builtin_ctzll(~used);
    }

    // Boundary of the removed cap: edges of removed vertices whose
    // neighbour across the edge survives (bit k of bm: edge k of the slot).
    const unsigned long long L0 = C.L0, L1 = C.L1;
    // Which slots survive the cut, as bytes every lane can look up.
    S.kept[lane] = (uint8_t)kept0;
    if (two) S.kept[lane + 64] = (uint8_t)kept1;   // (no live triangle refers to these slots otherwise)
    wave_sync();
    auto boundary = [&](uint32_t T) -> int {
      const int a = T & 255, bq = (T >> 8) & 255, cq = (T >> 16) & 255;
      const int m0 = S.kept[S.E[bq * kPlanes + a] & (kVerts - 1)];
      const int m1 = S.kept[S.E[cq * kPlanes + bq] & (kVerts - 1)];
      const int m2 = S.kept[S.E[a * kPlanes + cq] & (kVerts - 1)];
      return m0 | (m1 << 1) | (m2 << 2);
    };
    const int bm0 = out0 ? boundary(C.t0) : 0;
    const int bm1 = out1 ? boundary(C.t1) : 0;
    const int nbl = __popc(bm0) + __popc(bm1);
    int B;
    const int pre = wave_excl_scan(nbl, &B);

    const unsigned long long F0 = ~L0 | M0, F1 = ~L1 | M1;   // free slots after the cut
    const int nf0 = __popcll(F0);
    if (B > nf0 + __popcll(F1)) return F_VERTS;
    if (lane == 0) {
      S.pl[p] = make_double4(q.x, q.y, q.z, h);
      S.pcand[p] = S.cjk[c];   // the neighbour itself: later shells reuse the candidate slots
    }
    // Boundary edges into a list, in prefix order.
    int e = pre;
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      if (sl == 1 && !two) break;
      const uint32_t T = sl ? C.t1 : C.t0;
      const int bm = sl ? bm1 : bm0;
      const int ta = T & 255, tb = (T >> 8) & 255, tc = (T >> 16) & 255;
      if (bm & 1) S.elist[e++] = (uint16_t)(ta | (tb << 8));
      if (bm & 2) S.elist[e++] = (uint16_t)(tb | (tc << 8));
      if (bm & 4) S.elist[e++] = (uint16_t)(tc | (ta << 8));
    }
    wave_sync();   // every E lookup above is done before any write below

    // One new vertex per boundary edge: the fan of triangles (x, y, p)
    // around the new face.  Boundary edge r goes to the free slot of rank r
    // (slots of the first register in lane order, then of the second), and
    // the lane holding that slot builds it in place.
    const double4 qp = make_double4(q.x, q.y, q.z, h);
    const int r0 = __popcll(F0 & lanes_below());
    const int r1 = nf0 + __popcll(F1 & lanes_below());
    const bool new0 = lane_on(F0) && r0 < B;
    const bool new1 = lane_on(F1) && r1 < B;
    if (new0) {
      const int xy = S.elist[r0];
      const int x = xy & 255, y = xy >> 8;
      C.t0 = (uint32_t)(x | (y << 8) | (p << 16));
      intersect3(S.pl[x], S.pl[y], qp, C.v0x, C.v0y, C.v0z);
      S.E[x * kPlanes + y] = (uint8_t)lane;
      S.E[y * kPlanes + p] = (uint8_t)lane;
      S.E[p * kPlanes + x] = (uint8_t)lane;
    }
    if (new1) {
      const int xy = S.elist[r1];
      const int x = xy & 255, y = xy >> 8;
      C.t1 = (uint32_t)(x | (y << 8) | (p << 16));
      intersect3(S.pl[x], S.pl[y], qp, C.v1x, C.v1y, C.v1z);
      S.E[x * kPlanes + y] = (uint8_t)(lane + 64);
      S.E[y * kPlanes + p] = (uint8_t)(lane + 64);
      S.E[p * kPlanes + x] = (uint8_t)(lane + 64);
    }
    wave_sync();
    const bool nl0 = kept0 || new0;
    const bool nl1 = kept1 || new1;
    C.L0 = __ballot(nl0);
    C.L1 = two || B > nf0 ? __ballot(nl1) : 0ull;
    stale = true;
    if (++since == 4) {
      C.rmax2 = farthest_bound(C);
      lim = 2.0 * C.rmax2;
      stale = false;
      since = 0;
    }
  }
  if (stale) C.rmax2 = farthest_bound(C);
  return 0;
}

// Faces, volume and centroid of the finished cell; writes the cell's outputs.
__device__ int finish_cell(TessLds& S, const TessArgs& A, const int s, const CellRegs& C) {
  const int lane = __lane_id();
  const bool live0 = lane_on(C.L0), live1 = lane_on(C.L1);
  // The candidate list is dead now: its storage takes the vertex copies.
  wave_sync();
  S.vx[lane] = C.v0x; S.vy[lane] = C.v0y; S.vz[lane] = C.v0z;
  S.tri[lane] = C.t0;
  if (C.L1 != 0ull) {
    S.vx[lane + 64] = C.v1x; S.vy[lane + 64] = C.v1y; S.vz[lane + 64] = C.v1z;
    S.tri[lane + 64] = C.t1;
  }
  S.first[lane] = kVerts;
  wave_sync();
  if (live0) {
    atomicMin(&S.first[C.t0 & 255], lane);
    atomicMin(&S.first[(C.t0 >> 8) & 255], lane);
    atomicMin(&S.first[(C.t0 >> 16) & 255], lane);
  }
  if (live1) {
    atomicMin(&S.first[C.t1 & 255], lane + 64);
    atomicMin(&S.first[(C.t1 >> 8) & 255], lane + 64);
    atomicMin(&S.first[(C.t1 >> 16) & 255], lane + 64);
  }
  wave_sync();
  unsigned long long ul = 0ull;
  if (live0) ul |= plane_bits(C.t0);
  if (live1) ul |= plane_bits(C.t1);
  const unsigned long long usedL = wave_or(ul);

  // Lane p integrates the polygon of face p as a fan from its first vertex:
  // the walk goes counter-clockwise seen from outside, so the area along the
  // outward normal is positive.
  const int p = lane;
  const bool valid = (usedL >> p) & 1ull;
  double Af = 0.0, fx = 0.0, fy = 0.0, fz = 0.0, dl = 0.0;
  bool walk_bad = false;
  if (valid) {
    const double4 P = S.pl[p];
    dl = sqrt(2.0 * P.w);
    const double idl = 1.0 / dl;
    const double nx = P.x * idl, ny = P.y * idl, nz = P.z * idl;
    const int tstart = S.first[p];
    const double ox = S.vx[tstart], oy = S.vy[tstart], oz = S.vz[tstart];
    int t = tstart, it = 0;
    double as = 0.0, mx = 0.0, my = 0.0, mz = 0.0;
    do {
      const uint32_t T = S.tri[t];
      const int a = T & 255, bq = (T >> 8) & 255, cq = (T >> 16) & 255;
      const int z = (a == p) ? cq : (bq == p ? a : bq);
      const int tn = S.E[p * kPlanes + z] & (kVerts - 1);
      const double x1 = S.vx[t] - ox, y1 = S.vy[t] - oy, z1 = S.vz[t] - oz;
      const double x2 = S.vx[tn] - ox, y2 = S.vy[tn] - oy, z2 = S.vz[tn] - oz;
      const double ar = 0.5 * ((y1 * z2 - z1 * y2) * nx + (z1 * x2 - x1 * z2) * ny + (x1 * y2 - y1 * x2) * nz);
      as += ar;
      mx += ar * (x1 + x2);
      my += ar * (y1 + y2);
      mz += ar * (z1 + z2);
      t = tn;
      ++it;
    } while (t != tstart && it < kVerts);
    walk_bad = (t != tstart);
    Af = as;
    const double i3a = 1.0 / (3.0 * as);
    fx = ox + mx * i3a;
    fy = oy + my * i3a;
    fz = oz + mz * i3a;
  }
  if (__ballot(walk_bad)) return F_WALK;
  // A plane that only touches the cell gives no face (non-positive area).
  const bool keep = valid && Af > 0.0;
  const double vol = keep ? Af * dl / 6.0 : 0.0;
  const double V = wave_sum(vol);
  const double iV = 1.0 / V;
  const double cxr = wave_sum(keep ? 0.75 * vol * fx : 0.0) * iV;
  const double cyr = wave_sum(keep ? 0.75 * vol * fy : 0.0) * iV;
  const double czr = wave_sum(keep ? 0.75 * vol * fz : 0.0) * iV;
  if (!(V > 0.0)) return F_VOLUME;

  int j = s, code = 13;
  if (keep) {
    const int pc = S.pcand[p];
    if (pc >= 0) {
      j = pc >> 5;
      code = pc & 31;
    } else {
      const int bp = -1 - pc;   // box plane: axis bp/2, sign by parity
      const int step = (bp >> 1) == 0 ? 1 : ((bp >> 1) == 1 ? 3 : 9);
      code = (bp & 1) ? 13 - step : 13 + step;
    }
  }
  const bool owned = keep && (j > s || (j == s && code > 13));
  const unsigned long long MK = __ballot(keep), MO = __ballot(owned);
  if (keep) {
    const int idx = __popcll(MK & lanes_below());
    const int orank = __popcll(MO & lanes_below());
    StageNbr nb;
    nb.j = j;
    nb.meta = code | ((owned ? 1 : 0) << 8) | (orank << 16);
    A.stage_nb[(int64_t)s * kMaxFaces + idx] = nb;
    StageGeo& F = A.stage_geo[(int64_t)s * kMaxFaces + idx];
    F.A = Af;
    F.f[0] = fx;
    F.f[1] = fy;
    F.f[2] = fz;
  }
  if (lane == 0) {
    A.counts[s] = ((unsigned long long)__popcll(MK) << 32) | (unsigned long long)__popcll(MO);
    double* gp = A.geo + 4 * (int64_t)s;
    gp[0] = V;
    gp[1] = cxr;
    gp[2] = cyr;
    gp[3] = czr;
  }
  return 0;
}

// The live vertices of the cell (relative to the generator, w = |v|^2),
// compacted into vl; returns their number, or 0 (no list) when there are
// more than kPruneVerts.
__device__ int vertex_list(const CellRegs& C, double4* vl) {
  const int n0 = __popcll(C.L0), n = n0 + __popcll(C.L1);
  if (n > kPruneVerts) return 0;
  if (lane_on(C.L0))
    vl[__popcll(C.L0 & lanes_below())] =
        make_double4(C.v0x, C.v0y, C.v0z, C.v0x * C.v0x + C.v0y * C.v0y + C.v0z * C.v0z);
  if (lane_on(C.L1))
    vl[n0 + __popcll(C.L1 & lanes_below())] =
        make_double4(C.v1x, C.v1y, C.v1z, C.v1x * C.v1x + C.v1y * C.v1y + C.v1z * C.v1z);
  wave_sync();
  return n;
}

// Points in the cell's own bucket.  Buckets are sized for the mean spacing,
// so a bucket holding cnt > 4 points marks a denser region, whose
// first-candidate radius shrinks: by cbrt(4/cnt) up to kDense points, and
// for a bucket with a sub-grid by cbrt(ppb/cnt), the ratio of the local
// spacing to the mean one, which keeps the expected number of candidates of
// a uniform region.  Uniform inputs (a few points per bucket) keep the
// grid's radius.
__device__ inline unsigned own_count(const TessArgs& A, const GridParams& g, const int b[3]) {
  const int64_t key = g.base + bucket_key(g.nb, b[0], b[1], b[2]);
  return (unsigned)(A.boff[key + 1] - A.boff[key]);
}

__device__ void defer_cell(const TessArgs& A, int s, double rmax2) {
  if (__lane_id() == 0) {
    const int idx = atomicAdd(&A.st->n_deferred, 1);
    A.deferred[idx] = s;
    A.rmax2[s] = rmax2;
  }
}

// Hands a cell with a dense bucket in its stencil to the dense first pass.
__device__ void defer_dense(const TessArgs& A, int s) {
  if (__lane_id() == 0) A.dcells[atomicAdd(&A.st->n_dense_cells, 1)] = s;
}

// Squared outer radius of the next shell after [sqrt(lo2), sqrt(hi2)), which
// held nc candidates: twice the farthest vertex (the shell the cell needs),
// at most twice sqrt(hi2), and at most the radius that holds about `want`
// more at the density found (so the shell seldom overflows the candidate
// slots; a cell that needs more goes on with another shell).
__device__ inline double next_shell(double rmax2, double lo2, double hi2, int nc, double want) {
  double n2 = fmin(4.0 * rmax2 * (1.0 + 1e-9), 4.0 * hi2);
  if (nc > 0) {
    const double lo3 = lo2 * sqrt(lo2), hi3 = hi2 * sqrt(hi2);
    const double r = cbrt(hi3 + want * (hi3 - lo3) / (double)nc);
    n2 = fmin(n2, fmax(r * r, hi2 * (1.0 + 1e-6)));
  }
  return n2;
}

// Builds the cell of internal generator s.
// MODE 0 (first pass of the cells the two-cell pass hands on): candidates
//   within the grid's filter radius; a cell whose candidates do not cover
//   twice its farthest vertex goes on with up to kShells1 more shells (when
//   it found at least kFewCands candidates), and one that still falls short
//   (or overflows the candidate slots) is deferred to the shell pass; a cell
//   with a dense bucket in its own bucket or stencil goes to MODE 1.
// MODE 1 (first pass of the cells near dense regions): the same with the
//   two-level gather.
// MODE 2 (shell pass): distance shells [lo, hi) processed in order, each
//   gathered from a stencil wide enough for it and narrowed until it fits
//   the candidate slots, until twice the farthest vertex lies inside the
//   shells done.  The first shell ends at twice the farthest vertex found
//   before, which bounds the true one (that cell contains the true cell).
template <int MODE>
__device__ void tess_cell(TessLds& S, const TessArgs& A, const int s, double4* vl = nullptr) {
  const int seg = A.sseg[s];
  const GridParams& g = A.segs[seg].g;   // read in place (wave-uniform loads), never copied
  const double r[3] = {A.spos[3 * (int64_t)s], A.spos[3 * (int64_t)s + 1], A.spos[3 * (int64_t)s + 2]};
  int b[3];
  double edge[3];   // distance from the generator to its bucket's nearer wall, per axis
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    b[a] = bucket_coord(r[a], g.inv_hb[a], g.nb[a]);
    const double t = r[a] - b[a] * g.hb[a];
    edge[a] = fmax(0.0, fmin(t, g.hb[a] - t));
  }
  CellRegs C;
  init_box(S, g, C);
  const unsigned cnt = uniform_i32((int)own_count(A, g, b));
  const bool dense = cnt > 4u;
  const double rloc = !dense ? g.r_filter
                              : g.r_filter * cbrt((cnt > (unsigned)kDense ? g.ppb : 4.0) / (double)cnt);

  if (MODE == 0 && cnt > (unsigned)kDense) {
    // Listed for the dense first pass by the sort, unless the bucket is
    // beyond what the sort orders: then the call fails (the sort has
    // flagged it) and the cell gets empty outputs here.
    if (cnt > (unsigned)kDenseMax) fail_cell(A, s, seg, F_DENSE);
    return;
  }
  if (MODE < 2) {
    const int ring = dense ? min(g.ring, ring_for(g, edge, rloc * rloc)) : g.ring;
    double reach = 1e300;
#pragma unroll
    for (int a = 0; a < 3; ++a) reach = fmin(reach, ring * g.hb[a] + edge[a]);
    double hi2 = fmin(reach * reach, rloc * rloc);
    int nc = gather<MODE != 0>(S, A, g, s, r, b, ring, 0.0, hi2);
    if (nc < 0) {
      defer_dense(A, s);
      return;
    }
    if (MODE == 0 && nc < kFewCands) {
      // A thin region: the first radius, sized for the mean spacing, holds
      // few neighbours.  It grows, in one wider gather, to the radius that
      // holds as many neighbours as the first radius holds on average at
      // the mean density (the count found gives the local density), when
      // that stencil stays narrow enough; otherwise the cell goes to the
      // shell pass as before.
      const double mean_cands = 4.18879020478639 * (g.r_filter * g.r_filter * g.r_filter) * g.ppb /
                                (g.hb[0] * g.hb[1] * g.hb[2]);   // (4 pi / 3) r^3 times the mean density
      const double rt = g.r_filter * cbrt(mean_cands / (double)max(nc, 1));
      const double nhi2 = rt * rt;
      const int nring = ring_for(g, edge, nhi2);
      if (nhi2 > hi2 && nring <= kThinRing && nring <= g.nb[0] && nring <= g.nb[1] && nring <= g.nb[2]) {
        nc = gather<false>(S, A, g, s, r, b, nring, 0.0, nhi2);
        if (nc < 0) {
          defer_dense(A, s);
          return;
        }
        hi2 = nhi2;
      }
    }
    if (nc > kCands) {
      if (__lane_id() == 0) atomicAdd(&A.st->n_overflow, 1);
      defer_cell(A, s, -1.0);
      return;
    }
    sort_candidates(S, nc);
    if (int bad = clip_candidates(S, nc, C)) {
      fail_cell(A, s, seg, bad);
      return;
    }
    // A cell whose candidates fell short of twice its farthest vertex goes
    // on with a few more shells here (irregular inputs need them often);
    // one that still falls short, or whose next shell overflows even when
    // narrowed, is deferred with its farthest-vertex bound.
    double lo2 = 0.0;
    int last = nc;   // candidates of the last gather, between sqrt(lo2) and sqrt(hi2)
    for (int shell = 0; !(4.0 * C.rmax2 <= hi2 * (1.0 - 1e-12)); ++shell) {
      const double nhi2 = next_shell(C.rmax2, lo2, hi2, last, 70.0);
      const int nring = ring_for(g, edge, nhi2);
      // (A thin region's cell, with few candidates found, needs wide shells
      // that only the shell pass's pruning keeps cheap.)
      if (shell == kShells1 || (MODE == 0 && nc < kFewCands) || nring > g.nb[0] || nring > g.nb[1] ||
          nring > g.nb[2]) {
        defer_cell(A, s, C.rmax2);
        return;
      }
      lo2 = hi2;
      hi2 = nhi2;
      int nc2 = gather<MODE != 0>(S, A, g, s, r, b, nring, lo2, hi2);
      if (nc2 < 0) {
        defer_dense(A, s);
        return;
      }
      // A shell that overflows (its radius may double) is narrowed, as in
      // the shell pass; the next shell goes on from there.
      for (int t = 0; nc2 > kCands && t < 2; ++t) {
        hi2 = lo2 + 0.5 * (hi2 - lo2);
        nc2 = gather<MODE != 0>(S, A, g, s, r, b, nring, lo2, hi2);
      }
      if (nc2 > kCands) {
        defer_cell(A, s, C.rmax2);
        return;
      }
      last = nc2;
      sort_candidates(S, nc2);
      if (int bad = clip_candidates(S, nc2, C)) {
        fail_cell(A, s, seg, bad);
        return;
      }
    }
  } else {
    // Shells [lo2, hi2) of growing radius.  Each next shell reaches twice
    // the current farthest vertex but at most twice the previous radius, so
    // a cell that still touched the starting box after the first pass does
    // not ask for a stencil as wide as the box at once.
    const double rm2 = A.rmax2[s];
    const double rf2 = rloc * rloc;
    double lo2 = 0.0;
    // The first shell holds about twice the first pass's expected
    // candidates (a wider one overflowed and was halved, often twice).
    double hi2 = rm2 > 0.0 ? fmin(4.0 * rm2 * (1.0 + 1e-9), 1.55 * rf2) : rf2;
    bool done = false;
    for (int shell = 0; shell < kShells && !done; ++shell) {
      const int ring = ring_for(g, edge, hi2);
      if (ring > g.nb[0] || ring > g.nb[1] || ring > g.nb[2]) {
        fail_cell(A, s, seg, F_BOX);
        return;
      }
      // Buckets, sub-bucket rows and points that cannot cut the cell are
      // left out (a cell next to a much denser region sees only the few
      // points that face it).  The first shell starts from the box, which
      // prunes nothing: it takes the plain gather.
      const int nv = shell > 0 ? vertex_list(C, vl) : 0;
      const double4* vlp = nv ? vl : nullptr;
      int nc = gather<true>(S, A, g, s, r, b, ring, lo2, hi2, vlp, nv);
      for (int tries = 0; nc > kCands && tries < 40; ++tries) {
        hi2 = lo2 + 0.5 * (hi2 - lo2);
        nc = gather<true>(S, A, g, s, r, b, ring, lo2, hi2, vlp, nv);
      }
      if (nc > kCands) {
        fail_cell(A, s, seg, F_CANDS);
        return;
      }
      sort_candidates(S, nc);
      if (int bad = clip_candidates(S, nc, C)) {
        fail_cell(A, s, seg, bad);
        return;
      }
      if (4.0 * C.rmax2 <= hi2 * (1.0 - 1e-12)) {
        done = true;
      } else {
        const double grow = fmin(4.0 * C.rmax2 * (1.0 + 1e-9), 4.0 * hi2);
        lo2 = hi2;
        hi2 = grow;
      }
    }
    if (!done) {
      fail_cell(A, s, seg, F_INCOMPLETE);
      return;
    }
  }
  if (int bad = finish_cell(S, A, s, C)) fail_cell(A, s, seg, bad);
}

// Four waves per SIMD, with some values of the two-level gather and the
// extra shells spilled (at three, without spills, it is slower).
// The cells of dense regions that the two-cell dense pass handed on, then
// the listed ones beyond its grid.
__global__ __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(4))) void k_tess_pass1_dense(
    TessArgs A) {
  __shared__ TessLds lds[kWaves];
  const int w = threadIdx.x >> 6;
  const int64_t nr = A.st->n_dredo;
  const int64_t nx = max((int64_t)0, (int64_t)A.st->n_dense_cells - A.dense_cap);
  for (int64_t it = (int64_t)blockIdx.x * kWaves + w; it < nr + nx; it += (int64_t)gridDim.x * kWaves)
    tess_cell<1>(lds[w], A, it < nr ? A.redo[it] : A.dcells[A.dense_cap + (it - nr)]);
}

__global__ __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(3))) void k_tess_pass2(TessArgs A) {
  __shared__ TessLds lds[kWaves];
  __shared__ double4 verts[kWaves][kPruneVerts];   // the cell's live vertices, for pruning candidates
  const int w = threadIdx.x >> 6;
  const int nd = A.st->n_deferred;
  for (int64_t it = (int64_t)blockIdx.x * kWaves + w; it < nd; it += (int64_t)gridDim.x * kWaves)
    tess_cell<2>(lds[w], A, A.deferred[it], verts[w]);
}

// ---------------------------------------------------------------------------
// The first passes with two cells per wavefront (lean and dense).
//
// One wavefront builds one cell above, and most of the work of a cut (the
// plane slot, the cap's boundary, the new vertices of the fan) occupies a
// few lanes while the others wait.  Here each half of the wavefront (32
// lanes) builds its own cell with the same steps, so one instruction serves
// two cells.  A half holds 64 vertex slots (two per lane), 40 plane slots
// and 48 candidates, 5 KB of LDS per cell, so 32 cells fit a CU (twice the
// one-cell pass): the usual cell of the uniform inputs (about 16 faces, 28
// vertices, 29 candidates) fits with room to spare.  A cell that needs more
// slots, more distance shells than its pass takes (one extra in the lean
// pass, three in the dense one), or (lean pass) a thin region's wider first
// radius is handed to the one-cell pass of its kind, which builds it as
// before; a lean cell whose stencil holds a dense bucket is listed for the
// dense passes.  Values that are uniform per cell are uniform per half here:
// held in each lane of the half, and the half's 32 bits of every ballot are
// its masks (the cut loop keeps its per-half flags as wavefront masks and
// counters in scalar registers instead).
// ---------------------------------------------------------------------------
constexpr int kPlanesP = 40;
constexpr int kVertsP = 64;
constexpr int kCandsP = 48;

struct __align__(16) PairLds {
  double4 pl[kPlanesP];
  union {
    struct {                           // while the cell is cut
      double4 cd[kCandsP];
      int32_t cjk[kCandsP];
      uint8_t order[kCandsP];
      uint16_t elist[kVertsP];
    };
    struct {                           // in the epilogue
      double vx[kVertsP], vy[kVertsP], vz[kVertsP];
      int32_t first[kPlanesP];
      uint32_t tri[kVertsP];
    };
  };
  int32_t pcand[kPlanesP];
  uint8_t E[kPlanesP * kPlanesP];
};
static_assert(sizeof(PairLds) <= 5120, "32 cells per CU");

__device__ __forceinline__ int hlane() { return __lane_id() & 31; }
// The 32 bits of a wavefront mask that belong to this lane's half.
__device__ __forceinline__ unsigned hbits(unsigned long long m) { return (unsigned)(m >> (__lane_id() & 32)); }
__device__ __forceinline__ unsigned hbelow() { return (1u << hlane()) - 1u; }
// All lanes of each half whose 32 bits of m are not all zero.
__device__ __forceinline__ unsigned long long halves_of(unsigned long long m) {
  return ((unsigned)m ? 0xffffffffull : 0ull) | ((m >> 32) ? 0xffffffff00000000ull : 0ull);
}

// Inclusive prefix sum within each half: row shifts by 1, 2, 4 and 8 inside
// each row of 16 lanes (lanes shifted in from outside the row read 0), then
// the last lane of row 0 added to row 1 and that of row 2 to row 3.  Called
// by the whole wavefront.
__device__ __forceinline__ int half_incl_scan(int x) {
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xF, 0xF, true);
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xF, 0xF, true);
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xF, 0xF, true);
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xF, 0xF, true);
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xA, 0xF, false);
  return x;
}

// Reductions over each half: within rows of 16 by quad permutes and row
// rotations, then row 0 into row 1 and row 2 into row 3; lanes 31 and 63
// end with the two halves' results.
#define MM_DPP_REDUCE_HALF(OP, x)                                                   \
  do {                                                                              \
    x = OP(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xF, 0xF, false));  \
    x = OP(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x4E, 0xF, 0xF, false));  \
    x = OP(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x124, 0xF, 0xF, false)); \
    x = OP(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x128, 0xF, 0xF, false)); \
    x = OP(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false)); \
  } while (0)

__device__ __forceinline__ unsigned half_pick(unsigned x) {
  const unsigned a = (unsigned)__builtin_amdgcn_readlane((int)x, 31);
  const unsigned b = (unsigned)__builtin_amdgcn_readlane((int)x, 63);
  return (__lane_id() & 32) ? b : a;
}

__device__ __forceinline__ unsigned half_umax32(unsigned x) {
  MM_DPP_REDUCE_HALF(op_max, x);
  return half_pick(x);
}


// Upper bound of the half's largest non-negative finite value (as
// wave_max_bound).
__device__ __forceinline__ double half_max_bound(double x) {
  const unsigned hi = (unsigned)((unsigned long long)__double_as_longlong(x) >> 32) + 1u;
  return __longlong_as_double((long long)((unsigned long long)half_umax32(hi) << 32));
}

// Butterfly sum within each half: every lane of a half ends with the
// bitwise-same result.
__device__ __forceinline__ double half_sum(double x) {
#pragma unroll
  for (int o = 16; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// One half's cell: vertex slots hl and hl + 32 of lane hl; L0w, L1w are the
// wavefront's live masks (this half's bits by hbits); np, rmax2 uniform per
// half.
struct PairRegs {
  unsigned long long L0w, L1w;
  uint32_t t0, t1;
  double v0x, v0y, v0z, v1x, v1y, v1z;
  double rmax2;
  int np;
};

__device__ void init_box_pair(PairLds& S, const GridParams& g, PairRegs& C) {
  const int hl = hlane();
  if (hl < 6) {
    const int ax = hl >> 1;
    const double sg = (hl & 1) ? -1.0 : 1.0;
    double d[3] = {0.0, 0.0, 0.0};
    d[ax] = sg * g.L[ax];
    S.pl[hl] = make_double4(d[0], d[1], d[2], 0.5 * (g.L[ax] * g.L[ax]));
    S.pcand[hl] = -1 - hl;
  }
  C.t0 = C.t1 = 0u;
  C.v0x = C.v0y = C.v0z = C.v1x = C.v1y = C.v1z = 0.0;
  if (hl < 8) {
    const int sx = (hl & 1) ? -1 : 1, sy = (hl & 2) ? -1 : 1, sz = (hl & 4) ? -1 : 1;
    const int px = sx > 0 ? 0 : 1, py = sy > 0 ? 2 : 3, pz = sz > 0 ? 4 : 5;
    int a1 = py, a2 = pz;
    if (sx * sy * sz < 0) { a1 = pz; a2 = py; }   // orientation: det(d_a, d_b, d_c) > 0
    C.t0 = (uint32_t)(px | (a1 << 8) | (a2 << 16));
    C.v0x = sx * (0.5 * g.L[0]);
    C.v0y = sy * (0.5 * g.L[1]);
    C.v0z = sz * (0.5 * g.L[2]);
    S.E[px * kPlanesP + a1] = (uint8_t)hl;
    S.E[a1 * kPlanesP + a2] = (uint8_t)hl;
    S.E[a2 * kPlanesP + px] = (uint8_t)hl;
  }
  wave_sync();
  C.L0w = __ballot(hl < 8);
  C.L1w = 0ull;
  C.np = 6;
  C.rmax2 = half_max_bound(hl < 8 ? C.v0x * C.v0x + C.v0y * C.v0y + C.v0z * C.v0z : 0.0);
}

__device__ inline double farthest_bound_pair(const PairRegs& C) {
  double m2 = 0.0;
  if (lane_on(C.L0w)) m2 = C.v0x * C.v0x + C.v0y * C.v0y + C.v0z * C.v0z;
  if (lane_on(C.L1w)) m2 = fmax(m2, C.v1x * C.v1x + C.v1y * C.v1y + C.v1z * C.v1z);
  return half_max_bound(m2);
}

// The gather of both halves: images with lo2 <= |d|^2 < hi2 from each
// half's stencil of half-width `ring`.  The lean pass takes four stencil
// buckets per lane at a time (the usual 125-bucket stencil in one memory
// round trip, as in the one-cell gather); the dense pass one (its stencils
// are small, and the registers spared shrink its spill: the polytropes'
// dense cells 6% faster than with two, 10% than with four).  Returns the
// number of images this half found (more than kCandsP: an overflow, of
// which only the first kCandsP are stored).
// Without RUNS (the lean pass) a stencil that holds a dense bucket gives -1;
// with RUNS a chunk of the stencil that holds one, in either half, is taken
// by the two-level gather of both halves.  Called by the whole wavefront
// (act: the half has a cell).
constexpr int kPairBuckets = 4;

__device__ int gather_runs_pair(PairLds& S, const TessArgs& A, const GridParams& g, const int s, const double r[3],
                                const int b[3], const int ring, const int chunk, const int nb, const int W3,
                                const WidthDiv& D, const double lo2, const double hi2, int nc);

template <bool RUNS>
__device__ int gather_pair(PairLds& S, const TessArgs& A, const GridParams& g, bool act, const int s,
                           const double r[3], const int b[3], const int ring, const double lo2, const double hi2) {
  const int hl = hlane();
  const int W = 2 * ring + 1, W3 = act ? W * W * W : 0;
  const WidthDiv D = width_div((unsigned)W);
  const int W3max = (int)wave_umax32((unsigned)W3);
  int nc = 0;
  bool dense = false;
  constexpr int NB = RUNS ? 1 : kPairBuckets;   // stencil buckets per lane and chunk
  for (int chunk = 0; chunk < W3max; chunk += 32 * NB) {
    StencilBucket B[NB];
    bool dn = false;
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      B[u] = stencil_bucket(A, g, b, ring, chunk + 32 * u + hl, W3, D);
      dn |= B[u].cnt > kDense;
    }
    if constexpr (RUNS) {
      if (__ballot(dn)) {
        nc = gather_runs_pair(S, A, g, s, r, b, ring, chunk, NB, W3, D, lo2, hi2, nc);
        continue;
      }
    } else {
      dense |= hbits(__ballot(dn)) != 0u;
    }
    int cmax = 0;
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      if (dense) B[u].cnt = 0;
      cmax = max(cmax, B[u].cnt);
    }
    const int maxc = (int)wave_umax32((unsigned)cmax);
    for (int k = 0; k < maxc; ++k) {
      double dx[NB], dy[NB], dz[NB], d2[NB];
      bool keep[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int j = B[u].bst + k;
        const bool v = k < B[u].cnt && j != s;
        double x = 0, y = 0, z = 0;
        if (v) {
          x = A.spos[3 * (int64_t)j];
          y = A.spos[3 * (int64_t)j + 1];
          z = A.spos[3 * (int64_t)j + 2];
        }
        dx[u] = (x + B[u].sx) - r[0];
        dy[u] = (y + B[u].sy) - r[1];
        dz[u] = (z + B[u].sz) - r[2];
        d2[u] = dx[u] * dx[u] + dy[u] * dy[u] + dz[u] * dz[u];
        keep[u] = v && d2[u] >= lo2 && d2[u] < hi2;
      }
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const unsigned mk = hbits(__ballot(keep[u]));
        if (keep[u]) {
          const int idx = nc + __popc(mk & hbelow());
          if (idx < kCandsP) {
            S.cd[idx] = make_double4(dx[u], dy[u], dz[u], 0.5 * d2[u]);
            S.cjk[idx] = ((B[u].bst + k) << 5) | B[u].code;
          }
        }
        nc += __popc(mk);
      }
    }
  }
  wave_sync();
  if (dense) return -1;
  return nc;   // all it found: above kCandsP only the first kCandsP are stored
}

// The two-level gather of one chunk of 32 nb stencil buckets per half (as
// gather_runs, with 32 lanes per cell): each bucket that meets the box
// around the query sphere contributes runs of consecutive points, a sparse
// bucket its whole range and a dense one the part of each sub-bucket row
// inside the box; each half takes its runs 32 at a time, a lane finding the
// bucket of its run by a binary search over the half's run prefix sums.
// The per-point test is the plain path's, so the candidates are the same.
__device__ int gather_runs_pair(PairLds& S, const TessArgs& A, const GridParams& g, const int s, const double r[3],
                                const int b[3], const int ring, const int chunk, const int nb, const int W3,
                                const WidthDiv& D, const double lo2, const double hi2, int nc) {
  const int hl = hlane();
  const int h0 = __lane_id() & 32;   // first lane of this half
  const double rq = sqrt(hi2) * (1.0 + 1e-9) + 1e-9 * fmin(g.hb[0], fmin(g.hb[1], g.hb[2]));
  for (int u = 0; u < nb; ++u) {
    int bb[3] = {0, 0, 0};
    int64_t key = 0;
    const StencilBucket B = stencil_bucket(A, g, b, ring, chunk + 32 * u + hl, W3, D, bb, &key);
    int nr = 0, pack = 0, base = 0;
    if (B.cnt > 0) {
      const double sh[3] = {B.sx, B.sy, B.sz};
      double qlo[3], qhi[3];
      bool meet = true;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        qlo[a] = (r[a] - rq) - sh[a];
        qhi[a] = (r[a] + rq) - sh[a];
        const double tlo = qlo[a] * g.inv_hb[a], thi = qhi[a] * g.inv_hb[a];
        if (thi < (double)bb[a] || (tlo >= (double)(bb[a] + 1) && bb[a] < g.nb[a] - 1)) meet = false;
      }
      if (meet) {
        if (B.cnt <= kDense || B.cnt > kDenseMax) {
          nr = 1;
        } else {
          const int ss = sub_size((unsigned)B.cnt);
          int l[3], m[3];
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            l[a] = sub_coord(qlo[a], g.inv_hb[a], bb[a], ss);
            m[a] = sub_coord(qhi[a], g.inv_hb[a], bb[a], ss) - l[a] + 1;
          }
          nr = m[1] * m[2];
          pack = ss | l[0] << 5 | m[0] << 10 | l[1] << 15 | m[1] << 20 | l[2] << 25;
          base = (int)A.sbase[key];
        }
      }
    }
    const int incl = half_incl_scan(nr);
    const int excl = incl - nr;
    const int total = (int)half_pick((unsigned)incl);
    const int tmax = (int)wave_umax32((unsigned)total);
    for (int t0 = 0; t0 < tmax; t0 += 32) {
      const int t = t0 + hl;
      // the last lane of the half whose runs start at or before t
      int ow = 0;
#pragma unroll
      for (int step = 16; step > 0; step >>= 1) {
        const int e = __shfl(excl, h0 + ow + step, 64);
        if (e <= t) ow += step;
      }
      const int src = h0 + ow;
      const int e_o = __shfl(excl, src, 64);
      const int bst_o = __shfl(B.bst, src, 64), cnt_o = __shfl(B.cnt, src, 64), code_o = __shfl(B.code, src, 64);
      const int pack_o = __shfl(pack, src, 64), base_o = __shfl(base, src, 64);
      int kx, ky, kz;
      decode(code_o, kx, ky, kz);
      const double sx = kx * g.L[0], sy = ky * g.L[1], sz = kz * g.L[2];
      int start = bst_o, count = t < total ? cnt_o : 0;
      if (pack_o != 0 && t < total) {
        const int ss = pack_o & 31, x0 = (pack_o >> 5) & 31, nx = (pack_o >> 10) & 31;
        const int y0 = (pack_o >> 15) & 31, ny = (pack_o >> 20) & 31, z0 = (pack_o >> 25) & 31;
        const int jr = t - e_o;
        const int ry = y0 + jr % ny, rz = z0 + jr / ny;
        const int ri = (rz * ss + ry) * ss + x0;
        const uint32_t* so = A.soffs + base_o;
        const int a0 = (int)so[ri], a1 = (int)so[ri + nx];
        start = bst_o + a0;
        count = a1 - a0;
      }
      const int maxc = (int)wave_umax32((unsigned)count);
      for (int k = 0; k < maxc; ++k) {
        const int j = start + k;
        const bool v = k < count && j != s;
        double x = 0, y = 0, z = 0;
        if (v) {
          x = A.spos[3 * (int64_t)j];
          y = A.spos[3 * (int64_t)j + 1];
          z = A.spos[3 * (int64_t)j + 2];
        }
        const double dx = (x + sx) - r[0], dy = (y + sy) - r[1], dz = (z + sz) - r[2];
        const double d2 = dx * dx + dy * dy + dz * dz;
        const bool keep = v && d2 >= lo2 && d2 < hi2;
        const unsigned mk = hbits(__ballot(keep));
        if (keep) {
          const int idx = nc + __popc(mk & hbelow());
          if (idx < kCandsP) {
            S.cd[idx] = make_double4(dx, dy, dz, 0.5 * d2);
            S.cjk[idx] = (j << 5) | code_o;
          }
        }
        nc += __popc(mk);
      }
    }
  }
  return nc;
}

// Candidates of each half ordered by distance, ties by neighbour and image
// (as sort_candidates).
__device__ void sort_pair(PairLds& S, const int nc) {
  const int hl = hlane();
  const int c0 = hl, c1 = hl + 32;
  int lt0 = 0, lt1 = 0;
  // Keys past the half's count read as +inf while ranking: no bound test
  // in the loop.
  constexpr double kInf = __builtin_huge_val();
  const double k0 = c0 < nc ? S.cd[c0].w : kInf, k1 = c1 < nc ? S.cd[c1].w : kInf;
  const int ncmax = (int)wave_umax32((unsigned)nc);
  if (c0 >= nc && c0 < ncmax) S.cd[c0].w = kInf;
  if (c1 >= nc && c1 < ncmax) S.cd[c1].w = kInf;
  wave_sync();
#pragma unroll 4
  for (int m = 0; m < ncmax; ++m) {
    const double km = S.cd[m].w;
    lt0 += km < k0;
    lt1 += km < k1;
  }
  if (c0 < nc) S.order[lt0] = (uint8_t)c0;
  else if (c0 < kCandsP) S.order[c0] = 0;
  if (c1 < nc) S.order[lt1] = (uint8_t)c1;
  else if (c1 < kCandsP) S.order[c1] = 0;
  wave_sync();
  const bool tie = (c0 < nc && S.order[lt0] != c0) || (c1 < nc && S.order[lt1] != c1);
  const bool htie = hbits(__ballot(tie)) != 0u;
  if (__ballot(htie) == 0ull) return;
  wave_sync();
  for (int rnd = 0; rnd < 2; ++rnd) {
    const int c = hl + 32 * rnd;
    if (htie && c < nc) {
      const double key = S.cd[c].w;
      const int id = S.cjk[c];
      int rank = 0;
      for (int m = 0; m < nc; ++m) {
        const double km = S.cd[m].w;
        rank += (km < key) || (km == key && (S.cjk[m] < id || (S.cjk[m] == id && m < c)));
      }
      S.order[rank] = (uint8_t)c;
    }
  }
  wave_sync();
}

// Cuts each half's cell by its ordered candidates (as clip_candidates).
// Returns 0 or a failure bit for this half's cell.
__device__ int clip_pair(PairLds& S, const int nc, PairRegs& C) {
  const int hl = hlane();
  constexpr unsigned long long LO = 0xffffffffull, HI = ~LO;
  // The per-half state is held as wavefront masks (a half's 32 bits all set
  // or all clear) and per-half counters, which the compiler keeps in scalar
  // registers: a lane's own flag is a select on the mask, and the loop's
  // control is scalar work apart from the compares behind its ballots.
  unsigned long long donew = __ballot(nc <= 0);   // halves that stopped
  unsigned long long stalew = 0ull;                // rmax2 older than the last cut
  unsigned long long failp = 0ull, failv = 0ull;  // halves out of plane or vertex slots
  int since0 = 0, since1 = 0;                      // cuts since each half's last bound
  double lim = 2.0 * C.rmax2;
  const int ncmax = (int)wave_umax32((unsigned)max(nc, 0));
  for (int k = 0; k < ncmax; ++k) {
    // A half that stopped, or ran out of candidates, stays idle: the loop
    // ends when both are.  (Slots past a half's count hold candidate 0.)
    unsigned long long actw = __ballot(k < nc) & ~donew;
    if (actw == 0ull) break;
    const int c = S.order[k];
    const double4 q = S.cd[c];
    const double h = q.w;
    // Stop test of each half: farther images cannot cut its cell.  A bound
    // older than the last cut is refreshed and the test taken again.
    const unsigned long long farw = __ballot(h >= lim) & actw;
    if (farw) {
      const double nb = farthest_bound_pair(C);
      const unsigned long long refw = farw & stalew;
      if (lane_on(refw)) {
        C.rmax2 = nb;
        lim = 2.0 * nb;
      }
      stalew &= ~refw;
      if (refw & LO) since0 = 0;
      if (refw & HI) since1 = 0;
      const unsigned long long stopw = (farw & ~refw) | (refw & __ballot(h >= lim));
      donew |= stopw;
      actw &= ~stopw;
    }
    const unsigned long long M0w = __ballot(q.x * C.v0x + q.y * C.v0y + q.z * C.v0z > h) & actw & C.L0w;
    const unsigned long long M1w = __ballot(q.x * C.v1x + q.y * C.v1y + q.z * C.v1z > h) & actw & C.L1w;
    const unsigned long long cutw = halves_of(M0w | M1w);   // the halves whose cell this cuts
    if (cutw == 0ull) continue;

    // Plane slot: the next unused one (a cell that needs more goes to the
    // one-cell pass, which reuses the slots of faces cut away).
    const unsigned p = (unsigned)C.np;
    const unsigned long long fullw = __ballot(p >= (unsigned)kPlanesP) & cutw;
    failp |= fullw;
    donew |= fullw;
    const unsigned long long gow = cutw & ~fullw;
    if (gow == 0ull) continue;
    if (lane_on(gow)) C.np = (int)p + 1;
    // The half's kept vertices as a set over its 64 slots (bit v: slot v,
    // the first register's 32 slots, then the second's).
    const unsigned long long K =
        (unsigned long long)hbits(C.L0w & ~M0w) | ((unsigned long long)hbits(C.L1w & ~M1w) << 32);
    auto boundary = [&](uint32_t T) -> int {
      const unsigned a = T & 255, bq = (T >> 8) & 255, cq = (T >> 16) & 255;
      const unsigned m0 = (unsigned)(K >> (S.E[__umul24(bq, kPlanesP) + a] & (kVertsP - 1)));
      const unsigned m1 = (unsigned)(K >> (S.E[__umul24(cq, kPlanesP) + bq] & (kVertsP - 1)));
      const unsigned m2 = (unsigned)(K >> (S.E[__umul24(a, kPlanesP) + cq] & (kVertsP - 1)));
      return (int)((m0 & 1u) | ((m1 & 1u) << 1) | ((m2 & 1u) << 2));
    };
    int bm0 = 0, bm1 = 0;
    if (lane_on(gow & M0w)) bm0 = boundary(C.t0);
    if (lane_on(gow & M1w)) bm1 = boundary(C.t1);
    const int nb = __popc(bm0) + __popc(bm1);
    const int incl = half_incl_scan(nb);
    const int pre = incl - nb;
    // Boundary edges of each half, and its free slots after the cut.
    const int B0 = __builtin_amdgcn_readlane(incl, 31), B1 = __builtin_amdgcn_readlane(incl, 63);
    const unsigned long long F0w = ~C.L0w | M0w, F1w = ~C.L1w | M1w;
    const int nfree0 = __popc((unsigned)F0w) + __popc((unsigned)F1w);
    const int nfree1 = __popc((unsigned)(F0w >> 32)) + __popc((unsigned)(F1w >> 32));
    const unsigned long long roomw = (B0 <= nfree0 ? LO : 0ull) | (B1 <= nfree1 ? HI : 0ull);
    failv |= gow & ~roomw;
    donew |= gow & ~roomw;
    const unsigned long long doitw = gow & roomw;
    if (doitw == 0ull) continue;
    if (lane_on(doitw) && hl == 0) {
      S.pl[p] = make_double4(q.x, q.y, q.z, h);
      // (the slot's byte offset is taken opaque: derived from the plane
      // row's address the compiler forms it with a 64-bit multiply-add)
      unsigned p4 = p << 2;
      asm volatile("" : "+v"(p4));
      *(int32_t*)((char*)S.pcand + p4) = S.cjk[c];
    }
    // Each removed vertex lists its boundary edges from position pre, the
    // first register's, then the second's (only when a removed vertex
    // lies there).
    if (lane_on(doitw & M0w)) {
      int e = pre;
      const int ta0 = C.t0 & 255, tb0 = (C.t0 >> 8) & 255, tc0 = (C.t0 >> 16) & 255;
      if (bm0 & 1) S.elist[e++] = (uint16_t)(ta0 | (tb0 << 8));
      if (bm0 & 2) S.elist[e++] = (uint16_t)(tb0 | (tc0 << 8));
      if (bm0 & 4) S.elist[e++] = (uint16_t)(tc0 | (ta0 << 8));
    }
    if (doitw & M1w) {
      if (lane_on(doitw & M1w)) {
        int e = pre + __popc(bm0);
        const int ta1 = C.t1 & 255, tb1 = (C.t1 >> 8) & 255, tc1 = (C.t1 >> 16) & 255;
        if (bm1 & 1) S.elist[e++] = (uint16_t)(ta1 | (tb1 << 8));
        if (bm1 & 2) S.elist[e++] = (uint16_t)(tb1 | (tc1 << 8));
        if (bm1 & 4) S.elist[e++] = (uint16_t)(tc1 | (ta1 << 8));
      }
    }
    wave_sync();   // every E lookup above is done before any write below

    // Boundary edge r goes to the free slot of rank r (the first register's
    // slots in lane order, then the second's); that lane builds the vertex.
    // The second register takes part only in a half with more boundary
    // edges than free slots in the first.
    const double4 qp = make_double4(q.x, q.y, q.z, h);
    const unsigned F0 = hbits(F0w);
    const int r0 = __popc(F0 & hbelow());
    const int B = (__lane_id() & 32) ? B1 : B0;
    const unsigned long long new0w = __ballot(r0 < B) & F0w & doitw;
    const unsigned long long spillw = (B0 > __popc((unsigned)F0w) ? LO : 0ull) |
                                      (B1 > __popc((unsigned)(F0w >> 32)) ? HI : 0ull);
    unsigned long long new1w = 0ull;
    int r1 = 0;
    if (doitw & spillw) {
      r1 = __popc(F0) + __popc(hbits(F1w) & hbelow());
      new1w = __ballot(r1 < B) & F1w & doitw;
    }
    if (lane_on(new0w)) {
      const unsigned xy = S.elist[r0];
      const unsigned x = xy & 255, y = xy >> 8;
      C.t0 = x | (y << 8) | (p << 16);
      intersect3(S.pl[x], S.pl[y], qp, C.v0x, C.v0y, C.v0z);
      S.E[__umul24(x, kPlanesP) + y] = (uint8_t)hl;
      S.E[__umul24(y, kPlanesP) + p] = (uint8_t)hl;
      S.E[__umul24(p, kPlanesP) + x] = (uint8_t)hl;
    }
    if (lane_on(new1w)) {
      const unsigned xy = S.elist[r1];
      const unsigned x = xy & 255, y = xy >> 8;
      C.t1 = x | (y << 8) | (p << 16);
      intersect3(S.pl[x], S.pl[y], qp, C.v1x, C.v1y, C.v1z);
      S.E[__umul24(x, kPlanesP) + y] = (uint8_t)(hl + 32);
      S.E[__umul24(y, kPlanesP) + p] = (uint8_t)(hl + 32);
      S.E[__umul24(p, kPlanesP) + x] = (uint8_t)(hl + 32);
    }
    wave_sync();
    C.L0w = (C.L0w & ~(M0w & doitw)) | new0w;
    C.L1w = (C.L1w & ~(M1w & doitw)) | new1w;
    // The bound is refreshed every fourth cut of a half.
    stalew |= doitw;
    if (doitw & LO) ++since0;
    if (doitw & HI) ++since1;
    const unsigned long long refw = (since0 == 4 ? LO : 0ull) | (since1 == 4 ? HI : 0ull);
    if (refw) {
      const double nb2 = farthest_bound_pair(C);
      if (lane_on(refw)) {
        C.rmax2 = nb2;
        lim = 2.0 * nb2;
      }
      stalew &= ~refw;
      if (refw & LO) since0 = 0;
      if (refw & HI) since1 = 0;
    }
  }
  if (stalew) {
    const double nb = farthest_bound_pair(C);
    if (lane_on(stalew)) C.rmax2 = nb;
  }
  return lane_on(failp) ? F_PLANES : lane_on(failv) ? F_VERTS : 0;
}

// Faces, volume and centroid of each half's finished cell (as finish_cell;
// each lane integrates planes hl and hl + 32).  Returns 0 or a failure bit.
__device__ int finish_pair(PairLds& S, const TessArgs& A, const bool act, const int s, const PairRegs& C) {
  const int hl = hlane();
  const bool live0 = act && lane_on(C.L0w), live1 = act && lane_on(C.L1w);
  wave_sync();
  S.vx[hl] = C.v0x; S.vy[hl] = C.v0y; S.vz[hl] = C.v0z;
  S.tri[hl] = C.t0;
  S.vx[hl + 32] = C.v1x; S.vy[hl + 32] = C.v1y; S.vz[hl + 32] = C.v1z;
  S.tri[hl + 32] = C.t1;
  S.first[hl] = kVertsP;
  if (hl + 32 < kPlanesP) S.first[hl + 32] = kVertsP;
  wave_sync();
  if (live0) {
    atomicMin(&S.first[C.t0 & 255], hl);
    atomicMin(&S.first[(C.t0 >> 8) & 255], hl);
    atomicMin(&S.first[(C.t0 >> 16) & 255], hl);
  }
  if (live1) {
    atomicMin(&S.first[C.t1 & 255], hl + 32);
    atomicMin(&S.first[(C.t1 >> 8) & 255], hl + 32);
    atomicMin(&S.first[(C.t1 >> 16) & 255], hl + 32);
  }
  wave_sync();

  // A plane slot is a face of the cell when a live vertex lies on it: its
  // first vertex was set above.
  double Af[2] = {0.0, 0.0}, fx[2] = {0.0, 0.0}, fy[2] = {0.0, 0.0}, fz[2] = {0.0, 0.0}, dl[2] = {0.0, 0.0};
  bool walk_bad = false;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int p = hl + 32 * k;
    const int tstart = p < kPlanesP ? S.first[p] : kVertsP;
    if (act && tstart < kVertsP) {
      const double4 P = S.pl[p];
      const double w2 = 2.0 * P.w;   // the plane's |d|^2
      const double idl = rsqrt_nr(w2);
      dl[k] = w2 * idl;
      const double nx = P.x * idl, ny = P.y * idl, nz = P.z * idl;
      const double ox = S.vx[tstart], oy = S.vy[tstart], oz = S.vz[tstart];
      int t = tstart, it = 0;
      double as = 0.0, mx = 0.0, my = 0.0, mz = 0.0;
      double x1 = 0.0, y1 = 0.0, z1 = 0.0;   // vertex t relative to the first
      do {
        const uint32_t T = S.tri[t];
        const int a = T & 255, bq = (T >> 8) & 255, cq = (T >> 16) & 255;
        const int z = (a == p) ? cq : (bq == p ? a : bq);
        const int tn = S.E[p * kPlanesP + z] & (kVertsP - 1);
        const double x2 = S.vx[tn] - ox, y2 = S.vy[tn] - oy, z2 = S.vz[tn] - oz;
        const double ar = 0.5 * ((y1 * z2 - z1 * y2) * nx + (z1 * x2 - x1 * z2) * ny + (x1 * y2 - y1 * x2) * nz);
        as += ar;
        mx += ar * (x1 + x2);
        my += ar * (y1 + y2);
        mz += ar * (z1 + z2);
        x1 = x2;
        y1 = y2;
        z1 = z2;
        t = tn;
        ++it;
      } while (t != tstart && it < kVertsP);
      walk_bad |= (t != tstart);
      Af[k] = as;
      const double i3a = rcp_nr(3.0 * as);
      fx[k] = ox + mx * i3a;
      fy[k] = oy + my * i3a;
      fz[k] = oz + mz * i3a;
    }
  }
  if (hbits(__ballot(walk_bad))) return F_WALK;
  bool keep[2];
  double vol[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    keep[k] = Af[k] > 0.0;   // zero unless a valid plane of an active half
    vol[k] = keep[k] ? Af[k] * dl[k] / 6.0 : 0.0;
  }
  const double V = half_sum(vol[0] + vol[1]);
  const double iV = rcp_nr(V);
  const double cxr = half_sum((keep[0] ? 0.75 * vol[0] * fx[0] : 0.0) + (keep[1] ? 0.75 * vol[1] * fx[1] : 0.0)) * iV;
  const double cyr = half_sum((keep[0] ? 0.75 * vol[0] * fy[0] : 0.0) + (keep[1] ? 0.75 * vol[1] * fy[1] : 0.0)) * iV;
  const double czr = half_sum((keep[0] ? 0.75 * vol[0] * fz[0] : 0.0) + (keep[1] ? 0.75 * vol[1] * fz[1] : 0.0)) * iV;
  if (act && !(V > 0.0)) return F_VOLUME;

  int jj[2] = {s, s}, code[2] = {13, 13};
  bool owned[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    if (keep[k]) {
      const int pc = S.pcand[hl + 32 * k];
      if (pc >= 0) {
        jj[k] = pc >> 5;
        code[k] = pc & 31;
      } else {
        const int bp = -1 - pc;   // box plane: axis bp/2, sign by parity
        const int step = (bp >> 1) == 0 ? 1 : ((bp >> 1) == 1 ? 3 : 9);
        code[k] = (bp & 1) ? 13 - step : 13 + step;
      }
    }
    owned[k] = keep[k] && (jj[k] > s || (jj[k] == s && code[k] > 13));
  }
  // Faces staged in plane-slot order (planes 0-31 in lane order, then the rest).
  const unsigned MK0 = hbits(__ballot(keep[0])), MK1 = hbits(__ballot(keep[1]));
  const unsigned MO0 = hbits(__ballot(owned[0])), MO1 = hbits(__ballot(owned[1]));
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    if (keep[k]) {
      const int idx = k ? __popc(MK0) + __popc(MK1 & hbelow()) : __popc(MK0 & hbelow());
      const int orank = k ? __popc(MO0) + __popc(MO1 & hbelow()) : __popc(MO0 & hbelow());
      StageNbr nb;
      nb.j = jj[k];
      nb.meta = code[k] | ((owned[k] ? 1 : 0) << 8) | (orank << 16);
      A.stage_nb[(int64_t)s * kMaxFaces + idx] = nb;
      StageGeo& F = A.stage_geo[(int64_t)s * kMaxFaces + idx];
      F.A = Af[k];
      F.f[0] = fx[k];
      F.f[1] = fy[k];
      F.f[2] = fz[k];
    }
  }
  if (act && hl == 0) {
    const int nk = __popc(MK0) + __popc(MK1), no = __popc(MO0) + __popc(MO1);
    A.counts[s] = ((unsigned long long)nk << 32) | (unsigned long long)no;
    double* gp = A.geo + 4 * (int64_t)s;
    gp[0] = V;
    gp[1] = cxr;
    gp[2] = cyr;
    gp[3] = czr;
  }
  return 0;
}

// Generator s: its position, bucket, and distance to its bucket's nearer
// wall per axis.
struct CellGeom {
  double r[3], edge[3];
  int b[3];
};

__device__ inline void cell_geom(const TessArgs& A, const GridParams& g, const int s, CellGeom& G) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    G.r[a] = A.spos[3 * (int64_t)s + a];
    G.b[a] = bucket_coord(G.r[a], g.inv_hb[a], g.nb[a]);
    const double t = G.r[a] - G.b[a] * g.hb[a];
    G.edge[a] = fmax(0.0, fmin(t, g.hb[a] - t));
  }
}

// Squared outer radius of the shell from sqrt(lo2) that holds about `want`
// of the nc candidates found between sqrt(lo2) and sqrt(hi2), at the density
// found (counts go as the shell's volume, r^3 - lo^3).
__device__ inline double shell_for(double lo2, double hi2, int nc, double want) {
  const double lo3 = lo2 * sqrt(lo2), hi3 = hi2 * sqrt(hi2);
  const double r = cbrt(lo3 + (want / (double)nc) * (hi3 - lo3));
  return r * r;
}

// Hands a cell to the one-cell first pass of its kind (lean or dense).
template <bool DENSE>
__device__ inline void redo_cell(const TessArgs& A, int s) {
  A.redo[atomicAdd(DENSE ? &A.st->n_dredo : &A.st->n_redo, 1)] = s;
}

// One cell per half of the wavefront (act: the half has a cell, s).
// DENSE = false: the lean first pass over every cell; cells of dense
// buckets are left to the dense passes (listed by the sort), and a cell
// whose stencil holds a dense bucket is listed for them.  DENSE = true: the
// cells of those lists, with the two-level gather.  Either way a cell the
// half cannot finish is handed to the one-cell pass of its kind.
// ONE: one segment, whose grid comes with the kernel's arguments (scalar
// loads at the start, instead of a load that waits for the cell's segment).
template <bool DENSE, bool ONE>
__device__ void pair_cell(PairLds& S, const TessArgs& A, bool act, const int s) {
  const int hl = hlane();
  const int seg = ONE ? 0 : A.sseg[s];
  const GridParams& g = ONE ? A.g1 : A.segs[seg].g;
  CellGeom G;
  cell_geom(A, g, s, G);
  const double* r = G.r;
  const int* b = G.b;
  const double* edge = G.edge;
  PairRegs C;
  init_box_pair(S, g, C);
  const unsigned cnt = own_count(A, g, b);
  if (!DENSE && act && cnt > (unsigned)kDense) {
    // Listed for the dense first pass by the sort (a bucket beyond what the
    // sort orders fails the call).
    if (cnt > (unsigned)kDenseMax && hl == 0) {
      seg_fail(A.st, A.segst, seg, F_DENSE, s);
      A.counts[s] = 0ull;
      A.geo[4 * (int64_t)s] = 0.0;
    }
    act = false;
  }
  const double rloc =
      cnt > 4u ? g.r_filter * cbrt((cnt > (unsigned)kDense ? g.ppb : 4.0) / (double)cnt) : g.r_filter;
  int ring = cnt > 4u ? min(g.ring, ring_for(g, edge, rloc * rloc)) : g.ring;
  double reach = 1e300;
#pragma unroll
  for (int a = 0; a < 3; ++a) reach = fmin(reach, ring * g.hb[a] + edge[a]);
  double lo2 = 0.0, hi2 = fmin(reach * reach, rloc * rloc);
  // The first radius, then, for a cell whose candidates do not reach twice
  // its farthest vertex, more distance shells as in the one-cell passes
  // (irregular inputs need one often): up to kShells1 in the dense pass,
  // one in the lean pass (below).  A cell still short, or whose shell needs
  // a wider stencil than the grid has, is handed on.
  // work: the half gathers and cuts in this round (a half whose cell is
  // complete takes no further candidates: cutting a cell again by planes it
  // already has can split, by rounding, the vertices that lie on them).
  bool work = act;
  for (int shell = 0;; ++shell) {
    int nc = gather_pair<DENSE>(S, A, g, work, s, r, b, ring, lo2, hi2);
    if (!DENSE && work && nc < 0) {
      if (hl == 0) A.dcells[atomicAdd(&A.st->n_dense_cells, 1)] = s;
      act = work = false;
    }
    // More candidates than slots (a compressed region): gather again with
    // the radius that holds about 38 of them at the density found (the cell
    // is the same at any radius; only the work changes).  Not for the dense
    // pass's later shells: there the other half waits through the second
    // gather, and the one-cell pass builds such a cell for less (the
    // polytropes 3% faster).
    const bool over = work && nc > kCandsP && (!DENSE || shell == 0);
    if (__ballot(over)) {
      if (over) hi2 = shell_for(lo2, hi2, nc, 38.0);
      const int nc2 = gather_pair<DENSE>(S, A, g, over, s, r, b, ring, lo2, hi2);
      if (over) nc = nc2;
    }
    // Too many candidates, or (lean pass, first radius) few: a thin region,
    // whose radius the one-cell pass widens.
    if (work && (nc > kCandsP || (!DENSE && shell == 0 && nc < kFewCands))) {
      if (hl == 0) redo_cell<DENSE>(A, s);
      act = work = false;
    }
    if (!work) nc = 0;
    sort_pair(S, nc);
    // A failure (plane or vertex slots): the one-cell pass builds the cell
    // again.
    if (clip_pair(S, nc, C) && work) {
      if (hl == 0) redo_cell<DENSE>(A, s);
      act = work = false;
    }
    bool go = work && !(4.0 * C.rmax2 <= hi2 * (1.0 - 1e-12));
    if constexpr (!DENSE) {
      // One more shell here (the one-cell passes take up to kShells1); a
      // cell still short is handed on.  The generator's geometry and the
      // LDS address are taken afresh, opaque to the compiler, so that
      // nothing derived from them stays live across the first cuts: the
      // pass keeps 128 VGPRs and 4 waves per SIMD (146 otherwise), and a
      // loop over shells would hold more.
      if (__ballot(go)) {
        int s2 = s;
        asm volatile("" : "+v"(s2));
        PairLds* Sp = &S;
        asm volatile("" : "+v"(Sp));
        PairLds& S2 = *Sp;
        const GridParams& g2 = ONE ? A.g1 : A.segs[A.sseg[s2]].g;
        CellGeom G2;
        cell_geom(A, g2, s2, G2);
        int ring2 = 0;
        if (go) {
          const double nhi2 = next_shell(C.rmax2, lo2, hi2, nc, 38.0);
          ring2 = ring_for(g2, G2.edge, nhi2);
          if (ring2 > g2.nb[0] || ring2 > g2.nb[1] || ring2 > g2.nb[2]) {
            if (hl == 0) redo_cell<DENSE>(A, s);
            act = go = false;
          } else {
            lo2 = hi2;
            hi2 = nhi2;
          }
        }
        int nc2 = gather_pair<DENSE>(S2, A, g2, go, s2, G2.r, G2.b, ring2, lo2, hi2);
        // A shell that overflows is narrowed once (the one-cell pass takes
        // the cell on if it still falls short).
        const bool over2 = go && nc2 > kCandsP;
        if (__ballot(over2)) {
          if (over2) hi2 = shell_for(lo2, hi2, nc2, 38.0);
          const int nc3 = gather_pair<DENSE>(S2, A, g2, over2, s2, G2.r, G2.b, ring2, lo2, hi2);
          if (over2) nc2 = nc3;
        }
        if (go && (nc2 < 0 || nc2 > kCandsP)) {
          if (hl == 0) {
            if (nc2 < 0) A.dcells[atomicAdd(&A.st->n_dense_cells, 1)] = s;
            else redo_cell<DENSE>(A, s);
          }
          act = go = false;
        }
        if (!go) nc2 = 0;
        sort_pair(S2, nc2);
        if (clip_pair(S2, nc2, C) && go) {
          if (hl == 0) redo_cell<DENSE>(A, s);
          act = go = false;
        }
        if (go && !(4.0 * C.rmax2 <= hi2 * (1.0 - 1e-12))) {
          if (hl == 0) redo_cell<DENSE>(A, s);
          act = false;
        }
      }
      break;
    }
    if (__ballot(go) == 0ull) break;
    if (go) {
      const double nhi2 = next_shell(C.rmax2, lo2, hi2, nc, 38.0);
      ring = ring_for(g, edge, nhi2);
      if (shell == kShells1 || ring > g.nb[0] || ring > g.nb[1] || ring > g.nb[2]) {
        if (hl == 0) redo_cell<DENSE>(A, s);
        act = go = false;
      } else {
        lo2 = hi2;
        hi2 = nhi2;
      }
    }
    work = go;
  }
  const int bad2 = finish_pair(S, A, act, s, C);
  if (act && bad2 && hl == 0) {
    seg_fail(A.st, A.segst, seg, bad2, s);
    A.counts[s] = 0ull;
    A.geo[4 * (int64_t)s] = 0.0;
  }
}

// Two cells per wavefront: cells 2w and 2w + 1 of the launch.
template <bool ONE>
__global__ __launch_bounds__(64) void k_tess_pair(TessArgs A) {
  __shared__ PairLds lds[2];
  const int64_t s64 = 2 * xcd_block() + (__lane_id() >> 5);
  const bool act = s64 < A.n;
  pair_cell<false, ONE>(lds[__lane_id() >> 5], A, act, act ? (int)s64 : 0);
}

// The listed cells of dense regions, two per wavefront: those of the dense
// buckets (listed by the sort) and those the first passes met a dense
// bucket for.  The list's length is known on the device only; the grid is
// sized by the host from the last tessellation's length (with a margin),
// the blocks beyond the list exit at once, and listed cells beyond the
// grid (dense_cap) go to the one-cell dense pass.  The
// blocks with work are spread evenly over the XCDs, each XCD taking one
// contiguous share of the list (a bucket's cells are listed together and
// share their neighbours).  One pair per one-wavefront block: a loop over
// pairs holds about 50 more registers (polytropes 19% slower), and blocks of
// two or four waves hold their LDS until the slowest wave ends (3% and 5%
// slower).  Four waves per SIMD, with some registers spilled (at two,
// without spills, or three the polytropes' dense cells take 30% or 7%
// longer).
template <bool ONE>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_tess_pair_dense(TessArgs A) {
  __shared__ PairLds lds[2];
  const int64_t nd = min((int64_t)A.st->n_dense_cells, A.dense_cap);
  const int64_t npair = (nd + 1) / 2;
  const int64_t per = (npair + kXcds - 1) / kXcds;   // pairs per XCD
  const int64_t k = blockIdx.x / kXcds;
  if (k >= per) return;
  const int64_t it = (blockIdx.x % kXcds) * per + k;
  if (it >= npair) return;
  const int64_t q = 2 * it + (__lane_id() >> 5);
  const bool act = q < nd;
  pair_cell<true, ONE>(lds[__lane_id() >> 5], A, act, A.dcells[act ? q : 2 * it]);
}

// The one-cell first pass over the cells the pair pass handed on.  Four
// waves per SIMD with a small spill (at three, without it, the polytropes'
// cell construction takes 3% longer).
__global__ __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(4))) void k_tess_pass1_redo(TessArgs A) {
  __shared__ TessLds lds[kWaves];
  const int w = threadIdx.x >> 6;
  const int nr = A.st->n_redo;
  for (int64_t it = (int64_t)blockIdx.x * kWaves + w; it < nr; it += (int64_t)gridDim.x * kWaves)
    tess_cell<0>(lds[w], A, A.redo[it]);
}

}  // namespace

int64_t launch_tessellate(const double* spos, int64_t n, const SegDesc* segs, const int32_t* sseg,
                          const unsigned long long* boff, const unsigned long long* sbase, const uint32_t* soffs,
                          StageNbr* stage_nb, StageGeo* stage_geo, unsigned long long* counts, double* geo,
                          double* rmax2, int32_t* deferred, int32_t* dcells, int32_t* redo, const TessHints& hints,
                          const GridParams* g_one, DevStatus* st_dev, SegStatus* segst, hipStream_t st) {
  if (n <= 0) return 0;
  // Grid of the two-cell dense pass: the last tessellation's dense-list
  // length and a quarter more (all cells when there is none yet).
  const int64_t dh = hints.dense_cells;
  const int64_t want = dh < 0 ? n : std::min<int64_t>(n, dh + dh / 4 + 256);
  const int64_t dense_cap = (want + 1) / 2 * 2;
  TessArgs A{spos,   n,     segs,     sseg,   boff,      sbase,  soffs, stage_nb, stage_geo, counts,
             geo,    rmax2, deferred, dcells, redo,      dense_cap, st_dev, segst, GridParams{}};
  if (g_one) A.g1 = *g_one;
  if (g_one)
    hipLaunchKernelGGL(k_tess_pair<true>, dim3((unsigned)((n + 1) / 2)), dim3(64), 0, st, A);
  else
    hipLaunchKernelGGL(k_tess_pair<false>, dim3((unsigned)((n + 1) / 2)), dim3(64), 0, st, A);
  // The handed-on and deferred counts are known on the device only.  Each
  // list pass gets blocks for the length the last tessellation's list had
  // and a quarter more (a wavefront per cell; at least 256 blocks), at most
  // 65536 (the cells of these lists differ widely in cost, so each block
  // takes few of them: the polytropes' cell construction 15% faster with
  // 65536 blocks than with 16384, 262144 no faster), and 65536 before any
  // length is known.  A block with no cell exits at once; a list longer
  // than its grid is walked with a grid stride.
  auto list_blocks = [n](int64_t hint) -> unsigned {
    const int64_t full = std::min<int64_t>((n + kWaves - 1) / kWaves, 65536);
    if (hint < 0) return (unsigned)full;
    const int64_t want_b = (hint + hint / 4 + kWaves - 1) / kWaves;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(full, std::max<int64_t>(want_b, 256)));
  };
  hipLaunchKernelGGL(k_tess_pass1_redo, dim3(list_blocks(hints.redo)), dim3(64 * kWaves), 0, st, A);
  // (The hand-off list of the lean pass has been read: the dense passes'
  // hand-offs reuse it.)
  if (g_one)
    hipLaunchKernelGGL(k_tess_pair_dense<true>, dim3((unsigned)(dense_cap / 2 + kXcds)), dim3(64), 0, st, A);
  else
    hipLaunchKernelGGL(k_tess_pair_dense<false>, dim3((unsigned)(dense_cap / 2 + kXcds)), dim3(64), 0, st, A);
  hipLaunchKernelGGL(k_tess_pass1_dense, dim3(list_blocks(hints.dense_redo)), dim3(64 * kWaves), 0, st, A);
  hipLaunchKernelGGL(k_tess_pass2, dim3(list_blocks(hints.deferred)), dim3(64 * kWaves), 0, st, A);
  return dense_cap;
}

}  // namespace mm
