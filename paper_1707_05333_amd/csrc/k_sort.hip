// Grid hash and counting sort of the mesh-generating points, plus the
// prefix-sum and fill kernels the rest of the path uses.
//
// The sort realises the neighbour search the paper leaves to a tree
// (Sec. 3, the fast nearest-neighbour search): points are binned into a
// periodic grid of buckets, bucket-major with x fastest, so that the
// candidate stencil of a cell reads contiguous runs of positions.  Inside a
// bucket points keep their caller order, which makes the internal order, and
// every result downstream of it, independent of atomic scheduling.
#include <algorithm>

#include "mm_internal.h"

namespace mm {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ inline unsigned long long wave_incl_scan(unsigned long long x) {
  const int lane = __lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned long long y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  return x;
}

// Exclusive scan of one value per thread over a 256-thread block.
__device__ unsigned long long block_excl_scan(unsigned long long x, unsigned long long* total) {
  __shared__ unsigned long long wsum[kScanThreads / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const unsigned long long inc = wave_incl_scan(x);
  if (lane == 63) wsum[wid] = inc;
  __syncthreads();
  unsigned long long base = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kScanThreads / 64; ++k) {
    if (k < wid) base += wsum[k];
    tot += wsum[k];
  }
  __syncthreads();
  *total = tot;
  return base + inc - x;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const unsigned long long* in, int64_t n,
                                                              unsigned long long* part) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  unsigned long long s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k * kScanThreads + threadIdx.x;
    if (i < n) s += in[i];
  }
  unsigned long long tot;
  block_excl_scan(s, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Exclusive scan of the per-tile sums in place, by one block.
__global__ __launch_bounds__(kScanThreads) void k_scan_top(unsigned long long* part, int64_t m) {
  unsigned long long carry = 0;
  for (int64_t base = 0; base < m; base += kScanTile) {
    unsigned long long v[kScanItems];
    unsigned long long s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      const int64_t i = base + (int64_t)threadIdx.x * kScanItems + k;
      v[k] = (i < m) ? part[i] : 0ull;
      s += v[k];
    }
    unsigned long long tot;
    unsigned long long run = carry + block_excl_scan(s, &tot);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      const int64_t i = base + (int64_t)threadIdx.x * kScanItems + k;
      if (i < m) part[i] = run;
      run += v[k];
    }
    carry += tot;
    __syncthreads();
  }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_down(const unsigned long long* in, int64_t n,
                                                            const unsigned long long* part,
                                                            unsigned long long* out) {
  __shared__ unsigned long long tile[kScanTile];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k * kScanThreads + threadIdx.x;
    tile[k * kScanThreads + threadIdx.x] = (i < n) ? in[i] : 0ull;
  }
  __syncthreads();
  unsigned long long v[kScanItems];
  unsigned long long s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = tile[threadIdx.x * kScanItems + k];
    s += v[k];
  }
  unsigned long long tot;
  unsigned long long run = part[blockIdx.x] + block_excl_scan(s, &tot);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    tile[threadIdx.x * kScanItems + k] = run;
    run += v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k * kScanThreads + threadIdx.x;
    if (i < n) out[i] = tile[k * kScanThreads + threadIdx.x];
  }
  // The last tile also writes the grand total at out[n].
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == kScanThreads - 1) out[n] = run;
}

__global__ void k_fill_u64(unsigned long long* p, unsigned long long v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_status_reset(DevStatus* s, SegStatus* segst, int nseg) {
  const int t = threadIdx.x;
  if (t == 0) {
    s->flags = 0;
    s->n_deferred = 0;
    s->n_overflow = 0;
    s->max_faces = 0;
    s->bad_cell = 0x7fffffff;
    s->n_faces = 0;
    s->n_csr = 0;
    s->asym_cell = -1;
    s->asym_nbr = -1;
  }
  for (int k = t; k < nseg; k += blockDim.x) {
    SegStatus& g = segst[k];
    g.dt_bits = 0x7ff0000000000000ull;   // +inf
    g.flags = 0;
    g.bad_cell = 0x7fffffff;
    for (int q = 0; q < 4; ++q) g.floor_hits[q] = 0;
  }
}

// Bucket key of every used slot: the segment's first bucket plus the bucket
// of the point in that segment's grid.  Unused slots get key -1.
__global__ void k_hash(const double* __restrict__ pos, int64_t n_slots, const int32_t* __restrict__ slot_seg,
                       const SegDesc* __restrict__ segs, int32_t* __restrict__ key, unsigned long long* bcount,
                       DevStatus* st, SegStatus* segst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_slots) return;
  const int seg = slot_seg ? slot_seg[i] : 0;
  if (seg < 0) {
    key[i] = -1;
    return;
  }
  const GridParams& g = segs[seg].g;
  const double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
  const bool ok = (x >= 0.0) && (x < g.L[0]) && (y >= 0.0) && (y < g.L[1]) && (z >= 0.0) && (z < g.L[2]);
  int64_t k = g.base;
  if (ok) {
    const int bx = bucket_coord(x, g.inv_hb[0], g.nb[0]);
    const int by = bucket_coord(y, g.inv_hb[1], g.nb[1]);
    const int bz = bucket_coord(z, g.inv_hb[2], g.nb[2]);
    k += bucket_key(g.nb, bx, by, bz);
  } else {
    seg_fail(st, segst, seg, F_BADPOS, (int)i);
  }
  key[i] = (int32_t)k;
  atomicAdd(&bcount[k], 1ull);
}

__global__ void k_scatter(const int32_t* __restrict__ key, int64_t n_slots, const unsigned long long* __restrict__ boff,
                          unsigned long long* cursor, int32_t* __restrict__ perm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_slots) return;
  const int k = key[i];
  if (k < 0) return;
  const unsigned long long slot = boff[k] + atomicAdd(&cursor[k], 1ull);
  perm[slot] = (int32_t)i;
}

// Per bucket: a bucket of at most kDense points gets its slot order back
// (insertion sort of a handful); a denser one records the size of its
// sub-offset table (s^3 + 1), joins the list the block sort takes, and
// lists its cells (sorted positions) for the tessellation's dense first
// pass, with one atomic per bucket.
// Buckets above kDenseMax points fail the call (their points stay where the
// scatter put them and are read whole).
__global__ void k_bucket_prep(const unsigned long long* __restrict__ boff, int64_t nbt, int32_t* perm,
                              const int32_t* __restrict__ slot_seg, unsigned long long* __restrict__ sub_size_out,
                              int32_t* __restrict__ dense, int32_t* __restrict__ dcells, DevStatus* st,
                              SegStatus* segst) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbt) return;
  const int64_t lo = (int64_t)boff[b], hi = (int64_t)boff[b + 1];
  const int64_t cnt = hi - lo;
  if (cnt <= kDense) {
    sub_size_out[b] = 0;
    for (int64_t a = lo + 1; a < hi; ++a) {
      const int32_t v = perm[a];
      int64_t c = a - 1;
      while (c >= lo && perm[c] > v) {
        perm[c + 1] = perm[c];
        --c;
      }
      perm[c + 1] = v;
    }
    return;
  }
  if (cnt > kDenseMax) {
    sub_size_out[b] = 0;
    seg_fail(st, segst, slot_seg ? slot_seg[perm[lo]] : 0, F_DENSE, (int)lo);
    return;
  }
  const int s = sub_size((unsigned)cnt);
  sub_size_out[b] = (unsigned long long)(s * s * s + 1);
  dense[atomicAdd(&st->n_dense, 1)] = (int32_t)b;
  const int c0 = atomicAdd(&st->n_dense_cells, (int)cnt);
  for (int64_t i = 0; i < cnt; ++i) dcells[c0 + i] = (int32_t)(lo + i);
}

// Orders the points of each dense bucket by sub-bucket (x fastest), then by
// slot, with a bitonic sort of (sub-bucket << 32 | slot) keys in LDS, and
// writes the bucket's sub-bucket offsets: entry k counts its points in
// sub-buckets below k (k = 0 .. s^3).  One block per bucket of the list.
constexpr int kDenseThreads = 256;

__global__ __launch_bounds__(kDenseThreads) void k_dense_order(
    const int32_t* __restrict__ dense, const DevStatus* __restrict__ st, const unsigned long long* __restrict__ boff,
    const unsigned long long* __restrict__ sbase, const double* __restrict__ pos,
    const int32_t* __restrict__ slot_seg, const SegDesc* __restrict__ segs, int32_t* __restrict__ perm,
    uint32_t* __restrict__ soffs) {
  __shared__ unsigned long long kv[kDenseMax];
  const int nd = st->n_dense;
  const int t = threadIdx.x;
  for (int it = blockIdx.x; it < nd; it += gridDim.x) {
    const int64_t b = dense[it];
    const int64_t lo = (int64_t)boff[b];
    const int cnt = (int)((int64_t)boff[b + 1] - lo);
    const int s = sub_size((unsigned)cnt);
    int p2 = 1;
    while (p2 < cnt) p2 <<= 1;
    const int seg = slot_seg ? slot_seg[perm[lo]] : 0;
    const GridParams& g = segs[seg].g;
    for (int i = t; i < p2; i += kDenseThreads) {
      unsigned long long k = ~0ull;
      if (i < cnt) {
        const int32_t q = perm[lo + i];
        int sc[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const double x = pos[3 * (int64_t)q + a];
          sc[a] = sub_coord(x, g.inv_hb[a], bucket_coord(x, g.inv_hb[a], g.nb[a]), s);
        }
        k = ((unsigned long long)((sc[2] * s + sc[1]) * s + sc[0]) << 32) | (uint32_t)q;
      }
      kv[i] = k;
    }
    __syncthreads();
    for (int k = 2; k <= p2; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int i = t; i < p2; i += kDenseThreads) {
          const int ixj = i ^ j;
          if (ixj > i) {
            const unsigned long long a = kv[i], c = kv[ixj];
            if (((i & k) == 0) == (a > c)) {
              kv[i] = c;
              kv[ixj] = a;
            }
          }
        }
        __syncthreads();
      }
    }
    for (int i = t; i < cnt; i += kDenseThreads) perm[lo + i] = (int32_t)(uint32_t)(kv[i] & 0xffffffffull);
    const int ns = s * s * s;
    uint32_t* so = soffs + sbase[b];
    for (int k = t; k <= ns; k += kDenseThreads) {
      // first position whose sub-bucket is k or more
      const unsigned long long key = (unsigned long long)k << 32;
      int l = 0, h = cnt;
      while (l < h) {
        const int m = (l + h) >> 1;
        if (kv[m] < key) l = m + 1;
        else h = m;
      }
      so[k] = (uint32_t)l;
    }
    __syncthreads();
  }
}

__global__ void k_gather_pos(const double* __restrict__ pos, const int32_t* __restrict__ perm,
                             const int32_t* __restrict__ slot_seg, int64_t n, double* __restrict__ spos,
                             int32_t* __restrict__ sseg) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int64_t q = perm[s];
  spos[3 * s] = pos[3 * q];
  spos[3 * s + 1] = pos[3 * q + 1];
  spos[3 * s + 2] = pos[3 * q + 2];
  sseg[s] = slot_seg ? slot_seg[q] : 0;
}

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

size_t scan_tmp_elems(int64_t n) { return (size_t)((n + kScanTile - 1) / kScanTile) + 1; }

void scan_u64(const unsigned long long* in, unsigned long long* out, int64_t n, unsigned long long* tmp,
              hipStream_t st) {
  if (n <= 0) {
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, out, 0ull, (int64_t)1);
    return;
  }
  const int64_t tiles = (n + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)tiles), dim3(kScanThreads), 0, st, in, n, tmp);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, st, tmp, tiles);
  hipLaunchKernelGGL(k_scan_down, dim3((unsigned)tiles), dim3(kScanThreads), 0, st, in, n, tmp, out);
}

void launch_fill_u64(unsigned long long* p, unsigned long long v, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_u64, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, v, n);
}

void launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, v, n);
}

__global__ void k_remesh_reset(DevStatus* s) {
  if (threadIdx.x == 0) {
    s->n_deferred = 0;
    s->n_overflow = 0;
    s->n_faces = 0;
    s->n_csr = 0;
  }
}

void launch_remesh_reset(DevStatus* s, hipStream_t st) {
  hipLaunchKernelGGL(k_remesh_reset, dim3(1), dim3(64), 0, st, s);
}

void launch_status_reset(DevStatus* s, SegStatus* segst, int nseg, hipStream_t st) {
  hipLaunchKernelGGL(k_status_reset, dim3(1), dim3(256), 0, st, s, segst, nseg);
}

void launch_sort(const double* pos, int64_t n_slots, const int32_t* slot_seg, int64_t n, const SegDesc* segs,
                 int64_t nbt, unsigned long long* bcount, unsigned long long* boff, unsigned long long* scan_tmp,
                 unsigned long long* sbase, uint32_t* soffs, int32_t* key, int32_t* perm, int32_t* sseg,
                 double* spos, int32_t* dcells, DevStatus* st_dev, SegStatus* segst, hipStream_t st) {
  launch_fill_u64(bcount, 0ull, nbt, st);
  launch_fill_i32(&st_dev->n_dense, 0, 4, st);   // n_dense, n_dense_cells, n_redo and n_dredo
  hipLaunchKernelGGL(k_hash, dim3(blocks_for(n_slots, 256)), dim3(256), 0, st, pos, n_slots, slot_seg, segs, key,
                     bcount, st_dev, segst);
  scan_u64(bcount, boff, nbt, scan_tmp, st);
  launch_fill_u64(bcount, 0ull, nbt, st);
  hipLaunchKernelGGL(k_scatter, dim3(blocks_for(n_slots, 256)), dim3(256), 0, st, key, n_slots, boff, bcount, perm);
  // bcount (the scatter's cursors) now takes the sub-table sizes and key
  // (read by the scatter) the list of dense buckets.
  hipLaunchKernelGGL(k_bucket_prep, dim3(blocks_for(nbt, 256)), dim3(256), 0, st, boff, nbt, perm, slot_seg, bcount,
                     key, dcells, st_dev, segst);
  scan_u64(bcount, sbase, nbt, scan_tmp, st);
  const unsigned dense_blocks = (unsigned)std::min<int64_t>(std::max<int64_t>(nbt / kDense, 1), 2048);
  hipLaunchKernelGGL(k_dense_order, dim3(dense_blocks), dim3(kDenseThreads), 0, st, key, st_dev, boff, sbase, pos,
                     slot_seg, segs, perm, soffs);
  hipLaunchKernelGGL(k_gather_pos, dim3(blocks_for(n, 256)), dim3(256), 0, st, pos, perm, slot_seg, n, spos, sseg);
}

}  // namespace mm
