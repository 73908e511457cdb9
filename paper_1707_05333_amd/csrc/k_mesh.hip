// Mesh assembly after the tessellation: unique faces (each stored once, by
// the cell with the lower internal index), the per-cell face lists used to
// apply every face flux to both of its cells with opposite signs (Sec. 4,
// update of the charges), the per-cell neighbour entries of the
// least-squares gradient (centroid displacements and weights, Sec. 4.1) and
// the inverse of each cell's 3x3 least-squares matrix.  Also the exports of
// the mesh to the caller's point order.
//
// Per-cell lists use a sliced ELL layout: cells are taken in slices of 64
// consecutive internal cells, a slice is as wide as its longest list, and
// entry e of cell s sits at soff[s / 64] + 64 e + s % 64.  A wavefront
// that walks the lists of 64 consecutive cells in step then reads one
// contiguous row per step.
#include "mm_internal.h"

namespace mm {

namespace {

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

constexpr int kGroup = 8;                        // lanes per cell in the assembly
constexpr int kMeshThreads = 256;
constexpr int kCellsPerBlock = kMeshThreads / kGroup;

// 64 times the longest list of each slice of 64 cells (one wavefront per slice).
__global__ __launch_bounds__(256) void k_slice_width(const unsigned long long* __restrict__ counts, int64_t n,
                                                     unsigned long long* __restrict__ sw) {
  const int64_t k = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int64_t s = 64 * k + __lane_id();
  const int64_t nslices = (n + 63) / 64;
  int w = s < n ? (int)(counts[s] >> 32) : 0;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) w = max(w, __shfl_xor(w, o, 64));
  if (k < nslices && __lane_id() == 0) sw[k] = 64ull * (unsigned long long)w;
}

// Eight lanes per cell; lane l takes the cell's faces l, l + 8, ... (a lane
// walks two or three faces: more cells per wavefront than with sixteen
// lanes, whose last lanes idle while the first take a second face).
// The packed prefix sum off[] holds, for cell s, the index of its first
// unique face in its low 32 bits.
template <typename R>
__global__ __launch_bounds__(kMeshThreads) void k_build_mesh(
    const double* __restrict__ spos, const double* __restrict__ geo, int64_t n, const SegDesc* __restrict__ segs,
    const int32_t* __restrict__ sseg, const StageNbr* __restrict__ stage_nb, const StageGeo* __restrict__ stage_geo,
    const unsigned long long* __restrict__ counts, const unsigned long long* __restrict__ off,
    const unsigned long long* __restrict__ soff, int64_t face_cap, int64_t sell_cap, Face* __restrict__ faces,
    int32_t* __restrict__ csr, NbrEntry<R>* __restrict__ nbr, double* __restrict__ minv, DevStatus* st,
    SegStatus* segst) {
  __shared__ int smax[kMeshThreads / 64];
  const int l = threadIdx.x & (kGroup - 1);
  const int64_t s = xcd_block() * kCellsPerBlock + (threadIdx.x / kGroup);
  const bool active = s < n;
  double m00 = 0, m01 = 0, m02 = 0, m11 = 0, m12 = 0, m22 = 0;
  int nf = 0, bad = 0, seg = 0;
  if (active) {
    seg = sseg[s];
    const double L[3] = {segs[seg].g.L[0], segs[seg].g.L[1], segs[seg].g.L[2]};
    nf = (int)(counts[s] >> 32);
    const int64_t face_base = (int64_t)(off[s] & 0xffffffffull);
    const int64_t slice = s >> 6;
    const int64_t sbase = (int64_t)soff[slice] + (s & 63);
    if ((int64_t)soff[slice + 1] > sell_cap) {   // lists beyond the list capacity
      nf = 0;
      bad |= F_FACECAP;
    }
    const double rx = spos[3 * s], ry = spos[3 * s + 1], rz = spos[3 * s + 2];
    const double cix = geo[4 * s + 1], ciy = geo[4 * s + 2], ciz = geo[4 * s + 3];
    for (int e = l; e < nf; e += kGroup) {
      const StageNbr Nb = stage_nb[s * kMaxFaces + e];
      const StageGeo F = stage_geo[s * kMaxFaces + e];
      const int j = Nb.j;
      const int code = Nb.meta & 255;
      const bool owned = (Nb.meta >> 8) & 1;
      const int orank = Nb.meta >> 16;
      int kx, ky, kz;
      decode(code, kx, ky, kz);
      // centroid displacement d = (c_j + s) - c_i = (r_j + s - r_i) + (c_j - r_j) - (c_i - r_i)
      const double drx = (spos[3 * (int64_t)j] + kx * L[0]) - rx;
      const double dry = (spos[3 * (int64_t)j + 1] + ky * L[1]) - ry;
      const double drz = (spos[3 * (int64_t)j + 2] + kz * L[2]) - rz;
      const double dx = drx + geo[4 * (int64_t)j + 1] - cix;
      const double dy = dry + geo[4 * (int64_t)j + 2] - ciy;
      const double dz = drz + geo[4 * (int64_t)j + 3] - ciz;
      const double wgt = F.A / (dx * dx + dy * dy + dz * dz);
      const int64_t slot = sbase + 64ll * e;
      NbrW<R> E{};
      E.o = j;
      E.wgt = (R)wgt;
      *nbr_w(nbr, slot) = E;
      R* D = nbr_d(nbr, slot);
      D[0] = (R)dx;
      D[1] = (R)dy;
      D[2] = (R)dz;
      m00 += wgt * dx * dx;
      m01 += wgt * dx * dy;
      m02 += wgt * dx * dz;
      m11 += wgt * dy * dy;
      m12 += wgt * dy * dz;
      m22 += wgt * dz * dz;
      int32_t entry = 0;
      if (owned) {
        const int64_t fid = face_base + orank;
        if (fid < face_cap) {
          Face out;
          out.i = (int32_t)s;
          out.j = j;
          out.code = code;
          out.seg = seg;
          out.A = F.A;
          out.f[0] = F.f[0];
          out.f[1] = F.f[1];
          out.f[2] = F.f[2];
          faces[fid] = out;
          entry = (int32_t)fid;
        } else {
          bad |= F_FACECAP;
        }
      } else {
        // The same face in the neighbour's list: neighbour s, opposite image.
        // Two staged entries per 16-byte load (rows are 512-byte aligned).
        const int want = 26 - code;
        const int nfj = (int)(counts[j] >> 32);
        const int4* row = reinterpret_cast<const int4*>(stage_nb + (int64_t)j * kMaxFaces);
        // Eight entries per round, their loads issued together.
        int found_meta = -1;
        for (int t = 0; t < nfj && found_meta < 0; t += 8) {
          int4 G[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) G[u] = row[(t >> 1) + u];   // rows hold kMaxFaces entries: in bounds
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int e0 = t + 2 * u;
            if (found_meta < 0 && e0 < nfj && G[u].x == (int)s && (G[u].y & 255) == want) found_meta = G[u].y;
            if (found_meta < 0 && e0 + 1 < nfj && G[u].z == (int)s && (G[u].w & 255) == want) found_meta = G[u].w;
          }
        }
        if (found_meta < 0 || !((found_meta >> 8) & 1)) {
          bad |= F_ASYM;
          st->asym_cell = (int)s;
          st->asym_nbr = j;
        } else {
          const int64_t fid = (int64_t)(off[j] & 0xffffffffull) + (found_meta >> 16);
          if (fid < face_cap) entry = (int32_t)(fid | 0x80000000ll);
          else bad |= F_FACECAP;
        }
      }
      csr[slot] = entry;
    }
  }
  // Least-squares matrix summed over the group's lanes, and its failures.
#pragma unroll
  for (int o = kGroup / 2; o > 0; o >>= 1) {
    m00 += __shfl_xor(m00, o, kGroup);
    m01 += __shfl_xor(m01, o, kGroup);
    m02 += __shfl_xor(m02, o, kGroup);
    m11 += __shfl_xor(m11, o, kGroup);
    m12 += __shfl_xor(m12, o, kGroup);
    m22 += __shfl_xor(m22, o, kGroup);
    bad |= __shfl_xor(bad, o, kGroup);
  }
  if (active && l == 0) {
    // Inverse of the symmetric least-squares matrix by its adjugate.
    const double a00 = m11 * m22 - m12 * m12;
    const double a01 = m02 * m12 - m01 * m22;
    const double a02 = m01 * m12 - m02 * m11;
    const double a11 = m00 * m22 - m02 * m02;
    const double a12 = m02 * m01 - m00 * m12;
    const double a22 = m00 * m11 - m01 * m01;
    const double det = m00 * a00 + m01 * a01 + m02 * a02;
    double* mi = minv + 6 * s;
    if (nf > 0) {
      mi[0] = a00 / det;
      mi[1] = a01 / det;
      mi[2] = a02 / det;
      mi[3] = a11 / det;
      mi[4] = a12 / det;
      mi[5] = a22 / det;
    } else {
      for (int k = 0; k < 6; ++k) mi[k] = 0.0;
    }
    if (bad) seg_fail(st, segst, seg, bad, (int)s);
  }
  // Largest face count of the block.
  int mx = nf;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o, 64));
  if (__lane_id() == 0) smax[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = smax[0];
    for (int k = 1; k < kMeshThreads / 64; ++k) t = max(t, smax[k]);
    if (t > 0) atomicMax(&st->max_faces, t);
  }
}

__global__ void k_copy_totals(const unsigned long long* off, int64_t n, DevStatus* st) {
  if (threadIdx.x == 0) {
    st->n_faces = off[n] & 0xffffffffull;
    st->n_csr = off[n] >> 32;
  }
}

__global__ void k_export_cells(int64_t n, const int32_t* __restrict__ perm, const double* __restrict__ spos,
                               const double* __restrict__ geo, double* V, double* centroid) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int64_t q = perm[s];
  if (V) V[q] = geo[4 * s];
  if (centroid) {
    for (int a = 0; a < 3; ++a) centroid[3 * q + a] = spos[3 * s + a] + geo[4 * s + 1 + a];
  }
}

__global__ void k_export_faces(int64_t nf, const int32_t* __restrict__ perm, const double* __restrict__ spos,
                               const Face* __restrict__ faces, int32_t* fi, int32_t* fj, int32_t* fc, double* fA,
                               double* ff) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const Face F = faces[f];
  if (fi) fi[f] = perm[F.i];
  if (fj) fj[f] = perm[F.j];
  if (fc) fc[f] = F.code;
  if (fA) fA[f] = F.A;
  if (ff) {
    for (int a = 0; a < 3; ++a) ff[3 * f + a] = spos[3 * (int64_t)F.i + a] + F.f[a];
  }
}

}  // namespace

void launch_build_mesh(const double* spos, const double* geo, int64_t n, const SegDesc* segs, const int32_t* sseg,
                       const StageNbr* stage_nb, const StageGeo* stage_geo, const unsigned long long* counts,
                       const unsigned long long* off, unsigned long long* sw, unsigned long long* soff,
                       unsigned long long* scan_tmp, int64_t face_cap, int64_t sell_cap, Face* faces, int32_t* csr,
                       void* nbr, int precision, double* minv, DevStatus* st_dev, SegStatus* segst, hipStream_t st) {
  if (n > 0) {
    const int64_t nslices = (n + 63) / 64;
    hipLaunchKernelGGL(k_slice_width, dim3(blocks_for(nslices, 4)), dim3(256), 0, st, counts, n, sw);
    scan_u64(sw, soff, nslices, scan_tmp, st);
    if (precision == 1)   // MM_MIXED
      hipLaunchKernelGGL(k_build_mesh<float>, dim3(blocks_for(n, kCellsPerBlock)), dim3(kMeshThreads), 0, st, spos,
                         geo, n, segs, sseg, stage_nb, stage_geo, counts, off, soff, face_cap, sell_cap, faces, csr,
                         (NbrEntry<float>*)nbr, minv, st_dev, segst);
    else
      hipLaunchKernelGGL(k_build_mesh<double>, dim3(blocks_for(n, kCellsPerBlock)), dim3(kMeshThreads), 0, st, spos,
                         geo, n, segs, sseg, stage_nb, stage_geo, counts, off, soff, face_cap, sell_cap, faces, csr,
                         (NbrEntry<double>*)nbr, minv, st_dev, segst);
  }
  hipLaunchKernelGGL(k_copy_totals, dim3(1), dim3(64), 0, st, off, n, st_dev);
}

void launch_export_mesh(int64_t n, int64_t nf, const int32_t* perm, const double* spos, const double* geo,
                        const Face* faces, double* V, double* centroid, int32_t* fi, int32_t* fj, int32_t* fc,
                        double* fA, double* ff, hipStream_t st) {
  if (n > 0)
    hipLaunchKernelGGL(k_export_cells, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, perm, spos, geo, V, centroid);
  if (nf > 0)
    hipLaunchKernelGGL(k_export_faces, dim3(blocks_for(nf, 256)), dim3(256), 0, st, nf, perm, spos, faces, fi, fj,
                       fc, fA, ff);
}

}  // namespace mm
