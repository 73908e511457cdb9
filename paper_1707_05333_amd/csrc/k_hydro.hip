// Finite-volume kernels of the moving-mesh step (Sec. 4 of the paper), in
// the library's internal (bucket-sorted) cell order.  State arrays are
// cell-major rows (U [n][5], gradients [n][5][3]) so a gather of one
// neighbour reads one contiguous row.  R is double (MM_FP64) or float
// (MM_MIXED: state arithmetic in float, geometry and charge sums in double).
#include <algorithm>

#include "mm_internal.h"

namespace mm {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int kThreads = 256;

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// Orders a wavefront's LDS accesses: everything before is visible to every
// lane of the wavefront after.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// a / b: correctly rounded in double; in float (the mixed-precision state
// arithmetic) through the hardware reciprocal, within about one ulp.
template <typename T>
__device__ inline T quot(T a, T b) {
  return a / b;
}
template <>
__device__ inline float quot<float>(float a, float b) {
  return a * __builtin_amdgcn_rcpf(b);
}

// Floors of Sec. 4.1 on conserved densities: a density below the floor is
// raised keeping velocity and pressure; a pressure below the floor is raised
// keeping density and velocity.  Returns 1 if any floor fired.
template <typename T>
__device__ inline int apply_floors(T U[5], T g1, T rho_floor, T p_floor) {
  int hit = 0;
  const T rho = U[0];
  if (rho < rho_floor) {
    T vx = 0, vy = 0, vz = 0, P = p_floor;
    if (rho > T(0)) {
      const T ir = quot(T(1), rho);
      vx = U[1] * ir;
      vy = U[2] * ir;
      vz = U[3] * ir;
      P = g1 * (U[4] - T(0.5) * (U[1] * vx + U[2] * vy + U[3] * vz));
    }
    P = P > p_floor ? P : p_floor;
    U[0] = rho_floor;
    U[1] = rho_floor * vx;
    U[2] = rho_floor * vy;
    U[3] = rho_floor * vz;
    U[4] = quot(P, g1) + T(0.5) * rho_floor * (vx * vx + vy * vy + vz * vz);
    hit = 1;
  }
  const T ke = quot(T(0.5) * (U[1] * U[1] + U[2] * U[2] + U[3] * U[3]), U[0]);
  const T P = g1 * (U[4] - ke);
  if (P < p_floor) {
    U[4] = quot(p_floor, g1) + ke;
    hit = 1;
  }
  return hit;
}

// Time derivative of the state from its gradient (Sec. 4.1): -div F(U) by
// the chain rule, plus w . grad U when following the generator.
// g[3q + d] = d U_q / d x_d.
template <typename T>
__device__ inline void state_rate(const T U[5], const T g[15], const T wv[3], T g1, bool moving, T out[5]) {
  const T rho = U[0];
  const T ir = quot(T(1), rho);
  const T v[3] = {U[1] * ir, U[2] * ir, U[3] * ir};
  const T vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  const T P = g1 * (U[4] - T(0.5) * rho * vv);
  T dP[3], divv = 0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    dP[d] = g1 * (g[12 + d] - (v[0] * g[3 + d] + v[1] * g[6 + d] + v[2] * g[9 + d]) + T(0.5) * vv * g[d]);
    divv += (g[3 * (1 + d) + d] - v[d] * g[d]) * ir;
  }
  T div[5];
  div[0] = g[3 + 0] + g[6 + 1] + g[9 + 2];
#pragma unroll
  for (int a = 0; a < 3; ++a)
    div[1 + a] = v[0] * g[3 * (1 + a)] + v[1] * g[3 * (1 + a) + 1] + v[2] * g[3 * (1 + a) + 2] + U[1 + a] * divv +
                 dP[a];
  div[4] = v[0] * (g[12] + dP[0]) + v[1] * (g[13] + dP[1]) + v[2] * (g[14] + dP[2]) + (U[4] + P) * divv;
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    T adv = 0;
    if (moving) adv = wv[0] * g[3 * q] + wv[1] * g[3 * q + 1] + wv[2] * g[3 * q + 2];
    out[q] = adv - div[q];
  }
}

// Pressure a face solver takes from a conserved state.  In FP32 the
// difference E - rho v^2 / 2 resolves a pressure only down to about 6e-8 of
// the kinetic energy density, so a state floored at a pressure below that
// (cold gas moving fast) can come back slightly negative; the FP32 solver
// raises it to the floor.  FP64 states pass through unchanged.
template <typename T>
__device__ inline T face_pressure(T P, T p_floor) {
  if constexpr (sizeof(T) == 4) return P > p_floor ? P : p_floor;
  return P;
}

// Euler flux along unit normal n of a face-frame state (rho, v, P).
// ig1 = 1 / (gamma - 1).
template <typename T>
__device__ inline void euler_flux(T rho, const T v[3], T P, const T n[3], T ig1, T F[5]) {
  const T u = v[0] * n[0] + v[1] * n[1] + v[2] * n[2];
  const T E = P * ig1 + T(0.5) * rho * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  F[0] = rho * u;
  F[1] = rho * u * v[0] + P * n[0];
  F[2] = rho * u * v[1] + P * n[1];
  F[3] = rho * u * v[2] + P * n[2];
  F[4] = (E + P) * u;
}

// Flux across a face with unit normal n moving with velocity wt (Sec. 4,
// items 3-5): both lab-frame states are boosted to the face frame, HLLC (or
// HLL when hll is set) with Davis wave-speed bounds gives the face-frame
// flux, and the flux is boosted back (mass flux unchanged; momentum + wt F_rho; energy + wt.F_m +
// |wt|^2/2 F_rho).  The reciprocal densities are formed once per side.
template <typename T>
__device__ inline void moving_flux(const T UL[5], const T UR[5], const T n[3], const T wt[3], T gamma, bool hll,
                                   T p_floor, T F[5]) {
  const T g1 = gamma - T(1);
  const T ig1 = quot(T(1), g1);
  const T rL = UL[0], rR = UR[0];
  const T irL = quot(T(1), rL), irR = quot(T(1), rR);
  T vL[3], vR[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    vL[a] = UL[1 + a] * irL;
    vR[a] = UR[1 + a] * irR;
  }
  const T PL = face_pressure(g1 * (UL[4] - T(0.5) * (UL[1] * vL[0] + UL[2] * vL[1] + UL[3] * vL[2])), p_floor);
  const T PR = face_pressure(g1 * (UR[4] - T(0.5) * (UR[1] * vR[0] + UR[2] * vR[1] + UR[3] * vR[2])), p_floor);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    vL[a] -= wt[a];
    vR[a] -= wt[a];
  }
  const T uL = vL[0] * n[0] + vL[1] * n[1] + vL[2] * n[2];
  const T uR = vR[0] * n[0] + vR[1] * n[1] + vR[2] * n[2];
  const T cL = sqrt(gamma * PL * irL), cR = sqrt(gamma * PR * irR);
  const T SL = fmin(uL - cL, uR - cR);
  const T SR = fmax(uL + cL, uR + cR);
  T Ff[5];
  if (SL >= T(0)) {
    euler_flux(rL, vL, PL, n, ig1, Ff);
  } else if (SR < T(0)) {
    euler_flux(rR, vR, PR, n, ig1, Ff);
  } else if (hll) {
    // HLL: the one state between the bounding waves that conserves the
    // integral over the fan, F = (SR FL - SL FR + SL SR (UR - UL)) / (SR - SL).
    T FL[5], FR[5];
    euler_flux(rL, vL, PL, n, ig1, FL);
    euler_flux(rR, vR, PR, n, ig1, FR);
    const T EL = PL * ig1 + T(0.5) * rL * (vL[0] * vL[0] + vL[1] * vL[1] + vL[2] * vL[2]);
    const T ER = PR * ig1 + T(0.5) * rR * (vR[0] * vR[0] + vR[1] * vR[1] + vR[2] * vR[2]);
    const T dU[5] = {rR - rL, rR * vR[0] - rL * vL[0], rR * vR[1] - rL * vL[1], rR * vR[2] - rL * vL[2], ER - EL};
    const T iw = quot(T(1), SR - SL), sLR = SL * SR;
#pragma unroll
    for (int q = 0; q < 5; ++q) Ff[q] = (SR * FL[q] - SL * FR[q] + sLR * dU[q]) * iw;
  } else {
    const T Ss = quot(PR - PL + rL * uL * (SL - uL) - rR * uR * (SR - uR), rL * (SL - uL) - rR * (SR - uR));
    const bool left = Ss >= T(0);
    const T rK = left ? rL : rR, uK = left ? uL : uR, PK = left ? PL : PR, SK = left ? SL : SR;
    const T irK = left ? irL : irR;
    const T* vK = left ? vL : vR;
    T FK[5];
    euler_flux(rK, vK, PK, n, ig1, FK);
    const T EK = PK * ig1 + T(0.5) * rK * (vK[0] * vK[0] + vK[1] * vK[1] + vK[2] * vK[2]);
    const T a = SK - uK;
    const T fac = quot(rK * a, SK - Ss);
    const T du = Ss - uK;
    Ff[0] = FK[0] + SK * (fac - rK);
#pragma unroll
    for (int q = 0; q < 3; ++q) Ff[1 + q] = FK[1 + q] + SK * (fac * (vK[q] + du * n[q]) - rK * vK[q]);
    Ff[4] = FK[4] + SK * (fac * (EK * irK + du * (Ss + quot(PK * irK, a))) - EK);
  }
  const T w2 = wt[0] * wt[0] + wt[1] * wt[1] + wt[2] * wt[2];
  F[0] = Ff[0];
#pragma unroll
  for (int a = 0; a < 3; ++a) F[1 + a] = Ff[1 + a] + wt[a] * Ff[0];
  F[4] = Ff[4] + wt[0] * Ff[1] + wt[1] * Ff[2] + wt[2] * Ff[3] + T(0.5) * w2 * Ff[0];
}

// Entropy column on one face (Sec. 4.3): the face-frame flux of X = rho A,
// carried by the mass flux with the entropic function A of the side the
// contact leaves behind (upwind side when all waves go one way; the HLL
// average with hll), and the face's shock Mach number
// sqrt(1 + (gamma+1)/(2 gamma) max(0, p*/P_K - 1)) maximised over both
// sides, with p* the HLLC star pressure.  UL, UR are the face states after
// the face floors; AL, AR the entropic functions of the reconstruction.
template <typename T>
__device__ inline void entropy_flux(const T UL[5], const T UR[5], const T n[3], const T wt[3], T gamma, bool hll,
                                    T p_floor, T AL, T AR, T& FX, float& mach) {
  const T g1 = gamma - T(1);
  const T rL = UL[0], rR = UR[0];
  const T irL = quot(T(1), rL), irR = quot(T(1), rR);
  T vL[3], vR[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    vL[a] = UL[1 + a] * irL;
    vR[a] = UR[1 + a] * irR;
  }
  const T PL = face_pressure(g1 * (UL[4] - T(0.5) * (UL[1] * vL[0] + UL[2] * vL[1] + UL[3] * vL[2])), p_floor);
  const T PR = face_pressure(g1 * (UR[4] - T(0.5) * (UR[1] * vR[0] + UR[2] * vR[1] + UR[3] * vR[2])), p_floor);
  const T uL = (vL[0] - wt[0]) * n[0] + (vL[1] - wt[1]) * n[1] + (vL[2] - wt[2]) * n[2];
  const T uR = (vR[0] - wt[0]) * n[0] + (vR[1] - wt[1]) * n[1] + (vR[2] - wt[2]) * n[2];
  const T cL = sqrt(gamma * PL * irL), cR = sqrt(gamma * PR * irR);
  const T SL = fmin(uL - cL, uR - cR);
  const T SR = fmax(uL + cL, uR + cR);
  const T Ss = quot(PR - PL + rL * uL * (SL - uL) - rR * uR * (SR - uR), rL * (SL - uL) - rR * (SR - uR));
  const T ps = PL + rL * (SL - uL) * (Ss - uL);
  const T k = quot(gamma + T(1), T(2) * gamma);
  const T ML = sqrt(T(1) + k * fmax(T(0), quot(ps, PL) - T(1)));
  const T MR = sqrt(T(1) + k * fmax(T(0), quot(ps, PR) - T(1)));
  mach = (float)fmax(ML, MR);
  const T XL = rL * AL, XR = rR * AR;
  if (SL >= T(0)) {
    FX = XL * uL;
  } else if (SR < T(0)) {
    FX = XR * uR;
  } else if (hll) {
    FX = quot(SR * XL * uL - SL * XR * uR + SL * SR * (XR - XL), SR - SL);
  } else {
    const bool left = Ss >= T(0);
    const T rK = left ? rL : rR, uK = left ? uL : uR, SK = left ? SL : SR;
    const T fac = quot(rK * (SK - uK), SK - Ss);
    FX = (rK * uK + SK * (fac - rK)) * (left ? AL : AR);
  }
}

// Duffell-MacFadyen limit on one face (Sec. 4.1): the extrapolation D from
// the centroid to the face may not exceed theta times the jump dU to the
// neighbour, nor oppose its sign.  Returns beta D with
// beta = min(1, max(0, theta dU / D)), which is D, 0 or theta dU, so no
// division is needed; theta <= 0 switches the limit off (beta = 1).
template <typename T>
__device__ inline T dm_limited(T theta, T dU, T D) {
  if (theta <= T(0)) return D;
  const T t = theta * dU;
  if (!(t * D > T(0))) return T(0);   // opposite signs, or a zero jump or extrapolation
  return fabs(t) < fabs(D) ? t : D;
}

// ---------------------------------------------------------------------------

// Merges a per-cell timestep into its segment's minimum.  A block whose
// cells all belong to one segment (the usual case) reduces in LDS and issues
// one atomic; otherwise each wavefront does, or each cell of a wavefront
// that straddles segments.  Positive doubles order as their bit patterns.
__device__ void seg_min_dt(double v, int seg, bool active, SegStatus* segst) {
  __shared__ double red[kThreads / 64];
  __shared__ int sseg0[kThreads / 64 + 1];
  const int lane = __lane_id(), wid = threadIdx.x >> 6;
  const unsigned long long act = __ballot(active);
  const int first = act ? __ffsll((long long)act) - 1 : 0;
  const int seg0 = __shfl(seg, first, 64);
  const bool uniform = __ballot(active && seg != seg0) == 0ull;
  double m = active ? v : 1e300;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmin(m, __shfl_xor(m, o, 64));
  if (lane == 0) {
    red[wid] = m;
    sseg0[wid] = !act ? -1 : (uniform ? seg0 : -2);   // -1: no cell, -2: mixed
  }
  __syncthreads();
  int bseg = -1;
  bool block_uniform = true;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
    const int q = sseg0[k];
    if (q == -1) continue;
    if (q == -2 || (bseg >= 0 && q != bseg)) block_uniform = false;
    bseg = q;
  }
  if (block_uniform) {
    if (threadIdx.x == 0 && bseg >= 0) {
      double t = red[0];
      for (int k = 1; k < (int)(blockDim.x >> 6); ++k) t = fmin(t, red[k]);
      if (t < 1e300) atomicMin(&segst[bseg].dt_bits, (unsigned long long)__double_as_longlong(t));
    }
  } else if (uniform) {
    if (lane == first && act && m < 1e300)
      atomicMin(&segst[seg0].dt_bits, (unsigned long long)__double_as_longlong(m));
  } else if (active && v < 1e300) {
    atomicMin(&segst[seg].dt_bits, (unsigned long long)__double_as_longlong(v));
  }
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_cell_state(const SegDesc* __restrict__ segs,
                                                         const int32_t* __restrict__ sseg, int64_t n,
                                                         const double* __restrict__ Qc,
                                                         const int32_t* __restrict__ perm,
                                                         const double* __restrict__ geo, double* __restrict__ Qs,
                                                         R* __restrict__ U, double* __restrict__ w, DevStatus* st,
                                                         SegStatus* segst) {
  const int64_t s = xcd_block() * blockDim.x + threadIdx.x;
  const bool active = s < n;
  double dti = 1e300;
  int seg = 0;
  if (active) {
    seg = sseg[s];
    const HydroParams& hp = segs[seg].hp;
    const int64_t q = perm[s];
    double Q[5], u[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) Q[k] = Qc[5 * q + k];
    if (Qs) {
#pragma unroll
      for (int k = 0; k < 5; ++k) Qs[5 * s + k] = Q[k];
    }
    const double V = geo[4 * s];
    const double crx = geo[4 * s + 1], cry = geo[4 * s + 2], crz = geo[4 * s + 3];
#pragma unroll
    for (int k = 0; k < 5; ++k) u[k] = Q[k] / V;
    const double gamma = hp.gamma, g1 = gamma - 1.0;
    if (apply_floors(u, g1, hp.rho_floor, hp.p_floor)) atomicAdd(&segst[seg].floor_hits[0], 1ull);
    // Mesh velocity and timestep (Sec. 4.2).
    const double rho = u[0];
    const double vx = u[1] / rho, vy = u[2] / rho, vz = u[3] / rho;
    const double P = g1 * (u[4] - 0.5 * (u[1] * vx + u[2] * vy + u[3] * vz));
    const double cs = sqrt(gamma * P / rho);
    const double Rr = cbrt(3.0 * V / (4.0 * kPi));
    const double dn = sqrt(crx * crx + cry * cry + crz * crz);
    const double zeta = hp.zeta;
    double ramp;
    if (dn < 0.9 * zeta * Rr) ramp = 0.0;
    else if (dn <= 1.1 * zeta * Rr) ramp = (dn - 0.9 * zeta * Rr) / (0.2 * zeta * Rr);
    else ramp = 1.0;
    double dwx = 0.0, dwy = 0.0, dwz = 0.0;
    if (dn > 0.0 && ramp > 0.0) {
      const double chi = hp.chi;
      dwx = chi * cs * ramp * crx / dn;
      dwy = chi * cs * ramp * cry / dn;
      dwz = chi * cs * ramp * crz / dn;
    }
    const double eta = hp.eta;
    const double wx = eta * vx + dwx, wy = eta * vy + dwy, wz = eta * vz + dwz;
    const double rx = vx - wx, ry = vy - wy, rz = vz - wz;
    dti = hp.cfl * Rr / (cs + sqrt(rx * rx + ry * ry + rz * rz));
    w[3 * s] = wx;
    w[3 * s + 1] = wy;
    w[3 * s + 2] = wz;
#pragma unroll
    for (int k = 0; k < 5; ++k) U[5 * s + k] = (R)u[k];
    if (!(dti > 0.0 && dti < 1e300)) {
      seg_fail(st, segst, seg, F_NONFINITE, (int)s);
      dti = 1e300;
    }
  }
  seg_min_dt(dti, seg, active, segst);
}

// Least-squares gradient about the centroids with the S10 limiter (Sec. 4.1);
// with U_half set, the half-step predictor is applied in the same pass.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_gradient(const SegDesc* __restrict__ segs,
                                                       const int32_t* __restrict__ sseg, int64_t n,
                                                       const R* __restrict__ U,
                                                       const unsigned long long* __restrict__ counts,
                                                       const unsigned long long* __restrict__ soff,
                                                       const NbrEntry<R>* __restrict__ nbr,
                                                       const double* __restrict__ minv, int limit, R* __restrict__ G,
                                                       const double* __restrict__ w, const SegStatus* dt_src,
                                                       double dt_fixed, R* __restrict__ Uh,
                                                       FluxCell<R>* __restrict__ rec, const double* __restrict__ geo,
                                                       const double* __restrict__ spos, SegStatus* segst) {
  const int64_t s = xcd_block() * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int nf = (int)(counts[s] >> 32);
  const int64_t slot0 = sell_slot(soff, s, 0);   // entry e at slot0 + 64 e
  R ui[5], umax[5], umin[5], b[15];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    ui[q] = U[5 * s + q];
    umax[q] = ui[q];
    umin[q] = ui[q];
  }
#pragma unroll
  for (int k = 0; k < 15; ++k) b[k] = R(0);
  // Two entries' loads in flight at once pay in FP64 (10% faster) but not
  // with the smaller FP32 entries (10% slower).
  constexpr int kUnroll = sizeof(R) == 8 ? 2 : 1;
#pragma unroll kUnroll
  for (int e = 0; e < nf; ++e) {
    const NbrW<R> E = *nbr_w(nbr, slot0 + 64 * e);
    const R* dd = nbr_d(nbr, slot0 + 64 * e);
    const R dx = dd[0], dy = dd[1], dz = dd[2], wg = E.wgt;
    const R* uo = U + 5 * (int64_t)E.o;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      const R v = uo[q];
      const R t = wg * (v - ui[q]);
      b[3 * q] += t * dx;
      b[3 * q + 1] += t * dy;
      b[3 * q + 2] += t * dz;
      umax[q] = v > umax[q] ? v : umax[q];
      umin[q] = v < umin[q] ? v : umin[q];
    }
  }
  const double* mi = minv + 6 * s;
  const R m00 = (R)mi[0], m01 = (R)mi[1], m02 = (R)mi[2], m11 = (R)mi[3], m12 = (R)mi[4], m22 = (R)mi[5];
  R g[15];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    const R bx = b[3 * q], by = b[3 * q + 1], bz = b[3 * q + 2];
    g[3 * q] = m00 * bx + m01 * by + m02 * bz;
    g[3 * q + 1] = m01 * bx + m11 * by + m12 * bz;
    g[3 * q + 2] = m02 * bx + m12 * by + m22 * bz;
  }
  const int seg = sseg[s];
  const bool lim = limit < kLimitMaskBit0 ? limit != kLimitOff
                                          : ((segs[seg].hp.limit_mask >> (limit - kLimitMaskBit0)) & 1) != 0;
  if (lim) {
    // alpha = min(1, min_j psi_j) with psi_j = (U^max - U_i) / D_j for
    // D_j > 0 and (U^min - U_i) / D_j for D_j < 0.  Over the neighbours with
    // D_j > 0 the smallest quotient is the one with the largest D_j
    // (correctly rounded division is monotone), and likewise for D_j < 0,
    // so two divisions per component give the same value as one per
    // neighbour.
    R dpos[5], dneg[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) dpos[q] = dneg[q] = R(0);
    for (int e = 0; e < nf; ++e) {
      const R* dd = nbr_d(nbr, slot0 + 64 * e);
      const R dx = dd[0], dy = dd[1], dz = dd[2];
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        const R D = g[3 * q] * dx + g[3 * q + 1] * dy + g[3 * q + 2] * dz;
        dpos[q] = D > dpos[q] ? D : dpos[q];
        dneg[q] = D < dneg[q] ? D : dneg[q];
      }
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      R alpha = R(1);
      if (dpos[q] > R(0)) {
        const R psi = quot(umax[q] - ui[q], dpos[q]);
        alpha = psi < alpha ? psi : alpha;
      }
      if (dneg[q] < R(0)) {
        const R psi = quot(umin[q] - ui[q], dneg[q]);
        alpha = psi < alpha ? psi : alpha;
      }
      g[3 * q] *= alpha;
      g[3 * q + 1] *= alpha;
      g[3 * q + 2] *= alpha;
    }
  }
  if (G) {
#pragma unroll
    for (int k = 0; k < 15; ++k) G[15 * s + k] = g[k];
  }
  if (rec) {
    FluxCell<R> C;
#pragma unroll
    for (int q = 0; q < 5; ++q) C.U[q] = ui[q];
#pragma unroll
    for (int k = 0; k < 15; ++k) C.G[k] = g[k];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      C.w[a] = w[3 * s + a];
      C.c[a] = geo[4 * s + 1 + a];
      C.r[a] = spos[3 * s + a];
    }
    rec[s] = C;
  }
  if (Uh) {
    const HydroParams& hp = segs[seg].hp;
    const double dt = seg_dt(segs, dt_src, seg, dt_fixed);
    const R wv[3] = {(R)w[3 * s], (R)w[3 * s + 1], (R)w[3 * s + 2]};
    R rt[5], uh[5];
    state_rate(ui, g, wv, (R)(hp.gamma - 1.0), hp.predictor_frame == 0, rt);
    const R hdt = (R)(0.5 * dt);
#pragma unroll
    for (int q = 0; q < 5; ++q) uh[q] = ui[q] + hdt * rt[q];
    if (apply_floors(uh, (R)(hp.gamma - 1.0), (R)hp.rho_floor, (R)hp.p_floor))
      atomicAdd(&segst[seg].floor_hits[1], 1ull);
#pragma unroll
    for (int q = 0; q < 5; ++q) Uh[5 * s + q] = uh[q];
  }
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_predict(const SegDesc* __restrict__ segs,
                                                      const int32_t* __restrict__ sseg, int64_t n,
                                                      const R* __restrict__ U, const R* __restrict__ G,
                                                      const double* __restrict__ w, const SegStatus* dt_src,
                                                      double dt_fixed, R* __restrict__ Uh, SegStatus* segst) {
  const int64_t s = xcd_block() * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int seg = sseg[s];
  const HydroParams& hp = segs[seg].hp;
  R ui[5], g[15], rt[5], uh[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) ui[q] = U[5 * s + q];
#pragma unroll
  for (int k = 0; k < 15; ++k) g[k] = G[15 * s + k];
  const R wv[3] = {(R)w[3 * s], (R)w[3 * s + 1], (R)w[3 * s + 2]};
  const double dt = seg_dt(segs, dt_src, seg, dt_fixed);
  state_rate(ui, g, wv, (R)(hp.gamma - 1.0), hp.predictor_frame == 0, rt);
  const R hdt = (R)(0.5 * dt);
#pragma unroll
  for (int q = 0; q < 5; ++q) uh[q] = ui[q] + hdt * rt[q];
  if (apply_floors(uh, (R)(hp.gamma - 1.0), (R)hp.rho_floor, (R)hp.p_floor))
    atomicAdd(&segst[seg].floor_hits[1], 1ull);
#pragma unroll
  for (int q = 0; q < 5; ++q) Uh[5 * s + q] = uh[q];
}

// Scheme values one face needs from its segment.  When a wavefront's faces
// all belong to one segment (every launch of a single simulation, and all
// but the boundary wavefronts of a batch) they come through scalar loads.
struct FaceParams {
  double L[3];
  double theta, gamma, rho_floor, p_floor, dt;
  bool hll;
};

__device__ inline FaceParams face_params(const SegDesc* segs, const SegStatus* dt_src, double dt_fixed, int seg) {
  const int s0 = __builtin_amdgcn_readfirstlane(seg);
  const int sg = __all(seg == s0) ? s0 : seg;
  const HydroParams& hp = segs[sg].hp;
  FaceParams P;
  P.L[0] = hp.L[0];
  P.L[1] = hp.L[1];
  P.L[2] = hp.L[2];
  P.theta = hp.theta;
  P.gamma = hp.gamma;
  P.rho_floor = hp.rho_floor;
  P.p_floor = hp.p_floor;
  P.hll = hp.riemann == kRiemannHll;
  P.dt = seg_dt(segs, dt_src, sg, dt_fixed);
  return P;
}

// One thread per unique face (Sec. 4 items 1-5, Sec. 4.1 reconstruction):
// phi = dt A F, F the lab-frame flux from the owner i toward j.  Each XCD
// takes one contiguous eighth of the face list (faces are in owner order, so
// the cells it gathers stay in its L2) and its wavefronts stride through it.
// With ENT the entropy column's face flux and the face's shock Mach number
// are written as well (Sec. 4.3).
// The owners of a wavefront's faces are a few consecutive cells, but its 64
// neighbours are scattered: rather than each lane fetching its neighbour's
// record alone (every load instruction then touches 64 cache lines), the
// wavefront fetches the 64 records together, consecutive lanes taking
// consecutive 16-byte pieces of one record, and hands them over in LDS.
constexpr int kFluxThreads = 128;

template <typename R, bool ENT>
__global__ __launch_bounds__(kFluxThreads, sizeof(R) == 8 ? 6 : 8) void k_flux(const SegDesc* __restrict__ segs, int64_t nf_host,
                                                       const unsigned long long* __restrict__ nf_dev,
                                                       const Face* __restrict__ faces,
                                                       const FluxCell<R>* __restrict__ rec, const SegStatus* dt_src,
                                                       double dt_fixed, R* __restrict__ phi, SegStatus* segst,
                                                       const XCell<R>* __restrict__ recx, R* __restrict__ phiX,
                                                       float* __restrict__ machF) {
  constexpr int kPieces = (int)(sizeof(FluxCell<R>) / sizeof(uint4));
  static_assert(sizeof(FluxCell<R>) % sizeof(uint4) == 0, "records are whole 16-byte pieces");
  __shared__ uint4 stage[kFluxThreads / 64][64 * kPieces];
  const int lane = __lane_id();
  uint4* const own = stage[threadIdx.x >> 6];
  const int64_t nf = nf_dev ? std::min<int64_t>((int64_t)*nf_dev, nf_host) : nf_host;
  const int64_t xcd = blockIdx.x % kXcds, kb = blockIdx.x / kXcds;
  const int64_t nbx = ((int64_t)gridDim.x - xcd + kXcds - 1) / kXcds;
  const int64_t lo = nf * xcd / kXcds, hi = nf * (xcd + 1) / kXcds;
  for (int64_t f0 = lo + kb * blockDim.x + (threadIdx.x & ~63); f0 < hi; f0 += nbx * blockDim.x) {
    const int64_t f = f0 + lane;
    const bool valid = f < hi;
    Face F;
    if (valid) F = faces[f];
    const int jl = valid ? F.j : 0;   // a lane past the end fetches record 0 and ignores it
    // Piece q = lane + 64 k of the wavefront's records is piece q % kPieces
    // of the record of lane q / kPieces.
#pragma unroll
    for (int k = 0; k < kPieces; ++k) {
      const int q = lane + 64 * k;
      const int j = __shfl(jl, q / kPieces);
      own[q] = reinterpret_cast<const uint4*>(rec + j)[q % kPieces];
    }
    wave_sync();
    if (valid) {
      const FluxCell<R> A = rec[F.i];
      const FluxCell<R>& B = *reinterpret_cast<const FluxCell<R>*>(own + lane * kPieces);
      const int seg = F.seg;
      const FaceParams hp = face_params(segs, dt_src, dt_fixed, seg);
      int kx, ky, kz;
      decode(F.code, kx, ky, kz);
      // Geometry in double: r_j + s - r_i, face centre and centroid offsets.
      const double drx = (B.r[0] + kx * hp.L[0]) - A.r[0];
      const double dry = (B.r[1] + ky * hp.L[1]) - A.r[1];
      const double drz = (B.r[2] + kz * hp.L[2]) - A.r[2];
      const double len = sqrt(drx * drx + dry * dry + drz * drz);
      const double ilen = 1.0 / len;
      const double nx = drx * ilen, ny = dry * ilen, nz = drz * ilen;
      // Face velocity (Sec. 4 item 1): bisector's normal speed at the face
      // centre plus the mean generator velocity.
      const double sn = ((A.w[0] - B.w[0]) * (F.f[0] - 0.5 * drx) + (A.w[1] - B.w[1]) * (F.f[1] - 0.5 * dry) +
                         (A.w[2] - B.w[2]) * (F.f[2] - 0.5 * drz)) * ilen;
      const R wt[3] = {(R)(sn * nx + 0.5 * (A.w[0] + B.w[0])), (R)(sn * ny + 0.5 * (A.w[1] + B.w[1])),
                       (R)(sn * nz + 0.5 * (A.w[2] + B.w[2]))};
      const R nrm[3] = {(R)nx, (R)ny, (R)nz};
      // f - c_i and f - (c_j + s), with f and c relative to the generators.
      const R fi[3] = {(R)(F.f[0] - A.c[0]), (R)(F.f[1] - A.c[1]), (R)(F.f[2] - A.c[2])};
      const R fj[3] = {(R)(F.f[0] - drx - B.c[0]), (R)(F.f[1] - dry - B.c[1]), (R)(F.f[2] - drz - B.c[2])};
      const R theta = (R)hp.theta;
      R UL[5], UR[5];
  #pragma unroll
      for (int q = 0; q < 5; ++q) {
        const R ui = A.U[q], uj = B.U[q];
        const R Di = A.G[3 * q] * fi[0] + A.G[3 * q + 1] * fi[1] + A.G[3 * q + 2] * fi[2];
        const R Dj = B.G[3 * q] * fj[0] + B.G[3 * q + 1] * fj[1] + B.G[3 * q + 2] * fj[2];
        UL[q] = ui + dm_limited(theta, uj - ui, Di);
        UR[q] = uj + dm_limited(theta, ui - uj, Dj);
      }
      const R g1 = (R)(hp.gamma - 1.0);
      // A side whose reconstruction would need a floor takes its cell's
      // half-step state (already floored): extrapolating each component
      // across a large density jump can pair a small density with a large
      // momentum, a velocity no floor repairs.
      bool fbL, fbR;
      {
        R t[5];
  #pragma unroll
        for (int q = 0; q < 5; ++q) t[q] = UL[q];
        fbL = apply_floors(t, g1, (R)hp.rho_floor, (R)hp.p_floor) != 0;
  #pragma unroll
        for (int q = 0; q < 5; ++q) t[q] = UR[q];
        fbR = apply_floors(t, g1, (R)hp.rho_floor, (R)hp.p_floor) != 0;
      }
      if (fbL) {
  #pragma unroll
        for (int q = 0; q < 5; ++q) UL[q] = A.U[q];
      }
      if (fbR) {
  #pragma unroll
        for (int q = 0; q < 5; ++q) UR[q] = B.U[q];
      }
      const int hit = (int)fbL + (int)fbR;
      if (hit) atomicAdd(&segst[seg].floor_hits[2], (unsigned long long)hit);
      const R rL0 = UL[0], rR0 = UR[0];
      R Fx[5];
      moving_flux(UL, UR, nrm, wt, (R)hp.gamma, hp.hll, (R)hp.p_floor, Fx);
      const R scale = (R)(hp.dt * F.A);
  #pragma unroll
      for (int q = 0; q < 5; ++q) phi[5 * f + q] = scale * Fx[q];
      if constexpr (ENT) {
        const XCell<R> XA = recx[F.i], XB = recx[F.j];
        const R Di = XA.g[0] * fi[0] + XA.g[1] * fi[1] + XA.g[2] * fi[2];
        const R Dj = XB.g[0] * fj[0] + XB.g[1] * fj[1] + XB.g[2] * fj[2];
        const R XL = fbL ? XA.X : XA.X + dm_limited(theta, XB.X - XA.X, Di);
        const R XR = fbR ? XB.X : XB.X + dm_limited(theta, XA.X - XB.X, Dj);
        R FX;
        float mach;
        entropy_flux(UL, UR, nrm, wt, (R)hp.gamma, hp.hll, (R)hp.p_floor, quot(XL, rL0), quot(XR, rR0), FX,
                     mach);
        phiX[f] = scale * FX;
        machF[f] = mach;
      }
    }
    wave_sync();   // every lane has read its record before the next pieces land
  }
}

// Entropy column (Sec. 4.3): X = S / V of each internal cell, S gathered.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_entropy_state(int64_t n, const int32_t* __restrict__ perm,
                                                            const double* __restrict__ geo,
                                                            const double* __restrict__ Sc, double* __restrict__ Ss,
                                                            R* __restrict__ X) {
  const int64_t s = xcd_block() * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const double S = Sc[perm[s]];
  Ss[s] = S;
  X[s] = (R)(S / geo[4 * s]);
}

// Gradient of the entropy column, with the same least squares and S10
// limiter as k_gradient (one component); then either the half-step value
// X + dt/2 (-div(X v) + w . grad X) or the face kernel's record.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_entropy_gradient(
    const SegDesc* __restrict__ segs, const int32_t* __restrict__ sseg, int64_t n, const R* __restrict__ X,
    const unsigned long long* __restrict__ counts, const unsigned long long* __restrict__ soff,
    const NbrEntry<R>* __restrict__ nbr, const double* __restrict__ minv, int limit, const R* __restrict__ U,
    const R* __restrict__ G, const double* __restrict__ w, const SegStatus* dt_src, R* __restrict__ Xh,
    XCell<R>* __restrict__ recx) {
  const int64_t s = xcd_block() * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int nf = (int)(counts[s] >> 32);
  const int64_t slot0 = sell_slot(soff, s, 0);   // entry e at slot0 + 64 e
  const R xi = X[s];
  R xmax = xi, xmin = xi, b[3] = {R(0), R(0), R(0)};
  for (int e = 0; e < nf; ++e) {
    const NbrW<R> E = *nbr_w(nbr, slot0 + 64 * e);
    const R* dd = nbr_d(nbr, slot0 + 64 * e);
    const R v = X[E.o];
    const R t = E.wgt * (v - xi);
    b[0] += t * dd[0];
    b[1] += t * dd[1];
    b[2] += t * dd[2];
    xmax = v > xmax ? v : xmax;
    xmin = v < xmin ? v : xmin;
  }
  const double* mi = minv + 6 * s;
  const R m00 = (R)mi[0], m01 = (R)mi[1], m02 = (R)mi[2], m11 = (R)mi[3], m12 = (R)mi[4], m22 = (R)mi[5];
  R g[3] = {m00 * b[0] + m01 * b[1] + m02 * b[2], m01 * b[0] + m11 * b[1] + m12 * b[2],
            m02 * b[0] + m12 * b[1] + m22 * b[2]};
  const int seg = sseg[s];
  const HydroParams& hp = segs[seg].hp;
  const bool lim = limit < kLimitMaskBit0 ? limit != kLimitOff
                                          : ((hp.limit_mask >> (limit - kLimitMaskBit0)) & 1) != 0;
  if (lim) {
    R dpos = R(0), dneg = R(0);
    for (int e = 0; e < nf; ++e) {
      const R* dd = nbr_d(nbr, slot0 + 64 * e);
      const R D = g[0] * dd[0] + g[1] * dd[1] + g[2] * dd[2];
      dpos = D > dpos ? D : dpos;
      dneg = D < dneg ? D : dneg;
    }
    R alpha = R(1);
    if (dpos > R(0)) {
      const R psi = quot(xmax - xi, dpos);
      alpha = psi < alpha ? psi : alpha;
    }
    if (dneg < R(0)) {
      const R psi = quot(xmin - xi, dneg);
      alpha = psi < alpha ? psi : alpha;
    }
    g[0] *= alpha;
    g[1] *= alpha;
    g[2] *= alpha;
  }
  if (Xh) {
    const R* u = U + 5 * s;
    const R* gr = G + 15 * s;
    const R ir = quot(R(1), u[0]);
    const R v[3] = {u[1] * ir, u[2] * ir, u[3] * ir};
    R divv = R(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) divv += (gr[3 * (1 + a) + a] - v[a] * gr[a]) * ir;
    R rate = -(v[0] * g[0] + v[1] * g[1] + v[2] * g[2] + xi * divv);
    if (hp.predictor_frame == 0) rate += (R)w[3 * s] * g[0] + (R)w[3 * s + 1] * g[1] + (R)w[3 * s + 2] * g[2];
    const double dt = seg_dt(segs, dt_src, seg, 0.0);
    Xh[s] = xi + (R)(0.5 * dt) * rate;
  }
  if (recx) recx[s] = XCell<R>{xi, {g[0], g[1], g[2]}};
}

template <typename R>
__global__ void k_pack_flux_cells(int64_t n, const R* __restrict__ U, const R* __restrict__ G,
                                  const double* __restrict__ w, const double* __restrict__ geo,
                                  const double* __restrict__ spos, FluxCell<R>* __restrict__ rec) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  FluxCell<R> C;
#pragma unroll
  for (int q = 0; q < 5; ++q) C.U[q] = U[5 * s + q];
#pragma unroll
  for (int k = 0; k < 15; ++k) C.G[k] = G[15 * s + k];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    C.w[a] = w[3 * s + a];
    C.c[a] = geo[4 * s + 1 + a];
    C.r[a] = spos[3 * s + a];
  }
  rec[s] = C;
}

// Per-cell sum of the face fluxes through the CSR list in a fixed order:
// the owner side loses phi, the neighbour side gains it (Sec. 4, update of
// the charges).  Accumulation in double.
template <typename R>
__device__ inline void cell_flux_sum(int64_t s, const unsigned long long* counts, const unsigned long long* soff,
                                     const int32_t* csr, const R* phi, double acc[5]) {
  const int nf = (int)(counts[s] >> 32);
  const int32_t* list = csr + sell_slot(soff, s, 0);   // entry e at list[64 e]
#pragma unroll
  for (int q = 0; q < 5; ++q) acc[q] = 0.0;
  // Unrolled so the loads of four entries are in flight together (the sum
  // keeps its order).
#pragma unroll 4
  for (int e = 0; e < nf; ++e) {
    const int32_t cf = list[64 * e];
    const int64_t fid = cf & 0x7fffffff;
    const double sg = cf < 0 ? 1.0 : -1.0;
#pragma unroll
    for (int q = 0; q < 5; ++q) acc[q] += sg * (double)phi[5 * fid + q];
  }
}

// The charges, positions and entropy charges after the step, in internal
// order: Qn may be Qs (each thread reads its own row before writing it).
// Nothing in the caller's arrays changes here; k_commit copies the results
// out once every failure of the step is known.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_update(const SegDesc* __restrict__ segs,
                                                     const int32_t* __restrict__ sseg, int64_t n,
                                                     const unsigned long long* __restrict__ counts,
                                                     const unsigned long long* __restrict__ soff,
                                                     const int32_t* __restrict__ csr, const R* __restrict__ phi,
                                                     const double* __restrict__ geo, const int32_t* __restrict__ perm,
                                                     const double* Qs, double* Qn,
                                                     const double* __restrict__ spos, const double* __restrict__ w,
                                                     const double* __restrict__ posc, double* __restrict__ pn,
                                                     const SegStatus* dt_src, DevStatus* st, SegStatus* segst,
                                                     bool drift_from_slots, double* Ss,
                                                     const R* __restrict__ phiX, const float* __restrict__ machF,
                                                     float* __restrict__ machs) {
  const int64_t s = xcd_block() * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int seg = sseg[s];
  const HydroParams& hp = segs[seg].hp;
  double acc[5], Q[5];
  cell_flux_sum(s, counts, soff, csr, phi, acc);
#pragma unroll
  for (int q = 0; q < 5; ++q) Q[q] = Qs[5 * s + q] + acc[q];
  const double V = geo[4 * s];
  const double gamma = hp.gamma, g1 = gamma - 1.0;
  // Entropy switch (Sec. 4.3): the cell's largest face Mach number decides
  // whether its pressure follows the entropy (no shock) or the energy.
  double Snew = 0.0;
  float mx = 0.0f;
  bool from_entropy = false;
  if (Ss) {
    const int nfc = (int)(counts[s] >> 32);
    const int32_t* list = csr + sell_slot(soff, s, 0);
    double accX = 0.0;
#pragma unroll 4
    for (int e = 0; e < nfc; ++e) {
      const int32_t cf = list[64 * e];
      const int64_t fid = cf & 0x7fffffff;
      accX += (cf < 0 ? 1.0 : -1.0) * (double)phiX[fid];
      mx = fmaxf(mx, machF[fid]);
    }
    Snew = Ss[s] + accX;
    if ((double)mx < hp.mach_threshold) {
      const double m = Q[0];
      const double P = (Snew / m) * pow(m / V, gamma);
      Q[4] = P * V / g1 + 0.5 * (Q[1] * Q[1] + Q[2] * Q[2] + Q[3] * Q[3]) / m;
      from_entropy = true;
    }
  }
  // Floors at the cell centre after the step, with the volume of the mesh
  // the fluxes used.
  double u[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) u[q] = Q[q] / V;
  const bool floored = apply_floors(u, g1, hp.rho_floor, hp.p_floor);
  if (floored) {
    atomicAdd(&segst[seg].floor_hits[3], 1ull);
#pragma unroll
    for (int q = 0; q < 5; ++q) Q[q] = u[q] * V;
  }
  if (Ss) {
    if (!from_entropy || floored) {
      // The energy was integrated (or floored): the entropy follows the state.
      const double ir = 1.0 / u[0];
      const double P = g1 * (u[4] - 0.5 * (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) * ir);
      Snew = Q[0] * P / pow(u[0], gamma);
    }
  }
  int bad = 0;
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    Qn[5 * s + q] = Q[q];
    if (!isfinite(Q[q])) bad = 1;
  }
  // Drift by the full step with periodic wrap, from the start-of-step
  // position (the caller's slot when the mesh is a half-step one).
  const double dt = seg_dt(segs, dt_src, seg, 0.0);
  const int64_t c = drift_from_slots ? perm[s] : 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double x = (drift_from_slots ? posc[3 * c + a] : spos[3 * s + a]) + w[3 * s + a] * dt;
    if (x < 0.0) x += hp.L[a];
    if (x >= hp.L[a]) x -= hp.L[a];
    pn[3 * s + a] = x;
  }
  if (Ss) {
    Ss[s] = Snew;
    if (machs) machs[s] = mx;
    if (!isfinite(Snew)) bad = 1;
  }
  if (bad) seg_fail(st, segst, seg, F_NONFINITE, (int)s);
}

// Copies the step's results of every segment whose step raised no failure
// into the caller's slot-order arrays (charges, positions, mesh velocities,
// and with the entropy column its charges and Mach numbers).  A segment
// with a failure keeps its state as it was before the step, and so does
// every segment when the shared face capacity overflowed.
__global__ __launch_bounds__(kThreads) void k_commit(const int32_t* __restrict__ sseg, int64_t n,
                                                     const int32_t* __restrict__ perm, const DevStatus* __restrict__ st,
                                                     const SegStatus* __restrict__ segst,
                                                     const double* __restrict__ Qn, const double* __restrict__ pn,
                                                     const double* __restrict__ w, const double* __restrict__ Ss,
                                                     const float* __restrict__ machs, double* __restrict__ Qc,
                                                     double* __restrict__ posc, double* __restrict__ wc,
                                                     double* __restrict__ Sc, float* __restrict__ machc) {
  const int64_t s = xcd_block() * blockDim.x + threadIdx.x;
  if (s >= n) return;
  if (segst[sseg[s]].flags || (st->flags & F_FACECAP)) return;
  const int64_t c = perm[s];
#pragma unroll
  for (int q = 0; q < 5; ++q) Qc[5 * c + q] = Qn[5 * s + q];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    posc[3 * c + a] = pn[3 * s + a];
    wc[3 * c + a] = w[3 * s + a];
  }
  if (Sc) {
    Sc[c] = Ss[s];
    if (machc) machc[c] = machs[s];
  }
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_accumulate(int64_t n, const unsigned long long* __restrict__ counts,
                                                         const unsigned long long* __restrict__ soff,
                                                         const int32_t* __restrict__ csr, const R* __restrict__ phi,
                                                         const int32_t* __restrict__ perm, double* __restrict__ dQc) {
  const int64_t s = xcd_block() * blockDim.x + threadIdx.x;
  if (s >= n) return;
  double acc[5];
  cell_flux_sum(s, counts, soff, csr, phi, acc);
  const int64_t c = perm[s];
#pragma unroll
  for (int q = 0; q < 5; ++q) dQc[5 * c + q] = acc[q];
}

template <typename R>
__global__ void k_gather_rows(const R* __restrict__ src, const int32_t* __restrict__ perm, int64_t n, int width,
                              R* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * width) return;
  const int64_t s = t / width, k = t - s * width;
  dst[t] = src[(int64_t)perm[s] * width + k];
}

template <typename R>
__global__ void k_scatter_rows(const R* __restrict__ src, const int32_t* __restrict__ perm, int64_t n, int width,
                               R* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * width) return;
  const int64_t s = t / width, k = t - s * width;
  dst[(int64_t)perm[s] * width + k] = src[t];
}

__global__ void k_copy_rows(const double* __restrict__ src, double* __restrict__ dst, int64_t count) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) dst[t] = src[t];
}

// Charges from primitives (Sec. 4.3): Q = (rho, rho v, P/(gamma-1) + rho v^2/2) V.
// prim and Q may be the same array (each thread reads its row before writing it).
__global__ void k_init_charges(const SegDesc* __restrict__ segs, const int32_t* __restrict__ sseg, int64_t n,
                               const double* prim, const int32_t* __restrict__ perm,
                               const double* __restrict__ geo, double* Q, int only_fresh) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int seg = sseg[s];
  if (only_fresh && !segs[seg].fresh) return;
  const double gamma = segs[seg].hp.gamma;
  const int64_t c = perm[s];
  const double V = geo[4 * s];
  const double rho = prim[5 * c], vx = prim[5 * c + 1], vy = prim[5 * c + 2], vz = prim[5 * c + 3],
               P = prim[5 * c + 4];
  const double ke = 0.5 * rho * (vx * vx + vy * vy + vz * vz);
  Q[5 * c] = rho * V;
  Q[5 * c + 1] = rho * vx * V;
  Q[5 * c + 2] = rho * vy * V;
  Q[5 * c + 3] = rho * vz * V;
  Q[5 * c + 4] = (P / (gamma - 1.0) + ke) * V;
}

// Entropy charges S = m P rho^-gamma (Sec. 4.3) of primitive states, in
// caller order.
__global__ void k_init_entropy(const SegDesc* __restrict__ segs, const int32_t* __restrict__ sseg, int64_t n,
                               const double* prim, const int32_t* __restrict__ perm,
                               const double* __restrict__ geo, double* S) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const double gamma = segs[sseg[s]].hp.gamma;
  const int64_t c = perm[s];
  const double rho = prim[5 * c], P = prim[5 * c + 4];
  S[c] = rho * geo[4 * s] * P / pow(rho, gamma);
}

}  // namespace

void launch_init_entropy(const SegDesc* segs, const int32_t* sseg, int64_t n, const double* prim_slots,
                         const int32_t* perm, const double* geo, double* S_slots, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_init_entropy, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, st, segs, sseg, n,
                     prim_slots, perm, geo, S_slots);
}

template <typename R>
void launch_cell_state(const SegDesc* segs, const int32_t* sseg, int64_t n, const double* Q_slots,
                       const int32_t* perm, const double* geo, double* Qs, R* U, double* w, DevStatus* st_dev,
                       SegStatus* segst, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_cell_state<R>, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, st, segs, sseg, n, Q_slots,
                     perm, geo, Qs, U, w, st_dev, segst);
}

template <typename R>
void launch_gradient(const SegDesc* segs, const int32_t* sseg, int64_t n, const R* U,
                     const unsigned long long* counts, const unsigned long long* soff, const NbrEntry<R>* nbr,
                     const double* minv, int limit, R* G, const double* w, const SegStatus* dt_src, double dt_fixed,
                     R* U_half, FluxCell<R>* rec, const double* geo, const double* spos, SegStatus* segst,
                     hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_gradient<R>, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, st, segs, sseg, n, U, counts,
                     soff, nbr, minv, limit, G, w, dt_src, dt_fixed, U_half, rec, geo, spos, segst);
}

template <typename R>
void launch_pack_flux_cells(int64_t n, const R* U, const R* G, const double* w, const double* geo,
                            const double* spos, FluxCell<R>* rec, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_pack_flux_cells<R>, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, st, n, U, G, w, geo,
                     spos, rec);
}

template <typename R>
void launch_predict(const SegDesc* segs, const int32_t* sseg, int64_t n, const R* U, const R* G, const double* w,
                    const SegStatus* dt_src, double dt_fixed, R* U_half, SegStatus* segst, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_predict<R>, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, st, segs, sseg, n, U, G, w,
                     dt_src, dt_fixed, U_half, segst);
}

template <typename R>
void launch_flux(const SegDesc* segs, int64_t nf_host, const unsigned long long* nf_dev, const Face* faces,
                 const FluxCell<R>* rec, const SegStatus* dt_src, double dt_fixed, R* phi, SegStatus* segst,
                 hipStream_t st, const XCell<R>* recx, R* phiX, float* machF) {
  if (nf_host <= 0) return;
  // Enough resident blocks to fill the chip; each strides through its XCD's
  // part of the (device-counted) face list.  The kernel splits the list into
  // kXcds ranges by blockIdx.x % kXcds, so the grid is a whole multiple of
  // kXcds blocks (at least one per range) or a range would be left undone.
  const int64_t want = std::min<int64_t>(blocks_for(nf_host, kFluxThreads), 8192);
  const unsigned blocks = (unsigned)((want + kXcds - 1) / kXcds * kXcds);
  if (recx)
    hipLaunchKernelGGL((k_flux<R, true>), dim3(blocks), dim3(kFluxThreads), 0, st, segs, nf_host, nf_dev, faces,
                       rec, dt_src, dt_fixed, phi, segst, recx, phiX, machF);
  else
    hipLaunchKernelGGL((k_flux<R, false>), dim3(blocks), dim3(kFluxThreads), 0, st, segs, nf_host, nf_dev, faces,
                       rec, dt_src, dt_fixed, phi, segst, nullptr, nullptr, nullptr);
}

template <typename R>
void launch_entropy_state(int64_t n, const int32_t* perm, const double* geo, const double* S_slots, double* Ss,
                          R* X, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_entropy_state<R>, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, st, n, perm, geo,
                     S_slots, Ss, X);
}

template <typename R>
void launch_entropy_gradient(const SegDesc* segs, const int32_t* sseg, int64_t n, const R* X,
                             const unsigned long long* counts, const unsigned long long* soff, const NbrEntry<R>* nbr,
                             const double* minv, int limit, const R* U, const R* G, const double* w,
                             const SegStatus* dt_src, R* Xh, XCell<R>* recx, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_entropy_gradient<R>, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, st, segs, sseg, n, X,
                     counts, soff, nbr, minv, limit, U, G, w, dt_src, Xh, recx);
}

template <typename R>
void launch_update(const SegDesc* segs, const int32_t* sseg, int64_t n, const unsigned long long* counts,
                   const unsigned long long* soff, const int32_t* csr, const R* phi, const double* geo,
                   const int32_t* perm, double* Qs, const double* spos, const double* w, const double* pos_slots,
                   double* pn, const SegStatus* dt_src, DevStatus* st_dev, SegStatus* segst, hipStream_t st,
                   bool drift_from_slots, double* Ss, const R* phiX, const float* machF, float* machs) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_update<R>, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, st, segs, sseg, n, counts, soff,
                     csr, phi, geo, perm, Qs, Qs, spos, w, pos_slots, pn, dt_src, st_dev, segst, drift_from_slots, Ss,
                     phiX, machF, machs);
}

void launch_commit(const int32_t* sseg, int64_t n, const int32_t* perm, const DevStatus* st_dev,
                   const SegStatus* segst, const double* Qn, const double* pn, const double* w, const double* Ss,
                   const float* machs, double* Q_slots, double* pos_slots, double* w_slots, double* S_slots,
                   float* mach_slots, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_commit, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, st, sseg, n, perm, st_dev, segst, Qn, pn, w,
                     Ss, machs, Q_slots, pos_slots, w_slots, S_slots, mach_slots);
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_half_park(const SegDesc* __restrict__ segs,
                                                        const int32_t* __restrict__ sseg, int64_t n,
                                                        const int32_t* __restrict__ perm, const R* __restrict__ Uh,
                                                        const double* __restrict__ w, const SegStatus* dt_src,
                                                        const double* __restrict__ posc, double* __restrict__ pos_half,
                                                        R* __restrict__ Uhc, double* __restrict__ wc) {
  const int64_t s = xcd_block() * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int seg = sseg[s];
  const HydroParams& hp = segs[seg].hp;
  const double hdt = 0.5 * seg_dt(segs, dt_src, seg, 0.0);
  const int64_t c = perm[s];
#pragma unroll
  for (int q = 0; q < 5; ++q) Uhc[5 * c + q] = Uh[5 * s + q];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double wa = w[3 * s + a];
    wc[3 * c + a] = wa;
    double x = posc[3 * c + a] + wa * hdt;
    if (x < 0.0) x += hp.L[a];
    if (x >= hp.L[a]) x -= hp.L[a];
    pos_half[3 * c + a] = x;
  }
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_half_unpark(int64_t n, const int32_t* __restrict__ perm,
                                                          const R* __restrict__ Uhc, const double* __restrict__ wc,
                                                          const double* __restrict__ Qc, R* __restrict__ Uh,
                                                          double* __restrict__ w, double* __restrict__ Qs) {
  const int64_t s = xcd_block() * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int64_t c = perm[s];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    Uh[5 * s + q] = Uhc[5 * c + q];
    Qs[5 * s + q] = Qc[5 * c + q];
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) w[3 * s + a] = wc[3 * c + a];
}

template <typename R>
void launch_half_park(const SegDesc* segs, const int32_t* sseg, int64_t n, const int32_t* perm, const R* Uh,
                      const double* w, const SegStatus* dt_src, const double* pos_slots, double* pos_half,
                      R* Uh_slots, double* w_slots, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_half_park<R>, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, st, segs, sseg, n, perm, Uh,
                     w, dt_src, pos_slots, pos_half, Uh_slots, w_slots);
}

template <typename R>
void launch_half_unpark(int64_t n, const int32_t* perm, const R* Uh_slots, const double* w_slots,
                        const double* Q_slots, R* Uh, double* w, double* Qs, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_half_unpark<R>, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, st, n, perm, Uh_slots,
                     w_slots, Q_slots, Uh, w, Qs);
}

template <typename R>
void launch_accumulate(int64_t n, const unsigned long long* counts, const unsigned long long* soff, const int32_t* csr,
                       const R* phi, const int32_t* perm, double* dQ_slots, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_accumulate<R>, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, st, n, counts, soff, csr,
                     phi, perm, dQ_slots);
}

template <typename R>
void launch_gather_rows(const R* src_slots, const int32_t* perm, int64_t n, int width, R* dst, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_gather_rows<R>, dim3(blocks_for(n * width, kThreads)), dim3(kThreads), 0, st, src_slots, perm,
                     n, width, dst);
}

template <typename R>
void launch_scatter_rows(const R* src, const int32_t* perm, int64_t n, int width, R* dst_slots, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_scatter_rows<R>, dim3(blocks_for(n * width, kThreads)), dim3(kThreads), 0, st, src, perm, n,
                     width, dst_slots);
}

void launch_init_charges(const SegDesc* segs, const int32_t* sseg, int64_t n, const double* prim_slots,
                         const int32_t* perm, const double* geo, double* Q_slots, int only_fresh, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_init_charges, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, st, segs, sseg, n, prim_slots,
                     perm, geo, Q_slots, only_fresh);
}

void launch_copy_rows(const double* src, double* dst, int64_t n, int width, hipStream_t st) {
  const int64_t count = n * width;
  if (count <= 0) return;
  hipLaunchKernelGGL(k_copy_rows, dim3(blocks_for(count, kThreads)), dim3(kThreads), 0, st, src, dst, count);
}

#define MM_INSTANTIATE(R)                                                                                          \
  template void launch_cell_state<R>(const SegDesc*, const int32_t*, int64_t, const double*, const int32_t*,      \
                                     const double*, double*, R*, double*, DevStatus*, SegStatus*, hipStream_t);   \
  template void launch_gradient<R>(const SegDesc*, const int32_t*, int64_t, const R*, const unsigned long long*,  \
                                   const unsigned long long*, const NbrEntry<R>*, const double*, int, R*,         \
                                   const double*, const SegStatus*, double, R*, FluxCell<R>*, const double*,      \
                                   const double*, SegStatus*, hipStream_t);                                       \
  template void launch_pack_flux_cells<R>(int64_t, const R*, const R*, const double*, const double*,              \
                                          const double*, FluxCell<R>*, hipStream_t);                              \
  template void launch_predict<R>(const SegDesc*, const int32_t*, int64_t, const R*, const R*, const double*,     \
                                  const SegStatus*, double, R*, SegStatus*, hipStream_t);                         \
  template void launch_flux<R>(const SegDesc*, int64_t, const unsigned long long*, const Face*,                    \
                               const FluxCell<R>*, const SegStatus*, double, R*, SegStatus*, hipStream_t,         \
                               const XCell<R>*, R*, float*);                                                      \
  template void launch_entropy_state<R>(int64_t, const int32_t*, const double*, const double*, double*, R*,       \
                                        hipStream_t);                                                             \
  template void launch_entropy_gradient<R>(const SegDesc*, const int32_t*, int64_t, const R*,                     \
                                           const unsigned long long*, const unsigned long long*,                  \
                                           const NbrEntry<R>*, const double*, int, const R*, const R*,            \
                                           const double*, const SegStatus*, R*, XCell<R>*, hipStream_t);          \
  template void launch_update<R>(const SegDesc*, const int32_t*, int64_t, const unsigned long long*,              \
                                 const unsigned long long*, const int32_t*, const R*, const double*,              \
                                 const int32_t*, double*, const double*, const double*, const double*, double*,   \
                                 const SegStatus*, DevStatus*, SegStatus*, hipStream_t, bool, double*, const R*,  \
                                 const float*, float*);                                                           \
  template void launch_half_park<R>(const SegDesc*, const int32_t*, int64_t, const int32_t*, const R*,            \
                                    const double*, const SegStatus*, const double*, double*, R*, double*,         \
                                    hipStream_t);                                                                 \
  template void launch_half_unpark<R>(int64_t, const int32_t*, const R*, const double*, const double*, R*,         \
                                      double*, double*, hipStream_t);                                             \
  template void launch_accumulate<R>(int64_t, const unsigned long long*, const unsigned long long*,               \
                                     const int32_t*, const R*, const int32_t*, double*, hipStream_t);             \
  template void launch_gather_rows<R>(const R*, const int32_t*, int64_t, int, R*, hipStream_t);                   \
  template void launch_scatter_rows<R>(const R*, const int32_t*, int64_t, int, R*, hipStream_t);

MM_INSTANTIATE(double)
MM_INSTANTIATE(float)

}  // namespace mm
