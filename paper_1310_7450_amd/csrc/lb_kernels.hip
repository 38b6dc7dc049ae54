// gfx950 kernels of lbnlm: the fused pull / velocity-gradient / inlM stress /
// forcing / BGK sweep, its observation variant, the per-channel FP64
// reduction and the step-counter advance.
//
// Layout: ten fields per node (nine populations in the order
// (0,0),(1,0),(0,1),(-1,0),(0,-1),(1,1),(-1,1),(-1,-1),(1,-1), then the
// previous stress trace), stored as tiles of 64 consecutive nodes (row by
// row, x fastest, every channel starting on a tile): a tile holds field 0 of
// its 64 nodes, then field 1, ... (structure of arrays inside a 64-node
// tile, 2.5 KB in FP32). A slot holds the post-collision population of the
// previous step at its source node; the sweep pulls it along the lattice
// velocity (Sec. II.A, Eq. (lbupdate)), or from the same node with the
// opposite velocity where the link crosses a wall (half-way bounce-back,
// Sec. II.B).
//
// One wavefront marches up a strip of rows. It keeps the provisional
// velocity u~ = j/sum_i n_i of three consecutive row blocks in registers, so
// the central differences of Sec. II.C need no LDS: x neighbours come from
// lane moves, y neighbours from the previous/next block.
//  * narrow channels (nx a power of two up to 64) put whole periods into
//    lane groups of nx lanes (sweep_kernel);
//  * channels with nx a multiple of 64 run strips of 64 aligned columns
//    (sweep_wide64_kernel): every load is one aligned 64-lane run of a tile,
//    addressed from a wave-uniform tile base, and the x-shifted pulls are
//    DPP lane shifts of the aligned loads, with the two edge columns loaded
//    separately; this keeps the address arithmetic scalar;
//  * other widths run generic 64-column strips with wrapped lanes
//    (sweep_kernel, WIDE).
// The physics of one node (stencil, stress, forcing, collision) is one
// device function shared by all of them.
#include "lb_internal.h"

namespace lbnlm {
namespace {

#ifndef LB_WG_WAVES
#define LB_WG_WAVES 4
#endif
// Rows of loads in flight per wavefront in the vector sweep. A state that
// stays in the last-level cache (cached stores) runs best with two: the
// third row's registers push the FP32 kernel into accumulator registers
// (76 of them against 11), whose moves cost more than the deeper prefetch
// gains. A state written with nontemporal stores, streamed from HBM, runs
// best with three.
#ifndef LB_VEC_DEPTH
#define LB_VEC_DEPTH 2
#endif
#ifndef LB_VEC_DEPTH_NT
#define LB_VEC_DEPTH_NT 3
#endif

template <typename T>
__device__ __forceinline__ T shfl(T v, int src) {
  return __shfl(v, src, 64);
}

template <typename T>
__device__ __forceinline__ constexpr T weight(int i) {
  return i == 0 ? T(4.0 / 9.0) : (i < 5 ? T(1.0 / 9.0) : T(1.0 / 36.0));
}

template <typename T>
__device__ __forceinline__ T recip(T v) {
  if constexpr (sizeof(T) == 4) return __builtin_amdgcn_rcpf(v);
  return T(1) / v;
}
// Square root: FP32 takes the hardware instruction (1 ulp, like the
// reciprocal above) instead of the correctly rounded sequence.
template <typename T>
__device__ __forceinline__ T root(T v) {
  if constexpr (sizeof(T) == 4) return __builtin_amdgcn_sqrtf(v);
  return sqrt(v);
}

// Lane moves across the whole wavefront: shift_up gives lane i the value of
// lane i-1 (lane 0 gets `edge`), shift_down gives lane i the value of lane
// i+1 (lane 63 gets `edge`).
__device__ __forceinline__ int dpp_shr(int edge, int v) {
  return __builtin_amdgcn_update_dpp(edge, v, 0x138, 0xf, 0xf, false);
}
__device__ __forceinline__ int dpp_shl(int edge, int v) {
  return __builtin_amdgcn_update_dpp(edge, v, 0x130, 0xf, 0xf, false);
}
template <typename T>
__device__ __forceinline__ T shift_up(T edge, T v) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, dpp_shr(__builtin_bit_cast(int, edge), __builtin_bit_cast(int, v)));
  } else {
    const long long e = __builtin_bit_cast(long long, edge), x = __builtin_bit_cast(long long, v);
    const int lo = dpp_shr((int)e, (int)x), hi = dpp_shr((int)(e >> 32), (int)(x >> 32));
    return __builtin_bit_cast(T, ((long long)hi << 32) | (unsigned int)lo);
  }
}
template <typename T>
__device__ __forceinline__ T shift_down(T edge, T v) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, dpp_shl(__builtin_bit_cast(int, edge), __builtin_bit_cast(int, v)));
  } else {
    const long long e = __builtin_bit_cast(long long, edge), x = __builtin_bit_cast(long long, v);
    const int lo = dpp_shl((int)e, (int)x), hi = dpp_shl((int)(e >> 32), (int)(x >> 32));
    return __builtin_bit_cast(T, ((long long)hi << 32) | (unsigned int)lo);
  }
}
template <typename T>
__device__ __forceinline__ T lane_value(T v, int l) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
  } else {
    const long long x = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)x, l), hi = __builtin_amdgcn_readlane((int)(x >> 32), l);
    return __builtin_bit_cast(T, ((long long)hi << 32) | (unsigned int)lo);
  }
}

// Pulls the nine post-streaming populations of node (x, y), 0 <= y < ny;
// row = index of node (0, y).
// uw6 = u_w/6 of the top wall during the previous step: the populations
// reflected there gained -/+ u_w/6 (a_i c_ix u_w / cs2 for the diagonals).
template <typename T>
__device__ __forceinline__ void pull(const T *__restrict__ A, long long row, int nx, int ny, int x,
                                     int y, T uw6, T f[9]) {
  const int xm = (x == 0) ? nx - 1 : x - 1;
  const int xp = (x == nx - 1) ? 0 : x + 1;
  const long long dn = row - nx, up = row + nx;
  const bool bot = (y == 0), top = (y == ny - 1);
  f[0] = A[slot(0, row + x)];
  f[1] = A[slot(1, row + xm)];
  f[3] = A[slot(3, row + xp)];
  f[2] = A[bot ? slot(4, row + x) : slot(2, dn + x)];
  f[5] = A[bot ? slot(7, row + x) : slot(5, dn + xm)];
  f[6] = A[bot ? slot(8, row + x) : slot(6, dn + xp)];
  f[4] = A[top ? slot(2, row + x) : slot(4, up + x)];
  f[7] = A[top ? slot(5, row + x) : slot(7, up + xp)] - (top ? uw6 : T(0));
  f[8] = A[top ? slot(6, row + x) : slot(8, up + xm)] + (top ? uw6 : T(0));
}

// Slot of population q of node m of a channel relative to the channel's first
// slot (channels start on a tile boundary, so slot(q, off + m) = kPlanes *
// off + lslot(q, m)); 32-bit, for channels of fewer than 2^32 / kPlanes
// nodes.
__device__ __forceinline__ unsigned lslot(int q, unsigned m) {
  return ((m >> 6) * kPlanes + q) * kTile + (m & (kTile - 1));
}

// pull() on a channel's own slots (C = the channel's first slot).
__device__ __forceinline__ void pull_local(const double *__restrict__ C, int nx, int ny, int x, int y, double uw6,
                                           double f[9]) {
  const unsigned row = (unsigned)y * nx;
  const unsigned xm = (x == 0) ? nx - 1 : x - 1, xp = (x == nx - 1) ? 0 : x + 1;
  const unsigned dn = row - nx, up = row + nx;
  const bool bot = (y == 0), top = (y == ny - 1);
  f[0] = C[lslot(0, row + x)];
  f[1] = C[lslot(1, row + xm)];
  f[3] = C[lslot(3, row + xp)];
  f[2] = C[bot ? lslot(4, row + x) : lslot(2, dn + x)];
  f[5] = C[bot ? lslot(7, row + x) : lslot(5, dn + xm)];
  f[6] = C[bot ? lslot(8, row + x) : lslot(6, dn + xp)];
  f[4] = C[top ? lslot(2, row + x) : lslot(4, up + x)];
  f[7] = C[top ? lslot(5, row + x) : lslot(7, up + xp)] - (top ? uw6 : 0.0);
  f[8] = C[top ? lslot(6, row + x) : lslot(8, up + xm)] + (top ? uw6 : 0.0);
}

// Zeroth and first moments of the stored values: sd = sum_i f_i, m = sum_i
// c_i f_i. With SHIFT the stored values are n_i - a_i, so sd is the density
// deviation rho - 1 (kept separate so FP32 does not round it against 1) and
// the momentum is unchanged.
template <typename T>
__device__ __forceinline__ void moments(const T f[9], T &sd, T &mx, T &my) {
  sd = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
  mx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
  my = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
}

template <typename T>
struct U2 {
  T x, y;
};

template <typename T>
__device__ __forceinline__ U2<T> shfl2(U2<T> v, int src) {
  return U2<T>{shfl(v.x, src), shfl(v.y, src)};
}

// Provisional velocity u~ = (m + f/2) / sum_i n_i (reading R2 of the design
// notes: the stencil uses the velocity before the flow-induced density).
// With SHIFT the populations are stored relative to the equilibrium at the
// row's reference velocity (ur, 0), mx is the momentum beyond ur and the x
// component returned is u~_x - ur, kept small so that FP32 resolves it.
// No fused multiply-adds here or in the two helpers below: the nodes of a row
// and the halo columns beside a strip take these terms through differently
// shared code and must still round them identically (an x-uniform state
// stays exactly x-uniform).
template <typename T, bool SHIFT>
__device__ __forceinline__ U2<T> u_tilde(T sd, T mx, T my, T fx, T ur) {
#pragma clang fp contract(off)
  const T inv = recip<T>(SHIFT ? T(1) + sd : sd);
  if constexpr (SHIFT) return U2<T>{(mx + T(0.5) * fx - ur * sd) * inv, my * inv};
  return U2<T>{(mx + T(0.5) * fx) * inv, my * inv};
}

// FP32 storage: a population emitted by a node of row y is stored as
// n_i - a_i - E_i(ur_y), E_i(u) = a_i (3 c_ix u + (4.5 c_ix^2 - 1.5) u^2) the
// equilibrium excess at density 1 and velocity (u, 0). A value pulled from
// row y' != y therefore changes by E_i(ur_y') - E_i(ur_y); one reflected at a
// wall comes from the same node's opposite population and changes by
// E_opp(ur_y) - E_i(ur_y) = -6 a_i c_ix ur_y. Both are formed from
// differences, so the small stored values stay exact to FP32 rounding.
template <typename T>
__device__ __forceinline__ T ref_shift(T a, T cx, T us, T ud) {
#pragma clang fp contract(off)
  return a * (us - ud) * (T(3) * cx + (T(4.5) * cx * cx - T(1.5)) * (us + ud));
}
template <typename T>
__device__ __forceinline__ void to_row_reference(T f[9], T urd, T urc, T uru, bool bot, bool top) {
#pragma clang fp contract(off)
  constexpr T w1 = T(1.0 / 9.0), w5 = T(1.0 / 36.0);
  // from below (c_y = +1): 2 (c_x 0), 5 (+1), 6 (-1)
  f[2] += bot ? T(0) : ref_shift(w1, T(0), urd, urc);
  f[5] += bot ? -urc * T(1.0 / 6.0) : ref_shift(w5, T(1), urd, urc);
  f[6] += bot ? urc * T(1.0 / 6.0) : ref_shift(w5, T(-1), urd, urc);
  // from above (c_y = -1): 4 (0), 7 (-1), 8 (+1)
  f[4] += top ? T(0) : ref_shift(w1, T(0), uru, urc);
  f[7] += top ? urc * T(1.0 / 6.0) : ref_shift(w5, T(-1), uru, urc);
  f[8] += top ? -urc * T(1.0 / 6.0) : ref_shift(w5, T(1), uru, urc);
}

// Zou and He's velocity boundary on the top node row (Sec. II.B, the moving
// wall of planar Couette flow): the three populations a node of row ny - 1
// lacks after streaming (c_y = -1: 4, 7, 8) follow from the six it has. No
// flow through the wall gives the density s = f0 + f1 + f3 + 2 (f2 + f5 +
// f6); the normal non-equilibrium part bounces back, f4 = f2; the diagonals
// keep f7 + f8 = f5 + f6 and supply the x momentum for which the provisional
// velocity (m + f/2)/s is the wall's (uw, 0). With SHIFT the values are
// relative to the equilibrium at density 1 and the row reference (ur, 0):
// s is then the density deviation and the momentum the one beyond ur,
// (uw - ur) + s uw - f/2, and the relations between stored values are the
// same (the reference terms of 4 and 2, and of 7 + 8 and 5 + 6, are equal).
template <typename T, bool SHIFT>
__device__ __forceinline__ void zou_he_top(T f[9], T uw, T ur, T fx) {
#pragma clang fp contract(off)
  const T s = (f[0] + f[1] + f[3]) + T(2) * (f[2] + f[5] + f[6]);
  const T m = SHIFT ? (uw - ur) + s * uw - T(0.5) * fx : s * uw - T(0.5) * fx;
  const T d87 = m - ((f[1] - f[3]) + (f[5] - f[6]));
  const T s78 = f[5] + f[6];
  f[4] = f[2];
  f[8] = T(0.5) * (s78 + d87);
  f[7] = T(0.5) * (s78 - d87);
}
// x momentum a node of the top row gave a Zou-He wall in the previous step:
// what it emitted upwards (its own stored 5 and 6, a5 - a6) minus what the
// completion f supplies (f8 - f7). With SHIFT the reduction adds -ur/6 per
// node (the reference terms of both differences).
template <typename T>
__device__ __forceinline__ double zh_drag(T a5, T a6, const T f[9]) {
  return ((double)a5 - (double)a6) - ((double)f[8] - (double)f[7]);
}

// Wave-wide sum over a lane group of width GW (power of two).
template <int GW>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int m = 1; m < GW; m <<= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Channel constants in the arithmetic type.
template <typename T>
struct Coef {
  T om, kf, sp, G, inv_tau, inv_gc, lgt;
  bool stress_on;
  __device__ explicit Coef(const ChanDev &c)
      : om(T(c.omega)), kf(T(c.kf)), sp(T(c.sp)), G(T(c.G)), inv_tau(T(c.inv_tau)),
        inv_gc(T(c.inv_gc)), lgt(T(c.lgt)), stress_on(c.G > 0.0) {}
};

// Instantaneous stress (Eqs. (nlmaxwell), (sigtsum)) for the velocity
// gradient k_ab = d_b u_a: tau_M from the shear rate, then the steady sum
// through the relation it satisfies by Eq. (smalld),
// sigma - tau_M (kappa sigma + sigma kappa^T) = G tau_M D, solved in closed
// form (Cramer) for (sigma_xx, sigma_xy, sigma_yy). The relaxation rate
// vanishes only for tau = inf and D = 0; any finite tau_M then gives the
// right sigma = 0 (every right-hand side is zero), so tau_M = 1 is taken
// there instead of a branch.
template <typename T>
__device__ __forceinline__ void inlm_stress(T kxx, T kxy, T kyx, T kyy, const Coef<T> &q, T &sxx, T &sxy,
                                            T &syy) {
  const T Dxx = T(2) * kxx, Dxy = kxy + kyx, Dyy = T(2) * kyy;
  const T II = T(0.5) * (Dxx * Dxx + T(2) * Dxy * Dxy + Dyy * Dyy);
  const T r0 = q.inv_tau + root(II) * q.inv_gc;
  const T rate = r0 > T(0) ? r0 : T(1);
  {
    const T tM = recip<T>(rate);
    const T ka = tM * kxx, kb = tM * kxy, kc = tM * kyx, kd = tM * kyy;
    const T gt = q.G * tM;
    const T r1 = gt * Dxx, r2 = gt * Dxy, r3 = gt * Dyy;
    const T m11 = T(1) - T(2) * ka, m12 = T(-2) * kb, m21 = -kc;
    const T m22 = T(1) - ka - kd, m23 = -kb, m32 = T(-2) * kc, m33 = T(1) - T(2) * kd;
    const T c11 = m22 * m33 - m23 * m32;
    const T det = m11 * c11 - m12 * m21 * m33;
    const T idet = recip<T>(det);
    const T e2 = r2 * m33 - m23 * r3;
    sxx = (r1 * c11 - m12 * e2) * idet;
    sxy = (m11 * e2 - r1 * m21 * m33) * idet;
    syy = (m11 * (m22 * r3 - r2 * m32) - m12 * m21 * r3 + r1 * m21 * m32) * idet;
  }
}

// Everything that happens at one node once its populations and the stencil
// velocities are known: kappa (Sec. II.C), the inlM stress (Eqs.
// (nlmaxwell), (sigtsum)), the flow-induced density change (Eq. (rhoplus)),
// the density and velocity of Eq. (rhoj), and either the post-collision
// populations (equilibrium, forcing of Eq. (bodyforce), BGK) or the
// observables of the node.
// With SHIFT, f are stored relative to the row's reference (ur, 0), mx is
// the momentum beyond ur, the velocities lf, rt, dn, up carry u~_x minus
// their own row's reference, and kref = (ur_above - ur_below)/2 restores the
// reference's share of d_y u_x; the outputs are stored relative to ur.
// With VE the stress is the time-integrated one: sp holds (xx, xy, yy) of the
// previous step and sn receives those of this step.
template <typename T, bool SHIFT, bool OBS, bool VE>
__device__ __forceinline__ void node_update(const T f[9], T sd, T mx, T my, T Pc, T fx, U2<T> lf,
                                            U2<T> rt, U2<T> dn, U2<T> up, T ur, T kref, const Coef<T> &q,
                                            int nnp, const T sp[3], T sn[3], T out[9], T &trT_out,
                                            double obs[OF_COUNT]) {
  // velocity gradient kappa_ab = d_b u_a
  const T kxx = T(0.5) * (rt.x - lf.x);
  const T kxy = T(0.5) * (up.x - dn.x) + kref;
  const T kyx = T(0.5) * (rt.y - lf.y);
  const T kyy = T(0.5) * (up.y - dn.y);

  // tau_M of Eq. (nlmaxwell), then the steady series of Eq. (sigtsum) through
  // the relation it satisfies by Eq. (smalld),
  // sigma - tau_M (kappa sigma + sigma kappa^T) = G tau_M D, solved in closed
  // form (Cramer) for (sigma_xx, sigma_xy, sigma_yy).
  const T Dxx = T(2) * kxx, Dxy = kxy + kyx, Dyy = T(2) * kyy;
  T sxx = T(0), sxy = T(0), syy = T(0);
  if constexpr (VE) {
    // Time-integrated stress, Eq. (gkder) with d_t G = -G / tau_M(t): one
    // step with the upper-convected terms and the source explicit and the
    // relaxation implicit, sigma' = [sigma + kappa sigma + sigma kappa^T +
    // G D] / (1 + 1/tau_M), written as sigma plus its increment so that FP32
    // rounds only the increment.
    const T II = T(0.5) * (Dxx * Dxx + T(2) * Dxy * Dxy + Dyy * Dyy);
    const T rate = q.inv_tau + root(II) * q.inv_gc;  // 1 / tau_M
    const T d = recip<T>(T(1) + rate);
    const T cxx = T(2) * (kxx * sp[0] + kxy * sp[1]);
    const T cxy = kxx * sp[1] + kxy * sp[2] + kyx * sp[0] + kyy * sp[1];
    const T cyy = T(2) * (kyx * sp[1] + kyy * sp[2]);
    sxx = sp[0] + (cxx + q.G * Dxx - rate * sp[0]) * d;
    sxy = sp[1] + (cxy + q.G * Dxy - rate * sp[1]) * d;
    syy = sp[2] + (cyy + q.G * Dyy - rate * sp[2]) * d;
    sn[0] = sxx;
    sn[1] = sxy;
    sn[2] = syy;
  } else if (q.stress_on) {
    inlm_stress<T>(kxx, kxy, kyx, kyy, q, sxx, sxy, syy);
  }
  // non-Newtonian stress carried by the forcing (viscosity split)
  const T Txx = sxx - q.lgt * Dxx, Txy = sxy - q.lgt * Dxy, Tyy = syy - q.lgt * Dyy;
  const T trT = Txx + Tyy;
  const T Sxx = T(0.5) * (Txx - Tyy);  // traceless part; Sbar_yy = -Sxx
  // Eq. (rhoplus): r = dt d(delta rho)/dt with delta rho = -tr Sigma^nN /(cs2 d)
  const T rr = nnp ? T(-1.5) * (trT - Pc) : T(0);

  const T jx = mx + T(0.5) * fx, jy = my;
  // Eq. (rhoj): the equilibrium density is sum (n* + n)/2 = s + r/2, carried
  // as its deviation from 1 in the shifted storage
  const T sdev = SHIFT ? sd : sd - T(1);
  const T rho_dev = sdev + T(0.5) * rr;
  const T rho_e = SHIFT ? T(1) + rho_dev : sd + T(0.5) * rr;
  const T irho = recip<T>(rho_e);
  // SHIFT: jx is j_x - ur, so u_x - ur = (jx - ur rho_dev) / rho_e
  const T dux = (SHIFT ? jx - ur * rho_dev : jx) * irho;
  const T ux = SHIFT ? ur + dux : dux, uy = jy * irho;
  trT_out = trT;

  if constexpr (OBS) {
    // SHIFT: u_x - ur and j_x - ur; the reduction adds ur once per row, so
    // that row sums of equal values stay exact in any summation order
    obs[OF_UX] = SHIFT ? (double)dux : (double)ux;
    obs[OF_UY] = (double)uy;
    obs[OF_SXX] = (double)sxx;
    obs[OF_SXY] = (double)sxy;
    obs[OF_SYY] = (double)syy;
    obs[OF_RHOE_DEV] = (double)rho_dev;
    obs[OF_MASS_DEV] = (double)sdev + (nnp ? 1.5 * (double)Pc : 0.0);
    obs[OF_MOMX] = (double)mx;
    obs[OF_KXY] = (double)kxy;
    obs[OF_TRT] = (double)trT;
    obs[OF_KXX] = (double)kxx;
  } else {
    // equilibrium, forcing of Eq. (bodyforce) and BGK collision:
    // n*_i = (1 - om) n_i + om n^eq_i + F_i. For a pair of opposite
    // velocities c_i = -c_j the parts even in c (constant, (c.u)^2, (c.u)(c.f),
    // the stress term) are shared and the odd parts ((c.u), (c.f)) change sign.
    const T usq = ux * ux + uy * uy;
    const T uf = ux * fx;
    const T K0 = q.kf * (rr + T(1.5) * rr * usq - T(3) * uf);
    const T om1 = T(1) - q.om;
    // Equilibrium excess n^eq_i - a_i (- E_i(ur) with SHIFT). SHIFT expands it
    // around the reference so that only small differences are rounded:
    // a_i [rho_dev (1 + 3 cu + 4.5 cu^2 - 1.5 u^2) + 3 c.du + 4.5 (c.du)(c.(u+ur))
    //      - 1.5 du.(u + ur)], du = u - (ur, 0); with ur = 0 it is the plain
    // shifted form.
    T C0, Acu2, Bcu;
    if constexpr (SHIFT) {
      const T mix = dux * (ux + ur) + uy * uy;  // du.(u + ur)
      C0 = q.om * (rho_dev * (T(1) - T(1.5) * usq) - T(1.5) * mix) + K0;
      Acu2 = T(4.5) * (q.om * rho_dev - q.kf * rr);
      Bcu = T(3) * q.om * rho_dev;
    } else {
      C0 = q.om * rho_e * (T(1) - T(1.5) * usq) + K0;  // constant part
      Acu2 = T(4.5) * (q.om * rho_e - q.kf * rr);      // coefficient of (c.u)^2
      Bcu = T(3) * q.om * rho_e;                       // coefficient of (c.u), odd
    }
    const T E4 = SHIFT ? T(4.5) * q.om : T(0);  // (c.du)(c.(u+ur)), even
    const T B3 = SHIFT ? T(3) * q.om : T(0);    // c.du, odd
    const T Ccf = T(3) * q.kf * fx;             // 3 kf (c.f) for c_x = 1, odd
    const T Dcf = T(9) * q.kf * fx;             // 9 kf (c.u)(c.f) for c_x = 1, even
    const T spS = q.sp * Sxx, spT = T(2) * q.sp * Txy;
    const T usx = ux + ur;                      // (u + ur)_x (ur = 0 without SHIFT)
    constexpr T w0 = weight<T>(0), w1 = weight<T>(1), w5 = weight<T>(5);
    out[0] = om1 * f[0] + w0 * C0;
    {  // (1,0) and (-1,0): c.u = ux, c.f = fx, stress term Sxx
      const T cu = ux, cdu = dux, cs = usx;
      const T ev = w1 * (C0 + Acu2 * cu * cu + E4 * cdu * cs + spS + Dcf * cu);
      const T od = w1 * (Bcu * cu + B3 * cdu + Ccf);
      out[1] = om1 * f[1] + ev + od;
      out[3] = om1 * f[3] + ev - od;
    }
    {  // (0,1) and (0,-1): c.u = uy, c.f = 0, stress term -Sxx
      const T cu = uy;
      const T ev = w1 * (C0 + Acu2 * cu * cu + E4 * cu * cu - spS);
      const T od = w1 * (Bcu * cu + B3 * cu);
      out[2] = om1 * f[2] + ev + od;
      out[4] = om1 * f[4] + ev - od;
    }
    {  // (1,1) and (-1,-1): c.u = ux + uy, c.f = fx, stress term 2 Sxy
      const T cu = ux + uy, cdu = dux + uy, cs = usx + uy;
      const T ev = w5 * (C0 + Acu2 * cu * cu + E4 * cdu * cs + spT + Dcf * cu);
      const T od = w5 * (Bcu * cu + B3 * cdu + Ccf);
      out[5] = om1 * f[5] + ev + od;
      out[7] = om1 * f[7] + ev - od;
    }
    {  // (-1,1) and (1,-1): c.u = uy - ux, c.f = -fx, stress term -2 Sxy
      const T cu = uy - ux, cdu = uy - dux, cs = uy - usx;
      const T ev = w5 * (C0 + Acu2 * cu * cu + E4 * cdu * cs - spT - Dcf * cu);
      const T od = w5 * (Bcu * cu + B3 * cdu - Ccf);
      out[6] = om1 * f[6] + ev + od;
      out[8] = om1 * f[8] + ev - od;
    }
  }
}

// Momentum handed to the walls in the previous step: the reflected
// populations sit in the wall rows with the opposite velocity.
// With the FP32 reference ur the pulled values are n_i - a_i - E_i(ur), and
// n6 - n5 = f6 - f5 - ur/6, n7 - n8 = f7 - f8 - ur/6; the -ur/3 of each wall
// node is added per row in the reduction.
// At a Zou-He top wall the top row's share is ztop (zh_drag).
template <typename T>
__device__ __forceinline__ double wall_drag(const T f[9], int y, int ny, T uw6, bool zh, double ztop) {
  double d = 0.0;
  if (y == 0) d += 2.0 * ((double)f[6] - (double)f[5]);
  // a moving top wall also received the momentum its reflection added
  if (y == ny - 1) d += zh ? ztop : 2.0 * ((double)f[7] - (double)f[8]) + 2.0 * (double)uw6;
  return d;
}

// Workgroup w of n runs on XCD w % 8; the work item it takes, such that
// each XCD takes a contiguous range of the n items (neighbouring items then
// share their halo rows through that XCD's L2).
__device__ __forceinline__ int xcd_item(int w, int n) {
  const int q = n >> 3, rem = n & 7, j = w & 7;
  return j * q + (j < rem ? j : rem) + (w >> 3);
}

__device__ __forceinline__ int strip_index(const SweepArgs &a) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  return xcd_item(blockIdx.x, a.n_wg) * LB_WG_WAVES + wave;
}

template <typename T, bool SHIFT, int TXW, bool WIDE, bool OBS, bool VE>
__global__ void __launch_bounds__(64 * LB_WG_WAVES) sweep_kernel(SweepArgs a) {
  constexpr int TYW = 64 / TXW;
  const int lane = threadIdx.x & 63;
  const int sidx = strip_index(a);
  if (sidx >= a.n_strips) return;
  const Strip st = a.strips[sidx];
  const ChanDev c = a.ch[st.ch];
  const T *__restrict__ A = static_cast<const T *>(a.A);
  T *__restrict__ B = static_cast<T *>(a.B);
  const int nx = c.nx, ny = c.ny;
  const long long t = c.t + a.k;
  const T fx = (t < c.t_startup) ? T(c.g) : T(0);
  // moving top wall: its velocity at step t (stencil ghost) and u_w/6 of step
  // t - 1, whose reflected links step t pulls
  const T uwg = (t < c.t_startup) ? T(c.uw) : T(0);
  const T uw6 = (!c.zh && t >= 1 && t - 1 < c.t_startup) ? T(c.uw / 6.0) : T(0);
  const Coef<T> q(c);

  int lx, ly, x, hx = 0;
  bool colok;
  if (WIDE) {
    // 64 columns from x0; lanes past the end of the channel wrap onto valid
    // columns and only supply neighbours
    lx = lane;
    ly = 0;
    const int xr = st.x0 + lane;
    x = xr % nx;
    colok = xr < nx;
    // x halo: even lanes pull the column left of the strip, odd lanes the
    // column right of it
    hx = (lane & 1) ? (st.x0 + 64) % nx : (st.x0 - 1 + nx) % nx;
  } else {
    lx = lane & (TXW - 1);
    ly = lane / TXW;
    x = lx;
    colok = true;
  }
  const int left_src = WIDE ? (lane == 0 ? 0 : lane - 1) : ly * TXW + ((lx + TXW - 1) & (TXW - 1));
  const int right_src = WIDE ? (lane == 63 ? 63 : lane + 1) : ly * TXW + ((lx + 1) & (TXW - 1));
  const long long base = c.off;

  auto clampy = [&](int y) { return y < 0 ? 0 : (y >= ny ? ny - 1 : y); };
  // FP32 reference velocity of row y (0 in FP64)
  auto ref = [&](int y) -> T {
    if constexpr (SHIFT) return a.uref[c.row_off + clampy(y)];
    return T(0);
  };
  // a row's loads (the pulled populations and P), then the populations
  // relative to that row's reference ur: split so that the loads of several
  // rows can be in flight before any is used
  struct RowLoad {
    T f[9], P;
  };
  auto load_row = [&](int y, RowLoad &L) {
    const int yc = clampy(y);
    const long long row = base + (long long)yc * nx;
    pull<T>(A, row, nx, ny, x, yc, uw6, L.f);
    L.P = A[slot(9, row + x)];
  };
  auto finish_row = [&](int y, const RowLoad &L, T f[9], T &Pv, T &ur) {
    const int yc = clampy(y);
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = L.f[i];
    Pv = L.P;
    ur = ref(yc);
    if constexpr (SHIFT) to_row_reference(f, ref(yc - 1), ur, ref(yc + 1), yc == 0, yc == ny - 1);
    if (c.zh && yc == ny - 1) zou_he_top<T, SHIFT>(f, uwg, ur, fx);
  };
  auto halo_u = [&](int y) -> U2<T> {
    const int yc = clampy(y);
    T f[9], sd, mx, my;
    pull<T>(A, base + (long long)yc * nx, nx, ny, hx, yc, uw6, f);
    const T ur = ref(yc);
    if constexpr (SHIFT) to_row_reference(f, ref(yc - 1), ur, ref(yc + 1), yc == 0, yc == ny - 1);
    if (c.zh && yc == ny - 1) zou_he_top<T, SHIFT>(f, uwg, ur, fx);
    moments<T>(f, sd, mx, my);
    return u_tilde<T, SHIFT>(sd, mx, my, fx, ur);
  };
  // viscoelastic model: the stress of the previous step at (x, y)
  const T *__restrict__ SA = static_cast<const T *>(a.SA);
  T *__restrict__ SB = static_cast<T *>(a.SB);
  auto load_sigma = [&](int y, T sg[3]) {
    if constexpr (VE) {
      const long long o = base + (long long)clampy(y) * nx + x;
#pragma unroll
      for (int p = 0; p < 3; ++p) sg[p] = SA[sslot(p, o)];
    } else {
      sg[0] = sg[1] = sg[2] = T(0);
    }
  };

  T fc[9], fn[9], Pc, Pn, urc, urn, sgc[3], sgn[3];
  U2<T> uPrev, uCur, uNext, uhCur = {T(0), T(0)}, uhNext = {T(0), T(0)};
  // the loads of the row groups below the strip, at its start and after it
  // (the first one the loop takes) go out together
  RowLoad Lp, Lc, Ln;
  load_row(st.y0 - TYW + ly, Lp);
  load_row(st.y0 + ly, Lc);
  load_row(st.y0 + TYW + ly, Ln);
  {
    T ftmp[9], Ptmp, sd, mx, my, urp;
    finish_row(st.y0 - TYW + ly, Lp, ftmp, Ptmp, urp);
    moments<T>(ftmp, sd, mx, my);
    uPrev = u_tilde<T, SHIFT>(sd, mx, my, fx, urp);
  }
  T sdc, mxc, myc;
  finish_row(st.y0 + ly, Lc, fc, Pc, urc);
  load_sigma(st.y0 + ly, sgc);
  moments<T>(fc, sdc, mxc, myc);
  uCur = u_tilde<T, SHIFT>(sdc, mxc, myc, fx, urc);
  if (WIDE) uhCur = halo_u(st.y0);

#pragma unroll 1
  for (int yb = st.y0; yb < st.y1; yb += TYW) {
    T sdn, mxn, myn;
    if (yb != st.y0) load_row(yb + TYW + ly, Ln);
    finish_row(yb + TYW + ly, Ln, fn, Pn, urn);
    load_sigma(yb + TYW + ly, sgn);
    if (WIDE) uhNext = halo_u(yb + TYW);
    moments<T>(fn, sdn, mxn, myn);
    uNext = u_tilde<T, SHIFT>(sdn, mxn, myn, fx, urn);
    const int y = yb + ly;

    U2<T> dn, up;
    if (TYW == 1) {
      dn = uPrev;
      up = uNext;
    } else {
      const U2<T> dc = shfl2(uCur, lane - TXW < 0 ? 0 : lane - TXW);
      const U2<T> dp = shfl2(uPrev, lane + (TYW - 1) * TXW > 63 ? 63 : lane + (TYW - 1) * TXW);
      const U2<T> uc = shfl2(uCur, lane + TXW > 63 ? 63 : lane + TXW);
      const U2<T> un = shfl2(uNext, lane - (TYW - 1) * TXW < 0 ? 0 : lane - (TYW - 1) * TXW);
      dn = (ly > 0) ? dc : dp;
      up = (ly < TYW - 1) ? uc : un;
    }
    U2<T> lf = shfl2(uCur, left_src);
    U2<T> rt = shfl2(uCur, right_src);
    if (WIDE) {
      const U2<T> hl = shfl2(uhCur, 0), hr = shfl2(uhCur, 1);
      if (lane == 0) lf = hl;
      if (lane == 63) rt = hr;
    }
    // no-slip ghosts behind the half-way walls, u~(-1) = -u~(0) and
    // u~(ny) = 2 u_w - u~(ny-1), or behind a Zou-He node wall
    // u~(ny) = 2 u_w - u~(ny-2); with SHIFT the ghost rows take the mirrored
    // references -ur and 2 u_w - ur, so their deltas are just mirrored
    if (y == 0) dn = U2<T>{-uCur.x, -uCur.y};
    if (y == ny - 1) {
      const U2<T> m = c.zh ? dn : uCur;
      up = U2<T>{(SHIFT ? T(0) : T(2) * uwg) - m.x, -m.y};
    }
    T kref = T(0);
    if constexpr (SHIFT) {
      const T urd = (y == 0) ? -urc : ref(y - 1);
      const T uru = (y >= ny - 1) ? T(2) * uwg - (c.zh ? urd : urc) : ref(y + 1);
      kref = T(0.5) * (uru - urd);
    }

    // Every lane computes; only valid lanes store. Lanes past the strip or
    // outside the channel read clamped rows and their results are dropped.
    const bool ok = (y < st.y1) && colok;
    T out[9], trT, sg[3];
    double obs[OF_COUNT];
    node_update<T, SHIFT, OBS, VE>(fc, sdc, mxc, myc, Pc, fx, lf, rt, dn, up, urc, kref, q, c.nnp, sgc, sg, out,
                                   trT, obs);
    if constexpr (OBS) {
      double ztop = 0.0;
      if (c.zh && y == ny - 1) {
        const long long o = base + (long long)y * nx + x;
        ztop = zh_drag<T>(A[slot(5, o)], A[slot(6, o)], fc);
      }
      obs[OF_DRAG] = wall_drag<T>(fc, y, ny, uw6, c.zh, ztop);
      constexpr int GW = WIDE ? 64 : TXW;
#pragma unroll
      for (int f = 0; f < OF_COUNT; ++f) obs[f] = group_sum<GW>(ok ? obs[f] : 0.0);
      const bool writer = WIDE ? (lane == 0) : (lx == 0);
      if (writer && y < st.y1) {
        const long long pr = (long long)c.poff + (long long)y * c.nxs + (WIDE ? st.x0 / 64 : 0);
        double *dst = a.part + pr * OF_COUNT;
#pragma unroll
        for (int f = 0; f < OF_COUNT; ++f) dst[f] = obs[f];
      }
    } else {
      if (ok) {
        const long long o = base + (long long)y * nx + x;
#pragma unroll
        for (int i = 0; i < 9; ++i) B[slot(i, o)] = out[i];
        B[slot(9, o)] = trT;
        if constexpr (VE) {
#pragma unroll
          for (int p = 0; p < 3; ++p) SB[sslot(p, o)] = sg[p];
        }
      }
    }

    uPrev = uCur;
    uCur = uNext;
    uhCur = uhNext;
    urc = urn;
#pragma unroll
    for (int p = 0; p < 3; ++p) sgc[p] = sgn[p];
#pragma unroll
    for (int i = 0; i < 9; ++i) fc[i] = fn[i];
    Pc = Pn;
    sdc = sdn;
    mxc = mxn;
    myc = myn;
  }
}

// Two steps per launch for the narrow widths (nx = 1, 2, ..., 64: a row
// fits TXW = nx lanes and a wavefront holds TYW = 64 / nx rows), for the
// instantaneous model. A workgroup of two wavefronts takes the strip of rows
// [y0, y1) of one channel through steps t and t+1 with the narrow sweep's
// row machine in both:
//  * wavefront 0 (stage A, step t) marches groups of TYW rows from
//    max(y0 - 2, 0) to min(y1 + 2, ny), reading the state, and writes each
//    group's post-collision populations and trace into a ring of groups in
//    LDS;
//  * wavefront 1 (stage B, step t+1) marches the groups of [y0, y1), pulling
//    from the ring (any row of the last few groups, by index), and stores.
// A row of the channel is whole in one group, so no column beyond it is
// needed. Stage B runs L iterations behind stage A (L = 3, or 4 and 5 when
// a group holds 2 and 1 rows), or sooner at the end of the strip, so that
// every group it reads is in the ring; one barrier per iteration orders the
// ring's writes and reads. Per node the arithmetic is the narrow sweep's.
constexpr int kN2Ring = 8;  // groups in the ring
template <typename T, bool SHIFT, int TXW>
__global__ void __launch_bounds__(128) sweep_narrow2_kernel(SweepArgs a) {
  constexpr int TYW = 64 / TXW;
  constexpr int L = 3 + 2 / TYW;  // stage B's lag in iterations
  static_assert(L <= kN2Ring, "the ring must hold the groups stage B reads");
  __shared__ T ring[kN2Ring][kPlanes][64];
  const int lane = threadIdx.x & 63;
  const bool isA = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) == 0;
  const int sidx = xcd_item(blockIdx.x, a.n_wg);
  if (sidx >= a.n_strips) return;  // the whole workgroup, before any barrier
  const Strip st = a.strips[sidx];
  const ChanDev c = a.ch[st.ch];
  const T *__restrict__ A = static_cast<const T *>(a.A);
  T *__restrict__ B = static_cast<T *>(a.B);
  const int nx = c.nx, ny = c.ny;
  const long long t = c.t + a.k, ts = isA ? t : t + 1;  // this stage's step
  const T fx = (ts < c.t_startup) ? T(c.g) : T(0);
  const T uwg = (ts < c.t_startup) ? T(c.uw) : T(0);
  const T uw6 = (!c.zh && ts >= 1 && ts - 1 < c.t_startup) ? T(c.uw / 6.0) : T(0);
  const Coef<T> q(c);
  const int lx = lane & (TXW - 1), ly = lane / TXW, x = lx;
  const int left_src = ly * TXW + ((lx + TXW - 1) & (TXW - 1));
  const int right_src = ly * TXW + ((lx + 1) & (TXW - 1));
  const long long base = c.off;
  auto clampy = [&](int y) { return y < 0 ? 0 : (y >= ny ? ny - 1 : y); };
  auto ref = [&](int y) -> T {
    if constexpr (SHIFT) return a.uref[c.row_off + clampy(y)];
    return T(0);
  };
  // the groups of the two stages
  const int yA0 = st.y0 - 2 < 0 ? 0 : st.y0 - 2, yA1 = st.y1 + 2 > ny ? ny : st.y1 + 2;
  const int nA = (yA1 - yA0 + TYW - 1) / TYW, nB = (st.y1 - st.y0 + TYW - 1) / TYW;
  const int ys = isA ? yA0 : st.y0;  // this stage's first group

  // stage A's source: the state (the narrow sweep's pull)
  auto pull_mem = [&](int y, T f[9], T &Pv) {
    const int yc = clampy(y);
    const long long row = base + (long long)yc * nx;
    pull<T>(A, row, nx, ny, x, yc, uw6, f);
    Pv = A[slot(9, row + x)];
  };
  // stage B's source: row r, column col of step t from the ring (rows
  // outside stage A's range read a row inside it; their values are unused)
  auto at = [&](int r, int p, int col) -> T {
    const int rr = (r < yA0 ? yA0 : (r >= yA1 ? yA1 - 1 : r)) - yA0;
    const int g = rr / TYW;
    return ring[g & (kN2Ring - 1)][p][(rr - g * TYW) * TXW + col];
  };
  auto pull_ring = [&](int y, T f[9], T &Pv) {
    const int yc = clampy(y);
    const bool bot = (yc == 0), top = (yc == ny - 1);
    const int xm = (x == 0) ? nx - 1 : x - 1, xp = (x == nx - 1) ? 0 : x + 1;
    f[0] = at(yc, 0, x);
    f[1] = at(yc, 1, xm);
    f[3] = at(yc, 3, xp);
    f[2] = bot ? at(yc, 4, x) : at(yc - 1, 2, x);
    f[5] = bot ? at(yc, 7, x) : at(yc - 1, 5, xm);
    f[6] = bot ? at(yc, 8, x) : at(yc - 1, 6, xp);
    f[4] = top ? at(yc, 2, x) : at(yc + 1, 4, x);
    f[7] = top ? at(yc, 5, x) - uw6 : at(yc + 1, 7, xp);
    f[8] = top ? at(yc, 6, x) + uw6 : at(yc + 1, 8, xm);
    Pv = at(yc, 9, x);
  };
  // a row's pulled populations and P (split from the rest so that stage A
  // can have the loads of several groups in flight), then the populations
  // relative to the row's reference, moments and u~
  struct RowLoad {
    T f[9], P;
  };
  auto fetch = [&](int y, RowLoad &L) {
    if (isA) pull_mem(y, L.f, L.P);
    else pull_ring(y, L.f, L.P);
  };
  auto finish = [&](int y, const RowLoad &L, T f[9], T &Pv, T &ur, T &sd, T &mx, T &my, U2<T> &u) {
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = L.f[i];
    Pv = L.P;
    const int yc = clampy(y);
    ur = ref(yc);
    if constexpr (SHIFT) to_row_reference(f, ref(yc - 1), ur, ref(yc + 1), yc == 0, yc == ny - 1);
    if (c.zh && yc == ny - 1) zou_he_top<T, SHIFT>(f, uwg, ur, fx);
    moments<T>(f, sd, mx, my);
    u = u_tilde<T, SHIFT>(sd, mx, my, fx, ur);
  };

  T fc[9], Pc, urc, sdc, mxc, myc;
  U2<T> uPrev, uCur;
  RowLoad Ln;
  // the group below this stage's first and the first; stage A also fetches
  // the second (stage B cannot yet: stage A has not written all its rows)
  auto start = [&]() {
    RowLoad Lp, Lc;
    fetch(ys - TYW + ly, Lp);
    fetch(ys + ly, Lc);
    if (isA) fetch(ys + TYW + ly, Ln);
    T ftmp[9], Ptmp, urp, sd, mx, my;
    finish(ys - TYW + ly, Lp, ftmp, Ptmp, urp, sd, mx, my, uPrev);
    finish(ys + ly, Lc, fc, Pc, urc, sdc, mxc, myc, uCur);
  };
  // group g of this stage: fetch and finish the next group, update this one
  auto group = [&](int g) {
    const int yb = ys + g * TYW;
    T fn[9], Pn, urn, sdn, mxn, myn;
    U2<T> uNext;
    if (g != 0 || !isA) fetch(yb + TYW + ly, Ln);
    finish(yb + TYW + ly, Ln, fn, Pn, urn, sdn, mxn, myn, uNext);
    const int y = yb + ly;
    U2<T> dn, up;
    if (TYW == 1) {
      dn = uPrev;
      up = uNext;
    } else {
      const U2<T> dc = shfl2(uCur, lane - TXW < 0 ? 0 : lane - TXW);
      const U2<T> dp = shfl2(uPrev, lane + (TYW - 1) * TXW > 63 ? 63 : lane + (TYW - 1) * TXW);
      const U2<T> uc = shfl2(uCur, lane + TXW > 63 ? 63 : lane + TXW);
      const U2<T> un = shfl2(uNext, lane - (TYW - 1) * TXW < 0 ? 0 : lane - (TYW - 1) * TXW);
      dn = (ly > 0) ? dc : dp;
      up = (ly < TYW - 1) ? uc : un;
    }
    const U2<T> lf = shfl2(uCur, left_src), rt = shfl2(uCur, right_src);
    if (y == 0) dn = U2<T>{-uCur.x, -uCur.y};
    if (y == ny - 1) {
      const U2<T> m = c.zh ? dn : uCur;
      up = U2<T>{(SHIFT ? T(0) : T(2) * uwg) - m.x, -m.y};
    }
    T kref = T(0);
    if constexpr (SHIFT) {
      const T urd = (y == 0) ? -urc : ref(y - 1);
      const T uru = (y >= ny - 1) ? T(2) * uwg - (c.zh ? urd : urc) : ref(y + 1);
      kref = T(0.5) * (uru - urd);
    }
    T out[9], trT, sg[3];
    const T sp[3] = {T(0), T(0), T(0)};
    double obs[OF_COUNT];
    node_update<T, SHIFT, false, false>(fc, sdc, mxc, myc, Pc, fx, lf, rt, dn, up, urc, kref, q, c.nnp, sp, sg, out,
                                        trT, obs);
    if (isA) {
      // the whole group goes into the ring (rows past stage A's range are
      // never read)
      T *slotp = &ring[g & (kN2Ring - 1)][0][0];
#pragma unroll
      for (int i = 0; i < 9; ++i) slotp[i * 64 + lane] = out[i];
      slotp[9 * 64 + lane] = trT;
    } else if (y < st.y1 && y < ny) {
      const long long o = base + (long long)y * nx + x;
#pragma unroll
      for (int i = 0; i < 9; ++i) B[slot(i, o)] = out[i];
      B[slot(9, o)] = trT;
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) fc[i] = fn[i];
    Pc = Pn;
    urc = urn;
    sdc = sdn;
    mxc = mxn;
    myc = myn;
    uPrev = uCur;
    uCur = uNext;
  };

  // Iteration j: stage A runs group j (after starting at j = 0). Stage B
  // runs group b once stage A has written every group it reads, the groups
  // up to b + L - 1 or stage A's last, nA - 1: at iteration
  // jB(b) = max(min(b + L, nA), jB(0) + b), having started (groups -1 and
  // 0) at min(L - 1, nA). One barrier per iteration.
  const int jS = (L - 1 < nA) ? L - 1 : nA, jB0 = (L < nA) ? L : nA;
  auto jB = [&](int b) {
    const int r = (b + L < nA) ? b + L : nA;
    return (r > jB0 + b) ? r : jB0 + b;
  };
  const int niter = (nA > jB(nB - 1) + 1) ? nA : jB(nB - 1) + 1;
  if (isA) start();
  int bnext = 0;
#pragma unroll 1
  for (int j = 0; j < niter; ++j) {
    if (isA) {
      if (j < nA) group(j);
    } else {
      if (j == jS) start();
      if (bnext < nB && j == jB(bnext)) group(bnext++);
    }
    __syncthreads();
  }
}

// FP64 step of the instantaneous or time-integrated model over tiles of
// kMainTileX x kMainTileY nodes, one workgroup per tile and one thread per
// node. Each thread pulls its node and keeps the populations; u~ of the tile
// and of the ring of one node around it go to LDS, and after one barrier each
// thread has its four stencil velocities (no-slip ghosts behind the walls, as
// in the strip sweeps) and runs the node update. Each XCD takes a contiguous
// run of the tile list, which the host orders as blocks of neighbouring tiles
// (they share the halo populations they pull through that XCD's L2).
constexpr int kMainUX = kMainTileX + 2, kMainUY = kMainTileY + 2;
constexpr int kMainRing = 2 * kMainUX + 2 * kMainTileY;
static_assert(kMainTileX * kMainTileY == kMainThreads, "one node per thread");
static_assert(kMainRing <= kMainThreads, "at most one ring node per thread");

template <bool VE, bool NT>
__global__ void __launch_bounds__(kMainThreads) sweep_tile_kernel(SweepArgs a) {
  __shared__ double su[2][kMainUY][kMainUX];
  const Strip tl = a.strips[xcd_item(blockIdx.x, gridDim.x)];
  const ChanDev c = a.ch[tl.ch];
  if (!c.active) return;  // frozen channel (uniform over the workgroup)
  const int nx = c.nx, ny = c.ny;
  const long long t = c.t + a.k;
  const double fx = (t < c.t_startup) ? c.g : 0.0;
  const double uwg = (t < c.t_startup) ? c.uw : 0.0;
  const double uw6 = (!c.zh && t >= 1 && t - 1 < c.t_startup) ? c.uw / 6.0 : 0.0;
  const Coef<double> q(c);
  const double *__restrict__ Ac = static_cast<const double *>(a.A) + c.off * kPlanes;
  double *__restrict__ Bc = static_cast<double *>(a.B) + c.off * kPlanes;
  const bool wide = nx >= kMainTileX + 2;  // then halo columns wrap at most once
  auto wrapx = [&](int x) {
    if (wide) return x < 0 ? x + nx : (x >= nx ? x - nx : x);
    const int r = x % nx;
    return r < 0 ? r + nx : r;
  };
  auto clampy = [&](int y) { return y < 0 ? 0 : (y >= ny ? ny - 1 : y); };
  // this thread's node and (threads below kMainRing) one node of the ring:
  // the row below, the row above, one column on either side; both pulled
  // before either is used (rows outside the channel pull a row inside and
  // store nothing)
  const int jo = threadIdx.x / kMainTileX, io = threadIdx.x - jo * kMainTileX;
  const int yo = tl.y0 + jo, xo = tl.x0 + io;
  const int h = threadIdx.x;
  int hj, hi;
  if (h < kMainUX) {
    hj = 0;
    hi = h;
  } else if (h < 2 * kMainUX) {
    hj = kMainTileY + 1;
    hi = h - kMainUX;
  } else {
    const int r = h - 2 * kMainUX;
    hj = 1 + (r >> 1);
    hi = (r & 1) ? kMainUX - 1 : 0;
  }
  const int hy = tl.y0 - 1 + hj;
  const bool ring = h < kMainRing;
  const unsigned m = (unsigned)clampy(yo) * nx + wrapx(xo);
  double f[9], fh[9], sgc[3] = {0.0, 0.0, 0.0};
  pull_local(Ac, nx, ny, wrapx(xo), clampy(yo), uw6, f);
  if (c.zh && clampy(yo) == ny - 1) zou_he_top<double, false>(f, uwg, 0.0, fx);
  const double Pc = Ac[lslot(9, m)];
  if constexpr (VE) {
    const double *__restrict__ SAc = static_cast<const double *>(a.SA) + c.off * kStressPlanes;
#pragma unroll
    for (int p = 0; p < 3; ++p) sgc[p] = SAc[((m >> 6) * kStressPlanes + p) * kTile + (m & (kTile - 1))];
  }
  if (ring) pull_local(Ac, nx, ny, wrapx(tl.x0 - 1 + hi), clampy(hy), uw6, fh);
  if (ring && c.zh && clampy(hy) == ny - 1) zou_he_top<double, false>(fh, uwg, 0.0, fx);
  double sd, mx, my;
  moments<double>(f, sd, mx, my);
  const U2<double> uc = u_tilde<double, false>(sd, mx, my, fx, 0.0);
  if (yo < ny) {
    su[0][jo + 1][io + 1] = uc.x;
    su[1][jo + 1][io + 1] = uc.y;
  }
  if (ring && hy >= 0 && hy < ny) {
    double hs, hx, hv;
    moments<double>(fh, hs, hx, hv);
    const U2<double> u = u_tilde<double, false>(hs, hx, hv, fx, 0.0);
    su[0][hj][hi] = u.x;
    su[1][hj][hi] = u.y;
  }
  __syncthreads();
  if (yo >= tl.y1 || xo >= nx) return;
  const int js = jo + 1, is = io + 1;
  const U2<double> lf{su[0][js][is - 1], su[1][js][is - 1]};
  const U2<double> rt{su[0][js][is + 1], su[1][js][is + 1]};
  U2<double> dn{su[0][js - 1][is], su[1][js - 1][is]};
  U2<double> up{su[0][js + 1][is], su[1][js + 1][is]};
  if (yo == 0) dn = U2<double>{-uc.x, -uc.y};
  if (yo == ny - 1) up = c.zh ? U2<double>{2.0 * uwg - dn.x, -dn.y} : U2<double>{2.0 * uwg - uc.x, -uc.y};
  double out[9], trT, sg[3], obs[OF_COUNT];
  node_update<double, false, false, VE>(f, sd, mx, my, Pc, fx, lf, rt, dn, up, 0.0, 0.0, q, c.nnp, sgc, sg, out,
                                        trT, obs);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    if constexpr (NT) __builtin_nontemporal_store(out[i], &Bc[lslot(i, m)]);
    else Bc[lslot(i, m)] = out[i];
  }
  if constexpr (NT) __builtin_nontemporal_store(trT, &Bc[lslot(9, m)]);
  else Bc[lslot(9, m)] = trT;
  if constexpr (VE) {
    double *__restrict__ SBc = static_cast<double *>(a.SB) + c.off * kStressPlanes;
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      double *d = &SBc[((m >> 6) * kStressPlanes + p) * kTile + (m & (kTile - 1))];
      if constexpr (NT) __builtin_nontemporal_store(sg[p], d);
      else *d = sg[p];
    }
  }
}

// Aligned 64-column strips of a channel whose width is a multiple of 64
// (and at least 128). Row y of the strip is tile (off + y nx + x0)/64; lane
// l owns column x0 + l.
template <typename T, bool SHIFT, bool OBS, bool VE>
__global__ void __launch_bounds__(64 * LB_WG_WAVES) sweep_wide64_kernel(SweepArgs a) {
  const int lane = threadIdx.x & 63;
  const int sidx = strip_index(a);
  if (sidx >= a.n_strips) return;
  const Strip st = a.strips[sidx];
  const ChanDev c = a.ch[st.ch];
  const T *__restrict__ A = static_cast<const T *>(a.A);
  T *__restrict__ B = static_cast<T *>(a.B);
  const int nx = c.nx, ny = c.ny;
  const long long t = c.t + a.k;
  const T fx = (t < c.t_startup) ? T(c.g) : T(0);
  // moving top wall: its velocity at step t (stencil ghost) and u_w/6 of step
  // t - 1, whose reflected links step t pulls
  const T uwg = (t < c.t_startup) ? T(c.uw) : T(0);
  const T uw6 = (!c.zh && t >= 1 && t - 1 < c.t_startup) ? T(c.uw / 6.0) : T(0);
  const Coef<T> q(c);

  const int tiles_row = nx >> 6;                 // tiles per row
  const long long tile0 = (c.off + st.x0) >> 6;  // tile of row 0 of this strip
  const int xt = st.x0 >> 6;                     // tile column of the strip
  // tile offsets (in tiles) of the left and right neighbour columns' tiles
  const int dl = (xt == 0) ? tiles_row - 1 : -1;
  const int dr = (xt == tiles_row - 1) ? -(tiles_row - 1) : 1;
  constexpr int F = kTile;  // stride between fields inside a tile

  // Wave-uniform addressing: tile index of row y in this strip's column and
  // in the columns left/right of it; ld() reads one field of one column of a
  // tile (every lane the same address).
  auto tile = [&](int y) -> long long { return tile0 + (long long)y * tiles_row; };
  // wave-uniform loads go through the scalar unit: A is not written during
  // the sweep, so it can be read as constant memory
  typedef const __attribute__((address_space(4))) T *cptr;
  const cptr Ac = (cptr)(A);
  auto ld = [&](long long tl, int col, int p) -> T { return Ac[(tl * kPlanes + p) * F + col]; };
  auto run = [&](long long tl, int p) -> T { return A[(tl * kPlanes + p) * F + lane]; };
  // FP32 reference velocity of row y (0 in FP64), rows clamped to the channel
  auto ref = [&](int y) -> T {
    if constexpr (SHIFT) return a.uref[c.row_off + (y < 0 ? 0 : (y >= ny ? ny - 1 : y))];
    return T(0);
  };

  // Pull of row y (0 <= y < ny) for every lane from aligned runs of the
  // strip's own tiles; the x-shifted directions are lane shifts whose edge
  // lanes take the neighbouring column's value.
  auto pull_row = [&](int y, T f[9], T &Pv) {
    const bool bot = (y == 0), top = (y == ny - 1);
    const long long t0 = tile(y), td = bot ? t0 : tile(y - 1), tu = top ? t0 : tile(y + 1);
    f[0] = run(t0, 0);
    f[1] = shift_up(ld(t0 + dl, 63, 1), run(t0, 1));
    f[3] = shift_down(ld(t0 + dr, 0, 3), run(t0, 3));
    Pv = run(t0, 9);
    if (bot) {
      f[2] = run(t0, 4);
      f[5] = run(t0, 7);
      f[6] = run(t0, 8);
    } else {
      f[2] = run(td, 2);
      f[5] = shift_up(ld(td + dl, 63, 5), run(td, 5));
      f[6] = shift_down(ld(td + dr, 0, 6), run(td, 6));
    }
    if (top) {
      f[4] = run(t0, 2);
      f[7] = run(t0, 5) - uw6;
      f[8] = run(t0, 6) + uw6;
    } else {
      f[4] = run(tu, 4);
      f[7] = shift_down(ld(tu + dr, 0, 7), run(tu, 7));
      f[8] = shift_up(ld(tu + dl, 63, 8), run(tu, 8));
    }
    if constexpr (SHIFT) to_row_reference(f, ref(y - 1), ref(y), ref(y + 1), bot, top);
    if (c.zh && top) zou_he_top<T, SHIFT>(f, uwg, ref(y), fx);
  };
  // u~ of the column left of the strip (column 63 of the left tile) and of
  // the column right of it (column 0 of the right tile), from wave-uniform
  // pulls.
  auto halo_u = [&](int y, U2<T> &uL, U2<T> &uR) {
    const bool bot = (y == 0), top = (y == ny - 1);
    const long long t0 = tile(y), L0 = t0 + dl, R0 = t0 + dr;
    T a[9], b[9];
    a[0] = ld(L0, 63, 0);
    a[1] = ld(L0, 62, 1);
    a[3] = ld(t0, 0, 3);
    b[0] = ld(R0, 0, 0);
    b[1] = ld(t0, 63, 1);
    b[3] = ld(R0, 1, 3);
    if (bot) {
      a[2] = ld(L0, 63, 4);
      a[5] = ld(L0, 63, 7);
      a[6] = ld(L0, 63, 8);
      b[2] = ld(R0, 0, 4);
      b[5] = ld(R0, 0, 7);
      b[6] = ld(R0, 0, 8);
    } else {
      const long long td = tile(y - 1);
      a[2] = ld(td + dl, 63, 2);
      a[5] = ld(td + dl, 62, 5);
      a[6] = ld(td, 0, 6);
      b[2] = ld(td + dr, 0, 2);
      b[5] = ld(td, 63, 5);
      b[6] = ld(td + dr, 1, 6);
    }
    if (top) {
      a[4] = ld(L0, 63, 2);
      a[7] = ld(L0, 63, 5) - uw6;
      a[8] = ld(L0, 63, 6) + uw6;
      b[4] = ld(R0, 0, 2);
      b[7] = ld(R0, 0, 5) - uw6;
      b[8] = ld(R0, 0, 6) + uw6;
    } else {
      const long long tu = tile(y + 1);
      a[4] = ld(tu + dl, 63, 4);
      a[7] = ld(tu, 0, 7);
      a[8] = ld(tu + dl, 62, 8);
      b[4] = ld(tu + dr, 0, 4);
      b[7] = ld(tu + dr, 1, 7);
      b[8] = ld(tu, 63, 8);
    }
    const T urc = ref(y);
    if constexpr (SHIFT) {
      to_row_reference(a, ref(y - 1), urc, ref(y + 1), bot, top);
      to_row_reference(b, ref(y - 1), urc, ref(y + 1), bot, top);
    }
    if (c.zh && top) {
      zou_he_top<T, SHIFT>(a, uwg, urc, fx);
      zou_he_top<T, SHIFT>(b, uwg, urc, fx);
    }
    T sd, mx, my;
    moments<T>(a, sd, mx, my);
    uL = u_tilde<T, SHIFT>(sd, mx, my, fx, urc);
    moments<T>(b, sd, mx, my);
    uR = u_tilde<T, SHIFT>(sd, mx, my, fx, urc);
  };
  auto clampy = [&](int y) { return y < 0 ? 0 : (y >= ny ? ny - 1 : y); };
  // viscoelastic model: the stress of the previous step, one tile row of the
  // stress buffers (three fields per 64-node tile) per row
  const T *__restrict__ SA = static_cast<const T *>(a.SA);
  T *__restrict__ SB = static_cast<T *>(a.SB);
  auto load_sigma = [&](int y, T sg[3]) {
    if constexpr (VE) {
#pragma unroll
      for (int p = 0; p < 3; ++p) sg[p] = SA[(tile(y) * kStressPlanes + p) * F + lane];
    } else {
      sg[0] = sg[1] = sg[2] = T(0);
    }
  };

  T fc[9], fn[9], Pc, Pn, sgc[3], sgn[3];
  U2<T> uPrev, uCur, uNext, uLc, uRc, uLn, uRn;
  {
    T ftmp[9], Ptmp, sd, mx, my;
    pull_row(clampy(st.y0 - 1), ftmp, Ptmp);
    moments<T>(ftmp, sd, mx, my);
    uPrev = u_tilde<T, SHIFT>(sd, mx, my, fx, ref(st.y0 - 1));
  }
  T sdc, mxc, myc;
  pull_row(st.y0, fc, Pc);
  load_sigma(st.y0, sgc);
  moments<T>(fc, sdc, mxc, myc);
  uCur = u_tilde<T, SHIFT>(sdc, mxc, myc, fx, ref(st.y0));
  halo_u(st.y0, uLc, uRc);

#pragma unroll 1
  for (int y = st.y0; y < st.y1; ++y) {
    const int yn = clampy(y + 1);
    T sdn, mxn, myn;
    pull_row(yn, fn, Pn);
    load_sigma(yn, sgn);
    halo_u(yn, uLn, uRn);
    moments<T>(fn, sdn, mxn, myn);
    uNext = u_tilde<T, SHIFT>(sdn, mxn, myn, fx, ref(yn));

    U2<T> dn = uPrev, up = uNext;
    const U2<T> lf{shift_up(uLc.x, uCur.x), shift_up(uLc.y, uCur.y)};
    const U2<T> rt{shift_down(uRc.x, uCur.x), shift_down(uRc.y, uCur.y)};
    // no-slip ghosts behind the half-way walls; with SHIFT the ghost rows take
    // the mirrored references -ur and 2 u_w - ur (see sweep_kernel)
    const T urc = ref(y);
    if (y == 0) dn = U2<T>{-uCur.x, -uCur.y};
    if (y == ny - 1) {
      const U2<T> m = c.zh ? dn : uCur;
      up = U2<T>{(SHIFT ? T(0) : T(2) * uwg) - m.x, -m.y};
    }
    T kref = T(0);
    if constexpr (SHIFT) {
      const T urd = (y == 0) ? -urc : ref(y - 1);
      const T uru = (y == ny - 1) ? T(2) * uwg - (c.zh ? urd : urc) : ref(y + 1);
      kref = T(0.5) * (uru - urd);
    }

    T out[9], trT, sg[3];
    double obs[OF_COUNT];
    node_update<T, SHIFT, OBS, VE>(fc, sdc, mxc, myc, Pc, fx, lf, rt, dn, up, urc, kref, q, c.nnp, sgc, sg, out,
                                   trT, obs);
    if constexpr (OBS) {
      const double ztop = (c.zh && y == ny - 1) ? zh_drag<T>(run(tile(y), 5), run(tile(y), 6), fc) : 0.0;
      obs[OF_DRAG] = wall_drag<T>(fc, y, ny, uw6, c.zh, ztop);
#pragma unroll
      for (int f = 0; f < OF_COUNT; ++f) obs[f] = group_sum<64>(obs[f]);
      if (lane == 0) {
        const long long pr = (long long)c.poff + (long long)y * c.nxs + xt;
        double *dst = a.part + pr * OF_COUNT;
#pragma unroll
        for (int f = 0; f < OF_COUNT; ++f) dst[f] = obs[f];
      }
    } else {
      T *w = B + tile(y) * (kPlanes * F);
#pragma unroll
      for (int i = 0; i < 9; ++i) w[i * F + lane] = out[i];
      w[9 * F + lane] = trT;
      if constexpr (VE) {
        T *ws = SB + tile(y) * (kStressPlanes * F);
#pragma unroll
        for (int p = 0; p < 3; ++p) ws[p * F + lane] = sg[p];
      }
    }

    uPrev = uCur;
    uCur = uNext;
    uLc = uLn;
    uRc = uRn;
#pragma unroll
    for (int p = 0; p < 3; ++p) sgc[p] = sgn[p];
#pragma unroll
    for (int i = 0; i < 9; ++i) fc[i] = fn[i];
    Pc = Pn;
    sdc = sdn;
    mxc = mxn;
    myc = myn;
  }
}

// Vector accesses of NPL consecutive elements.
template <typename T, int NPL>
struct Vec;
template <>
struct Vec<float, 4> {
  typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct Vec<double, 2> {
  typedef double type __attribute__((ext_vector_type(2)));
};
template <>
struct Vec<float, 2> {
  typedef float type __attribute__((ext_vector_type(2)));
};
template <>
struct Vec<double, 1> {
  typedef double type __attribute__((ext_vector_type(1)));
};

// Side values of a row of a vector strip (see sweep_vec_kernel), packed as
// (dy + 1) | tile << 2 | column << 4 | field << 11 with tile 0: column left
// of the strip's tiles, 1: right of them, 2: first tile, 3: last tile.
#define SIDE(dy, t, col, p) ((dy) + 1 | (t) << 2 | (col) << 4 | (p) << 11)
constexpr int kSideIn[25] = {
    SIDE(0, 0, 63, 1),  SIDE(0, 1, 0, 3),   SIDE(-1, 0, 63, 5), SIDE(-1, 1, 0, 6),  SIDE(1, 1, 0, 7),
    SIDE(1, 0, 63, 8),  SIDE(0, 0, 63, 0),  SIDE(0, 0, 62, 1),  SIDE(0, 2, 0, 3),   SIDE(-1, 0, 63, 2),
    SIDE(-1, 0, 62, 5), SIDE(-1, 2, 0, 6),  SIDE(1, 0, 63, 4),  SIDE(1, 2, 0, 7),   SIDE(1, 0, 62, 8),
    SIDE(0, 1, 0, 0),   SIDE(0, 3, 63, 1),  SIDE(0, 1, 1, 3),   SIDE(-1, 1, 0, 2),  SIDE(-1, 3, 63, 5),
    SIDE(-1, 1, 1, 6),  SIDE(1, 1, 0, 4),   SIDE(1, 1, 1, 7),   SIDE(1, 3, 63, 8),  SIDE(0, 2, 0, 0)};
// bottom wall row: entries reading row y-1 take the bounce-back source (-1: unchanged)
constexpr int kSideBot[25] = {
    -1, -1, SIDE(0, 2, 0, 0), SIDE(0, 2, 0, 0), -1, -1, -1, -1, -1, SIDE(0, 0, 63, 4), SIDE(0, 0, 63, 7),
    SIDE(0, 0, 63, 8), -1, -1, -1, -1, -1, -1, SIDE(0, 1, 0, 4), SIDE(0, 1, 0, 7), SIDE(0, 1, 0, 8), -1, -1, -1, -1};
// top wall row: entries reading row y+1 take the bounce-back source
constexpr int kSideTop[25] = {
    -1, -1, -1, -1, SIDE(0, 2, 0, 0), SIDE(0, 2, 0, 0), -1, -1, -1, -1, -1, -1, SIDE(0, 0, 63, 2),
    SIDE(0, 0, 63, 5), SIDE(0, 0, 63, 6), -1, -1, -1, -1, -1, -1, SIDE(0, 1, 0, 2), SIDE(0, 1, 0, 5),
    SIDE(0, 1, 0, 6), -1};
#undef SIDE

// Aligned strips of 64 NPL columns of a channel whose width is a multiple of
// that: lane l owns the NPL consecutive columns x0 + NPL l + k, k < NPL, which
// sit in one tile (tile x0/64 + l/(64/NPL), first column NPL (l % (64/NPL))),
// so every field of a row is one NPL-element access per lane (16 bytes for
// four FP32 nodes). A pull along +x
// takes element k-1 of the same lane, and for k = 0 element NPL-1 of lane l-1
// (a DPP lane shift; lane 0 takes the column left of the strip); a pull along
// -x mirrors it.
//
// The march is software-pipelined two rows deep: while row y is computed,
// the loads of row y+2 are in flight and row y+1 (loaded one iteration
// earlier) is assembled for the stencil. The 24 values a row needs from the
// columns beside the strip (the six edge populations of the shifted pulls and
// the nine pulled populations of each neighbour column, for its u~) come in
// one lane-indexed vector load, lane i holding value i, so that they complete
// in order with the row's other loads; they are read out with readlane.
template <typename T, bool SHIFT, bool OBS, int NPL, bool NT, bool VE, bool ZH>
__global__ void __launch_bounds__(64 * LB_WG_WAVES) sweep_vec_kernel(SweepArgs a) {
  typedef typename Vec<T, NPL>::type V;
  constexpr int LPT = 64 / NPL;  // lanes per tile
  const int lane = threadIdx.x & 63;
  const int sidx = strip_index(a);
  if (sidx >= a.n_strips) return;
  const Strip st = a.strips[sidx];
  const ChanDev c = a.ch[st.ch];
  const T *__restrict__ A = static_cast<const T *>(a.A);
  T *__restrict__ B = static_cast<T *>(a.B);
  const int nx = c.nx, ny = c.ny;
  const long long t = c.t + a.k;
  const T fx = (t < c.t_startup) ? T(c.g) : T(0);
  // moving top wall: its velocity at step t (stencil ghost) and u_w/6 of step
  // t - 1, whose reflected links step t pulls
  const T uwg = (t < c.t_startup) ? T(c.uw) : T(0);
  const T uw6 = (!c.zh && t >= 1 && t - 1 < c.t_startup) ? T(c.uw / 6.0) : T(0);
  const Coef<T> q(c);

  const int tiles_row = nx >> 6;        // tiles per row
  const long long tile00 = c.off >> 6;  // tile of node (0, 0)
  const int xt = st.x0 >> 6;            // first tile column of the strip
  const int xe = xt + NPL - 1;          // last tile column of the strip
  const int xl = (xt == 0) ? tiles_row - 1 : xt - 1;  // tile column left of the strip
  const int xr = (xe == tiles_row - 1) ? 0 : xe + 1;  // tile column right of the strip
  const int lt = lane / LPT;            // tile of this lane inside the strip
  const int lo = NPL * (lane % LPT);    // first column of this lane inside its tile
  constexpr int F = kTile;

  auto tile = [&](int y, int tx) __attribute__((always_inline)) -> long long { return tile00 + (long long)y * tiles_row + tx; };
  // one field of this lane's NPL columns of row y
  // The time-integrated model's cached step (state and stress about 218 MB
  // per buffer on 4096 x 1024 FP32, near the last-level cache's 256 MB)
  // reads its rows with nontemporal loads: the buffer it reads is dead once
  // read, and letting it go first keeps more of what the previous step wrote
  // (+3 points there; the same loads cost 1 point on the instantaneous
  // model's 168 MB buffers and 6 on the streamed 10.7 GB ones).
  auto vrun = [&](int y, int p) __attribute__((always_inline)) -> V {
    const V *src = reinterpret_cast<const V *>(A + (tile(y, xt + lt) * kPlanes + p) * F + lo);
    if constexpr (VE && !NT && !OBS) return __builtin_nontemporal_load(src);
    return *src;
  };

  // Side values of a row, by lane i < 24 (kSide* below): lanes 0..5 hold the
  // edge populations of the shifted pulls, lanes 6..14 the pulled
  // populations of the column left of the strip, lanes 15..23 those of the
  // column right of it; wall rows take the bounce-back sources. With FP32
  // storage lanes 24..26 hold the reference velocities of rows y-1, y, y+1
  // (clamped to the channel), so that they arrive with the row's loads and
  // not through a dependent load in the row step. Other lanes read node
  // (x0, y). Each lane decodes its entry into an element offset
  // relative to row 0: once per strip for interior rows, again on the wall
  // rows (bottom, top, or both when ny = 1).
  auto side_off = [&](int code) __attribute__((always_inline)) -> long long {
    const int dy = (code & 3) - 1, tsel = (code >> 2) & 3, col = (code >> 4) & 127, p = code >> 11;
    // a blend of values, not a choice between the captured variables (which
    // the compiler would turn into a load through a chosen address and so
    // keep those variables in scratch memory)
    const int tc = (tsel == 0) * xl + (tsel == 1) * xr + (tsel == 2) * xt + (tsel == 3) * xe;
    return ((tile00 + (long long)dy * tiles_row + tc) * kPlanes + p) * F + col;
  };
  const int li = lane < 24 ? lane : 24;
  const int c_in = kSideIn[li];
  const int c_bot = kSideBot[li] >= 0 ? kSideBot[li] : c_in;
  const int c_top = kSideTop[li] >= 0 ? kSideTop[li] : c_in;
  const int c_both = kSideBot[li] >= 0 ? kSideBot[li] : c_top;
  const long long o_in = side_off(c_in);
  const long long row_stride = (long long)tiles_row * kPlanes * F;  // elements per row

  // Raw loads of row y: the ten runs (fields 0, 1, 3, 9 of row y; 2, 5, 6 of
  // row y-1 or, at the bottom wall, 4, 7, 8 of row y; 4, 7, 8 of row y+1 or,
  // at the top wall, 2, 5, 6 of row y) and the side values.
  // viscoelastic model: the stress of the previous step comes with each
  // row's loads (three fields of this lane's NPL columns)
  const T *__restrict__ SA = static_cast<const T *>(a.SA);
  T *__restrict__ SB = static_cast<T *>(a.SB);
  struct Raw {
    V sg[VE ? 3 : 1];
    V r[10];
    T side;
  };
  auto load_raw = [&](int y, Raw &R) __attribute__((always_inline)) {
    const bool bot = (y == 0), top = (y == ny - 1);
    const int yd = bot ? y : y - 1, yu = top ? y : y + 1;
    R.r[0] = vrun(y, 0);
    R.r[1] = vrun(y, 1);
    R.r[3] = vrun(y, 3);
    R.r[9] = vrun(y, 9);
    R.r[2] = vrun(yd, bot ? 4 : 2);
    R.r[5] = vrun(yd, bot ? 7 : 5);
    R.r[6] = vrun(yd, bot ? 8 : 6);
    R.r[4] = vrun(yu, top ? 2 : 4);
    R.r[7] = vrun(yu, top ? 5 : 7);
    R.r[8] = vrun(yu, top ? 6 : 8);
    long long o = o_in;
    if (bot || top)  // wall rows only
      o = side_off(bot * top * c_both + bot * (1 - top) * c_bot + (1 - bot) * c_top);
    const T *ps = A + o + (long long)y * row_stride;
    if constexpr (SHIFT) {
      const int yr = y + lane - 25;
      const T *pu = a.uref + c.row_off + (yr < 0 ? 0 : (yr >= ny ? ny - 1 : yr));
      ps = (lane >= 24 && lane <= 26) ? pu : ps;
    }
    R.side = *ps;
    if constexpr (VE) {
#pragma unroll
      for (int p = 0; p < 3; ++p)
        R.sg[p] = *reinterpret_cast<const V *>(SA + (tile(y, xt + lt) * kStressPlanes + p) * F + lo);
    }
  };
  // Pulled populations, P, moments and u~ of the NPL columns of row y, and u~
  // of the two columns beside the strip.
  auto assemble = [&](int y, const Raw &R, T f[9][NPL], T P[NPL], T sd[NPL], T mx[NPL], T my[NPL],
                      U2<T> u[NPL], U2<T> &uL, U2<T> &uR, T ur3[3]) __attribute__((always_inline)) {
    const bool bot = (y == 0), top = (y == ny - 1);
    auto from_left = [&](const V &r, T edge, T out[NPL]) __attribute__((always_inline)) {
      out[0] = shift_up(edge, r[NPL - 1]);
#pragma unroll
      for (int k = 1; k < NPL; ++k) out[k] = r[k - 1];
    };
    auto from_right = [&](const V &r, T edge, T out[NPL]) __attribute__((always_inline)) {
#pragma unroll
      for (int k = 0; k < NPL - 1; ++k) out[k] = r[k + 1];
      out[NPL - 1] = shift_down(edge, r[0]);
    };
    auto split = [&](const V &r, T out[NPL]) __attribute__((always_inline)) {
#pragma unroll
      for (int k = 0; k < NPL; ++k) out[k] = r[k];
    };
    split(R.r[0], f[0]);
    from_left(R.r[1], lane_value(R.side, 0), f[1]);
    from_right(R.r[3], lane_value(R.side, 1), f[3]);
    split(R.r[9], P);
    split(R.r[2], f[2]);
    split(R.r[4], f[4]);
    if (bot) {
      split(R.r[5], f[5]);
      split(R.r[6], f[6]);
    } else {
      from_left(R.r[5], lane_value(R.side, 2), f[5]);
      from_right(R.r[6], lane_value(R.side, 3), f[6]);
    }
    if (top) {
      split(R.r[7], f[7]);
      split(R.r[8], f[8]);
#pragma unroll
      for (int k = 0; k < NPL; ++k) {
        f[7][k] -= uw6;
        f[8][k] += uw6;
      }
    } else {
      from_right(R.r[7], lane_value(R.side, 4), f[7]);
      from_left(R.r[8], lane_value(R.side, 5), f[8]);
    }
    // a Zou-He top wall completes the top row's populations from above (a
    // variant of its own: the completion's registers cost the plain sweep
    // about a fifth of a point of occupancy headroom)
    const bool zhtop = ZH && top && c.zh;
    // FP32: every pulled value relative to this row's reference
    const T urd = SHIFT ? lane_value(R.side, 24) : T(0);
    const T urc = SHIFT ? lane_value(R.side, 25) : T(0);
    const T uru = SHIFT ? lane_value(R.side, 26) : T(0);
    ur3[0] = urd;
    ur3[1] = urc;
    ur3[2] = uru;
#pragma unroll
    for (int k = 0; k < NPL; ++k) {
      T g[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) g[i] = f[i][k];
      if constexpr (SHIFT) to_row_reference(g, urd, urc, uru, bot, top);
      if (zhtop) zou_he_top<T, SHIFT>(g, uwg, urc, fx);
      if (SHIFT || zhtop) {
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i][k] = g[i];
      }
      moments<T>(g, sd[k], mx[k], my[k]);
      u[k] = u_tilde<T, SHIFT>(sd[k], mx[k], my[k], fx, urc);
    }
    // side lanes 6..14 / 15..23 hold populations 0,1,3,2,5,6,4,7,8
    T l[9], r[9];
    l[0] = lane_value(R.side, 6);
    l[1] = lane_value(R.side, 7);
    l[3] = lane_value(R.side, 8);
    l[2] = lane_value(R.side, 9);
    l[5] = lane_value(R.side, 10);
    l[6] = lane_value(R.side, 11);
    l[4] = lane_value(R.side, 12);
    l[7] = lane_value(R.side, 13);
    l[8] = lane_value(R.side, 14);
    r[0] = lane_value(R.side, 15);
    r[1] = lane_value(R.side, 16);
    r[3] = lane_value(R.side, 17);
    r[2] = lane_value(R.side, 18);
    r[5] = lane_value(R.side, 19);
    r[6] = lane_value(R.side, 20);
    r[4] = lane_value(R.side, 21);
    r[7] = lane_value(R.side, 22);
    r[8] = lane_value(R.side, 23);
    const T wc = top ? uw6 : T(0);  // a select: no branch in the row step
    l[7] -= wc;
    l[8] += wc;
    r[7] -= wc;
    r[8] += wc;
    if constexpr (SHIFT) {
      to_row_reference(l, urd, urc, uru, bot, top);
      to_row_reference(r, urd, urc, uru, bot, top);
    }
    if (zhtop) {
      zou_he_top<T, SHIFT>(l, uwg, urc, fx);
      zou_he_top<T, SHIFT>(r, uwg, urc, fx);
    }
    T s0, m0, n0;
    moments<T>(l, s0, m0, n0);
    uL = u_tilde<T, SHIFT>(s0, m0, n0, fx, urc);
    moments<T>(r, s0, m0, n0);
    uR = u_tilde<T, SHIFT>(s0, m0, n0, fx, urc);
  };
  auto clampy = [&](int y) __attribute__((always_inline)) { return y < 0 ? 0 : (y >= ny ? ny - 1 : y); };

  // The march runs upwards from y0, or downwards from y1 - 1 (the step's
  // direction, reversed on flipped strips); "prev" and "next" are the rows
  // behind and ahead of the current one.
  const bool down = (a.down != 0) != (st.flip != 0);
  const int dir = down ? -1 : 1;
  const int yfirst = down ? st.y1 - 1 : st.y0;
  // Rows the ring loads: the strip and its two halo rows. Its last loads run
  // past the far halo row and are never assembled; they re-read that halo
  // row (fetched a row or two earlier, so from cache) instead of new rows.
  auto ring_row = [&](int y) __attribute__((always_inline)) {
    return clampy(y < st.y0 - 1 ? st.y0 - 1 : (y > st.y1 ? st.y1 : y));
  };
  const int nrows = st.y1 - st.y0;
  T fc[9][NPL], Pc[NPL], sdc[NPL], mxc[NPL], myc[NPL];
  U2<T> uPrev[NPL], uCur[NPL], uLc, uRc;
  T urC[3];  // reference velocities of rows y-1, y, y+1 for the current row
  T sgc[3][NPL];  // viscoelastic model: stress of the previous step, current row
  auto take_sigma = [&](const Raw &R, T sg[3][NPL]) __attribute__((always_inline)) {
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int k = 0; k < NPL; ++k) sg[p][k] = VE ? R.sg[VE ? p : 0][k] : T(0);
  };
  // ring of raw rows: the row i steps ahead of the first lives in slot i mod D
  constexpr int D = NT ? LB_VEC_DEPTH_NT : LB_VEC_DEPTH;
  Raw S[D];
  {
    // every load of the prologue is issued before the first is used, so the
    // strip pays one memory latency before its first row, not three
    Raw Rp, Rf;
    const int yp = clampy(yfirst - dir);
    load_raw(yp, Rp);
    load_raw(yfirst, Rf);
#pragma unroll
    for (int k = 1; k < D; ++k) load_raw(ring_row(yfirst + dir * k), S[k]);
    T ftmp[9][NPL], Ptmp[NPL], s0[NPL], m0[NPL], n0[NPL], ur_unused[3];
    U2<T> hl, hr;
    assemble(yp, Rp, ftmp, Ptmp, s0, m0, n0, uPrev, hl, hr, ur_unused);
    assemble(yfirst, Rf, fc, Pc, sdc, mxc, myc, uCur, uLc, uRc, urC);
    take_sigma(Rf, sgc);
  }

  // Row y: start the loads of the row D ahead, assemble the next row (loaded
  // D - 1 rows earlier), update and store row y.
  auto row_step = [&](int y, Raw &Rload, const Raw &Rasm) __attribute__((always_inline)) {
    load_raw(ring_row(y + dir * D), Rload);  // unconditional: a branch here costs more than the loads
    T fn[9][NPL], Pn[NPL], sdn[NPL], mxn[NPL], myn[NPL], urN[3];
    U2<T> uNext[NPL], uLn, uRn;
    assemble(clampy(y + dir), Rasm, fn, Pn, sdn, mxn, myn, uNext, uLn, uRn, urN);
    T sgn[3][NPL], sgo[3][NPL];
    take_sigma(Rasm, sgn);

    T out[9][NPL], trT[NPL];
    double obs[OF_COUNT];
    if constexpr (OBS) {
#pragma unroll
      for (int f = 0; f < OF_COUNT; ++f) obs[f] = 0.0;
    }
    // the row's reference and its share of d_y u_x (ghost rows mirrored)
    const T urc = urC[1];
    T kref = T(0);
    if constexpr (SHIFT) {
      const T urd = (y == 0) ? -urc : urC[0];
      const T uru = (y == ny - 1) ? T(2) * uwg - (c.zh ? urd : urc) : urC[2];
      kref = T(0.5) * (uru - urd);
    }
    // the top row's own stored 5 and 6 (what it emitted upwards), for the
    // momentum a Zou-He wall took (observation only)
    V a5{}, a6{};
    if constexpr (OBS && ZH) {
      if (c.zh && y == ny - 1) {
        a5 = vrun(y, 5);
        a6 = vrun(y, 6);
      }
    }
#pragma unroll
    for (int k = 0; k < NPL; ++k) {
      U2<T> lf, rt;
      if (k == 0) {
        lf = U2<T>{shift_up(uLc.x, uCur[NPL - 1].x), shift_up(uLc.y, uCur[NPL - 1].y)};
      } else {
        lf = uCur[k - 1];
      }
      if (k == NPL - 1) {
        rt = U2<T>{shift_down(uRc.x, uCur[0].x), shift_down(uRc.y, uCur[0].y)};
      } else {
        rt = uCur[k + 1];
      }
      U2<T> dn = down ? uNext[k] : uPrev[k], up = down ? uPrev[k] : uNext[k];
      // no-slip ghosts behind the half-way walls, or behind a Zou-He node
      // wall mirrored through the wall row
      if (y == 0) dn = U2<T>{-uCur[k].x, -uCur[k].y};
      if (y == ny - 1) {
        const U2<T> m = c.zh ? dn : uCur[k];
        up = U2<T>{(SHIFT ? T(0) : T(2) * uwg) - m.x, -m.y};
      }
      T g[9], o[9], tr;
#pragma unroll
      for (int i = 0; i < 9; ++i) g[i] = fc[i][k];
      double ob[OF_COUNT];
      const T sp[3] = {sgc[0][k], sgc[1][k], sgc[2][k]};
      T sn[3];
      node_update<T, SHIFT, OBS, VE>(g, sdc[k], mxc[k], myc[k], Pc[k], fx, lf, rt, dn, up, urc, kref, q, c.nnp, sp,
                                     sn, o, tr, ob);
      if constexpr (VE) {
#pragma unroll
        for (int p = 0; p < 3; ++p) sgo[p][k] = sn[p];
      }
      if constexpr (OBS) {
        ob[OF_DRAG] = wall_drag<T>(g, y, ny, uw6, c.zh, zh_drag<T>(a5[k], a6[k], g));
#pragma unroll
        for (int f = 0; f < OF_COUNT; ++f) obs[f] += ob[f];
      } else {
#pragma unroll
        for (int i = 0; i < 9; ++i) out[i][k] = o[i];
        trT[k] = tr;
      }
    }
    if constexpr (OBS) {
#pragma unroll
      for (int f = 0; f < OF_COUNT; ++f) obs[f] = group_sum<64>(obs[f]);
      if (lane == 0) {
        const long long pr = (long long)c.poff + (long long)y * c.nxs + st.x0 / (64 * NPL);
        double *dst = a.part + pr * OF_COUNT;
#pragma unroll
        for (int f = 0; f < OF_COUNT; ++f) dst[f] = obs[f];
      }
    } else {
      T *w = B + tile(y, xt + lt) * (kPlanes * F) + lo;
      V v[kPlanes];
#pragma unroll
      for (int k = 0; k < NPL; ++k) {
#pragma unroll
        for (int i = 0; i < 9; ++i) v[i][k] = out[i][k];
        v[9][k] = trT[k];
      }
      if constexpr (NT) {
#pragma unroll
        for (int i = 0; i < kPlanes; ++i) __builtin_nontemporal_store(v[i], reinterpret_cast<V *>(w + i * F));
      } else {
#pragma unroll
        for (int i = 0; i < kPlanes; ++i) *reinterpret_cast<V *>(w + i * F) = v[i];
      }
      if constexpr (VE) {
        T *ws = SB + tile(y, xt + lt) * (kStressPlanes * F) + lo;
#pragma unroll
        for (int p = 0; p < 3; ++p) {
          V vs;
#pragma unroll
          for (int k = 0; k < NPL; ++k) vs[k] = sgo[p][k];
          if constexpr (NT) __builtin_nontemporal_store(vs, reinterpret_cast<V *>(ws + p * F));
          else *reinterpret_cast<V *>(ws + p * F) = vs;
        }
      }
    }

    uLc = uLn;
    uRc = uRn;
    urC[0] = urN[0];
    urC[1] = urN[1];
    urC[2] = urN[2];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int k = 0; k < NPL; ++k) sgc[p][k] = sgn[p][k];
#pragma unroll
    for (int k = 0; k < NPL; ++k) {
      uPrev[k] = uCur[k];
      uCur[k] = uNext[k];
      Pc[k] = Pn[k];
      sdc[k] = sdn[k];
      mxc[k] = mxn[k];
      myc[k] = myn[k];
#pragma unroll
      for (int i = 0; i < 9; ++i) fc[i][k] = fn[i][k];
    }
  };

  // unrolled D times so that the ring slots are fixed registers
#pragma unroll 1
  for (int i = 0; i < nrows; i += D) {
#pragma unroll
    for (int j = 0; j < D; ++j)
      if (j == 0 || i + j < nrows) row_step(yfirst + dir * (i + j), S[j], S[(j + 1) % D]);
  }
}

// ---------------------------------------------------------------------------
// Two steps per launch for vector-class channels without the pressure
// drive (either stress model, any top wall; FP32 storage relative to the
// row references or plain FP64). One workgroup of two wavefronts takes an
// output strip of columns [x0, x1) and rows [y0, y1) through steps t and
// t+1 without writing step t to memory; each lane holds NPL adjacent nodes
// of a row (two, or four for streamed FP32 states of the instantaneous
// model):
//  * the window is the 64 NPL columns starting HL NPL columns left of x0
//    (HL = ceil(2 / NPL) lanes, wrapped periodically), with one column
//    beside it on either side as the vector sweep has;
//  * wavefront 0 runs stage A (step t): the vector sweep's row machine over
//    the window for rows max(y0-2, 0) .. min(y1+2, ny)-1, read from the
//    state; each row's post-collision populations and trace (and with the
//    time-integrated model the stress sigma(t)) go into a ring of four rows
//    in LDS instead of memory;
//  * wavefront 1 runs stage B (step t+1): the same machine reading its rows
//    from that ring, three rows behind stage A, and stores rows y0 .. y1-1
//    of lanes HL .. 63-HL to the other buffer.
// The two stages share one loop with one barrier per row. Splitting them
// over two wavefronts halves what each keeps in registers, so that two or
// three wavefronts fit a SIMD and one's arithmetic covers the other's waits.
// After step t the window's two outermost columns on each side lack valid
// neighbours for step t+1; the lanes holding them store nothing, so every
// stored node saw only values of the exact step-t state. Per node the
// arithmetic is the vector sweep's (same helpers, same pull, reference
// shifts and collision), so the result equals two one-step sweeps to the
// rounding of the operations. A moving top wall takes each stage's own
// step's velocity.
constexpr int kV2Ring = 4;

// Side values of stage A's rows, by lane i < 24: (row offset, column offset
// from the window start, field), with the wall rows' bounce-back sources;
// the same meaning as kSideIn/kSideBot/kSideTop for the columns beside a
// window that need not start on a tile. The table is written for a window
// of 256 columns (offsets 255..257 on the right); v2_side<W> moves the
// right side to a window of W columns. Lanes 24..26 carry the row
// references (FP32 storage).
struct SideEntry {
  int dy, dc, p;
};
// interior rows, packed as (dy + 1) | (dc + 2) << 2 | p << 12
#define V2SIDE(dy, dc, p) ((dy) + 1 | ((dc) + 2) << 2 | (p) << 12)
constexpr int kV2Side[24] = {
    V2SIDE(0, -1, 1),   V2SIDE(0, 256, 3),  V2SIDE(-1, -1, 5), V2SIDE(-1, 256, 6), V2SIDE(1, 256, 7),
    V2SIDE(1, -1, 8),   V2SIDE(0, -1, 0),   V2SIDE(0, -2, 1),  V2SIDE(0, 0, 3),    V2SIDE(-1, -1, 2),
    V2SIDE(-1, -2, 5),  V2SIDE(-1, 0, 6),   V2SIDE(1, -1, 4),  V2SIDE(1, 0, 7),    V2SIDE(1, -2, 8),
    V2SIDE(0, 256, 0),  V2SIDE(0, 255, 1),  V2SIDE(0, 257, 3), V2SIDE(-1, 256, 2), V2SIDE(-1, 255, 5),
    V2SIDE(-1, 257, 6), V2SIDE(1, 256, 4),  V2SIDE(1, 257, 7), V2SIDE(1, 255, 8)};
#undef V2SIDE
template <int W>
__device__ __forceinline__ SideEntry v2_side(int i, bool bot, bool top) {
  const int code = kV2Side[i];
  SideEntry e{(code & 3) - 1, ((code >> 2) & 1023) - 2, code >> 12};
  if (e.dc >= 255) e.dc += W - 256;
  if (bot && e.dy < 0) {
    // entries 2, 3: edge values of pulls the wall row takes from its own
    // node (unused); the side columns' pops 2, 5, 6 bounce back from 4, 7, 8
    const bool edge = (i == 2 || i == 3);
    const int col = (i < 15) ? -1 : W;
    const int back = e.p == 2 ? 4 : (e.p == 5 ? 7 : 8);
    e = edge ? SideEntry{0, 0, 0} : SideEntry{0, col, back};
  }
  if (top && e.dy > 0) {
    const bool edge = (i == 4 || i == 5);
    const int col = (i < 15) ? -1 : W;
    const int back = e.p == 4 ? 2 : (e.p == 7 ? 5 : 6);
    e = edge ? SideEntry{0, 0, 0} : SideEntry{0, col, back};
  }
  return e;
}

template <typename T, int NPL, bool NT, bool VE, bool WALL>
__global__ void __launch_bounds__(64 * kTwoStepWaves, VE ? 1 : kTwoStepWaves) sweep_vec2_kernel(SweepArgs a) {
  // FP32: storage relative to the row references; FP64: plain storage
  constexpr bool SHIFT = sizeof(T) == 4;
  constexpr int W = 64 * NPL;                 // window columns
  constexpr int HL = (2 + NPL - 1) / NPL;     // lanes per side without valid step t+1
  typedef typename Vec<T, NPL>::type V;
  // the ring of step-t rows: populations and trace, and with VE the stress
  // sigma(t) (sizeof(T) x NPL x 5 KB per workgroup, x 6.5 KB with VE)
  constexpr int RP = kPlanes + (VE ? kStressPlanes : 0);
  __shared__ V ring[kV2Ring][RP][64];
  const int lane = threadIdx.x & 63;
  // wave 0 runs stage A, wave 1 stage B of the same strip
  const bool isA = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) == 0;
  const int sidx = xcd_item(blockIdx.x, a.n_wg);
  if (sidx >= a.n_strips) return;  // the whole workgroup, before any barrier
  const Strip st = a.strips[sidx];
  const ChanDev c = a.ch[st.ch];
  const T *__restrict__ A = static_cast<const T *>(a.A);
  T *__restrict__ B = static_cast<T *>(a.B);
  const int nx = c.nx, ny = c.ny;
  const long long t = c.t + a.k;
  const T fxA = (t < c.t_startup) ? T(c.g) : T(0);
  const T fxB = (t + 1 < c.t_startup) ? T(c.g) : T(0);
  const T fx = isA ? fxA : fxB;
  // WALL: a moving top wall at this stage's step ts: its velocity (stencil
  // ghost) and, for the half-way wall, u_w/6 of step ts - 1, whose reflected
  // links step ts pulls; or the Zou-He completion of the top row
  const long long ts = isA ? t : t + 1;
  const T uwg = (WALL && ts < c.t_startup) ? T(c.uw) : T(0);
  const T uw6 = (WALL && !c.zh && ts >= 1 && ts - 1 < c.t_startup) ? T(c.uw / 6.0) : T(0);
  const Coef<T> q(c);
  constexpr int F = kTile;
  const long long tile00 = c.off >> 6;
  const int tiles_row = nx >> 6;
  const long long row_stride = (long long)tiles_row * kPlanes * F;
  auto rowbase = [&](int y) __attribute__((always_inline)) { return (tile00 + (long long)y * tiles_row) * (kPlanes * F); };
  // column of window offset dc, wrapped, as an element offset inside a row
  const int w0 = st.x0 - HL * NPL;
  auto colpart = [&](int dc) __attribute__((always_inline)) -> long long {
    int col = w0 + dc;
    col += (col < 0) ? nx : 0;
    col -= (col >= nx) ? nx : 0;
    return (long long)(col >> 6) * (kPlanes * F) + (col & 63);
  };
  const long long lcol = colpart(NPL * lane);
  // VE: the stress fields, three planes per tile of 64 nodes
  const T *__restrict__ SA = static_cast<const T *>(a.SA);
  T *__restrict__ SB = static_cast<T *>(a.SB);
  auto srow = [&](int y) __attribute__((always_inline)) {
    return (tile00 + (long long)y * tiles_row) * (kStressPlanes * F);
  };
  const long long scol = (long long)(((w0 + NPL * lane + nx) % nx) >> 6) * (kStressPlanes * F) +
                         ((w0 + NPL * lane + nx) % nx & 63);
  auto clampy = [&](int y) __attribute__((always_inline)) { return y < 0 ? 0 : (y >= ny ? ny - 1 : y); };

  // ---- rows of the two stages
  const int A0 = st.y0 - 2 < 0 ? 0 : st.y0 - 2, A1 = st.y1 + 2 > ny ? ny : st.y1 + 2;
  const int R0 = st.y0 - 1 < 0 ? 0 : st.y0 - 1, R1 = st.y1 + 1 > ny ? ny : st.y1 + 1;
  const int iend = st.y1 + 3;  // iterations [A0, iend): stage B updates row i - 3
  // stage B's stores: lanes whose columns lie in [x0, x1)
  const bool store_lane = lane >= HL && NPL * (lane - HL) < st.x1 - st.x0;
  // FP32: row references of rows A0-1 .. A0+62 (clamped), lane j holding
  // row A0-1+j: stage B reads those of its rows from here (strips have at
  // most 56 rows, so rows A0-1 .. A1 fit)
  T uall = T(0);
  if constexpr (SHIFT) uall = a.uref[c.row_off + clampy(A0 - 1 + lane)];
  auto ref = [&](int y) __attribute__((always_inline)) {
    return SHIFT ? lane_value(uall, clampy(y) - (A0 - 1)) : T(0);
  };

  // ---- stage A: raw loads of a row of the state (window and side values)
  struct Raw {
    V r[10];
    V sg[VE ? 3 : 1];  // VE: the stress of the previous step at the row's own nodes
    T side;
  };
  const int li = lane < 24 ? lane : 0;
  // element offset of this lane's side value relative to the row (decoded
  // again on wall rows: a choice between precomputed offsets would keep them
  // in scratch memory)
  auto side_offset = [&](bool bot, bool top) __attribute__((always_inline)) -> long long {
    const SideEntry e = v2_side<W>(li, bot, top);
    return (lane < 24) ? (long long)e.dy * row_stride + colpart(e.dc) + (long long)e.p * F : lcol;
  };
  const long long o_in = side_offset(false, false);
  auto load_raw = [&](int y, Raw &R) __attribute__((always_inline)) {
    const bool bot = (y == 0), top = (y == ny - 1);
    const long long rb = rowbase(y);
    const long long rd = bot ? rb : rb - row_stride, ru = top ? rb : rb + row_stride;
    auto run = [&](long long base, int p) __attribute__((always_inline)) {
      return *reinterpret_cast<const V *>(A + base + lcol + (long long)p * F);
    };
    R.r[0] = run(rb, 0);
    R.r[1] = run(rb, 1);
    R.r[3] = run(rb, 3);
    R.r[9] = run(rb, 9);
    R.r[2] = run(rd, bot ? 4 : 2);
    R.r[5] = run(rd, bot ? 7 : 5);
    R.r[6] = run(rd, bot ? 8 : 6);
    R.r[4] = run(ru, top ? 2 : 4);
    R.r[7] = run(ru, top ? 5 : 7);
    R.r[8] = run(ru, top ? 6 : 8);
    long long o = o_in;
    if (bot || top) o = side_offset(bot, top);  // wall rows only
    const T *ps = A + rb + o;
    if constexpr (VE) {
#pragma unroll
      for (int p = 0; p < 3; ++p) R.sg[p] = *reinterpret_cast<const V *>(SA + srow(y) + scol + (long long)p * F);
    }
    if constexpr (SHIFT) {
      const int yr = y + lane - 25;
      const T *pu = a.uref + c.row_off + (yr < 0 ? 0 : (yr >= ny ? ny - 1 : yr));
      ps = (lane >= 24 && lane <= 26) ? pu : ps;
    }
    R.side = *ps;
  };
  // ---- stage B: the same row from the LDS ring of step-t rows (no side
  // values: lanes 0 and 63, which would use them, store nothing)
  auto load_lds = [&](int y, Raw &R) __attribute__((always_inline)) {
    const bool bot = (y == 0), top = (y == ny - 1);
    const int sc = y & (kV2Ring - 1), sd = bot ? sc : ((y - 1) & (kV2Ring - 1)), su = top ? sc : ((y + 1) & (kV2Ring - 1));
    R.r[0] = ring[sc][0][lane];
    R.r[1] = ring[sc][1][lane];
    R.r[3] = ring[sc][3][lane];
    R.r[9] = ring[sc][9][lane];
    R.r[2] = ring[sd][bot ? 4 : 2][lane];
    R.r[5] = ring[sd][bot ? 7 : 5][lane];
    R.r[6] = ring[sd][bot ? 8 : 6][lane];
    R.r[4] = ring[su][top ? 2 : 4][lane];
    R.r[7] = ring[su][top ? 5 : 7][lane];
    R.r[8] = ring[su][top ? 6 : 8][lane];
    if constexpr (VE) {
#pragma unroll
      for (int p = 0; p < 3; ++p) R.sg[p] = ring[sc][kPlanes + p][lane];
    }
    R.side = T(0);
  };

  // Pulled populations, P, moments and u~ of the window's columns of row y,
  // and (stage A) u~ of the two columns beside it (the vector sweep's
  // assembly, fixed walls), with the row references urd, urc, uru.
  auto assemble = [&](int y, const Raw &R, T urd, T urc, T uru, T f[9][NPL], T P[NPL], T sd[NPL], T mx[NPL],
                      T my[NPL], U2<T> u[NPL], U2<T> &uL, U2<T> &uR) __attribute__((always_inline)) {
    const bool bot = (y == 0), top = (y == ny - 1);
    auto from_left = [&](const V &r, T edge, T out[NPL]) __attribute__((always_inline)) {
      out[0] = shift_up(edge, r[NPL - 1]);
#pragma unroll
      for (int k = 1; k < NPL; ++k) out[k] = r[k - 1];
    };
    auto from_right = [&](const V &r, T edge, T out[NPL]) __attribute__((always_inline)) {
#pragma unroll
      for (int k = 0; k < NPL - 1; ++k) out[k] = r[k + 1];
      out[NPL - 1] = shift_down(edge, r[0]);
    };
    auto split = [&](const V &r, T out[NPL]) __attribute__((always_inline)) {
#pragma unroll
      for (int k = 0; k < NPL; ++k) out[k] = r[k];
    };
    split(R.r[0], f[0]);
    from_left(R.r[1], lane_value(R.side, 0), f[1]);
    from_right(R.r[3], lane_value(R.side, 1), f[3]);
    split(R.r[9], P);
    split(R.r[2], f[2]);
    split(R.r[4], f[4]);
    if (bot) {
      split(R.r[5], f[5]);
      split(R.r[6], f[6]);
    } else {
      from_left(R.r[5], lane_value(R.side, 2), f[5]);
      from_right(R.r[6], lane_value(R.side, 3), f[6]);
    }
    if (top) {
      split(R.r[7], f[7]);
      split(R.r[8], f[8]);
      if constexpr (WALL) {
#pragma unroll
        for (int k = 0; k < NPL; ++k) {
          f[7][k] -= uw6;
          f[8][k] += uw6;
        }
      }
    } else {
      from_right(R.r[7], lane_value(R.side, 4), f[7]);
      from_left(R.r[8], lane_value(R.side, 5), f[8]);
    }
    const bool zhtop = WALL && top && c.zh;
#pragma unroll
    for (int k = 0; k < NPL; ++k) {
      T g[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) g[i] = f[i][k];
      if constexpr (SHIFT) to_row_reference(g, urd, urc, uru, bot, top);
      if (zhtop) zou_he_top<T, SHIFT>(g, uwg, urc, fx);
#pragma unroll
      for (int i = 0; i < 9; ++i) f[i][k] = g[i];
      moments<T>(g, sd[k], mx[k], my[k]);
      u[k] = u_tilde<T, SHIFT>(sd[k], mx[k], my[k], fx, urc);
    }
    uL = uR = U2<T>{T(0), T(0)};
    if (isA) {
      T l[9], r[9];
      l[0] = lane_value(R.side, 6);
      l[1] = lane_value(R.side, 7);
      l[3] = lane_value(R.side, 8);
      l[2] = lane_value(R.side, 9);
      l[5] = lane_value(R.side, 10);
      l[6] = lane_value(R.side, 11);
      l[4] = lane_value(R.side, 12);
      l[7] = lane_value(R.side, 13);
      l[8] = lane_value(R.side, 14);
      r[0] = lane_value(R.side, 15);
      r[1] = lane_value(R.side, 16);
      r[3] = lane_value(R.side, 17);
      r[2] = lane_value(R.side, 18);
      r[5] = lane_value(R.side, 19);
      r[6] = lane_value(R.side, 20);
      r[4] = lane_value(R.side, 21);
      r[7] = lane_value(R.side, 22);
      r[8] = lane_value(R.side, 23);
      if constexpr (WALL) {
        const T wc = top ? uw6 : T(0);
        l[7] -= wc;
        l[8] += wc;
        r[7] -= wc;
        r[8] += wc;
      }
      if constexpr (SHIFT) {
        to_row_reference(l, urd, urc, uru, bot, top);
        to_row_reference(r, urd, urc, uru, bot, top);
      }
      if (zhtop) {
        zou_he_top<T, SHIFT>(l, uwg, urc, fx);
        zou_he_top<T, SHIFT>(r, uwg, urc, fx);
      }
      T s0, m0, n0;
      moments<T>(l, s0, m0, n0);
      uL = u_tilde<T, SHIFT>(s0, m0, n0, fx, urc);
      moments<T>(r, s0, m0, n0);
      uR = u_tilde<T, SHIFT>(s0, m0, n0, fx, urc);
    }
  };

  // Update of row y from its assembled state (fc ..., uCur, side u~, the
  // references) and u~ of the rows below and above; out and trT receive
  // the new populations and trace.
  auto update = [&](int y, T fc[9][NPL], const T Pc[NPL], const T sdc[NPL], const T mxc[NPL], const T myc[NPL],
                    const U2<T> uPrev[NPL], const U2<T> uCur[NPL], const U2<T> uNext[NPL], U2<T> uLc, U2<T> uRc,
                    const T urC[3], const T sgc[VE ? 3 : 1][NPL], V out[RP]) __attribute__((always_inline)) {
    const T urc = urC[1];
    const T urd = (y == 0) ? -urc : urC[0];
    const T uru = (y == ny - 1) ? T(2) * uwg - (WALL && c.zh ? urd : urc) : urC[2];
    // FP32: the references' share of d_y u_x (ghost rows mirrored); FP64
    // stores plain populations and has none
    const T kref = SHIFT ? T(0.5) * (uru - urd) : T(0);
#pragma unroll
    for (int k = 0; k < NPL; ++k) {
      U2<T> lf, rt;
      if (k == 0) lf = U2<T>{shift_up(uLc.x, uCur[NPL - 1].x), shift_up(uLc.y, uCur[NPL - 1].y)};
      else lf = uCur[k - 1];
      if (k == NPL - 1) rt = U2<T>{shift_down(uRc.x, uCur[0].x), shift_down(uRc.y, uCur[0].y)};
      else rt = uCur[k + 1];
      U2<T> dn = uPrev[k], up = uNext[k];
      if (y == 0) dn = U2<T>{-uCur[k].x, -uCur[k].y};
      // no-slip ghosts behind the half-way walls (moving at u_w above), or
      // behind a Zou-He node wall mirrored through the wall row
      if (y == ny - 1) {
        const U2<T> m = (WALL && c.zh) ? dn : uCur[k];
        up = U2<T>{(SHIFT ? T(0) : T(2) * uwg) - m.x, -m.y};
      }
      T g[9], o[9], tr, sn[3];
#pragma unroll
      for (int i = 0; i < 9; ++i) g[i] = fc[i][k];
      const T sp[3] = {VE ? sgc[0][k] : T(0), VE ? sgc[VE ? 1 : 0][k] : T(0), VE ? sgc[VE ? 2 : 0][k] : T(0)};
      double ob[OF_COUNT];
      node_update<T, SHIFT, false, VE>(g, sdc[k], mxc[k], myc[k], Pc[k], fx, lf, rt, dn, up, urc, kref, q, c.nnp, sp,
                                       sn, o, tr, ob);
#pragma unroll
      for (int i = 0; i < 9; ++i) out[i][k] = o[i];
      out[9][k] = tr;
      if constexpr (VE) {
#pragma unroll
        for (int p = 0; p < 3; ++p) out[kPlanes + p][k] = sn[p];
      }
    }
  };

  // The state each wave carries from one iteration to the next: its
  // assembled current row and u~ of the rows below and at it (stage A: row
  // i and the raw loads of row i+1; stage B: row i-3).
  T fc[9][NPL], Pc[NPL], sdc[NPL], mxc[NPL], myc[NPL], urC[3], sgc[VE ? 3 : 1][NPL];
  U2<T> uPrev[NPL], uCur[NPL], uLc, uRc;
  Raw R;
  // VE: the stress of the previous step at a row's nodes, from its loads
  auto take_sigma = [&](const Raw &Q, T sg[VE ? 3 : 1][NPL]) __attribute__((always_inline)) {
#pragma unroll
    for (int p = 0; p < (VE ? 3 : 1); ++p)
#pragma unroll
      for (int k = 0; k < NPL; ++k) sg[p][k] = VE ? Q.sg[p][k] : T(0);
  };
  if (isA) {
    Raw Rp;
    const int yp = clampy(A0 - 1);
    load_raw(yp, Rp);
    load_raw(A0, R);
    T ftmp[9][NPL], Ptmp[NPL], s0[NPL], m0[NPL], n0[NPL];
    U2<T> hl, hr;
    // row references (FP32; zero in FP64, which stores plain populations)
    auto refs = [&](const Raw &Q, T u[3]) __attribute__((always_inline)) {
#pragma unroll
      for (int j = 0; j < 3; ++j) u[j] = SHIFT ? lane_value(Q.side, 24 + j) : T(0);
    };
    T urp[3];
    refs(Rp, urp);
    assemble(yp, Rp, urp[0], urp[1], urp[2], ftmp, Ptmp, s0, m0, n0, uPrev, hl, hr);
    refs(R, urC);
    assemble(A0, R, urC[0], urC[1], urC[2], fc, Pc, sdc, mxc, myc, uCur, uLc, uRc);
    take_sigma(R, sgc);
    load_raw(clampy(A0 + 1), R);
  } else {
#pragma unroll
    for (int k = 0; k < NPL; ++k) {
      uPrev[k] = uCur[k] = U2<T>{T(0), T(0)};
      Pc[k] = sdc[k] = mxc[k] = myc[k] = T(0);
#pragma unroll
      for (int j = 0; j < 9; ++j) fc[j][k] = T(0);
    }
    uLc = uRc = U2<T>{T(0), T(0)};
    urC[0] = urC[1] = urC[2] = T(0);
#pragma unroll
    for (int j = 0; j < 10; ++j) R.r[j] = V{};
#pragma unroll
    for (int j = 0; j < (VE ? 3 : 1); ++j) R.sg[j] = V{};
    R.side = T(0);
    take_sigma(R, sgc);
  }

  // Iteration i. Stage A (rows [A0, A1)): assembles row i+1 from the loads
  // issued in the previous iteration, updates row i into ring slot i mod 4,
  // then issues the loads of row i+2. Stage B: assembles row i-2 from the
  // ring (rows [R0, R1)), updates row i-3 and stores it (rows [y0, y1)).
  // One barrier per iteration orders stage A's ring writes before stage B's
  // reads three iterations later, and stage B's reads before the slot is
  // written again; both waves run every iteration.
  auto iteration = [&](int i) __attribute__((always_inline)) {
    const int r = isA ? i + 1 : i - 2, y = isA ? i : i - 3;
    const bool do_asm = isA ? (i < A1) : (r >= R0 && r < R1);
    const bool do_upd = isA ? (i < A1) : (y >= st.y0 && y < st.y1);
    T fn[9][NPL], Pn[NPL], sdn[NPL], mxn[NPL], myn[NPL], urN[3], sgn[VE ? 3 : 1][NPL];
    U2<T> uNext[NPL], uLn, uRn;
    if (do_asm) {
      if (!isA) load_lds(r, R);
      const int rr = clampy(r);
#pragma unroll
      for (int j = 0; j < 3; ++j) urN[j] = !SHIFT ? T(0) : (isA ? lane_value(R.side, 24 + j) : ref(rr - 1 + j));
      assemble(rr, R, urN[0], urN[1], urN[2], fn, Pn, sdn, mxn, myn, uNext, uLn, uRn);
      take_sigma(R, sgn);
    } else {
#pragma unroll
      for (int p = 0; p < (VE ? 3 : 1); ++p)
#pragma unroll
        for (int k = 0; k < NPL; ++k) sgn[p][k] = T(0);
#pragma unroll
      for (int k = 0; k < NPL; ++k) {
        uNext[k] = U2<T>{T(0), T(0)};
        Pn[k] = sdn[k] = mxn[k] = myn[k] = T(0);
#pragma unroll
        for (int j = 0; j < 9; ++j) fn[j][k] = T(0);
      }
      uLn = uRn = U2<T>{T(0), T(0)};
      urN[0] = urN[1] = urN[2] = T(0);
    }
    if (do_upd) {
      V out[RP];
      update(y, fc, Pc, sdc, mxc, myc, uPrev, uCur, uNext, uLc, uRc, urC, sgc, out);
      if (isA) {
        const int slot = y & (kV2Ring - 1);
#pragma unroll
        for (int p = 0; p < RP; ++p) ring[slot][p][lane] = out[p];
      } else if (store_lane) {
        T *w = B + rowbase(y) + lcol;
#pragma unroll
        for (int p = 0; p < kPlanes; ++p) {
          if constexpr (NT) __builtin_nontemporal_store(out[p], reinterpret_cast<V *>(w + (long long)p * F));
          else *reinterpret_cast<V *>(w + (long long)p * F) = out[p];
        }
        if constexpr (VE) {
          T *ws = SB + srow(y) + scol;
#pragma unroll
          for (int p = 0; p < 3; ++p) {
            if constexpr (NT) __builtin_nontemporal_store(out[kPlanes + p], reinterpret_cast<V *>(ws + (long long)p * F));
            else *reinterpret_cast<V *>(ws + (long long)p * F) = out[kPlanes + p];
          }
        }
      }
    }
    uLc = uLn;
    uRc = uRn;
    urC[0] = urN[0];
    urC[1] = urN[1];
    urC[2] = urN[2];
#pragma unroll
    for (int p = 0; p < (VE ? 3 : 1); ++p)
#pragma unroll
      for (int k = 0; k < NPL; ++k) sgc[p][k] = sgn[p][k];
#pragma unroll
    for (int k = 0; k < NPL; ++k) {
      uPrev[k] = uCur[k];
      uCur[k] = uNext[k];
      Pc[k] = Pn[k];
      sdc[k] = sdn[k];
      mxc[k] = mxn[k];
      myc[k] = myn[k];
#pragma unroll
      for (int j = 0; j < 9; ++j) fc[j][k] = fn[j][k];
    }
    // the loads of row i+2 (clamped to the lattice), in flight across the
    // barrier
    if (isA && i + 1 < A1) load_raw(clampy(i + 2), R);
    __syncthreads();
  };
  // unrolled twice: the two-deep state swaps stay in fixed registers (the
  // trip count is the same for both wavefronts, so they pass the same
  // barriers)
#pragma unroll 1
  for (int i = A0; i < iend; i += 2) {
    iteration(i);
    if (i + 1 < iend) iteration(i + 1);
  }
}

__global__ void __launch_bounds__(256) reduce_kernel(const ChanDev *ch, const double *part,
                                                     double *prof, double *prev_ux, double *scal,
                                                     const float *uref, int update_residual,
                                                     int steps_since) {
  const ChanDev c = ch[blockIdx.x];
  __shared__ double red[7][256];
  double mass = 0, momx = 0, flux = 0, drag = 0, umax = 0, dmax = 0, bad = 0;
  for (int y = threadIdx.x; y < c.ny; y += blockDim.x) {
    double rs[OF_COUNT];
#pragma unroll
    for (int f = 0; f < OF_COUNT; ++f) rs[f] = 0.0;
    for (int xs = 0; xs < c.nxs; ++xs) {
      const double *src = part + ((long long)c.poff + (long long)y * c.nxs + xs) * OF_COUNT;
#pragma unroll
      for (int f = 0; f < OF_COUNT; ++f) rs[f] += src[f];
    }
    // FP32 storage: the row's reference velocity, left out of the node
    // values of u_x, j_x and the wall momentum (0 for FP64)
    const double ur = (double)uref[c.row_off + y];
    rs[OF_UX] += c.nx * ur;
    rs[OF_MOMX] += c.nx * ur;
    if (y == 0) rs[OF_DRAG] -= c.nx * ur / 3.0;
    if (y == c.ny - 1) rs[OF_DRAG] -= c.nx * ur / (c.zh ? 6.0 : 3.0);
    double *dst = prof + ((long long)c.row_off + y) * OF_COUNT;
#pragma unroll
    for (int f = 0; f < OF_COUNT; ++f) {
      dst[f] = rs[f] / c.nx;
      if (!isfinite(rs[f])) bad = 1;
    }
    mass += rs[OF_MASS_DEV];
    momx += rs[OF_MOMX];
    flux += rs[OF_UX];
    drag += rs[OF_DRAG];
    const double ub = rs[OF_UX] / c.nx;
    umax = fmax(umax, fabs(ub));
    const double pv = prev_ux[c.row_off + y];
    const double d = fabs(ub - pv);
    dmax = (d != d) ? INFINITY : fmax(dmax, d);
    if (update_residual) prev_ux[c.row_off + y] = ub;
  }
  red[0][threadIdx.x] = mass;
  red[1][threadIdx.x] = momx;
  red[2][threadIdx.x] = flux;
  red[3][threadIdx.x] = drag;
  red[4][threadIdx.x] = umax;
  red[5][threadIdx.x] = dmax;
  red[6][threadIdx.x] = bad;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
      for (int k = 4; k < 7; ++k) red[k][threadIdx.x] = fmax(red[k][threadIdx.x], red[k][threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double *o = scal + (long long)blockIdx.x * CS_COUNT;
    o[CS_MASS_DEV] = red[0][0];
    o[CS_MOMX] = red[1][0];
    o[CS_FLUX] = red[2][0];
    o[CS_DRAG] = red[3][0];
    const double *pr = prof + (long long)c.row_off * OF_COUNT;
    const double um = (c.ny & 1) ? pr[(c.ny / 2) * OF_COUNT + OF_UX]
                                 : 0.5 * (pr[(c.ny / 2 - 1) * OF_COUNT + OF_UX] + pr[(c.ny / 2) * OF_COUNT + OF_UX]);
    o[CS_UMID] = um;
    o[CS_UMAX] = red[4][0];
    const bool nan = red[6][0] > 0;
    o[CS_NAN] = nan ? 1.0 : 0.0;
    if (update_residual) {
      // R = max_y |ubar(t) - ubar(t - K)| / (K max_y |ubar(t)|); +inf when a
      // previous profile is missing or the data are not finite
      const double dm = red[5][0], um2 = red[4][0];
      double R;
      if (nan || !(dm < INFINITY)) R = INFINITY;
      else if (um2 == 0.0) R = (dm == 0.0) ? 0.0 : INFINITY;
      else R = dm / ((double)steps_since * um2);
      o[CS_RESIDUAL] = R;
    }
  }
}

// Generalised periodic boundaries (Sec. II.B), applied to the state a step
// has just written: a population that the next pull carries across the
// period (+x out of the outlet column x = nx-1 into the inlet, -x out of the
// inlet column into the outlet) becomes the equilibrium at the far end's
// density plus its own non-equilibrium part. With the moments (rho, j) of its
// source node, a density shift d = p+-/cs2 - mean column density adds
// a_i [d + (4.5 (c.j)^2 - 1.5 j^2) (1/(rho + d) - 1/rho)]. Diagonal links
// that meet a wall are reflected, not carried, and stay. One workgroup per
// channel; the column means are taken before anything is changed.
template <typename T, bool SHIFT>
__global__ void __launch_bounds__(256) gpbc_kernel(T *B, const ChanDev *ch, int k, const float *uref) {
  const ChanDev c = ch[blockIdx.x];
  if (!c.gpbc || !c.active) return;
  const long long t = c.t + k;
  const double dp = (t < c.t_startup) ? c.pd : 0.0;
  const int nx = c.nx, ny = c.ny;
  auto node = [&](int x, int y) -> long long { return c.off + (long long)y * nx + x; };
  // density and momentum of a node (FP32: stored relative to the equilibrium
  // at density 1 and the row's reference velocity, which carries momentum ur)
  auto load9 = [&](long long n, int y, double f[9], double &rho, double &jx, double &jy) {
    double s = 0;
    jx = jy = 0;
    for (int i = 0; i < 9; ++i) {
      f[i] = (double)B[slot(i, n)];
      s += f[i];
    }
    jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
    jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
    if (SHIFT) jx += (double)uref[c.row_off + y];
    rho = SHIFT ? 1.0 + s : s;
  };
  __shared__ double red[2][256];
  double si = 0, so = 0;
  for (int y = threadIdx.x; y < ny; y += blockDim.x) {
    double f[9], r, jx, jy;
    load9(node(0, y), y, f, r, jx, jy);
    si += r;
    load9(node(nx - 1, y), y, f, r, jx, jy);
    so += r;
  }
  red[0][threadIdx.x] = si;
  red[1][threadIdx.x] = so;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      red[0][threadIdx.x] += red[0][threadIdx.x + st];
      red[1][threadIdx.x] += red[1][threadIdx.x + st];
    }
    __syncthreads();
  }
  const double d_in = 1.0 + 1.5 * dp - red[1][0] / ny;   // links entering the inlet
  const double d_out = 1.0 - 1.5 * dp - red[0][0] / ny;  // links entering the outlet
  auto fix = [&](long long n, double d, int i0, int i1, int i2, int y) {
    double f[9], r, jx, jy;
    load9(n, y, f, r, jx, jy);
    const double j2 = jx * jx + jy * jy, w = 1.0 / (r + d) - 1.0 / r;
    const int ids[3] = {i0, i1, i2};
    for (int q = 0; q < 3; ++q) {
      const int i = ids[q];
      const int cy = (i == 5 || i == 6) ? 1 : ((i == 7 || i == 8) ? -1 : 0);
      if (y + cy < 0 || y + cy >= ny) continue;  // met a wall: reflected
      const double cx = (i == 1 || i == 5 || i == 8) ? 1.0 : -1.0;
      const double cj = cx * jx + cy * jy;
      const double a = (i < 5) ? 1.0 / 9.0 : 1.0 / 36.0;
      B[slot(i, n)] = (T)(f[i] + a * (d + (4.5 * cj * cj - 1.5 * j2) * w));
    }
  };
  for (int y = threadIdx.x; y < ny; y += blockDim.x) {
    fix(node(nx - 1, y), d_in, 1, 5, 8, y);
    fix(node(0, y), d_out, 3, 6, 7, y);
  }
}

// FP32 storage: moves the reference velocity of every row of the active
// channels to the row's current x-averaged u_x (prof, from the last
// observation) and restates the stored populations of the row: a value
// stored relative to E_i(uo) becomes one relative to E_i(un) by adding
// E_i(uo) - E_i(un), formed as a difference. One workgroup per row.
__global__ void __launch_bounds__(256) rereference_kernel(float *A, const ChanDev *ch, int n_ch,
                                                          const double *prof, float *uref) {
  const int r = blockIdx.x;  // row over all channels
  int lo = 0, hi = n_ch - 1;
  while (lo < hi) {  // the channel holding row r: last one with row_off <= r
    const int mid = (lo + hi + 1) / 2;
    if (ch[mid].row_off <= r) lo = mid;
    else hi = mid - 1;
  }
  const ChanDev c = ch[lo];
  if (!c.active) return;
  const float uo = uref[r];
  const double unx = prof[(long long)r * OF_COUNT + OF_UX];
  if (!(unx == unx) || fabs(unx) > 1.0) return;  // not finite or not a velocity: keep the old one
  const float un = (float)unx;
  float d[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const float cx = (i == 1 || i == 5 || i == 8) ? 1.f : ((i == 3 || i == 6 || i == 7) ? -1.f : 0.f);
    d[i] = ref_shift(weight<float>(i), cx, uo, un);
  }
  const int y = r - c.row_off;
  for (int x = threadIdx.x; x < c.nx; x += blockDim.x) {
    const long long n = c.off + (long long)y * c.nx + x;
#pragma unroll
    for (int i = 0; i < 9; ++i) A[slot(i, n)] += d[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) uref[r] = un;
}

// ---------------------------------------------------------------------------
// Stress as a force density (FP64, instantaneous model): the divergence of
// the non-Newtonian stress enters as an external force in Eq. (ns), the
// alternative Sec. II.C names. A step forms u~ at every node, Sigma^nN from
// the neighbours' u~, then collides with the force f = rho0 g + div Sigma^nN
// (central differences, ghost rows extrapolated linearly through the walls)
// in the body-force terms of the forcing. The step runs as one fused kernel
// over tiles (saf_fused_kernel); observation runs the same stages as
// node-wise passes over every channel, with scratch U (u~_x, u~_y) and T
// (Sigma^nN xx, xy, yy), plane-major over the nodes of the buffer.

// Channel holding node n (channels are laid out by increasing offset).
__device__ __forceinline__ int channel_of_node(const ChanDev *ch, int n_ch, long long n) {
  int lo = 0, hi = n_ch - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (ch[mid].off <= n) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

struct SafNode {
  ChanDev c;
  int x, y;
  long long t;
};

// Decodes node n; false for padding nodes and (unless all) frozen channels.
__device__ __forceinline__ bool saf_node(const ChanDev *ch, int n_ch, long long n, int k, bool all, SafNode &s) {
  s.c = ch[channel_of_node(ch, n_ch, n)];
  const long long loc = n - s.c.off;
  if (loc < 0 || loc >= (long long)s.c.nx * s.c.ny) return false;
  if (!all && !s.c.active) return false;
  s.y = (int)(loc / s.c.nx);
  s.x = (int)(loc - (long long)s.y * s.c.nx);
  s.t = s.c.t + k;
  return true;
}

// x and y neighbours' values of a node field F (plane-major, plane nodes),
// with the ghost rule of the caller.
__global__ void __launch_bounds__(256) saf_u_kernel(const double *__restrict__ A, const ChanDev *ch, int n_ch,
                                                    long long plane, int k, int all, double *__restrict__ U) {
  for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < plane;
       n += (long long)gridDim.x * blockDim.x) {
    SafNode q;
    if (!saf_node(ch, n_ch, n, k, all, q)) continue;
    const double g = (q.t < q.c.t_startup) ? q.c.g : 0.0;
    const double uw6 = (q.t >= 1 && q.t - 1 < q.c.t_startup) ? q.c.uw / 6.0 : 0.0;
    double f[9], sd, mx, my;
    pull<double>(A, q.c.off + (long long)q.y * q.c.nx, q.c.nx, q.c.ny, q.x, q.y, uw6, f);
    moments<double>(f, sd, mx, my);
    U[n] = (mx + 0.5 * g) / sd;
    U[plane + n] = my / sd;
  }
}

// kappa_ab = d_b u~_a of a node by central differences (x periodic; wall
// ghosts -u~ below, 2 u_w - u~ above for x, -u~ for y).
__device__ __forceinline__ void saf_kappa(const double *__restrict__ U, long long plane, const SafNode &q,
                                          double &kxx, double &kxy, double &kyx, double &kyy) {
  const ChanDev &c = q.c;
  const long long row = c.off + (long long)q.y * c.nx;
  const long long n = row + q.x;
  const int xm = (q.x == 0) ? c.nx - 1 : q.x - 1, xp = (q.x == c.nx - 1) ? 0 : q.x + 1;
  const double uwg = (q.t < c.t_startup) ? c.uw : 0.0;
  const double ux = U[n], uy = U[plane + n];
  const double uxd = (q.y > 0) ? U[n - c.nx] : -ux, uyd = (q.y > 0) ? U[plane + n - c.nx] : -uy;
  const double uxu = (q.y < c.ny - 1) ? U[n + c.nx] : 2.0 * uwg - ux;
  const double uyu = (q.y < c.ny - 1) ? U[plane + n + c.nx] : -uy;
  kxx = 0.5 * (U[row + xp] - U[row + xm]);
  kxy = 0.5 * (uxu - uxd);
  kyx = 0.5 * (U[plane + row + xp] - U[plane + row + xm]);
  kyy = 0.5 * (uyu - uyd);
}

__global__ void __launch_bounds__(256) saf_stress_kernel(const ChanDev *ch, int n_ch, long long plane, int k,
                                                         int all, const double *__restrict__ U,
                                                         double *__restrict__ Tn) {
  for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < plane;
       n += (long long)gridDim.x * blockDim.x) {
    SafNode q;
    if (!saf_node(ch, n_ch, n, k, all, q)) continue;
    double kxx, kxy, kyx, kyy;
    saf_kappa(U, plane, q, kxx, kxy, kyx, kyy);
    const Coef<double> cf(q.c);
    double sxx = 0, sxy = 0, syy = 0;
    if (cf.stress_on) inlm_stress<double>(kxx, kxy, kyx, kyy, cf, sxx, sxy, syy);
    Tn[n] = sxx - cf.lgt * 2.0 * kxx;
    Tn[plane + n] = sxy - cf.lgt * (kxy + kyx);
    Tn[2 * plane + n] = syy - cf.lgt * 2.0 * kyy;
  }
}

// f_Sigma = div Sigma^nN at a node: central differences, x periodic, ghost
// rows Sigma(-1) = 2 Sigma(0) - Sigma(1), Sigma(ny) = 2 Sigma(ny-1) -
// Sigma(ny-2) (one row: zero gradient).
__device__ __forceinline__ void saf_force(const double *__restrict__ Tn, long long plane, const SafNode &q,
                                          double &fsx, double &fsy) {
  const ChanDev &c = q.c;
  const long long row = c.off + (long long)q.y * c.nx;
  const long long n = row + q.x;
  const int xm = (q.x == 0) ? c.nx - 1 : q.x - 1, xp = (q.x == c.nx - 1) ? 0 : q.x + 1;
  double dn[3], up[3];
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    const double *P = Tn + p * plane;
    if (c.ny == 1) {
      dn[p] = up[p] = P[n];
    } else {
      dn[p] = (q.y > 0) ? P[n - c.nx] : 2.0 * P[n] - P[n + c.nx];
      up[p] = (q.y < c.ny - 1) ? P[n + c.nx] : 2.0 * P[n] - P[n - c.nx];
    }
  }
  fsx = 0.5 * (Tn[row + xp] - Tn[row + xm]) + 0.5 * (up[1] - dn[1]);
  fsy = 0.5 * (Tn[plane + row + xp] - Tn[plane + row + xm]) + 0.5 * (up[2] - dn[2]);
}

// One step of the stress-force path fused in one kernel, one workgroup per
// tile of kSafTX x kSafTY output nodes, each thread taking a column of
// kSafNPT of them (kSafRows rows apart): the taller tile repeats less of
// the ring work per node than one node per thread would, at the same
// number of wavefronts per CU. Each XCD takes a contiguous run of the tile
// list, which the host orders so that a run is a block of neighbouring
// tiles: adjacent tiles share the halo populations they pull and then find
// them in that XCD's L2. Each thread pulls its nodes and keeps the
// populations; u~ of the tile and of a ring of two nodes around it go to
// LDS, then Sigma^nN of the tile and a ring of one node, then each thread
// collides its nodes with div Sigma^nN from LDS. Columns wrap (x periodic; narrow channels repeat columns); rows
// outside the channel are the wall ghosts of saf_kappa and saf_force. The
// arithmetic is that of the three separate passes.
constexpr int kSafTX = kSafTileX, kSafTY = kSafTileY;
constexpr int kSafRows = kSafThreads / kSafTX;            // rows of threads
constexpr int kSafNPT = kSafTY / kSafRows;                // output nodes per thread
constexpr int kSafUX = kSafTX + 4, kSafUY = kSafTY + 4;  // u~ region
constexpr int kSafSX = kSafTX + 2, kSafSY = kSafTY + 2;  // Sigma^nN region
constexpr int kSafRing = 4 * kSafUX + 4 * kSafTY;       // u~ region minus the tile
static_assert(kSafRows * kSafTX == kSafThreads && kSafNPT * kSafRows == kSafTY,
              "a whole column of output nodes per thread");
static_assert(kSafRing <= kSafThreads, "at most one ring node per thread");

template <bool NT>
__global__ void __launch_bounds__(kSafThreads) saf_fused_kernel(const double *__restrict__ A,
                                                                double *__restrict__ B, const ChanDev *ch,
                                                                const Strip *tiles, int k) {
  __shared__ double su[2][kSafUY][kSafUX];
  __shared__ double sT[3][kSafSY][kSafSX];
  constexpr int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  constexpr int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  const Strip tl = tiles[xcd_item(blockIdx.x, gridDim.x)];
  const ChanDev c = ch[tl.ch];
  if (!c.active) return;  // frozen channel (uniform over the workgroup)
  const int nx = c.nx, ny = c.ny;
  const long long t = c.t + k;
  const double g = (t < c.t_startup) ? c.g : 0.0;
  const double uwg = (t < c.t_startup) ? c.uw : 0.0;
  const double uw6 = (!c.zh && t >= 1 && t - 1 < c.t_startup) ? c.uw / 6.0 : 0.0;
  const Coef<double> cf(c);
  const double *__restrict__ Ac = A + c.off * kPlanes;
  double *__restrict__ Bc = B + c.off * kPlanes;
  const bool wide = nx >= kSafTX + 4;  // then halo columns wrap at most once
  auto wrapx = [&](int x) {
    if (wide) return x < 0 ? x + nx : (x >= nx ? x - nx : x);
    const int r = x % nx;
    return r < 0 ? r + nx : r;
  };
  auto clampy = [&](int y) { return y < 0 ? 0 : (y >= ny ? ny - 1 : y); };
  // This thread's nodes (a column of kSafNPT, kSafRows rows apart), whose
  // populations it keeps to the collision, and (threads below kSafRing) one
  // node of the ring of two around the tile: two rows below, two above, two
  // columns on either side. All are pulled before any is used, so that
  // their loads overlap; rows outside the channel pull a row inside and
  // store nothing.
  const int jo = threadIdx.x / kSafTX, io = threadIdx.x - jo * kSafTX;
  const int xo = tl.x0 + io, xw = wrapx(xo);
  const int h = threadIdx.x;
  int hj, hi;
  if (h < 2 * kSafUX) {
    hj = h / kSafUX;
    hi = h - hj * kSafUX;
  } else if (h < 4 * kSafUX) {
    const int r = h - 2 * kSafUX;
    hj = kSafTY + 2 + r / kSafUX;
    hi = r % kSafUX;
  } else {
    const int r = h - 4 * kSafUX, side = r & 3;
    hj = 2 + (r >> 2);
    hi = side < 2 ? side : kSafUX - 4 + side;
  }
  const int hy = tl.y0 - 2 + hj;
  const bool ring = h < kSafRing;
  double f[kSafNPT][9], fh[9], Pc[kSafNPT];
  unsigned m[kSafNPT];
#pragma unroll
  for (int s = 0; s < kSafNPT; ++s) {
    const int yc = clampy(tl.y0 + jo + s * kSafRows);
    m[s] = (unsigned)yc * nx + xw;
    pull_local(Ac, nx, ny, xw, yc, uw6, f[s]);
    Pc[s] = Ac[lslot(9, m[s])];
  }
  if (ring) pull_local(Ac, nx, ny, wrapx(tl.x0 - 2 + hi), clampy(hy), uw6, fh);
  double sd[kSafNPT], mx[kSafNPT], my[kSafNPT], inv[kSafNPT];
#pragma unroll
  for (int s = 0; s < kSafNPT; ++s) {
    moments<double>(f[s], sd[s], mx[s], my[s]);
    inv[s] = recip<double>(sd[s]);  // shared with the collision
    if (tl.y0 + jo + s * kSafRows < ny) {
      const U2<double> u = u_tilde<double, false>(sd[s], mx[s], my[s], g, 0.0);
      su[0][jo + s * kSafRows + 2][io + 2] = u.x;
      su[1][jo + s * kSafRows + 2][io + 2] = u.y;
    }
  }
  if (ring && hy >= 0 && hy < ny) {
    double hs, hx, hv;
    moments<double>(fh, hs, hx, hv);
    const U2<double> u = u_tilde<double, false>(hs, hx, hv, g, 0.0);
    su[0][hj][hi] = u.x;
    su[1][hj][hi] = u.y;
  }
  __syncthreads();
  // Sigma^nN of the tile and a ring of one node (kappa with the wall ghosts)
  for (int i = threadIdx.x; i < kSafSX * kSafSY; i += kSafThreads) {
    const int j = i / kSafSX, ii = i - j * kSafSX;
    const int y = tl.y0 - 1 + j;
    if (y < 0 || y >= ny) continue;
    const int ju = j + 1, iu = ii + 1;
    const double ux = su[0][ju][iu], uy = su[1][ju][iu];
    const double uxd = (y > 0) ? su[0][ju - 1][iu] : -ux, uyd = (y > 0) ? su[1][ju - 1][iu] : -uy;
    const double uxu = (y < ny - 1) ? su[0][ju + 1][iu] : 2.0 * uwg - ux;
    const double uyu = (y < ny - 1) ? su[1][ju + 1][iu] : -uy;
    const double kxx = 0.5 * (su[0][ju][iu + 1] - su[0][ju][iu - 1]);
    const double kxy = 0.5 * (uxu - uxd);
    const double kyx = 0.5 * (su[1][ju][iu + 1] - su[1][ju][iu - 1]);
    const double kyy = 0.5 * (uyu - uyd);
    double sxx = 0, sxy = 0, syy = 0;
    if (cf.stress_on) inlm_stress<double>(kxx, kxy, kyx, kyy, cf, sxx, sxy, syy);
    sT[0][j][ii] = sxx - cf.lgt * 2.0 * kxx;
    sT[1][j][ii] = sxy - cf.lgt * (kxy + kyx);
    sT[2][j][ii] = syy - cf.lgt * 2.0 * kyy;
  }
  __syncthreads();
  // collide and stream this thread's nodes
  if (xo >= nx) return;
#pragma unroll
  for (int s = 0; s < kSafNPT; ++s) {
    const int yo = tl.y0 + jo + s * kSafRows;
    if (yo >= tl.y1) continue;
    const int js = jo + s * kSafRows + 1, is = io + 1;
    double dn[3], up[3];
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      const double Tc = sT[p][js][is];
      if (ny == 1) {
        dn[p] = up[p] = Tc;
      } else {
        dn[p] = (yo > 0) ? sT[p][js - 1][is] : 2.0 * Tc - sT[p][js + 1][is];
        up[p] = (yo < ny - 1) ? sT[p][js + 1][is] : 2.0 * Tc - sT[p][js - 1][is];
      }
    }
    const double fsx = 0.5 * (sT[0][js][is + 1] - sT[0][js][is - 1]) + 0.5 * (up[1] - dn[1]);
    const double fsy = 0.5 * (sT[1][js][is + 1] - sT[1][js][is - 1]) + 0.5 * (up[2] - dn[2]);
    const double fx = g + fsx, fy = fsy;
    const double ux = (mx[s] + 0.5 * fx) * inv[s], uy = (my[s] + 0.5 * fy) * inv[s];
    const double usq = ux * ux + uy * uy, uf = ux * fx + uy * fy;
    const double om = c.omega, kf = c.kf;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const double cu = cx[q] * ux + cy[q] * uy, cfo = cx[q] * fx + cy[q] * fy;
      const double a = weight<double>(q);
      const double neq = a * sd[s] * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
      const double F = a * kf * (3.0 * cfo + 9.0 * cu * cfo - 3.0 * uf);
      const double v = f[s][q] - om * (f[s][q] - neq) + F;
      if constexpr (NT) __builtin_nontemporal_store(v, &Bc[lslot(q, m[s])]);
      else Bc[lslot(q, m[s])] = v;
    }
    if constexpr (NT) __builtin_nontemporal_store(Pc[s], &Bc[lslot(9, m[s])]);
    else Bc[lslot(9, m[s])] = Pc[s];
  }
}

// Observation of the stress-force path: one workgroup per row of every
// channel; the row sums go to the row's first x-strip partial (the others
// are zeroed) for reduce_kernel.
__global__ void __launch_bounds__(256) saf_observe_kernel(const double *__restrict__ A, const ChanDev *ch,
                                                          int n_ch, long long plane, const double *__restrict__ U,
                                                          const double *__restrict__ Tn, double *part) {
  __shared__ double red[OF_COUNT][256];
  const int r = blockIdx.x;
  int lo = 0, hi = n_ch - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (ch[mid].row_off <= r) lo = mid;
    else hi = mid - 1;
  }
  const ChanDev c = ch[lo];
  SafNode q;
  q.c = c;
  q.y = r - c.row_off;
  q.t = c.t;
  double acc[OF_COUNT];
#pragma unroll
  for (int f = 0; f < OF_COUNT; ++f) acc[f] = 0.0;
  const double g = (q.t < c.t_startup) ? c.g : 0.0;
  const double uw6 = (q.t >= 1 && q.t - 1 < c.t_startup) ? c.uw / 6.0 : 0.0;
  const Coef<double> cf(c);
  for (int x = threadIdx.x; x < c.nx; x += blockDim.x) {
    q.x = x;
    const long long n = c.off + (long long)q.y * c.nx + x;
    double f[9], sd, mx, my;
    pull<double>(A, c.off + (long long)q.y * c.nx, c.nx, c.ny, x, q.y, uw6, f);
    moments<double>(f, sd, mx, my);
    double kxx, kxy, kyx, kyy, fsx, fsy;
    saf_kappa(U, plane, q, kxx, kxy, kyx, kyy);
    saf_force(Tn, plane, q, fsx, fsy);
    double sxx = 0, sxy = 0, syy = 0;
    if (cf.stress_on) inlm_stress<double>(kxx, kxy, kyx, kyy, cf, sxx, sxy, syy);
    acc[OF_UX] += (mx + 0.5 * (g + fsx)) / sd;
    acc[OF_UY] += (my + 0.5 * fsy) / sd;
    acc[OF_SXX] += sxx;
    acc[OF_SXY] += sxy;
    acc[OF_SYY] += syy;
    acc[OF_RHOE_DEV] += sd - 1.0;
    acc[OF_MASS_DEV] += sd - 1.0;
    acc[OF_MOMX] += mx;
    acc[OF_KXY] += kxy;
    acc[OF_TRT] += Tn[n] + Tn[2 * plane + n];
    acc[OF_DRAG] += wall_drag<double>(f, q.y, c.ny, uw6, false, 0.0);
    acc[OF_KXX] += kxx;
  }
#pragma unroll
  for (int f = 0; f < OF_COUNT; ++f) red[f][threadIdx.x] = acc[f];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st)
      for (int f = 0; f < OF_COUNT; ++f) red[f][threadIdx.x] += red[f][threadIdx.x + st];
    __syncthreads();
  }
  double *dst = part + ((long long)c.poff + (long long)q.y * c.nxs) * OF_COUNT;
  for (int i = threadIdx.x; i < c.nxs * OF_COUNT; i += blockDim.x) dst[i] = (i < OF_COUNT) ? red[i][0] : 0.0;
}

__global__ void advance_kernel(ChanDev *ch, int n_ch, int steps) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_ch && ch[i].active) ch[i].t += steps;
}

template <typename T, bool SHIFT, int TXW, bool WIDE, bool VE>
hipError_t launch_cls(bool observe, const SweepArgs &a, hipStream_t s) {
  if (a.n_strips == 0) return hipSuccess;
  dim3 grid(a.n_wg), block(64 * LB_WG_WAVES);
  if (observe)
    hipLaunchKernelGGL((sweep_kernel<T, SHIFT, TXW, WIDE, true, VE>), grid, block, 0, s, a);
  else
    hipLaunchKernelGGL((sweep_kernel<T, SHIFT, TXW, WIDE, false, VE>), grid, block, 0, s, a);
  return hipGetLastError();
}

template <typename T, bool SHIFT, bool VE>
hipError_t launch_wide64(bool observe, const SweepArgs &a, hipStream_t s) {
  if (a.n_strips == 0) return hipSuccess;
  dim3 grid(a.n_wg), block(64 * LB_WG_WAVES);
  if (observe)
    hipLaunchKernelGGL((sweep_wide64_kernel<T, SHIFT, true, VE>), grid, block, 0, s, a);
  else
    hipLaunchKernelGGL((sweep_wide64_kernel<T, SHIFT, false, VE>), grid, block, 0, s, a);
  return hipGetLastError();
}

template <typename T, bool SHIFT, bool VE>
hipError_t launch_vec(bool observe, const SweepArgs &a, hipStream_t s) {
  if (a.n_strips == 0) return hipSuccess;
  constexpr int NPL = sizeof(T) == 4 ? LB_VEC_NPL32 : LB_VEC_NPL64;
  dim3 grid(a.n_wg), block(64 * LB_WG_WAVES);
  if (observe)
    hipLaunchKernelGGL((sweep_vec_kernel<T, SHIFT, true, NPL, false, VE, true>), grid, block, 0, s, a);
  else if (a.zh && a.nt)
    hipLaunchKernelGGL((sweep_vec_kernel<T, SHIFT, false, NPL, true, VE, true>), grid, block, 0, s, a);
  else if (a.zh)
    hipLaunchKernelGGL((sweep_vec_kernel<T, SHIFT, false, NPL, false, VE, true>), grid, block, 0, s, a);
  else if (a.nt)
    hipLaunchKernelGGL((sweep_vec_kernel<T, SHIFT, false, NPL, true, VE, false>), grid, block, 0, s, a);
  else
    hipLaunchKernelGGL((sweep_vec_kernel<T, SHIFT, false, NPL, false, VE, false>), grid, block, 0, s, a);
  return hipGetLastError();
}

template <typename T, bool SHIFT, bool VE>
hipError_t launch_model(int cls, bool observe, const SweepArgs &a, hipStream_t s) {
  switch (cls) {
    case 0: return launch_cls<T, SHIFT, 1, false, VE>(observe, a, s);
    case 1: return launch_cls<T, SHIFT, 2, false, VE>(observe, a, s);
    case 2: return launch_cls<T, SHIFT, 4, false, VE>(observe, a, s);
    case 3: return launch_cls<T, SHIFT, 8, false, VE>(observe, a, s);
    case 4: return launch_cls<T, SHIFT, 16, false, VE>(observe, a, s);
    case 5: return launch_cls<T, SHIFT, 32, false, VE>(observe, a, s);
    case 6: return launch_cls<T, SHIFT, 64, false, VE>(observe, a, s);
    case kWide64Class: return launch_wide64<T, SHIFT, VE>(observe, a, s);
    case kVecClass: return launch_vec<T, SHIFT, VE>(observe, a, s);
    default: return launch_cls<T, SHIFT, 64, true, VE>(observe, a, s);
  }
}

template <typename T, bool SHIFT>
hipError_t launch_prec(int cls, bool observe, const SweepArgs &a, hipStream_t s) {
  if (a.ve) {
    if (!a.SA || !a.SB) return hipErrorInvalidValue;
    return launch_model<T, SHIFT, true>(cls, observe, a, s);
  }
  return launch_model<T, SHIFT, false>(cls, observe, a, s);
}

}  // namespace

hipError_t launch_sweep(int fp32, int cls, bool observe, const SweepArgs &a, hipStream_t s) {
  return fp32 ? launch_prec<float, true>(cls, observe, a, s)
              : launch_prec<double, false>(cls, observe, a, s);
}

hipError_t launch_tiles(const SweepArgs &a, hipStream_t s) {
  if (a.n_strips == 0) return hipSuccess;
  const dim3 grid(a.n_strips), block(kMainThreads);
  if (a.ve) {
    if (a.nt) hipLaunchKernelGGL((sweep_tile_kernel<true, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((sweep_tile_kernel<true, false>), grid, block, 0, s, a);
  } else {
    if (a.nt) hipLaunchKernelGGL((sweep_tile_kernel<false, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((sweep_tile_kernel<false, false>), grid, block, 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_reduce(const ChanDev *ch, int n_ch, const double *part, double *prof,
                         double *prev_ux, double *scal, const float *uref, int update_residual,
                         int steps_since, hipStream_t s) {
  if (n_ch == 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_kernel, dim3(n_ch), dim3(256), 0, s, ch, part, prof, prev_ux, scal, uref,
                     update_residual, steps_since);
  return hipGetLastError();
}

hipError_t launch_gpbc(int fp32, void *B, const ChanDev *ch, int n_ch, int k, const float *uref, hipStream_t s) {
  if (n_ch == 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL((gpbc_kernel<float, true>), dim3(n_ch), dim3(256), 0, s, static_cast<float *>(B), ch, k,
                       uref);
  else
    hipLaunchKernelGGL((gpbc_kernel<double, false>), dim3(n_ch), dim3(256), 0, s, static_cast<double *>(B), ch,
                       k, uref);
  return hipGetLastError();
}

template <typename T, int NPL, bool VE>
void launch_two_step_t(const SweepArgs &a, hipStream_t s) {
  const dim3 grid(a.n_wg), block(64 * kTwoStepWaves);
  if (a.wall) {
    if (a.nt) hipLaunchKernelGGL((sweep_vec2_kernel<T, NPL, true, VE, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((sweep_vec2_kernel<T, NPL, false, VE, true>), grid, block, 0, s, a);
  } else {
    if (a.nt) hipLaunchKernelGGL((sweep_vec2_kernel<T, NPL, true, VE, false>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((sweep_vec2_kernel<T, NPL, false, VE, false>), grid, block, 0, s, a);
  }
}

hipError_t launch_narrow_two_step(bool fp32, int nx, const SweepArgs &a, hipStream_t s) {
  if (a.n_strips == 0) return hipSuccess;
  const dim3 grid(a.n_wg), block(128);
#define LB_N2(TT, SH, W) hipLaunchKernelGGL((sweep_narrow2_kernel<TT, SH, W>), grid, block, 0, s, a)
#define LB_N2_ALL(TT, SH)  \
  switch (nx) {            \
    case 1: LB_N2(TT, SH, 1); break;   \
    case 2: LB_N2(TT, SH, 2); break;   \
    case 4: LB_N2(TT, SH, 4); break;   \
    case 8: LB_N2(TT, SH, 8); break;   \
    case 16: LB_N2(TT, SH, 16); break; \
    case 32: LB_N2(TT, SH, 32); break; \
    case 64: LB_N2(TT, SH, 64); break; \
    default: return hipErrorInvalidValue; \
  }
  if (fp32) {
    LB_N2_ALL(float, true)
  } else {
    LB_N2_ALL(double, false)
  }
#undef LB_N2_ALL
#undef LB_N2
  return hipGetLastError();
}

template <typename T, bool SH>
int narrow2_blocks_per_cu() {
  int lo = 1 << 30;
  auto q = [&](const void *f) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, 128, 0) == hipSuccess && n > 0) lo = std::min(lo, n);
  };
  q(reinterpret_cast<const void *>(sweep_narrow2_kernel<T, SH, 1>));
  q(reinterpret_cast<const void *>(sweep_narrow2_kernel<T, SH, 2>));
  q(reinterpret_cast<const void *>(sweep_narrow2_kernel<T, SH, 4>));
  q(reinterpret_cast<const void *>(sweep_narrow2_kernel<T, SH, 8>));
  q(reinterpret_cast<const void *>(sweep_narrow2_kernel<T, SH, 16>));
  q(reinterpret_cast<const void *>(sweep_narrow2_kernel<T, SH, 32>));
  q(reinterpret_cast<const void *>(sweep_narrow2_kernel<T, SH, 64>));
  return lo == (1 << 30) ? 1 : lo;
}

int narrow_two_step_blocks_per_cu(bool fp32) {
  return fp32 ? narrow2_blocks_per_cu<float, true>() : narrow2_blocks_per_cu<double, false>();
}

hipError_t launch_two_step(bool fp32, const SweepArgs &a, hipStream_t s) {
  if (a.n_strips == 0) return hipSuccess;
  if (a.ve && (!a.SA || !a.SB)) return hipErrorInvalidValue;
  const int npl = two_step_npl(fp32, a.nt, a.ve);
  if (fp32 && npl == 4) {
    launch_two_step_t<float, 4, false>(a, s);
  } else if (fp32) {
    if (a.ve) launch_two_step_t<float, 2, true>(a, s);
    else launch_two_step_t<float, 2, false>(a, s);
  } else {
    if (a.ve) launch_two_step_t<double, 2, true>(a, s);
    else launch_two_step_t<double, 2, false>(a, s);
  }
  return hipGetLastError();
}

int two_step_blocks_per_cu(bool fp32, bool nt, bool ve) {
  int n = 0;
  constexpr int b = 64 * kTwoStepWaves;
  hipError_t e;
  if (fp32 && two_step_npl(fp32, nt, ve) == 4)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, sweep_vec2_kernel<float, 4, true, false, false>, b, 0);
  else if (fp32)
    e = ve ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, sweep_vec2_kernel<float, 2, false, true, false>, b, 0)
           : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, sweep_vec2_kernel<float, 2, false, false, false>, b, 0);
  else
    e = ve ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, sweep_vec2_kernel<double, 2, false, true, false>, b, 0)
           : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, sweep_vec2_kernel<double, 2, false, false, false>, b, 0);
  return (e == hipSuccess && n > 0) ? n : 1;
}

hipError_t launch_rereference(float *A, const ChanDev *ch, int n_ch, int total_rows, const double *prof,
                              float *uref, hipStream_t s) {
  if (n_ch == 0 || total_rows == 0) return hipSuccess;
  hipLaunchKernelGGL(rereference_kernel, dim3(total_rows), dim3(256), 0, s, A, ch, n_ch, prof, uref);
  return hipGetLastError();
}

static int saf_blocks(long long plane) {
  const long long b = (plane + 255) / 256;
  return (int)(b < 16384 ? b : 16384);
}

hipError_t launch_saf_fused(const double *A, double *B, const ChanDev *ch, const Strip *tiles, int n_tiles, int k,
                            int nt, hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
  if (nt) hipLaunchKernelGGL(saf_fused_kernel<true>, dim3(n_tiles), dim3(kSafThreads), 0, s, A, B, ch, tiles, k);
  else hipLaunchKernelGGL(saf_fused_kernel<false>, dim3(n_tiles), dim3(kSafThreads), 0, s, A, B, ch, tiles, k);
  return hipGetLastError();
}

hipError_t launch_saf_observe(const double *A, const ChanDev *ch, int n_ch, long long plane, int total_rows,
                              double *U, double *Tn, double *part, hipStream_t s) {
  if (n_ch == 0 || plane == 0 || total_rows == 0) return hipSuccess;
  const int nb = saf_blocks(plane);
  hipLaunchKernelGGL(saf_u_kernel, dim3(nb), dim3(256), 0, s, A, ch, n_ch, plane, 0, 1, U);
  hipLaunchKernelGGL(saf_stress_kernel, dim3(nb), dim3(256), 0, s, ch, n_ch, plane, 0, 1, U, Tn);
  hipLaunchKernelGGL(saf_observe_kernel, dim3(total_rows), dim3(256), 0, s, A, ch, n_ch, plane, U, Tn, part);
  return hipGetLastError();
}

hipError_t launch_advance(ChanDev *ch, int n_ch, int steps, hipStream_t s) {
  if (n_ch == 0 || steps == 0) return hipSuccess;
  hipLaunchKernelGGL(advance_kernel, dim3((n_ch + 255) / 256), dim3(256), 0, s, ch, n_ch, steps);
  return hipGetLastError();
}

}  // namespace lbnlm
