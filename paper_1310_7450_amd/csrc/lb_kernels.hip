// gfx950 kernels of lbnlm: the fused pull / velocity-gradient / inlM stress /
// forcing / BGK sweep, its observation variant, the per-channel FP64
// reduction and the step-counter advance.
//
// Layout: structure of arrays, ten planes (nine populations in the order
// (0,0),(1,0),(0,1),(-1,0),(0,-1),(1,1),(-1,1),(-1,-1),(1,-1), then the
// previous stress trace), each plane holding every channel's nodes row by
// row (x fastest). A plane slot holds the post-collision population of the
// previous step at its source node; the sweep pulls it along the lattice
// velocity (Sec. II.A, Eq. (lbupdate)), or from the same node with the
// opposite velocity where the link crosses a wall (half-way bounce-back,
// Sec. II.B).
//
// One wavefront marches up a strip of rows. It keeps the provisional
// velocity u~ = j/sum_i n_i of three consecutive row blocks in registers, so
// the central differences of Sec. II.C need no LDS: x neighbours come from
// lane shuffles, y neighbours from the previous/next block. A narrow channel
// (nx a power of two up to 64) puts whole periods into lane groups of nx
// lanes; a wide channel runs 64-lane strips whose two edge lanes only
// supply the x halo.
#include "lb_internal.h"

namespace lbnlm {
namespace {

template <typename T>
__device__ __forceinline__ T shfl(T v, int src) {
  return __shfl(v, src, 64);
}

template <typename T>
__device__ __forceinline__ constexpr T weight(int i) {
  return i == 0 ? T(4.0 / 9.0) : (i < 5 ? T(1.0 / 9.0) : T(1.0 / 36.0));
}

// Pulls the nine post-streaming populations of node (x, y), 0 <= y < ny.
template <typename T>
__device__ __forceinline__ void pull(const T *__restrict__ A, long long P, long long row, int nx,
                                     int ny, int x, int y, T f[9]) {
  const int xm = (x == 0) ? nx - 1 : x - 1;
  const int xp = (x == nx - 1) ? 0 : x + 1;
  const long long dn = row - nx, up = row + nx;
  const bool bot = (y == 0), top = (y == ny - 1);
  f[0] = A[row + x];
  f[1] = A[1 * P + row + xm];
  f[3] = A[3 * P + row + xp];
  f[2] = A[bot ? (4 * P + row + x) : (2 * P + dn + x)];
  f[5] = A[bot ? (7 * P + row + x) : (5 * P + dn + xm)];
  f[6] = A[bot ? (8 * P + row + x) : (6 * P + dn + xp)];
  f[4] = A[top ? (2 * P + row + x) : (4 * P + up + x)];
  f[7] = A[top ? (5 * P + row + x) : (7 * P + up + xp)];
  f[8] = A[top ? (6 * P + row + x) : (8 * P + up + xm)];
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

// Wave-wide sum over a lane group of width GW (power of two).
template <int GW>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int m = 1; m < GW; m <<= 1) v += __shfl_xor(v, m, 64);
  return v;
}

template <typename T, bool SHIFT, int TXW, bool WIDE, bool OBS>
__global__ void __launch_bounds__(256) sweep_kernel(SweepArgs a) {
  constexpr int TYW = 64 / TXW;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // Spread consecutive work over one XCD: workgroup w runs on XCD w % 8,
  // and each XCD takes a contiguous range of strips (vertical neighbours
  // share halo rows through that XCD's L2).
  const int w = blockIdx.x;
  const int q = a.n_wg >> 3, rem = a.n_wg & 7, j = w & 7;
  const int L = j * q + (j < rem ? j : rem) + (w >> 3);
  const int sidx = L * 4 + wave;
  if (sidx >= a.n_strips) return;
  const Strip st = a.strips[sidx];
  const ChanDev c = a.ch[st.ch];
  const T *__restrict__ A = static_cast<const T *>(a.A);
  T *__restrict__ B = static_cast<T *>(a.B);
  const long long P = a.plane;
  const int nx = c.nx, ny = c.ny;
  const long long t = c.t + a.k;
  const T fx = (t < c.t_startup) ? T(c.g) : T(0);

  int lx, ly, x;
  bool colok;
  if (WIDE) {
    lx = lane;
    ly = 0;
    const int xr = st.x0 + lane - 1;
    x = ((xr % nx) + nx) % nx;
    colok = (lane >= 1) && (lane <= 62) && (xr < nx);
  } else {
    lx = lane & (TXW - 1);
    ly = lane / TXW;
    x = lx;
    colok = true;
  }
  const int left_src = WIDE ? lane - 1 : ly * TXW + ((lx + TXW - 1) & (TXW - 1));
  const int right_src = WIDE ? lane + 1 : ly * TXW + ((lx + 1) & (TXW - 1));
  const long long base = c.off;

  auto clampy = [&](int y) { return y < 0 ? 0 : (y >= ny ? ny - 1 : y); };
  auto load_u = [&](int y, T f[9], T &Pv) -> U2<T> {
    const int yc = clampy(y);
    const long long row = base + (long long)yc * nx;
    pull<T>(A, P, row, nx, ny, x, yc, f);
    Pv = A[9 * P + row + x];
    T sd, mx, my;
    moments<T>(f, sd, mx, my);
    const T inv = T(1) / (SHIFT ? T(1) + sd : sd);
    return U2<T>{(mx + T(0.5) * fx) * inv, my * inv};
  };

  T fc[9], fn[9], Pc, Pn;
  U2<T> uPrev, uCur, uNext;
  {
    T ftmp[9], Ptmp;
    uPrev = load_u(st.y0 - TYW + ly, ftmp, Ptmp);
  }
  uCur = load_u(st.y0 + ly, fc, Pc);

  const T om = T(c.omega), kf = T(c.kf), sp = T(c.sp), Gm = T(c.G);
  const T inv_tau = T(c.inv_tau), inv_gc = T(c.inv_gc), lgt = T(c.lgt);
  const bool stress_on = c.G > 0.0;

#pragma unroll 1
  for (int yb = st.y0; yb < st.y1; yb += TYW) {
    uNext = load_u(yb + TYW + ly, fn, Pn);
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
    const U2<T> lf = shfl2(uCur, left_src < 0 ? 0 : left_src);
    const U2<T> rt = shfl2(uCur, right_src > 63 ? 63 : right_src);
    // no-slip ghosts behind the half-way walls
    if (y == 0) dn = U2<T>{-uCur.x, -uCur.y};
    if (y == ny - 1) up = U2<T>{-uCur.x, -uCur.y};

    // Every lane computes; only valid lanes store. Lanes past the strip or
    // outside the channel read clamped rows and their results are dropped.
    const bool ok = (y < st.y1) && colok;

    // velocity gradient kappa_ab = d_b u_a (Sec. II.C)
    const T kxx = T(0.5) * (rt.x - lf.x);
    const T kxy = T(0.5) * (up.x - dn.x);
    const T kyx = T(0.5) * (rt.y - lf.y);
    const T kyy = T(0.5) * (up.y - dn.y);

    // inlM stress: tau_M of Eq. (nlmaxwell), then the steady series of
    // Eq. (sigtsum) through the relation it satisfies by Eq. (smalld),
    // sigma - tau_M (kappa sigma + sigma kappa^T) = G tau_M D, solved in
    // closed form (Cramer) for (sigma_xx, sigma_xy, sigma_yy).
    const T Dxx = T(2) * kxx, Dxy = kxy + kyx, Dyy = T(2) * kyy;
    T sxx = T(0), sxy = T(0), syy = T(0);
    if (stress_on) {
      const T II = T(0.5) * (Dxx * Dxx + T(2) * Dxy * Dxy + Dyy * Dyy);
      const T rate = inv_tau + sqrt(II) * inv_gc;
      if (rate > T(0)) {
        const T tM = T(1) / rate;
        const T ka = tM * kxx, kb = tM * kxy, kc = tM * kyx, kd = tM * kyy;
        const T gt = Gm * tM;
        const T r1 = gt * Dxx, r2 = gt * Dxy, r3 = gt * Dyy;
        const T m11 = T(1) - T(2) * ka, m12 = T(-2) * kb, m21 = -kc;
        const T m22 = T(1) - ka - kd, m23 = -kb, m32 = T(-2) * kc, m33 = T(1) - T(2) * kd;
        const T c11 = m22 * m33 - m23 * m32;
        const T det = m11 * c11 - m12 * m21 * m33;
        const T idet = T(1) / det;
        const T e2 = r2 * m33 - m23 * r3;
        sxx = (r1 * c11 - m12 * e2) * idet;
        sxy = (m11 * e2 - r1 * m21 * m33) * idet;
        syy = (m11 * (m22 * r3 - r2 * m32) - m12 * m21 * r3 + r1 * m21 * m32) * idet;
      }
    }
    // non-Newtonian stress carried by the forcing (viscosity split)
    const T Txx = sxx - lgt * Dxx, Txy = sxy - lgt * Dxy, Tyy = syy - lgt * Dyy;
    const T trT = Txx + Tyy;
    const T Sxx = T(0.5) * (Txx - Tyy);  // traceless part; Sbar_yy = -Sxx
    // Eq. (rhoplus): r = dt d(delta rho)/dt with delta rho = -tr Sigma^nN /(cs2 d)
    const T rr = a.nnp ? T(-1.5) * (trT - Pc) : T(0);

    T sd, mx, my;
    moments<T>(fc, sd, mx, my);
    const T jx = mx + T(0.5) * fx, jy = my;
    // Eq. (rhoj): the equilibrium density is sum (n* + n)/2 = s + r/2, carried
    // as its deviation from 1 in the shifted storage
    const T sdev = SHIFT ? sd : sd - T(1);
    const T rho_dev = sdev + T(0.5) * rr;
    const T rho_e = SHIFT ? T(1) + rho_dev : sd + T(0.5) * rr;
    const T irho = T(1) / rho_e;
    const T ux = jx * irho, uy = jy * irho;

    if (OBS) {
      double v[OF_COUNT];
      v[OF_UX] = (double)ux;
      v[OF_UY] = (double)uy;
      v[OF_SXX] = (double)sxx;
      v[OF_SXY] = (double)sxy;
      v[OF_SYY] = (double)syy;
      v[OF_RHOE_DEV] = (double)rho_dev;
      v[OF_MASS_DEV] = (double)sdev + (a.nnp ? 1.5 * (double)Pc : 0.0);
      v[OF_MOMX] = (double)mx;
      v[OF_KXY] = (double)kxy;
      v[OF_TRT] = (double)trT;
      // x momentum handed to the walls in the previous step: the reflected
      // populations now sit in the wall rows with the opposite velocity
      double drag = 0.0;
      if (y == 0) drag += 2.0 * ((double)fc[6] - (double)fc[5]);
      if (y == ny - 1) drag += 2.0 * ((double)fc[7] - (double)fc[8]);
      v[OF_DRAG] = drag;
      v[OF_KXX] = (double)kxx;
      constexpr int GW = WIDE ? 64 : TXW;
#pragma unroll
      for (int f = 0; f < OF_COUNT; ++f) v[f] = group_sum<GW>(ok ? v[f] : 0.0);
      const bool writer = WIDE ? (lane == 0) : (lx == 0);
      if (writer && y < st.y1) {
        const long long pr = (long long)c.poff + (long long)y * c.nxs + (WIDE ? st.x0 / 62 : 0);
        double *dst = a.part + pr * OF_COUNT;
#pragma unroll
        for (int f = 0; f < OF_COUNT; ++f) dst[f] = v[f];
      }
    } else {
      // equilibrium, forcing of Eq. (bodyforce) and BGK collision
      const T usq = ux * ux + uy * uy;
      const T uf = ux * fx;
      const T K0 = kf * (rr + T(1.5) * rr * usq - T(3) * uf);
      const T eq0 = SHIFT ? (rho_dev - T(1.5) * rho_e * usq) : rho_e * (T(1) - T(1.5) * usq);
      const T Sxy2 = T(2) * Txy;
      const long long o = base + (long long)y * nx + x;
      T out[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        constexpr int cxs[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
        constexpr int cys[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
        const int cx = cxs[i], cy = cys[i];
        const T cu = T(cx) * ux + T(cy) * uy;
        const T cf = T(cx) * fx;
        const T Q = (i == 0) ? T(0)
                    : (i < 5 ? (cx != 0 ? Sxx : -Sxx) : (cx * cy > 0 ? Sxy2 : -Sxy2));
        const T wi = weight<T>(i);
        const T Fi = wi * (sp * Q + K0 + kf * (T(3) * cf - T(4.5) * rr * cu * cu + T(9) * cu * cf));
        const T eqi = wi * (eq0 + rho_e * (T(3) * cu + T(4.5) * cu * cu));
        out[i] = fc[i] - om * (fc[i] - eqi) + Fi;
      }
      if (ok) {
#pragma unroll
        for (int i = 0; i < 9; ++i) B[i * P + o] = out[i];
        B[9 * P + o] = trT;
      }
    }

    uPrev = uCur;
    uCur = uNext;
#pragma unroll
    for (int i = 0; i < 9; ++i) fc[i] = fn[i];
    Pc = Pn;
  }
}

// One workgroup per channel: sums the x partials of every row in a fixed
// order, writes x-averaged rows, channel totals and the steady residual.
__global__ void __launch_bounds__(256) reduce_kernel(const ChanDev *ch, const double *part,
                                                     double *prof, double *prev_ux, double *scal,
                                                     int update_residual, int steps_since) {
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

__global__ void advance_kernel(ChanDev *ch, int n_ch, int steps) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_ch && ch[i].active) ch[i].t += steps;
}

template <typename T, bool SHIFT, int TXW, bool WIDE>
hipError_t launch_cls(bool observe, const SweepArgs &a, hipStream_t s) {
  if (a.n_strips == 0) return hipSuccess;
  dim3 grid(a.n_wg), block(256);
  if (observe)
    hipLaunchKernelGGL((sweep_kernel<T, SHIFT, TXW, WIDE, true>), grid, block, 0, s, a);
  else
    hipLaunchKernelGGL((sweep_kernel<T, SHIFT, TXW, WIDE, false>), grid, block, 0, s, a);
  return hipGetLastError();
}

template <typename T, bool SHIFT>
hipError_t launch_prec(int cls, bool observe, const SweepArgs &a, hipStream_t s) {
  switch (cls) {
    case 0: return launch_cls<T, SHIFT, 1, false>(observe, a, s);
    case 1: return launch_cls<T, SHIFT, 2, false>(observe, a, s);
    case 2: return launch_cls<T, SHIFT, 4, false>(observe, a, s);
    case 3: return launch_cls<T, SHIFT, 8, false>(observe, a, s);
    case 4: return launch_cls<T, SHIFT, 16, false>(observe, a, s);
    case 5: return launch_cls<T, SHIFT, 32, false>(observe, a, s);
    case 6: return launch_cls<T, SHIFT, 64, false>(observe, a, s);
    default: return launch_cls<T, SHIFT, 64, true>(observe, a, s);
  }
}

}  // namespace

hipError_t launch_sweep(int fp32, int cls, bool observe, const SweepArgs &a, hipStream_t s) {
  return fp32 ? launch_prec<float, true>(cls, observe, a, s)
              : launch_prec<double, false>(cls, observe, a, s);
}

hipError_t launch_reduce(const ChanDev *ch, int n_ch, const double *part, double *prof,
                         double *prev_ux, double *scal, int update_residual, int steps_since,
                         hipStream_t s) {
  if (n_ch == 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_kernel, dim3(n_ch), dim3(256), 0, s, ch, part, prof, prev_ux, scal,
                     update_residual, steps_since);
  return hipGetLastError();
}

hipError_t launch_advance(ChanDev *ch, int n_ch, int steps, hipStream_t s) {
  if (n_ch == 0 || steps == 0) return hipSuccess;
  hipLaunchKernelGGL(advance_kernel, dim3((n_ch + 255) / 256), dim3(256), 0, s, ch, n_ch, steps);
  return hipGetLastError();
}

}  // namespace lbnlm
