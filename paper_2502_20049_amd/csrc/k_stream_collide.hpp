// Fused PSM stream-collide kernel (in-place AA pattern) for gfx950.
//
// One thread per lattice cell, 256-thread workgroups tiling (TX x TY) cells of
// one z-plane with TX in {64,128,256}: every wave64 covers 64 consecutive x of
// one row, so each of the Q direction arrays is read and written with
// coalesced (at most one element shifted) 64-lane accesses.  No MFMA: the
// update is a bandwidth-bound stencil of ~3-5 flop per byte.
//
// AA pattern (in place, one buffer): at even steps a cell reads its own Q
// slots and writes the post-collision value of direction k into its own slot
// of the opposite direction; at odd steps it reads slot (x - c_k, kbar) and
// writes direction k's post-collision value to slot (x + c_k, k).  In both
// parities "the post-collision value of kbar goes back to the slot f_k was
// read from", so one address per direction serves the load and the store.
// Face rules (cell-local, so they fit the pattern):
//   wall   odd read of an incoming k whose source is outside: own slot (x, k),
//          which holds f*_kbar of the previous even step;
//   inlet  as wall plus 6 w_k (c_k . u_in) on the odd read and on the odd
//          write of that slot (moving-wall bounce-back, rest density 1);
//   outlet the slot of an incoming k receives f*_k (not f*_kbar) in both
//          parities, so the next read sees the cell's own post-collision value.
#pragma once

#include <type_traits>
#include <utility>

#include "psm_internal.hpp"

namespace psm {

template <typename T>
struct Comp {
  using type = float;
};
template <>
struct Comp<double> {
  using type = double;
};

template <int... Ks, typename F>
__device__ __forceinline__ void sfor_impl(std::integer_sequence<int, Ks...>, F &&f) {
  (f(std::integral_constant<int, Ks>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void sfor(F &&f) {
  sfor_impl(std::make_integer_sequence<int, N>{}, f);
}

// Workgroups are dispatched round-robin over the 8 XCDs; remap so that each
// XCD walks a contiguous range of tiles (its own L2 sees neighbouring rows).
__device__ __forceinline__ uint32_t xcd_remap(uint32_t bid, uint32_t nblk) {
  const uint32_t nxcd = 8;
  const uint32_t xcd = bid % nxcd, loc = bid / nxcd;
  const uint32_t per = nblk / nxcd, rem = nblk % nxcd;
  return xcd < rem ? xcd * (per + 1) + loc : rem * (per + 1) + (xcd - rem) * per + loc;
}

template <typename T, typename R>
__device__ __forceinline__ R ldv(const char *p) {
  return (R)(*(const T *)p);
}
template <typename T, typename R>
__device__ __forceinline__ void stv(char *p, R v) {
  *(T *)p = (T)v;
}

// Whole-wave lane shifts (DPP wave_shr:1 / wave_shl:1): lane i receives lane
// i-1 (shr) or lane i+1 (shl); the lane without a source gets 0.  Every lane
// of the wave must be active.
__device__ __forceinline__ float wave_shr1(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float wave_shl1(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ bool wave_shr1(bool b) {
  return __builtin_amdgcn_update_dpp(0, b ? 1 : 0, 0x138, 0xf, 0xf, false) != 0;
}
__device__ __forceinline__ bool wave_shl1(bool b) {
  return __builtin_amdgcn_update_dpp(0, b ? 1 : 0, 0x130, 0xf, 0xf, false) != 0;
}

// Per-cell collision: TRT + Guo fluid collision blended with NS solid slots.
// Inverse central-moment transform along one axis: the populations at c = -1,
// 0, +1 of the central moments (m0, m1, m2) about u (linear in the moments).
template <typename R>
__device__ __forceinline__ void chim(R m0, R m1, R m2, R u, R (&o)[3]) {
#pragma clang fp contract(on)
  o[0] = R(0.5) * ((u * u - u) * m0 + (R(2) * u - R(1)) * m1 + m2);
  o[1] = (R(1) - u * u) * m0 - R(2) * u * m1 - m2;
  o[2] = R(0.5) * ((u * u + u) * m0 + (R(2) * u + R(1)) * m1 + m2);
}
template <typename R>
__device__ __forceinline__ void chim02(R m0, R m2, R u, R (&o)[3]) {  // m1 = 0
#pragma clang fp contract(on)
  o[0] = R(0.5) * ((u * u - u) * m0 + m2);
  o[1] = (R(1) - u * u) * m0 - m2;
  o[2] = R(0.5) * ((u * u + u) * m0 + m2);
}
template <typename R>
__device__ __forceinline__ void chim1(R m1, R u, R (&o)[3]) {  // m0 = m2 = 0
#pragma clang fp contract(on)
  o[0] = R(0.5) * (R(2) * u - R(1)) * m1;
  o[1] = R(-2) * u * m1;
  o[2] = R(0.5) * (R(2) * u + R(1)) * m1;
}

// Cumulant fluid collision (D3Q27, no body force), in deviation variables.
// The shear rate om = 1/tau relaxes the off-diagonal second-order cumulants
// and the deviators; every other rate is one: the trace goes to 3 c_s^2 and
// all cumulants of orders 3..6 to zero.  Then the post-collision central
// moments (about u) are those of a Gaussian with the relaxed covariance S
// (Isserlis): E[x^2 y^2] = Sxx Syy + 2 Sxy^2, E[x^2 y z] = Sxx Syz + 2 Sxy Sxz,
// E[x^2 y^2 z^2] = Sxx Syy Szz + 2 (Sxx Syz^2 + Syy Sxz^2 + Szz Sxy^2)
// + 8 Sxy Sxz Syz, odd orders zero.  Written as deviations from the rest
// state (S = I/3): the transform of the rest moments is the product of the
// 1-D weights (1/6, 2/3, 1/6) shifted by u, so
//   f*_k - w_k = dr w_k + rho (P_k + D_k),
// P = product-equilibrium minus rest weights, D = transform of the moment
// deviations (axis by axis: z, then y, then x).  Returns Om = f* - f.
template <typename R>
__device__ __forceinline__ void cumulant_fluid(const R (&f)[27], R dr, R rho, R inv, R ux, R uy, R uz, R om,
                                               R (&Om)[27]) {
  // contraction only within an expression: the same bits whatever the kernel
  // around it (the row kernels and the per-cell general path agree exactly)
#pragma clang fp contract(on)
  R pxx = 0, pyy = 0, pzz = 0, pxy = 0, pxz = 0, pyz = 0;
  sfor<27>([&](auto K) {
    constexpr int k = K;
    constexpr int ex = cx<27>(k), ey = cy<27>(k), ez = cz<27>(k);
    if constexpr (ex != 0) pxx += f[k];
    if constexpr (ey != 0) pyy += f[k];
    if constexpr (ez != 0) pzz += f[k];
    if constexpr (ex * ey == 1) pxy += f[k];
    if constexpr (ex * ey == -1) pxy -= f[k];
    if constexpr (ex * ez == 1) pxz += f[k];
    if constexpr (ex * ez == -1) pxz -= f[k];
    if constexpr (ey * ez == 1) pyz += f[k];
    if constexpr (ey * ez == -1) pyz -= f[k];
  });
  const R third = R(1) / R(3), d3 = dr * third;
  const R ecx = (pxx - d3) * inv - ux * ux, ecy = (pyy - d3) * inv - uy * uy, ecz = (pzz - d3) * inv - uz * uz;
  const R w1 = R(1) - om;
  const R dxy = w1 * (ecx - ecy), dxz = w1 * (ecx - ecz);
  const R ex_ = (dxy + dxz) * third, ey_ = ex_ - dxy, ez_ = ex_ - dxz;
  const R sxy = w1 * (pxy * inv - ux * uy), sxz = w1 * (pxz * inv - ux * uz), syz = w1 * (pyz * inv - uy * uz);
  // post-collision central moments minus their rest values
  const R M220 = (ex_ + ey_) * third + ex_ * ey_ + R(2) * sxy * sxy;
  const R M202 = (ex_ + ez_) * third + ex_ * ez_ + R(2) * sxz * sxz;
  const R M022 = (ey_ + ez_) * third + ey_ * ez_ + R(2) * syz * syz;
  const R M211 = (third + ex_) * syz + R(2) * sxy * sxz;
  const R M121 = (third + ey_) * sxz + R(2) * sxy * syz;
  const R M112 = (third + ez_) * sxy + R(2) * sxz * syz;
  const R M222 = (ex_ + ey_ + ez_) * (third * third) + (ex_ * ey_ + ex_ * ez_ + ey_ * ez_) * third + ex_ * ey_ * ez_ +
                 R(2) * ((third + ex_) * syz * syz + (third + ey_) * sxz * sxz + (third + ez_) * sxy * sxy) +
                 R(8) * sxy * sxz * syz;
  // z: G[a][b][cz] for the moment pairs (a, b) of x and y
  R G[3][3][3];
  G[0][0][0] = R(0.5) * ez_;
  G[0][0][1] = -ez_;
  G[0][0][2] = R(0.5) * ez_;
  chim1(sxz, uz, G[1][0]);
  chim1(syz, uz, G[0][1]);
  chim02(sxy, M112, uz, G[1][1]);
  chim02(ex_, M202, uz, G[2][0]);
  chim02(ey_, M022, uz, G[0][2]);
  chim1(M211, uz, G[2][1]);
  chim1(M121, uz, G[1][2]);
  chim02(M220, M222, uz, G[2][2]);
  // y, then x
  R H[3][3][3];  // H[a][cy][cz]
#pragma unroll
  for (int aa = 0; aa < 3; ++aa)
#pragma unroll
    for (int cz = 0; cz < 3; ++cz) {
      R o[3];
      chim(G[aa][0][cz], G[aa][1][cz], G[aa][2][cz], uy, o);
      H[aa][0][cz] = o[0];
      H[aa][1][cz] = o[1];
      H[aa][2][cz] = o[2];
    }
  R D[3][3][3];  // D[cx][cy][cz]
#pragma unroll
  for (int cy = 0; cy < 3; ++cy)
#pragma unroll
    for (int cz = 0; cz < 3; ++cz) {
      R o[3];
      chim(H[0][cy][cz], H[1][cy][cz], H[2][cy][cz], ux, o);
      D[0][cy][cz] = o[0];
      D[1][cy][cz] = o[1];
      D[2][cy][cz] = o[2];
    }
  // product equilibrium minus the rest weights, per axis w1d + d
  const R u2x = ux * ux, u2y = uy * uy, u2z = uz * uz;
  const R dxv[3] = {R(0.5) * (u2x - ux), -u2x, R(0.5) * (u2x + ux)};
  const R dyv[3] = {R(0.5) * (u2y - uy), -u2y, R(0.5) * (u2y + uy)};
  const R dzv[3] = {R(0.5) * (u2z - uz), -u2z, R(0.5) * (u2z + uz)};
  sfor<27>([&](auto K) {
    constexpr int k = K;
    constexpr int ix = cx<27>(k) + 1, iy = cy<27>(k) + 1, iz = cz<27>(k) + 1;
    constexpr double wx = ix == 1 ? 2.0 / 3.0 : 1.0 / 6.0, wy = iy == 1 ? 2.0 / 3.0 : 1.0 / 6.0,
                     wz = iz == 1 ? 2.0 / 3.0 : 1.0 / 6.0;
    const R tz = R(wz) + dzv[iz];
    const R P = dxv[ix] * ((R(wy) + dyv[iy]) * tz) + R(wx) * (dyv[iy] * tz + R(wy) * dzv[iz]);
    Om[k] = (dr * R(wt<27>(k)) + rho * (P + D[ix][iy][iz])) - f[k];
  });
}

// f holds deviations delta f; on return f holds the post-collision deviations.
// CM = 0: TRT with Guo forcing; CM = 1: the cumulant collision above (D3Q27,
// no body force) as the fluid part.
template <int Q, int SC, int NS, typename R, int CM = 0>
__device__ __forceinline__ void collide(R (&f)[Q], const SCArgs &a, R B0, const R (&us0)[3], R B1,
                                        const R (&us1)[3], R (&mom0)[3], R (&mom1)[3]) {
  constexpr int H = Lat<Q>::H;
  R dr = 0, jx = 0, jy = 0, jz = 0;
  sfor<Q>([&](auto K) {
    constexpr int k = K;
    dr += f[k];
    if constexpr (cx<Q>(k) > 0) jx += f[k];
    if constexpr (cx<Q>(k) < 0) jx -= f[k];
    if constexpr (cy<Q>(k) > 0) jy += f[k];
    if constexpr (cy<Q>(k) < 0) jy -= f[k];
    if constexpr (cz<Q>(k) > 0) jz += f[k];
    if constexpr (cz<Q>(k) < 0) jz -= f[k];
  });
  const R rho = R(1) + dr;
  R inv;
  if constexpr (std::is_same<R, float>::value)
    inv = __builtin_amdgcn_rcpf(rho);  // 1 ulp; FP32 arithmetic budget
  else
    inv = R(1) / rho;
  const bool hf = a.has_force != 0;
  const R Fx = (R)a.force[0], Fy = (R)a.force[1], Fz = (R)a.force[2];
  R ux, uy, uz;
  if (hf) {
    ux = (jx + R(0.5) * Fx) * inv;
    uy = (jy + R(0.5) * Fy) * inv;
    uz = (jz + R(0.5) * Fz) * inv;
  } else {
    ux = jx * inv;
    uy = jy * inv;
    uz = jz * inv;
  }
  const R usq = ux * ux + uy * uy + uz * uz;
  const R uF = ux * Fx + uy * Fy + uz * Fz;
  const R le = (R)a.lam_e, lo = (R)a.lam_o;
  const R ge = R(1) - R(0.5) * le, go = R(1) - R(0.5) * lo;

  R Bs0 = B0, Bs1 = B1;
  if constexpr (NS == 2) {
    const R sb = B0 + B1;
    if (sb > R(1)) {
      const R is = R(1) / sb;
      Bs0 = B0 * is;
      Bs1 = B1 * is;
    }
  }
  R fl = R(1);
  if constexpr (NS >= 1) fl -= Bs0;
  if constexpr (NS == 2) fl -= Bs1;
  R uss0 = 0, uss1 = 0;
  if constexpr (NS >= 1) uss0 = us0[0] * us0[0] + us0[1] * us0[1] + us0[2] * us0[2];
  if constexpr (NS == 2) uss1 = us1[0] * us1[0] + us1[1] * us1[1] + us1[2] * us1[2];
  R OmC[CM == 1 ? Q : 1];
  if constexpr (CM == 1) {
    static_assert(Q == 27, "the cumulant collision is written for D3Q27");
    cumulant_fluid<R>(f, dr, rho, inv, ux, uy, uz, le, OmC);
  }

  // rest direction
  {
    const R w = (R)wt<Q>(0);
    const R E = w * (dr - R(1.5) * rho * usq);
    R om;
    if constexpr (CM == 1) {
      om = OmC[0];
    } else {
      om = -le * (f[0] - E);
      if (hf) om += ge * (R(-3) * w * uF);
    }
    R out = f[0] + fl * om;
    if constexpr (NS >= 1) {
      const R Es = w * (dr - R(1.5) * rho * uss0);
      R s;
      if constexpr (SC == 1) s = Es - E;
      else if constexpr (SC == 2) s = -le * (f[0] - Es);
      else s = R(0);
      out += Bs0 * s;
    }
    if constexpr (NS == 2) {
      const R Es = w * (dr - R(1.5) * rho * uss1);
      R s;
      if constexpr (SC == 1) s = Es - E;
      else if constexpr (SC == 2) s = -le * (f[0] - Es);
      else s = R(0);
      out += Bs1 * s;
    }
    f[0] = out;
  }
  // direction pairs (i, i+H)
  sfor<H>([&](auto Kh) {
    constexpr int i = Kh + 1, ib = Kh + 1 + H;
    constexpr int ex = cx<Q>(i), ey = cy<Q>(i), ez = cz<Q>(i);
    const R w = (R)wt<Q>(i);
    const R av = f[i], bv = f[ib];
    const R cu = R(ex) * ux + R(ey) * uy + R(ez) * uz;
    const R E = w * (dr + rho * (R(4.5) * cu * cu - R(1.5) * usq));
    const R O = R(3) * w * rho * cu;
    R rp, rm;
    if constexpr (CM == 1) {
      rp = R(0.5) * (OmC[i] + OmC[ib]);
      rm = R(0.5) * (OmC[i] - OmC[ib]);
    } else {
      const R fp = R(0.5) * (av + bv), fm = R(0.5) * (av - bv);
      rp = -le * (fp - E);
      rm = -lo * (fm - O);
      if (hf) {
        const R cF = R(ex) * Fx + R(ey) * Fy + R(ez) * Fz;
        rp += ge * (w * (R(9) * cu * cF - R(3) * uF));
        rm += go * (R(3) * w * cF);
      }
    }
    R oa = av + fl * (rp + rm);
    R ob = bv + fl * (rp - rm);
    auto solid = [&](const R(&us)[3], R uss, R Bk, R(&mom)[3]) {
      const R cus = R(ex) * us[0] + R(ey) * us[1] + R(ez) * us[2];
      const R Es = w * (dr + rho * (R(4.5) * cus * cus - R(1.5) * uss));
      const R Os = R(3) * w * rho * cus;
      R sa, sb;
      if constexpr (SC == 1) {
        sa = (bv - E + O) - (av - Es - Os);
        sb = (av - E - O) - (bv - Es + Os);
      } else if constexpr (SC == 2) {
        sa = -le * (av - Es - Os);
        sb = -le * (bv - Es + Os);
      } else {
        sa = (bv - Es + Os) - (av - Es - Os);
        sb = (av - Es - Os) - (bv - Es + Os);
      }
      oa += Bk * sa;
      ob += Bk * sb;
      const R d = sa - sb;
      if constexpr (ex != 0) mom[0] += R(ex) * d;
      if constexpr (ey != 0) mom[1] += R(ey) * d;
      if constexpr (ez != 0) mom[2] += R(ez) * d;
    };
    if constexpr (NS >= 1) solid(us0, uss0, Bs0, mom0);
    if constexpr (NS == 2) solid(us1, uss1, Bs1, mom1);
    f[i] = oa;
    f[ib] = ob;
  });
  if constexpr (NS >= 1) {
    mom0[0] *= -Bs0;
    mom0[1] *= -Bs0;
    mom0[2] *= -Bs0;
  }
  if constexpr (NS == 2) {
    mom1[0] *= -Bs1;
    mom1[1] *= -Bs1;
    mom1[2] *= -Bs1;
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over a 256-thread workgroup: fixed lane tree per wave, then the four
// waves in order (every thread gets the result).
__device__ __forceinline__ double block_sum256(double v, double *sh) {
  v = wave_sum(v);
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  return ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

// Force/torque of body b from the solid kernel's per-workgroup partials, by
// one 256-thread workgroup: partials in increasing workgroup order (thread t
// takes every 256th), then the fixed tree above (deterministic).
__device__ __forceinline__ void ft_body_sum(const double *ftp, int max_bodies, int nblocks, int b, double *ft,
                                            double *sh) {
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int i = threadIdx.x; i < nblocks; i += 256) {
    const double *p = ftp + ((size_t)i * max_bodies + b) * 6;
#pragma unroll
    for (int c = 0; c < 6; ++c) acc[c] += p[c];
  }
  for (int c = 0; c < 6; ++c) {
    const double s = block_sum256(acc[c], sh);
    if (threadIdx.x == 0) ft[b * 6 + c] = s;
  }
}

// The extra last workgroup of the step's last fluid launch (the face rows, or
// the interior rows with the face rows as extra blocks on even D3Q19 steps)
// that also sums the F/T; the solid kernel, an earlier launch, has finished
// writing the partials.  Those launches need more registers than this, or
// stay within their occupancy step.
__device__ __forceinline__ bool ft_extra_block(const SCArgs &a) {
  if (a.ft_out == nullptr || blockIdx.x != a.ft_block) return false;
  __shared__ double sh[4];
  for (int b = 0; b < a.ft_nb; ++b) ft_body_sum(a.ftp, a.max_bodies, a.ft_nblocks, b, a.ft_out, sh);
  return true;
}

// Inlet term 6 w_k (c_k . u_in) of the velocity-inlet rule.  Not contracted
// into the add that applies it, so every kernel (whatever its code shape)
// rounds the face rule the same way.
template <int Q, typename R>
__device__ __forceinline__ R inlet_term(const SCArgs &a, int k) {
#pragma clang fp contract(off)
  return R(6.0 * wt<Q>(k)) *
         (R(cx<Q>(k)) * (R)a.u_in_d[0] + R(cy<Q>(k)) * (R)a.u_in_d[1] + R(cz<Q>(k)) * (R)a.u_in_d[2]);
}

__device__ __forceinline__ bool box_has(const IBox &b, int x, int y, int z) {
  return x >= b.lo[0] && x <= b.hi[0] && y >= b.lo[1] && y <= b.hi[1] && z >= b.lo[2] && z <= b.hi[2];
}

// Directions whose source x - c_k lies beyond face f (f = -x,+x,-y,+y,-z,+z):
// those with c_k along the face's inward normal.
template <int Q>
__host__ __device__ constexpr uint32_t face_dirs(int f) {
  uint32_t m = 0;
  for (int k = 0; k < Q; ++k) {
    const int e = f < 2 ? cx<Q>(k) : (f < 4 ? cy<Q>(k) : cz<Q>(k));
    if (e == ((f & 1) ? -1 : 1)) m |= 1u << k;
  }
  return m;
}

// Face kinds of every incoming direction of cell (x,y,z) (source x - c_k):
// bit k of bcm set when the source is outside a non-periodic face; outm / inm
// mark the outlet / inlet kinds (after the wall > inlet > outlet precedence).
// Per face: the cell's flag selects the face's direction set into the mask of
// the face's (uniform) kind; precedence is applied to the three masks.
template <int Q>
__device__ __forceinline__ void classify(const SCArgs &a, int x, int y, int z, uint32_t &bcm, uint32_t &outm,
                                         uint32_t &inm) {
  const bool on[6] = {x == 0, x == a.nx - 1, y == 0, y == a.ny - 1, z == 0, z == a.nz - 1};
  uint32_t mw = 0, mi = 0, mo = 0;
  sfor<6>([&](auto F) {
    constexpr int f = F;
    constexpr uint32_t dm = face_dirs<Q>(f);
    const int kd = a.periodic[f >> 1] ? K_NONE : a.bc[f];
    const uint32_t sel = on[f] ? dm : 0u;
    mw |= sel & (kd == K_WALL ? ~0u : 0u);
    mi |= sel & (kd == K_INLET ? ~0u : 0u);
    mo |= sel & (kd == K_OUTLET ? ~0u : 0u);
  });
  bcm = mw | mi | mo;
  inm = mi & ~mw;
  outm = mo & ~(mw | mi);
}

// Slot of direction k for cell (x,y,z) with full face handling (face cells,
// solid cells): own slot at even parity or for a face direction, else the
// slot (x - c_k, kbar) with periodic wrap.
template <int Q, typename T, int PAR>
__device__ __forceinline__ char *slot_general(const SCArgs &a, char *pdf, int k, int x, int y, int z, uint64_t n,
                                              uint32_t bcm) {
  (void)n;
  const size_t NS = (size_t)a.dS * sizeof(T);
  if (PAR == 0 || ((bcm >> k) & 1u))
    return pdf + (size_t)k * NS + (pdf_row(a, (uint32_t)y + (uint32_t)a.ny * (uint32_t)z) + (uint64_t)x) * sizeof(T);
  int sx = x - cx<Q>(k), sy = y - cy<Q>(k), sz = z - cz<Q>(k);
  if (sx < 0) sx += a.nx;
  if (sx >= a.nx) sx -= a.nx;
  if (sy < 0) sy += a.ny;
  if (sy >= a.ny) sy -= a.ny;
  if (sz < 0) sz += a.nz;
  if (sz >= a.nz) sz -= a.nz;
  const uint64_t src = pdf_row(a, (uint32_t)sy + (uint32_t)a.ny * (uint32_t)sz) + (uint64_t)sx;
  return pdf + (size_t)opp<Q>(k) * NS + (size_t)src * sizeof(T);
}

// Solid fraction of slot 0, plus the optional time-invariant offset field.
template <typename R>
__device__ __forceinline__ R solid_fraction(const SCArgs &a, uint64_t n) {
  R b = (R)a.B0[n];
  if (a.dB) b += (R)a.dB[n];
  return b;
}

// Does the tile / cell need the solid-fraction read?  B can only be nonzero
// inside the bodies' current boxes (the mapping keeps it so).
__device__ __forceinline__ bool boxes_touch(const SCArgs &a, int x0, int x1, int y0, int y1, int z0, int z1) {
  for (int b = 0; b < a.nbox; ++b) {
    const IBox &B = a.box[b];
    if (x1 >= B.lo[0] && x0 <= B.hi[0] && y1 >= B.lo[1] && y0 <= B.hi[1] && z1 >= B.lo[2] && z0 <= B.hi[2])
      return true;
  }
  return false;
}

// ---------------------------------------------------------------------------
// Fluid cells (every row).  Each wave64 covers 64 consecutive x of one row,
// so the row (y, z) is wave-uniform: every direction is one uniform 64-bit
// row base plus a 32-bit lane offset chosen from three (x-1, x, x+1, wrapped
// when x is periodic).  Rows inside the domain take the plain pattern; rows
// on a y or z face (EDGE) wrap the source row and take the y/z face rules as
// wave-uniform direction masks (selects, no branches).  Only the first and
// last cell of a row with a non-periodic x take a per-lane fix-up for the x
// faces.  With PSM, cells whose B is nonzero are left to the solid kernel.
// ---------------------------------------------------------------------------

// Directions k with c_k[axis] == sgn (the directions whose source lies
// outside the face on the -sgn side of that axis).
template <int Q>
__host__ __device__ constexpr uint32_t dirs_with(int axis, int sgn) {
  uint32_t m = 0;
  for (int k = 0; k < Q; ++k) {
    const int c = axis == 0 ? cx<Q>(k) : (axis == 1 ? cy<Q>(k) : cz<Q>(k));
    if (c == sgn) m |= 1u << k;
  }
  return m;
}

// Face rules as direction masks: a face that is on adds its directions to the
// mask of its kind.  Resolution (wall > inlet > outlet) happens in FaceMask.
struct FaceAcc {
  uint32_t w = 0, i = 0, o = 0;
  __device__ __forceinline__ void add(bool on, int kind, uint32_t dirs) {
    const uint32_t m = on ? dirs : 0u;
    w |= kind == K_WALL ? m : 0u;
    i |= kind == K_INLET ? m : 0u;
    o |= kind == K_OUTLET ? m : 0u;
  }
  // own slot / inlet term / outlet rule, per direction
  __device__ __forceinline__ uint32_t own() const { return w | i | o; }
  __device__ __forceinline__ uint32_t inlet() const { return i & ~w; }
  __device__ __forceinline__ uint32_t outlet() const { return o & ~(w | i); }
};

template <int Q, typename T, int PAR, bool EDGE>
struct RowCell {
  using R = typename Comp<T>::type;
  static constexpr uint32_t S = sizeof(T);
  const SCArgs &a;
  int y, z;
  uint32_t row;  // y + ny z
  bool lo_face, hi_face, xface;
  uint32_t o0, om, op;
  size_t NS, nxy;
  char *own_row;
  uint32_t own_m, in_m, out_m;
  FaceAcc yz, all;

  __device__ __forceinline__ RowCell(const SCArgs &args, int x, int y_, int z_, size_t rowbase)
      : a(args), y(y_), z(z_) {
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    nxy = (size_t)nx * (size_t)ny;
    const bool xper = a.periodic[0] != 0;
    lo_face = !xper && x == 0;       // sources x-1 are outside (face -x)
    hi_face = !xper && x == nx - 1;  // sources x+1 are outside (face +x)
    xface = lo_face || hi_face;
    int xm = x - 1, xp = x + 1;
    if (xm < 0) xm = xper ? xm + nx : 0;
    if (xp >= nx) xp = xper ? xp - nx : nx - 1;
    o0 = (uint32_t)x * S;
    om = (uint32_t)xm * S;
    op = (uint32_t)xp * S;
    NS = (size_t)a.dS * S;
    (void)rowbase;
    row = (uint32_t)y + (uint32_t)ny * (uint32_t)z;
    own_row = a.pdf + pdf_row(a, row) * S;
    // y/z face rules of this row (wave-uniform)
    if constexpr (EDGE) {
      const bool py = a.periodic[1] != 0, pz = a.periodic[2] != 0;
      yz.add(!py && y == 0, a.bc[2], dirs_with<Q>(1, 1));
      yz.add(!py && y == ny - 1, a.bc[3], dirs_with<Q>(1, -1));
      yz.add(!pz && z == 0, a.bc[4], dirs_with<Q>(2, 1));
      yz.add(!pz && z == nz - 1, a.bc[5], dirs_with<Q>(2, -1));
    }
    own_m = yz.own();
    in_m = yz.inlet();
    out_m = yz.outlet();
    all = yz;
    if (xface) {
      all.add(lo_face, a.bc[0], dirs_with<Q>(0, 1));
      all.add(hi_face, a.bc[1], dirs_with<Q>(0, -1));
    }
  }

  template <typename K>
  __device__ __forceinline__ char *own(K) const {
    return own_row + (size_t)(int)K::value * NS + o0;
  }
  // odd parity, no face: slot kbar of the source cell x - c_k, as a
  // wave-uniform row base and a 32-bit lane offset
  template <typename K>
  __device__ __forceinline__ char *src_base(K) const {
    constexpr int k = K::value;
    constexpr int ey = cy<Q>(k), ez = cz<Q>(k);
    char *rp;
    if constexpr (!EDGE) {
      // interior rows: the source row never wraps
      rp = a.pdf + pdf_row(a, row - (uint32_t)(ey + ez * a.ny)) * S;
    } else {
      int sy = y - ey, sz = z - ez;
      if (sy < 0) sy += a.ny;
      if (sy >= a.ny) sy -= a.ny;
      if (sz < 0) sz += a.nz;
      if (sz >= a.nz) sz -= a.nz;
      rp = a.pdf + pdf_row(a, (uint32_t)sy + (uint32_t)a.ny * (uint32_t)sz) * S;
    }
    return rp + (size_t)opp<Q>(k) * NS;
  }
  template <typename K>
  __device__ __forceinline__ uint32_t src_lane(K) const {
    constexpr int ex = cx<Q>(K::value);
    return ex == 1 ? om : (ex == -1 ? op : o0);
  }
  // slot of direction k: own slot at even parity or where the face mask has
  // k, else the source slot.  Base and lane offset are selected separately
  // (both candidates formed first, so the choice is a select): with a
  // wave-uniform mask the base stays scalar.
  template <typename K>
  __device__ __forceinline__ char *slot(K kk, uint32_t ownmask) const {
    if constexpr (PAR == 0) {
      return own(kk);
    } else {
      char *const ps = src_base(kk) + src_lane(kk);
      if constexpr (!EDGE) {
        return ps;  // interior rows have no y/z face directions
      } else {
        // both addresses formed first: the choice is between values (a
        // choice between two members would keep the object in private memory)
        char *const po = own(kk);
        return ((ownmask >> (int)K::value) & 1u) ? po : ps;
      }
    }
  }
  template <typename K>
  __device__ __forceinline__ R inlet_if(K, uint32_t inmask) const {
    const R t = inlet_term<Q, R>(a, (int)K::value);
    return ((inmask >> (int)K::value) & 1u) ? t : R(0);
  }

  // incoming populations f_k of the cell: the row's pattern (load_row),
  // then the x-face corrections of the row's first and last cell (load_fix)
  __device__ __forceinline__ void load(R f[Q]) const {
    load_row(f);
    load_fix(f);
  }
  __device__ __forceinline__ void load_row(R f[Q]) const {
    sfor<Q>([&](auto K) {
      constexpr int k = K;
      R v = ldv<T, R>(slot(K, own_m));
      if constexpr (PAR == 1 && EDGE) v += inlet_if(K, in_m);
      f[k] = v;
    });
  }
  __device__ __forceinline__ void load_fix(R f[Q]) const {
    if constexpr (PAR == 1) {
      if (xface) {
        // odd parity: directions whose rule the x faces change re-read the
        // cell's own slot
        const uint32_t own_x = all.own(), in_x = all.inlet();
        const uint32_t redo = (own_x ^ own_m) | (in_x ^ in_m);
        sfor<Q>([&](auto K) {
          constexpr int k = K;
          if ((redo >> k) & 1u) {
            R v = ldv<T, R>(own(K));
            if ((in_x >> k) & 1u) v += inlet_term<Q, R>(a, k);
            f[k] = v;
          }
        });
      }
    }
  }

  // post-collision populations back, with the face rules
  __device__ __forceinline__ void store(const R f[Q]) const {
    auto put = [&](auto K, uint32_t ownmask, uint32_t inmask, uint32_t outmask) {
      constexpr int k = K;
      R v = ((outmask >> k) & 1u) ? f[k] : f[opp<Q>(k)];
      if constexpr (PAR == 1) v += inlet_if(K, inmask);
      stv<T, R>(slot(K, ownmask), v);
    };
    if (!xface) {
      sfor<Q>([&](auto K) { put(K, own_m, in_m, out_m); });
    } else {
      // first or last cell of a row with a non-periodic x: a direction whose
      // source lies beyond the x face takes the merged rule, in its own
      // slot.  (Written with branches, unlike the row's path, so that the
      // compiler keeps the two paths apart instead of turning the row's
      // stores into per-lane selects.)
      const uint32_t own_x = all.own(), in_x = all.inlet(), out_x = all.outlet();
      const uint32_t changed = (own_x ^ own_m) | (in_x ^ in_m) | (out_x ^ out_m);
      sfor<Q>([&](auto K) {
        constexpr int k = K;
        if constexpr (cx<Q>(k) == 0) {
          put(K, own_m, in_m, out_m);
        } else {
          if ((changed >> k) & 1u) {
            R v = ((out_x >> k) & 1u) ? f[k] : f[opp<Q>(k)];
            if constexpr (PAR == 1) {
              if ((in_x >> k) & 1u) v += inlet_term<Q, R>(a, k);
            }
            stv<T, R>(own(K), v);
          } else {
            put(K, own_m, in_m, out_m);
          }
        }
      });
    }
  }
};

template <int Q, typename T, int PAR, bool EDGE, int CM = 0>
__device__ __forceinline__ void fluid_row_cell(const SCArgs &a, int x, int y, int z, size_t rowbase) {
  using R = typename Comp<T>::type;
  const RowCell<Q, T, PAR, EDGE> c(a, x, y, z, rowbase);
  R f[Q];
  c.load(f);
  R z3[3] = {0, 0, 0}, m0[3] = {0, 0, 0}, m1[3] = {0, 0, 0};
  collide<Q, 1, 0, R, CM>(f, a, R(0), z3, R(0), z3, m0, m1);
  c.store(f);
}

// A wave's cell: skip lanes past the row end and, with PSM, cells whose B is
// nonzero (those belong to the solid kernel); without PSM, with a static
// obstacle, obstacle cells and the fluid cells next to them (the obstacle
// kernel takes those).
template <typename R, bool PSM>
__device__ __forceinline__ bool fluid_lane(const SCArgs &a, int x, int y, int z, size_t rowbase) {
  if (x >= a.nx) return false;
  const int x0 = x & ~(a.TX - 1);
  if constexpr (PSM) {
    if (boxes_touch(a, x0, x0 + a.TX - 1, y, y, z, z) && solid_fraction<R>(a, rowbase + (size_t)x) != R(0))
      return false;
  } else {
    if (a.ocls) {
      const IBox &B = a.obox;
      if (x0 + a.TX - 1 >= B.lo[0] && x0 <= B.hi[0] && y >= B.lo[1] && y <= B.hi[1] && z >= B.lo[2] &&
          z <= B.hi[2] && a.ocls[rowbase + (size_t)x] != 0)
        return false;
    }
  }
  return true;
}

// Row r of the rows on a y or z face: the planes z = 0 and z = nz-1, then the
// rows y = 0 and y = ny-1 of the other planes (each row once).
__device__ __forceinline__ void edge_row_yz(const SCArgs &a, int r, int &y, int &z) {
  const int ny = a.ny, nz = a.nz;
  const int nzp = nz >= 2 ? 2 : 1;
  if (r < nzp * ny) {
    z = (r < ny) ? 0 : nz - 1;
    y = r % ny;
    return;
  }
  const int r2 = r - nzp * ny;
  const int nyp = ny >= 2 ? 2 : 1;
  z = 1 + r2 / nyp;
  y = (r2 % nyp) ? ny - 1 : 0;
}

// Rows on a y or z face, TY rows (of the list above) of TX cells per block.
template <int Q, typename T, int PAR, bool PSM, int CM = 0>
__device__ __forceinline__ void edge_block(const SCArgs &a, uint32_t bid) {
  const int tid = threadIdx.x;
  const int txi = (int)(bid % (uint32_t)a.ntx);
  const int r = __builtin_amdgcn_readfirstlane((int)(bid / (uint32_t)a.ntx) * a.TY + (tid >> a.lTX));
  if (r >= a.nfrows) return;
  int y, z;
  edge_row_yz(a, r, y, z);
  const int x = txi * a.TX + (tid & (a.TX - 1));
  const size_t rowbase = (size_t)a.nx * (size_t)y + (size_t)a.nx * (size_t)a.ny * (size_t)z;
  if (!fluid_lane<typename Comp<T>::type, PSM>(a, x, y, z, rowbase)) return;
  fluid_row_cell<Q, T, PAR, true, CM>(a, x, y, z, rowbase);
}

// Odd step, 16-bit storage, interior rows: a wave takes 128 consecutive
// cells of a row, two per lane (xa = x0 + 2 lane, xb = xa + 1), so every
// slot access is a 4-byte pair (2-byte accesses to y/z-shifted rows run at
// ~3 TB/s, 4-byte ones at ~5 TB/s on this chip).  The directions with
// c_kx != 0 need the pair shifted by one cell: the missing half comes from the
// neighbouring lane by DPP, and the wave's two edge elements (x0 - 1 and
// x0 + 128) are read and written one element each.  Every lane of the wave
// must be active; only active cells (fluid, in the row) store, and a value is
// stored only if its own cell is active.
template <int Q, bool PSM, int CM = 0>
__device__ __forceinline__ void fluid_seg_h2(const SCArgs &a, int x0, int y, int z, size_t rowbase) {
  using T = _Float16;
  using R = float;
  typedef _Float16 H2 __attribute__((ext_vector_type(2)));
  auto shr_pair = [](H2 v) {  // lane i <- lane i-1
    return __builtin_bit_cast(H2, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x138, 0xf, 0xf, false));
  };
  auto shl_pair = [](H2 v) {  // lane i <- lane i+1
    return __builtin_bit_cast(H2, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x130, 0xf, 0xf, false));
  };
  const int lane = threadIdx.x & 63;
  const int xa = x0 + 2 * lane, xb = xa + 1;
  const bool acta = fluid_lane<R, PSM>(a, xa, y, z, rowbase);
  const bool actb = fluid_lane<R, PSM>(a, xb, y, z, rowbase);
  const RowCell<Q, T, 1, false> ca(a, xa, y, z, rowbase), cb(a, xb, y, z, rowbase);
  const uint32_t oa = ca.o0;                                      // byte offset of the pair
  const uint32_t om0 = __builtin_amdgcn_readfirstlane(ca.om);     // element x0 - 1 (wrapped / clamped)
  const uint32_t op63 = __builtin_amdgcn_readlane(cb.op, 63);     // element x0 + 128
  // the aligned source pairs, and the wave's edge elements (kept in storage
  // precision until each cell needs them)
  H2 p[Q];
  T e[Q];
  sfor<Q>([&](auto K) {
    constexpr int k = K;
    constexpr int ex = cx<Q>(k);
    char *const rowk = ca.src_base(K);
    p[k] = *(const H2 *)(rowk + oa);
    if constexpr (ex != 0) e[k] = *(const T *)(rowk + (ex == 1 ? om0 : op63));
  });
  auto changed_of = [&](const RowCell<Q, T, 1, false> &c) -> uint32_t {
    return c.xface ? (c.all.own() ^ c.own_m) | (c.all.inlet() ^ c.in_m) | (c.all.outlet() ^ c.out_m) : 0u;
  };
  // first or last cell of a row with a non-periodic x: the directions the x
  // face changes take the merged rule in the cell's own slot
  auto face_store = [&](const RowCell<Q, T, 1, false> &c, const R *f, uint32_t ch) {
    const uint32_t in_x = c.all.inlet(), out_x = c.all.outlet();
    sfor<Q>([&](auto K) {
      constexpr int k = K;
      if constexpr (cx<Q>(k) != 0) {
        if ((ch >> k) & 1u) {
          R v = ((out_x >> k) & 1u) ? f[k] : f[opp<Q>(k)];
          if ((in_x >> k) & 1u) v += inlet_term<Q, R>(a, k);
          stv<T, R>(c.own(K), v);
        }
      }
    });
  };
  const uint32_t cha = changed_of(ca), chb = changed_of(cb);
  R z3[3] = {0, 0, 0}, m0[3] = {0, 0, 0}, m1[3] = {0, 0, 0};
  H2 o[Q];  // post-collision values to store: .x cell a, .y cell b
  {
    R f[Q];
    sfor<Q>([&](auto K) {
      constexpr int k = K;
      constexpr int ex = cx<Q>(k);
      if constexpr (ex == 0) {
        f[k] = (R)p[k].x;  // source xa
      } else if constexpr (ex == 1) {
        const H2 sh = shr_pair(p[k]);  // source xa - 1: high half of the previous pair
        f[k] = (R)(lane == 0 ? e[k] : sh.y);
      } else {
        f[k] = (R)p[k].y;  // source xa + 1
      }
    });
    ca.load_fix(f);
    collide<Q, 1, 0, R, CM>(f, a, R(0), z3, R(0), z3, m0, m1);
    sfor<Q>([&](auto K) { o[(int)K].x = (T)f[opp<Q>((int)K)]; });
    if (ca.xface && acta) face_store(ca, f, cha);
  }
  {
    R f[Q];
    sfor<Q>([&](auto K) {
      constexpr int k = K;
      constexpr int ex = cx<Q>(k);
      if constexpr (ex == 0) {
        f[k] = (R)p[k].y;  // source xb
      } else if constexpr (ex == 1) {
        f[k] = (R)p[k].x;  // source xb - 1 = xa
      } else {
        const H2 sh = shl_pair(p[k]);  // source xb + 1: low half of the next pair
        f[k] = (R)(lane == 63 ? e[k] : sh.x);
      }
    });
    cb.load_fix(f);
    collide<Q, 1, 0, R, CM>(f, a, R(0), z3, R(0), z3, m0, m1);
    sfor<Q>([&](auto K) { o[(int)K].y = (T)f[opp<Q>((int)K)]; });
    if (cb.xface && actb) face_store(cb, f, chb);
  }
  // every cell of the segment is a fluid cell away from the x faces (the
  // common case): the stores need no per-lane conditions but the wave's edges
  if (__all(acta && actb && !ca.xface && !cb.xface)) {
    sfor<Q>([&](auto K) {
      constexpr int k = K;
      constexpr int ex = cx<Q>(k);
      char *const rowk = ca.src_base(K);
      if constexpr (ex == 0) {
        *(H2 *)(rowk + oa) = o[k];
      } else if constexpr (ex == 1) {
        // element xa <- cell b, element xa + 1 <- cell a of the next lane
        // (lane 63: the next wave's, which stores it), element x0 - 1 <- cell a of lane 0
        const H2 nx_ = shl_pair(o[k]);
        H2 v;
        v.x = o[k].y;
        v.y = nx_.x;
        if (lane < 63) *(H2 *)(rowk + oa) = v;
        else *(T *)(rowk + oa) = o[k].y;
        if (lane == 0) *(T *)(rowk + om0) = o[k].x;
      } else {
        // element xa <- cell b of the previous lane (lane 0: the previous
        // wave's), element xa + 1 <- cell a, element x0 + 128 <- cell b of lane 63
        const H2 pv = shr_pair(o[k]);
        H2 v;
        v.x = pv.y;
        v.y = o[k].x;
        if (lane > 0) *(H2 *)(rowk + oa) = v;
        else *(T *)(rowk + oa + sizeof(T)) = o[k].x;
        if (lane == 63) *(T *)(rowk + op63) = o[k].y;
      }
    });
    return;
  }
  const bool acta_n = wave_shl1(acta), actb_p = wave_shr1(actb);
  auto put2 = [&](char *q, T lo, bool lo_ok, T hi, bool hi_ok) {
    if (lo_ok && hi_ok) {
      H2 v;
      v.x = lo;
      v.y = hi;
      *(H2 *)q = v;
    } else {
      if (lo_ok) *(T *)q = lo;
      if (hi_ok) *(T *)(q + sizeof(T)) = hi;
    }
  };
  sfor<Q>([&](auto K) {
    constexpr int k = K;
    constexpr int ex = cx<Q>(k);
    char *const rowk = ca.src_base(K);
    if constexpr (ex == 0) {
      put2(rowk + oa, o[k].x, acta, o[k].y, actb);
    } else if constexpr (ex == 1) {
      // element xa <- cell b, element xa + 1 <- cell a of the next lane,
      // element x0 - 1 <- cell a of lane 0
      const H2 nx_ = shl_pair(o[k]);
      put2(rowk + oa, o[k].y, actb, nx_.x, lane < 63 && acta_n);
      if (lane == 0 && acta && !((cha >> k) & 1u)) *(T *)(rowk + om0) = o[k].x;
    } else {
      // element xa <- cell b of the previous lane, element xa + 1 <- cell a,
      // element x0 + 128 <- cell b of lane 63
      const H2 pv = shr_pair(o[k]);
      put2(rowk + oa, pv.y, lane > 0 && actb_p, o[k].x, acta);
      if (lane == 63 && actb && !((chb >> k) & 1u)) *(T *)(rowk + op63) = o[k].y;
    }
  });
}

// Odd steps with 16-bit storage and rows of a multiple of 128 cells:
// interior rows in segments of 128 cells, one segment per wave
// (fluid_seg_h2).  Other row lengths take k_fluid.  The D3Q27 PSM
// instantiation is held to four waves per SIMD (130 -> 128 VGPRs, 12 bytes
// of spills per lane: rotor pair 3.28 -> 3.02 ms per call); five for D3Q19
// spills more and is slower.
template <int Q, bool PSM, int CM = 0>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu((Q == 27 && PSM) ? 4 : 1, 8))) void k_fluid_h2odd(
    const SCArgs a) {
  const int nsx = a.nx / 128;
  // wave-uniform (one segment per wave): the row arithmetic stays scalar
  const uint32_t seg = (uint32_t)__builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4u + (threadIdx.x >> 6)));
  const uint32_t nseg = (uint32_t)nsx * (uint32_t)(a.ny - 2) * (uint32_t)(a.nz - 2);
  if (seg >= nseg) return;  // wave-uniform
  const int sx = (int)(seg % (uint32_t)nsx);
  const uint32_t r = seg / (uint32_t)nsx;
  const int y = 1 + (int)(r % (uint32_t)(a.ny - 2));
  const int z = 1 + (int)(r / (uint32_t)(a.ny - 2));
  const size_t rowbase = (size_t)a.nx * (size_t)y + (size_t)a.nx * (size_t)a.ny * (size_t)z;
  fluid_seg_h2<Q, PSM, CM>(a, sx * 128, y, z, rowbase);
}

// Interior rows (1 <= y <= ny-2, 1 <= z <= nz-2), TY rows of TX cells per
// workgroup.
template <int Q, typename T, int PAR, bool PSM, int CM = 0>
__global__ __launch_bounds__(256) void k_fluid(const SCArgs a) {
  using R = typename Comp<T>::type;
  if constexpr (PAR == 0 && Q == 19) {
    if (ft_extra_block(a)) return;  // the step's last launch here (face rows ride along)
  }
  const int tid = threadIdx.x;
  if constexpr (PAR == 0 && Q == 19) {
    // even D3Q19 steps: the rows on the y/z faces ride along as extra blocks
    // (there the edge path needs no more registers than the interior one)
    if (blockIdx.x >= a.ntiles_i) {
      edge_block<Q, T, PAR, PSM, CM>(a, blockIdx.x - a.ntiles_i);
      return;
    }
  }
  const uint32_t tile = a.xcd_remap ? xcd_remap(blockIdx.x, a.ntiles_i) : blockIdx.x;
  const int txi = (int)(tile % (uint32_t)a.ntx);
  const uint32_t rr = tile / (uint32_t)a.ntx;
  const int tyi = (int)(rr % (uint32_t)a.nty_i);
  const int z = 1 + (int)(rr / (uint32_t)a.nty_i);
  const int x = txi * a.TX + (tid & (a.TX - 1));
  // TX >= 64: the row is the same over the wave
  const int y = __builtin_amdgcn_readfirstlane(1 + tyi * a.TY + (tid >> a.lTX));
  if (y > a.ny - 2) return;
  const size_t rowbase = (size_t)a.nx * (size_t)y + (size_t)a.nx * (size_t)a.ny * (size_t)z;
  if (!fluid_lane<R, PSM>(a, x, y, z, rowbase)) return;
  fluid_row_cell<Q, T, PAR, false, CM>(a, x, y, z, rowbase);
}


template <int Q, typename T, int PAR, bool PSM, int CM = 0>
__global__ __launch_bounds__(256) void k_fluid_edge(const SCArgs a) {
  if (ft_extra_block(a)) return;
  edge_block<Q, T, PAR, PSM, CM>(a, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Fluid cells with the general per-lane face handling, one thread per cell in
// linear order (the cross-check path of PSM_OPT_GENERAL_PATH).
// ---------------------------------------------------------------------------
template <int Q, typename T, int PAR, int CM = 0>
__device__ __forceinline__ void general_cell(const SCArgs &a, int x, int y, int z, uint64_t n, uint32_t bcm,
                                             uint32_t outm, uint32_t inm) {
  using R = typename Comp<T>::type;
  R f[Q];
  sfor<Q>([&](auto K) {
    constexpr int k = K;
    R v = ldv<T, R>(slot_general<Q, T, PAR>(a, a.pdf, k, x, y, z, n, bcm));
    if constexpr (PAR == 1) {
      if ((inm >> k) & 1u) v += inlet_term<Q, R>(a, k);
    }
    f[k] = v;
  });
  R z3[3] = {0, 0, 0}, m0[3] = {0, 0, 0}, m1[3] = {0, 0, 0};
  collide<Q, 1, 0, R, CM>(f, a, R(0), z3, R(0), z3, m0, m1);
  sfor<Q>([&](auto K) {
    constexpr int k = K;
    R v = ((outm >> k) & 1u) ? f[k] : f[opp<Q>(k)];
    if constexpr (PAR == 1) {
      if ((inm >> k) & 1u) v += inlet_term<Q, R>(a, k);
    }
    stv<T, R>(slot_general<Q, T, PAR>(a, a.pdf, k, x, y, z, n, bcm), v);
  });
}

template <int Q, typename T, int PAR, bool PSM, int CM = 0>
__global__ __launch_bounds__(256) void k_fluid_general(const SCArgs a) {
  using R = typename Comp<T>::type;
  const uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x;
  if (i >= (uint64_t)a.N) return;
  const int x = (int)(i % (uint64_t)a.nx);
  const int y = (int)((i / (uint64_t)a.nx) % (uint64_t)a.ny);
  const int z = (int)(i / ((uint64_t)a.nx * (uint64_t)a.ny));
  const uint64_t n = (uint64_t)x + (uint64_t)a.nx * ((uint64_t)y + (uint64_t)a.ny * (uint64_t)z);
  if constexpr (PSM) {
    if (boxes_touch(a, x, x, y, y, z, z) && solid_fraction<R>(a, n) != R(0)) return;
  } else {
    if (a.ocls && a.ocls[n] != 0) return;
  }
  uint32_t bcm, outm, inm;
  classify<Q>(a, x, y, z, bcm, outm, inm);
  general_cell<Q, T, PAR, CM>(a, x, y, z, n, bcm, outm, inm);
}

// ---------------------------------------------------------------------------
// Fluid cells next to a static obstacle (plain-LBM fields), one thread per
// listed cell: a link into an obstacle cell takes halfway bounce-back, the
// wall rule, ahead of the face kinds (wall > inlet > outlet).  Obstacle cells
// are never touched.
// ---------------------------------------------------------------------------
template <int Q, typename T, int PAR, int CM = 0>
__global__ __launch_bounds__(256) void k_obstacle(const SCArgs a) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= a.ocount) return;
  const uint32_t n = a.olist[2 * (size_t)i], lm = a.olist[2 * (size_t)i + 1];
  const uint32_t nx = (uint32_t)a.nx, nxy = nx * (uint32_t)a.ny;
  const uint32_t z = n / nxy, r = n - z * nxy, y = r / nx, x = r - y * nx;
  uint32_t bcm, outm, inm;
  classify<Q>(a, (int)x, (int)y, (int)z, bcm, outm, inm);
  bcm |= lm;
  outm &= ~lm;
  inm &= ~lm;
  general_cell<Q, T, PAR, CM>(a, (int)x, (int)y, (int)z, (uint64_t)n, bcm, outm, inm);
}

// ---------------------------------------------------------------------------
// Cells with a nonzero solid fraction (inside the bodies' current boxes):
// the PSM blend of eq. (4) with SC1/2/3 over up to two body slots, full face
// handling, and the force / torque of eqs. (10)-(11) on each body.  A fixed
// grid of workgroups walks groups of a.cpw consecutive 256-cell chunks of the
// boxes in a fixed order; a workgroup first lists the group's cells with
// B != 0 in LDS (ascending order), then updates the list in whole rounds of
// 256 cells (a short remainder waits for the workgroup's next group), so thin
// or sparse solids still fill whole waves.  NS: fraction slots of the field
// (the two-body blend exists only in the NS = 2 instantiation: one slot needs
// fewer registers, 3 waves per SIMD instead of 2 for D3Q19 FP32).  Per-body FP64 sums are
// kept per wave in LDS, added across the waves once and written once per
// workgroup (fixed order: deterministic).  A cell inside several boxes is
// taken by the lowest-index box.
// ---------------------------------------------------------------------------
// D3Q19 even steps with one fraction slot and FP32 or FP16 storage fit four
// waves per SIMD without spills (128 VGPRs; rotor box +1.1%); the other
// instantiations keep the compiler's choice (four waves there spill).
template <int Q, typename T, int PAR, int SC, int CM, int NS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(
    (PAR == 0 && NS == 1 && Q == 19 && sizeof(T) <= 4) ? 4 : 1, 8))) void k_solid(const SCArgs a) {
  using R = typename Comp<T>::type;
  __shared__ double wacc[4][PSM_MAX_BODIES][6];  // per-wave F/T sums (each wave writes only its own)
  // listed cells: fewer than 256 left over from earlier groups, then this group's
  constexpr int LCAP = SOLID_MAX_CPW * 256 + 256;
  __shared__ uint32_t cells_l[LCAP];
  __shared__ R bfrac_l[LCAP];
  __shared__ uint8_t meta_l[LCAP];
  __shared__ uint32_t wcnt[SOLID_MAX_CPW][4];
  const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63;
  if (tid < 4 * PSM_MAX_BODIES * 6) (&wacc[0][0][0])[tid] = 0.0;
  __syncthreads();
  const uint32_t cpw = (uint32_t)a.cpw;
  const uint32_t ngroups = (a.nchunks + cpw - 1) / cpw;
  const uint32_t nx = (uint32_t)a.nx, nxy = nx * (uint32_t)a.ny;
  uint32_t pending = 0;  // listed cells not yet updated (wave-uniform)
  for (uint32_t grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
    // 1. the group's cells with B != 0, appended to the list in ascending
    //    (chunk, thread) order with their slot-0 fraction and body ids
    uint32_t mine[SOLID_MAX_CPW];
    R bmine[SOLID_MAX_CPW];
    uint8_t mmine[SOLID_MAX_CPW];
    bool hit[SOLID_MAX_CPW];
#pragma unroll
    for (int j = 0; j < SOLID_MAX_CPW; ++j) {
      hit[j] = false;
      mine[j] = 0;
      bmine[j] = R(0);
      mmine[j] = 0;
      const uint32_t ch = grp * cpw + (uint32_t)j;
      if ((uint32_t)j < cpw && ch < a.nchunks) {
        int rb = 0;
        while (rb + 1 < a.nbox && ch >= a.cprefix[rb + 1]) ++rb;
        const IBox &G = a.box[rb];
        const uint64_t idx64 = (uint64_t)(ch - a.cprefix[rb]) * 256u + (uint64_t)tid;
        const uint32_t ex_ = (uint32_t)(G.hi[0] - G.lo[0] + 1), ey_ = (uint32_t)(G.hi[1] - G.lo[1] + 1);
        const uint64_t cells = (uint64_t)ex_ * ey_ * (uint64_t)(G.hi[2] - G.lo[2] + 1);
        if (idx64 < cells) {
          const uint32_t idx = (uint32_t)idx64;
          const uint32_t bz = idx / (ex_ * ey_), br = idx - bz * ex_ * ey_, by = br / ex_, bx = br - by * ex_;
          const int x = G.lo[0] + (int)bx, y = G.lo[1] + (int)by, z = G.lo[2] + (int)bz;
          bool act = true;
          for (int b = 0; b < rb; ++b)
            if (box_has(a.box[b], x, y, z)) act = false;
          const uint32_t n = (uint32_t)x + nx * (uint32_t)y + nxy * (uint32_t)z;
          const R b = solid_fraction<R>(a, n);
          mmine[j] = a.meta[n];
          hit[j] = act && b != R(0);
          mine[j] = n;
          bmine[j] = b;
        }
      }
      const unsigned long long bm = __ballot(hit[j]);
      if (lane == 0) wcnt[j][wid] = (uint32_t)__popcll(bm);
    }
    __syncthreads();
    uint32_t total = pending;
#pragma unroll
    for (int j = 0; j < SOLID_MAX_CPW; ++j) {
      const unsigned long long bm = __ballot(hit[j]);
      uint32_t off = total;
      for (int w = 0; w < wid; ++w) off += wcnt[j][w];
      if (hit[j]) {
        const uint32_t e = off + (uint32_t)__popcll(bm & ((1ull << lane) - 1ull));
        cells_l[e] = mine[j];
        bfrac_l[e] = bmine[j];
        meta_l[e] = mmine[j];
      }
      total += (wcnt[j][0] + wcnt[j][1]) + (wcnt[j][2] + wcnt[j][3]);
    }
    __syncthreads();
    // 2. the listed cells in whole rounds of 256 (the workgroup's last group:
    //    all of them); a short remainder waits for the next group, so that
    //    sparse boxes still fill the waves
    const bool last_grp = grp + gridDim.x >= ngroups;
    const uint32_t nproc = last_grp ? total : (total & ~255u);
    for (uint32_t base = 0; base < nproc; base += 256) {
      const uint32_t li = base + (uint32_t)tid;
      bool act = li < nproc;
      const uint32_t n = act ? cells_l[li] : 0u;
      const int z = (int)(n / nxy), y = (int)((n - (uint32_t)z * nxy) / nx),
                x = (int)(n - (uint32_t)z * nxy - (uint32_t)y * nx);
      R B0 = 0, B1 = 0;
      int b0 = 0, b1 = 0;
      bool two = false;
      if (act) {
        B0 = bfrac_l[li];
        const uint8_t m = meta_l[li];
        b0 = m & 15;
        if (b0 >= a.nb) b0 = 0;  // ids come from the mapping; never index past the body table
        if (NS == 2 && (m >> 4)) {
          b1 = (m >> 4) - 1;
          if (b1 >= a.nb) b1 = 0;
          B1 = (R)a.B1[n];
          two = true;
        }
      }
      R mom0[3] = {0, 0, 0}, mom1[3] = {0, 0, 0};
      const double xc = x + 0.5, yc = y + 0.5, zc = z + 0.5;
      if (__any(act)) {  // wave-uniform: waves past the list's end skip the update
        uint32_t bcm = 0, outm = 0, inm = 0;
        R f[Q];
        if (act) {
          classify<Q>(a, x, y, z, bcm, outm, inm);
          sfor<Q>([&](auto K) {
            constexpr int k = K;
            R v = ldv<T, R>(slot_general<Q, T, PAR>(a, a.pdf, k, x, y, z, n, bcm));
            if constexpr (PAR == 1) {
              if ((inm >> k) & 1u) v += inlet_term<Q, R>(a, k);
            }
            f[k] = v;
          });
        } else {
          sfor<Q>([&](auto K) { f[K] = R(0); });
        }
        R us0[3] = {0, 0, 0}, us1[3] = {0, 0, 0};
        for (int b = 0; b < a.nb; ++b) {  // uniform loop: body data stays scalar
          const BodyK &bd = a.body[b];
          if (act && (b0 == b || (two && b1 == b))) {
            const R rx = (R)(xc - bd.X[0]), ry = (R)(yc - bd.X[1]), rz = (R)(zc - bd.X[2]);
            const R wx = (R)bd.W[0], wy = (R)bd.W[1], wz = (R)bd.W[2];
            R u0 = (R)bd.V[0] + (wy * rz - wz * ry);
            R u1 = (R)bd.V[1] + (wz * rx - wx * rz);
            R u2 = (R)bd.V[2] + (wx * ry - wy * rx);
            if (b0 == b) {
              us0[0] = u0;
              us0[1] = u1;
              us0[2] = u2;
            }
            if (two && b1 == b) {
              us1[0] = u0;
              us1[1] = u1;
              us1[2] = u2;
            }
          }
        }
        if (NS == 2 && __any(two)) {
          collide<Q, SC, 2, R, CM>(f, a, B0, us0, B1, us1, mom0, mom1);
        } else {
          collide<Q, SC, 1, R, CM>(f, a, B0, us0, B1, us1, mom0, mom1);
        }
        if (act) {
          sfor<Q>([&](auto K) {
            constexpr int k = K;
            R v = ((outm >> k) & 1u) ? f[k] : f[opp<Q>(k)];
            if constexpr (PAR == 1) {
              if ((inm >> k) & 1u) v += inlet_term<Q, R>(a, k);
            }
            stv<T, R>(slot_general<Q, T, PAR>(a, a.pdf, k, x, y, z, n, bcm), v);
          });
        }
      }
      // force / torque on each body touched by these cells, summed per wave
      // (fixed lane tree, rounds in order) into the wave's own slots
      for (int b = 0; b < a.nb; ++b) {
        const bool has = act && (b0 == b || (two && b1 == b));
        if (!__any(has)) continue;  // wave-uniform
        const BodyK &bd = a.body[b];
        double v0 = 0, v1 = 0, v2 = 0;
        if (act && b0 == b) {
          v0 += (double)mom0[0];
          v1 += (double)mom0[1];
          v2 += (double)mom0[2];
        }
        if (act && two && b1 == b) {
          v0 += (double)mom1[0];
          v1 += (double)mom1[1];
          v2 += (double)mom1[2];
        }
        const double rx = xc - bd.X[0], ry = yc - bd.X[1], rz = zc - bd.X[2];
        double v3 = ry * v2 - rz * v1, v4 = rz * v0 - rx * v2, v5 = rx * v1 - ry * v0;
        v0 = wave_sum(v0);
        v1 = wave_sum(v1);
        v2 = wave_sum(v2);
        v3 = wave_sum(v3);
        v4 = wave_sum(v4);
        v5 = wave_sum(v5);
        if (lane == 0) {
          wacc[wid][b][0] += v0;
          wacc[wid][b][1] += v1;
          wacc[wid][b][2] += v2;
          wacc[wid][b][3] += v3;
          wacc[wid][b][4] += v4;
          wacc[wid][b][5] += v5;
        }
      }
    }
    // the remainder (fewer than 256, none after the last group) moves to the
    // front; the next group appends after it
    pending = total - nproc;
    __syncthreads();
    if (pending && nproc) {
      uint32_t c = 0;
      R bv = R(0);
      uint8_t mv = 0;
      if ((uint32_t)tid < pending) {
        c = cells_l[nproc + tid];
        bv = bfrac_l[nproc + tid];
        mv = meta_l[nproc + tid];
      }
      __syncthreads();
      if ((uint32_t)tid < pending) {
        cells_l[tid] = c;
        bfrac_l[tid] = bv;
        meta_l[tid] = mv;
      }
      __syncthreads();
    }
  }
  __syncthreads();
  if (tid < a.nb * 6) {
    const int b = tid / 6, c = tid % 6;
    a.ftp[((size_t)blockIdx.x * a.max_bodies + b) * 6 + c] = ((wacc[0][b][c] + wacc[1][b][c]) + wacc[2][b][c]) + wacc[3][b][c];
  }
}

}  // namespace psm
