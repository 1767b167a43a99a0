// Reverse-mode (adjoint) PSM step for one body, SC1, frozen solid fractions.
//
// Objective per step: J_t = wt * a . T(t), the torque of body 0 about X along
// the unit axis a (eq. (11), force on the body).  With gh = dJ/df*(x) (the
// adjoint of the post-collision values, gathered by transposing the
// streaming and the face rules) the step computes, per cell,
//   fhat_j = gh_j + (1 - B) [dOmega^F/df]^T gh + [dOmega^S/df]^T sh,
//   sh_i   = B (gh_i - wt m_i),   m_i = c_i . (a x r),  r = x_c - X,
//   dJ/dB += sum_i (gh_i - wt m_i) Omega^S_i - sum_i gh_i Omega^F_i,
//   dJ/dOmega += (a x r) . sum_i sh_i dfeq_i(rho, u_s)/du_s,
// where the transposed Jacobians of the TRT + Guo fluid collision and of SC1
// contract to O(Q) work through rho = sum f and u = (sum c f + F/2)/rho:
//   sum_i b_i dfeq_i/df_j = G_rho + G_u . (c_j - u)/rho,
//   dfeq_i/drho = feq_i/rho,  dfeq_i/du = w_i rho [3 c_i + 9 (c_i.u) c_i - 3 u],
//   dS_i/du = w_i [-3 F + 9 (c_i.F) c_i].
// The forward state (a copy of the PDF buffer) and both adjoint buffers are
// in the PDF buffer's layout: for a cell, one offset in elements serves all
// three (the adjoint buffers in the adjoint precision).
#include "k_stream_collide.hpp"

namespace psm {



// c . v for a lattice direction with compile-time components in {-1, 0, 1}
// (adds and subtracts only: a product by 0 or +-1 is not folded otherwise).
template <int EX, int EY, int EZ, typename R>
__device__ __forceinline__ R cdot(R vx, R vy, R vz) {
  constexpr int nz = (EX != 0) + (EY != 0) + (EZ != 0);
  static_assert(nz > 0, "rest direction has no dot product");
  R s;
  bool have = false;
  auto add = [&](int e, R v) {
    const R t = e > 0 ? v : -v;
    s = have ? s + t : t;
    have = true;
  };
  if constexpr (EX != 0) add(EX, vx);
  if constexpr (EY != 0) add(EY, vy);
  if constexpr (EZ != 0) add(EZ, vz);
  return s;
}

// v += k c for a lattice direction c
template <int EX, int EY, int EZ, typename R>
__device__ __forceinline__ void cacc(R &vx, R &vy, R &vz, R k) {
  if constexpr (EX == 1) vx += k;
  if constexpr (EX == -1) vx -= k;
  if constexpr (EY == 1) vy += k;
  if constexpr (EY == -1) vy -= k;
  if constexpr (EZ == 1) vz += k;
  if constexpr (EZ == -1) vz -= k;
}

// The step is written over opposite pairs (i, ib): for any per-direction
// vectors a, b, a_i b_i + a_ib b_ib = 2 (a+ b+ + a- b-) with a+- = (a_i +- a_ib)/2,
// and feq, the Guo term and their u-derivatives split into even and odd parts
// with c_ib = -c_i.  With phi_i = feq_i / rho, for any v:
//   sum_i v_i phi_i          = (1 - 3/2 u^2) W(v) + sum_pairs w [9 v+ cu^2 + 6 v- cu]
//   sum_i v_i dfeq_i/du / rho = sum_pairs w (6 v- + 18 v+ cu) c - 3 u W(v)
// where W(v) = sum_i w_i v_i and cu = c.u over the pair's first direction.  The
// fluid part takes v = b (b+ = le g+, b- = lo g-), the solid part v_i = sh_ib
// (v+ = sh+, v- = -sh-) at u and v = sh at u_s, the Guo derivative
// dS_i/du = w (-3 F + 9 (c.F) c) is even.  Collecting terms,
//   fhat_j = gh_j - (1 - B) b_j + (sh_jb - sh_j) + C0 + V . c_j
// with one scalar C0 and one vector V per cell, both sums over the pairs.
//
// One cell: x per lane, the row (y, z) shared by the wave.  Returns the
// cell's dJ/dOmega term.
template <int Q, typename T, int PAR, bool O32, bool FRC>
__device__ __forceinline__ double adjoint_cell(const AdjArgs &A, uint32_t row, uint32_t yy, uint32_t zz,
                                               uint32_t xx) {
  using R = typename Comp<T>::type;
  constexpr int H = Lat<Q>::H;
  const SCArgs &a = A.s;
  const uint32_t nx = (uint32_t)a.nx, ny = (uint32_t)a.ny, nz = (uint32_t)a.nz;
  const uint32_t n = row * nx + xx;
  const int x = (int)xx, y = (int)yy, z = (int)zz;
  // periodic neighbours (used only where the direction is not a face
  // direction of this cell): rows are wave-uniform, x per lane
  const uint32_t ym = yy == 0 ? ny - 1 : yy - 1, yp = yy + 1 == ny ? 0u : yy + 1;
  const uint32_t zm = zz == 0 ? nz - 1 : zz - 1, zp = zz + 1 == nz ? 0u : zz + 1;
  const uint32_t xm = xx == 0 ? nx - 1 : xx - 1, xp = xx + 1 == nx ? 0u : xx + 1;
  auto rowof = [&](int ey, int ez) -> uint32_t {
    return (ey < 0 ? ym : ey > 0 ? yp : yy) + ny * (ez < 0 ? zm : ez > 0 ? zp : zz);
  };
  auto xof = [&](int ex) -> uint32_t { return ex < 0 ? xm : ex > 0 ? xp : xx; };
  uint32_t bcm, outm, inm;
  classify<Q>(a, x, y, z, bcm, outm, inm);
  // forward state before the step, as deviations d_k = f_k - w_k, and the
  // adjoint gh of the post-collision values (transpose of the streaming)
  // Element offsets in 32 bits when every array spans fewer than 2^32 bytes
  // (a uniform base plus a 32-bit lane offset per access), else 64.
  using Off = typename std::conditional<O32, uint32_t, uint64_t>::type;
  const Off DS = (Off)a.dS, NX = (Off)nx;
  auto el = [&](int k, uint32_t r, uint32_t xe) -> Off {
    return (Off)(r >> a.lrb) * (Off)a.bst + (Off)(r & a.rbm) * NX + (Off)k * DS + (Off)xe;
  };
  auto F = [&](int k, uint32_t r, uint32_t xe) -> const T * {
    return (const T *)((const char *)A.fwd + (uint64_t)(el(k, r, xe) * (Off)sizeof(T)));
  };
  auto G = [&](int k, uint32_t r, uint32_t xe) -> R {
    return *(const R *)((const char *)A.ain + (uint64_t)(el(k, r, xe) * (Off)sizeof(R)));
  };
  auto O = [&](int k) -> R * { return (R *)((char *)A.aout + (uint64_t)(el(k, row, xx) * (Off)sizeof(R))); };
  R d[Q], gh[Q];
  if (bcm == 0) {  // no face direction: plain pulls / pushes with periodic wrap
    sfor<Q>([&](auto K) {
      constexpr int k = K;
      constexpr int ex = cx<Q>(k), ey = cy<Q>(k), ez = cz<Q>(k);
      if constexpr (PAR == 0 || k == 0) d[k] = (R)*F(k, row, xx);
      else d[k] = (R)*F(opp<Q>(k), rowof(-ey, -ez), xof(-ex));
      if constexpr (k == 0) gh[k] = G(0, row, xx);
      else gh[k] = G(k, rowof(ey, ez), xof(ex));
    });
  } else {
    sfor<Q>([&](auto K) {
      constexpr int k = K;
      constexpr int ex = cx<Q>(k), ey = cy<Q>(k), ez = cz<Q>(k);
      const T *own = F(k, row, xx);
      R v;
      if constexpr (PAR == 0 || k == 0) {
        v = (R)*own;
      } else {
        const T *p = ((bcm >> k) & 1u) ? own : F(opp<Q>(k), rowof(-ey, -ez), xof(-ex));
        v = (R)*p;
        if ((inm >> k) & 1u) v += inlet_term<Q, R>(a, k);
      }
      d[k] = v;
    });
    sfor<Q>([&](auto K) {
      constexpr int i = K;
      constexpr int ib = opp<Q>(i);
      constexpr int ex = cx<Q>(i), ey = cy<Q>(i), ez = cz<Q>(i);
      R g = 0;
      if constexpr (i == 0) {
        g = G(0, row, xx);
      } else {
        // f*_i(x) streams to x + c_i unless that neighbour's source (x) is
        // outside for it, i.e. unless direction ib is a face direction here
        if (!((bcm >> ib) & 1u)) g += G(i, rowof(ey, ez), xof(ex));
        else if (!((outm >> ib) & 1u)) g += G(ib, row, xx);  // bounced back into direction ib
        if ((outm >> i) & 1u) g += G(i, row, xx);              // outlet: f_i(x) = f*_i(x)
      }
      gh[i] = g;
    });
  }
  // forward recompute: rho, u, and the per-cell constants
  R drho = d[0], jx = 0, jy = 0, jz = 0;
  sfor<H>([&](auto P) {
    constexpr int i = P + 1, ib = opp<Q>(i);
    drho += d[i] + d[ib];
    cacc<cx<Q>(i), cy<Q>(i), cz<Q>(i)>(jx, jy, jz, d[i] - d[ib]);
  });
  const R rho = R(1) + drho, ir = R(1) / rho;
  // FRC = false: no body force, its terms dropped at compile time
  const R Fx = FRC ? (R)a.force[0] : R(0), Fy = FRC ? (R)a.force[1] : R(0), Fz = FRC ? (R)a.force[2] : R(0);
  const R ux = FRC ? (jx + R(0.5) * Fx) * ir : jx * ir, uy = FRC ? (jy + R(0.5) * Fy) * ir : jy * ir,
          uz = FRC ? (jz + R(0.5) * Fz) * ir : jz * ir;
  const R Frx = Fx * ir, Fry = Fy * ir, Frz = Fz * ir;
  const R usq = ux * ux + uy * uy + uz * uz, uF = FRC ? ux * Fx + uy * Fy + uz * Fz : R(0);
  const R B = solid_fraction<R>(a, n), fl = R(1) - B;
  const double rx = x + 0.5 - A.X[0], ry = y + 0.5 - A.X[1], rz = z + 0.5 - A.X[2];
  const R usx = (R)(A.V[0] + (A.W[1] * rz - A.W[2] * ry));
  const R usy = (R)(A.V[1] + (A.W[2] * rx - A.W[0] * rz));
  const R usz = (R)(A.V[2] + (A.W[0] * ry - A.W[1] * rx));
  const R uss = usx * usx + usy * usy + usz * usz;
  // a x r: torque lever per unit force along c_i
  const R arx = (R)(A.axis[1] * rz - A.axis[2] * ry), ary = (R)(A.axis[2] * rx - A.axis[0] * rz),
          arz = (R)(A.axis[0] * ry - A.axis[1] * rx);
  const R wtt = (R)A.wt;
  const R le = (R)a.lam_e, lo = (R)a.lam_o;
  const R ge = R(1) - R(0.5) * le, go = R(1) - R(0.5) * lo;
  const R dus = R(1.5) * (uss - usq);
  // rest direction
  R Wg, dJ;
  {
    const R w0 = (R)wt<Q>(0);
    const R fe = d[0] - w0 * (drho - rho * R(1.5) * usq);
    const R OF = FRC ? -le * fe - ge * R(3) * w0 * uF : -le * fe;
    const R OS = -w0 * rho * dus;
    Wg = w0 * gh[0];
    dJ = R(0.5) * gh[0] * (OS - OF);
  }
  R Vx = 0, Vy = 0, Vz = 0, C0 = 0, dS = 0, Wg2 = 0;
  sfor<H>([&](auto P) {
    constexpr int i = P + 1, ib = opp<Q>(i);
    constexpr int ex = cx<Q>(i), ey = cy<Q>(i), ez = cz<Q>(i);
    const R wi = (R)wt<Q>(i);
    const R gp = R(0.5) * (gh[i] + gh[ib]), gm = R(0.5) * (gh[i] - gh[ib]);
    const R dp = R(0.5) * (d[i] + d[ib]), dm = R(0.5) * (d[i] - d[ib]);
    const R cu = cdot<ex, ey, ez>(ux, uy, uz), cs = cdot<ex, ey, ez>(usx, usy, usz);
    const R cF = FRC ? cdot<ex, ey, ez>(Fx, Fy, Fz) : R(0), cFr = FRC ? cdot<ex, ey, ez>(Frx, Fry, Frz) : R(0);
    const R m = cdot<ex, ey, ez>(arx, ary, arz);
    const R cu2 = cu * cu, cs2 = cs * cs;
    // TRT + Guo (even / odd parts) and SC1 collision of the pair
    const R fpe = dp - wi * (drho + rho * (R(4.5) * cu2 - R(1.5) * usq));
    const R fme = dm - R(3) * wi * rho * cu;
    const R OFp = FRC ? -le * fpe + ge * wi * (R(9) * cu * cF - R(3) * uF) : -le * fpe;
    const R OFm = FRC ? -lo * fme + go * R(3) * wi * cF : -lo * fme;
    const R OSp = wi * rho * (R(4.5) * (cs2 - cu2) - dus);
    const R OSm = R(-2) * dm + R(3) * wi * rho * (cu + cs);
    const R qm = gm - wtt * m;
    dJ += gp * (OSp - OFp) + qm * OSm - gm * OFm;
    const R shp = B * gp, shm = B * qm;
    const R kap = wi * (fl * (R(6) * lo * gm + R(18) * gp * (FRC ? le * cu + ge * cFr : le * cu)) + R(6) * shm -
                        R(18) * shp * cu);
    cacc<ex, ey, ez>(Vx, Vy, Vz, kap);
    C0 += wi * (R(9) * shp * (cu2 + cs2) + R(6) * shm * cs -
                fl * gp * cu * (FRC ? R(9) * le * cu + R(18) * ge * cFr : R(9) * le * cu));
    dS += wi * (R(6) * shm + R(18) * shp * cs) * m;
    Wg2 += wi * gp;
  });
  Wg += R(2) * Wg2;
  const R Ws = B * Wg;
  if constexpr (FRC) {
    C0 += fl * Wg * (le * (R(1) + R(1.5) * usq) + R(3) * ge * (Frx * ux + Fry * uy + Frz * uz)) -
          R(1.5) * (usq + uss) * Ws;
    Vx -= R(3) * (fl * Wg * (le * ux + ge * Frx) - ux * Ws);
    Vy -= R(3) * (fl * Wg * (le * uy + ge * Fry) - uy * Ws);
    Vz -= R(3) * (fl * Wg * (le * uz + ge * Frz) - uz * Ws);
  } else {
    C0 += fl * Wg * (le * (R(1) + R(1.5) * usq)) - R(1.5) * (usq + uss) * Ws;
    Vx -= R(3) * (fl * Wg * (le * ux) - ux * Ws);
    Vy -= R(3) * (fl * Wg * (le * uy) - uy * Ws);
    Vz -= R(3) * (fl * Wg * (le * uz) - uz * Ws);
  }
  *O(0) = gh[0] - fl * le * gh[0] + C0;
  sfor<H>([&](auto P) {
    constexpr int i = P + 1, ib = opp<Q>(i);
    constexpr int ex = cx<Q>(i), ey = cy<Q>(i), ez = cz<Q>(i);
    const R gp = R(0.5) * (gh[i] + gh[ib]), gm = R(0.5) * (gh[i] - gh[ib]);
    const R shm = B * (gm - wtt * cdot<ex, ey, ez>(arx, ary, arz));
    const R vc = cdot<ex, ey, ez>(Vx, Vy, Vz);
    const R bp = le * gp, bm = lo * gm;
    *O(i) = gh[i] - fl * (bp + bm) - R(2) * shm + C0 + vc;
    *O(ib) = gh[ib] - fl * (bp - bm) + R(2) * shm + C0 - vc;
  });
  R *gB = (R *)A.dJdB;
  gB[n] += R(2) * dJ;
  return (double)(rho * (dS - R(3) * (arx * usx + ary * usy + arz * usz) * Ws));
}

// One wave per work unit of up to 64 cells of one row (ceil(nx / 64) units
// per row); one FP64 dJ/dOmega partial per workgroup.
// Without body force the FP32-arithmetic D3Q19 kernels fit five waves per
// SIMD (100 -> 96 VGPRs, 8-12 bytes of spills per lane; 128^3 rotor backward
// 0.130 -> 0.120 s); the others keep the compiler's choice.
template <int Q, typename T, int PAR, bool O32, bool FRC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu((Q == 19 && !FRC && sizeof(T) <= 4) ? 5 : 1, 8))) void
k_adjoint(const AdjArgs A) {
  const SCArgs &a = A.s;
  const uint32_t nx = (uint32_t)a.nx, ny = (uint32_t)a.ny;
  const uint32_t segs = (nx + 63u) >> 6, units = ny * (uint32_t)a.nz * segs;
  const uint32_t u = __builtin_amdgcn_readfirstlane(blockIdx.x * 4u + (threadIdx.x >> 6));
  double dom = 0.0;
  if (u < units) {
    const uint32_t row = u / segs, xx = (u - row * segs) * 64u + (threadIdx.x & 63u);
    const uint32_t zz = row / ny, yy = row - zz * ny;
    if (xx < nx) dom = adjoint_cell<Q, T, PAR, O32, FRC>(A, row, yy, zz, xx);
  }
  __shared__ double sh4[4];
  double v = wave_sum(dom);
  if ((threadIdx.x & 63) == 0) sh4[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) A.part[blockIdx.x] = ((sh4[0] + sh4[1]) + sh4[2]) + sh4[3];
}

template <int Q, typename T, bool O32, bool FRC>
static void go_adjoint(const AdjArgs &A, dim3 g, hipStream_t st) {
  if (A.parity == 0) hipLaunchKernelGGL((k_adjoint<Q, T, 0, O32, FRC>), g, dim3(256), 0, st, A);
  else hipLaunchKernelGGL((k_adjoint<Q, T, 1, O32, FRC>), g, dim3(256), 0, st, A);
}

template <int Q, typename T>
static void go_adjoint(const AdjArgs &A, dim3 g, hipStream_t st) {
  const bool frc = A.s.force[0] != 0.0 || A.s.force[1] != 0.0 || A.s.force[2] != 0.0;
  if (A.o32 && frc) go_adjoint<Q, T, true, true>(A, g, st);
  else if (A.o32) go_adjoint<Q, T, true, false>(A, g, st);
  else if (frc) go_adjoint<Q, T, false, true>(A, g, st);
  else go_adjoint<Q, T, false, false>(A, g, st);
}

hipError_t launch_adjoint(const psm_field &f, const AdjArgs &A, hipStream_t st) {
  const dim3 g(adjoint_blocks(f.cfg.nx, f.cfg.ny, f.cfg.nz));
  const int q = f.cfg.q, sto = f.cfg.storage;
  if (q == 19 && sto == PSM_F64) go_adjoint<19, double>(A, g, st);
  else if (q == 19 && sto == PSM_F32) go_adjoint<19, float>(A, g, st);
  else if (q == 19) go_adjoint<19, _Float16>(A, g, st);
  else if (sto == PSM_F64) go_adjoint<27, double>(A, g, st);
  else if (sto == PSM_F32) go_adjoint<27, float>(A, g, st);
  else go_adjoint<27, _Float16>(A, g, st);
  return hipGetLastError();
}

// out[0] += sum of p[0..n) in a fixed order (1024 strided partial sums, then
// a fixed wave / workgroup tree).
__global__ __launch_bounds__(1024) void k_sum_accumulate(const double *p, uint32_t n, double *out) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  uint32_t i = threadIdx.x;
  for (; i + 3 * 1024 < n; i += 4 * 1024) {
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] += p[i + u * 1024];
  }
  if (i < n) acc[0] += p[i];  // at most three strides remain
  if (i + 1024 < n) acc[1] += p[i + 1024];
  if (i + 2048 < n) acc[2] += p[i + 2048];
  double v = wave_sum((acc[0] + acc[1]) + (acc[2] + acc[3]));
  __shared__ double sh[16];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < 16; ++w) s += sh[w];
    out[0] += s;
  }
}

hipError_t launch_sum_accumulate(const double *p, uint32_t n, double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_accumulate, dim3(1), dim3(1024), 0, st, p, n, out);
  return hipGetLastError();
}

}  // namespace psm
