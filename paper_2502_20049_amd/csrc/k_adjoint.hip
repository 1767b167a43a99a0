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
// The adjoint PDFs are stored in the standard layout, two buffers.
#include "k_stream_collide.hpp"

namespace psm {



template <int Q, typename T>
__global__ __launch_bounds__(256) void k_adjoint(const AdjArgs A) {
  using R = typename Comp<T>::type;
  const SCArgs &a = A.s;
  const uint64_t n = (uint64_t)blockIdx.x * 256u + threadIdx.x;
  const bool act = n < (uint64_t)a.N;
  double dom = 0.0;
  if (act) {
    const int x = (int)(n % (uint64_t)a.nx);
    const int y = (int)((n / (uint64_t)a.nx) % (uint64_t)a.ny);
    const int z = (int)(n / ((uint64_t)a.nx * (uint64_t)a.ny));
    const uint64_t N = a.N;
    uint32_t bcm, outm, inm;
    classify<Q>(a, x, y, z, bcm, outm, inm);
    // forward state f(t) (full values f = w + delta f)
    char *fwd = (char *)A.fwd;
    R f[Q];
    sfor<Q>([&](auto K) {
      constexpr int k = K;
      R v = (A.parity == 0) ? ldv<T, R>(slot_general<Q, T, 0>(a, fwd, k, x, y, z, n, bcm))
                            : ldv<T, R>(slot_general<Q, T, 1>(a, fwd, k, x, y, z, n, bcm));
      if (A.parity == 1 && ((inm >> k) & 1u)) v += inlet_term<Q, R>(a, k);
      f[k] = v + R(wt<Q>(k));
    });
    // adjoint of the post-collision values: transpose of the streaming
    const R *ain = (const R *)A.ain;
    R gh[Q];
    sfor<Q>([&](auto K) {
      constexpr int i = K;
      constexpr int ib = opp<Q>(i);
      R g = 0;
      // f*_i(x) streams to x + c_i unless that neighbour's source (x) is
      // outside for it, i.e. unless direction ib is a face direction here
      if (!((bcm >> ib) & 1u)) {
        int px = x + cx<Q>(i), py = y + cy<Q>(i), pz = z + cz<Q>(i);
        if (px < 0) px += a.nx;
        if (px >= a.nx) px -= a.nx;
        if (py < 0) py += a.ny;
        if (py >= a.ny) py -= a.ny;
        if (pz < 0) pz += a.nz;
        if (pz >= a.nz) pz -= a.nz;
        const uint64_t m = (uint64_t)px + (uint64_t)a.nx * ((uint64_t)py + (uint64_t)a.ny * (uint64_t)pz);
        g += ain[(uint64_t)i * N + m];
      } else if (!((outm >> ib) & 1u)) {
        g += ain[(uint64_t)ib * N + n];  // bounced back by a wall / inlet into direction ib
      }
      if ((outm >> i) & 1u) g += ain[(uint64_t)i * N + n];  // outlet: f_i(x) = f*_i(x)
      gh[i] = g;
    });
    // forward recompute
    R rho = 0, jx = 0, jy = 0, jz = 0;
    sfor<Q>([&](auto K) {
      constexpr int k = K;
      rho += f[k];
      jx += R(cx<Q>(k)) * f[k];
      jy += R(cy<Q>(k)) * f[k];
      jz += R(cz<Q>(k)) * f[k];
    });
    const R Fx = (R)a.force[0], Fy = (R)a.force[1], Fz = (R)a.force[2];
    const R ux = (jx + R(0.5) * Fx) / rho, uy = (jy + R(0.5) * Fy) / rho, uz = (jz + R(0.5) * Fz) / rho;
    const R usq = ux * ux + uy * uy + uz * uz;
    R B = a.B0 ? (R)a.B0[n] : R(0);
    if (a.dB) B += (R)a.dB[n];
    const double rx = x + 0.5 - A.X[0], ry = y + 0.5 - A.X[1], rz = z + 0.5 - A.X[2];
    const R usx = (R)(A.V[0] + (A.W[1] * rz - A.W[2] * ry));
    const R usy = (R)(A.V[1] + (A.W[2] * rx - A.W[0] * rz));
    const R usz = (R)(A.V[2] + (A.W[0] * ry - A.W[1] * rx));
    const R uss = usx * usx + usy * usy + usz * usz;
    // a x r (torque lever per unit force along c_i)
    const R arx = (R)(A.axis[1] * rz - A.axis[2] * ry), ary = (R)(A.axis[2] * rx - A.axis[0] * rz),
            arz = (R)(A.axis[0] * ry - A.axis[1] * rx);
    const R wtt = (R)A.wt;
    const R le = (R)a.lam_e, lo = (R)a.lam_o;
    const R ge = R(1) - R(0.5) * le, go = R(1) - R(0.5) * lo;
    R feq[Q], feqs[Q], S[Q];
    sfor<Q>([&](auto K) {
      constexpr int i = K;
      const R w = (R)wt<Q>(i);
      const R cu = R(cx<Q>(i)) * ux + R(cy<Q>(i)) * uy + R(cz<Q>(i)) * uz;
      const R cs = R(cx<Q>(i)) * usx + R(cy<Q>(i)) * usy + R(cz<Q>(i)) * usz;
      feq[i] = w * rho * (R(1) + R(3) * cu + R(4.5) * cu * cu - R(1.5) * usq);
      feqs[i] = w * rho * (R(1) + R(3) * cs + R(4.5) * cs * cs - R(1.5) * uss);
      const R cF = R(cx<Q>(i)) * Fx + R(cy<Q>(i)) * Fy + R(cz<Q>(i)) * Fz;
      const R uF = ux * Fx + uy * Fy + uz * Fz;
      S[i] = w * (R(3) * (cF - uF) + R(9) * cu * cF);
    });
    R dJdB = 0;
    R sh[Q];
    sfor<Q>([&](auto K) {
      constexpr int i = K;
      constexpr int ib = opp<Q>(i);
      const R fp = R(0.5) * (f[i] + f[ib]), fm = R(0.5) * (f[i] - f[ib]);
      const R ep = R(0.5) * (feq[i] + feq[ib]), em = R(0.5) * (feq[i] - feq[ib]);
      const R sp = R(0.5) * (S[i] + S[ib]), sm = R(0.5) * (S[i] - S[ib]);
      const R omF = -le * (fp - ep) - lo * (fm - em) + ge * sp + go * sm;
      const R omS = (f[ib] - feq[ib]) - (f[i] - feqs[i]);
      const R mi = R(cx<Q>(i)) * arx + R(cy<Q>(i)) * ary + R(cz<Q>(i)) * arz;
      dJdB += (gh[i] - wtt * mi) * omS - gh[i] * omF;
      sh[i] = B * (gh[i] - wtt * mi);
    });
    // fluid part: b_i, d_i from the even / odd parts of gh
    R Grho = 0, Gux = 0, Guy = 0, Guz = 0;
    R Hrho = 0, Hux = 0, Huy = 0, Huz = 0, Krho = 0, Kx = 0, Ky = 0, Kz = 0;
    sfor<Q>([&](auto K) {
      constexpr int i = K;
      constexpr int ib = opp<Q>(i);
      constexpr int ex = cx<Q>(i), ey = cy<Q>(i), ez = cz<Q>(i);
      const R w = (R)wt<Q>(i);
      const R gp = R(0.5) * (gh[i] + gh[ib]), gm = R(0.5) * (gh[i] - gh[ib]);
      const R b = le * gp + lo * gm, d = ge * gp + go * gm;
      const R cu = R(ex) * ux + R(ey) * uy + R(ez) * uz;
      const R cs = R(ex) * usx + R(ey) * usy + R(ez) * usz;
      const R cF = R(ex) * Fx + R(ey) * Fy + R(ez) * Fz;
      // dfeq_i/du = w rho [3 c + 9 (c.u) c - 3 u]
      const R t1 = w * rho * R(3), t9 = w * rho * R(9) * cu;
      Grho += b * feq[i] / rho;
      Gux += b * (t1 * R(ex) + t9 * R(ex) - t1 * ux) + d * w * (R(-3) * Fx + R(9) * cF * R(ex));
      Guy += b * (t1 * R(ey) + t9 * R(ey) - t1 * uy) + d * w * (R(-3) * Fy + R(9) * cF * R(ey));
      Guz += b * (t1 * R(ez) + t9 * R(ez) - t1 * uz) + d * w * (R(-3) * Fz + R(9) * cF * R(ez));
      // solid part (SC1): sum_i sh_ib feq_i(u) and sum_i sh_i feq_i(u_s)
      const R sb = sh[ib];
      Hrho += sb * feq[i] / rho;
      Hux += sb * (t1 * R(ex) + t9 * R(ex) - t1 * ux);
      Huy += sb * (t1 * R(ey) + t9 * R(ey) - t1 * uy);
      Huz += sb * (t1 * R(ez) + t9 * R(ez) - t1 * uz);
      Krho += sh[i] * feqs[i] / rho;
      const R s9 = w * rho * R(9) * cs;
      Kx += sh[i] * (t1 * R(ex) + s9 * R(ex) - t1 * usx);
      Ky += sh[i] * (t1 * R(ey) + s9 * R(ey) - t1 * usy);
      Kz += sh[i] * (t1 * R(ez) + s9 * R(ez) - t1 * usz);
    });
    const R fl = R(1) - B;
    R *aout = (R *)A.aout;
    sfor<Q>([&](auto K) {
      constexpr int j = K;
      constexpr int jb = opp<Q>(j);
      const R cux = (R(cx<Q>(j)) - ux) / rho, cuy = (R(cy<Q>(j)) - uy) / rho, cuz = (R(cz<Q>(j)) - uz) / rho;
      const R gp = R(0.5) * (gh[j] + gh[jb]), gm = R(0.5) * (gh[j] - gh[jb]);
      const R vF = -le * gp - lo * gm + Grho + Gux * cux + Guy * cuy + Guz * cuz;
      const R vS = (sh[jb] - sh[j]) - (Hrho + Hux * cux + Huy * cuy + Huz * cuz) + Krho;
      aout[(uint64_t)j * N + n] = gh[j] + fl * vF + vS;
    });
    R *gB = (R *)A.dJdB;
    gB[n] += dJdB;
    dom = (double)(arx * Kx + ary * Ky + arz * Kz);
  }
  __shared__ double sh4[4];
  double v = wave_sum(dom);
  if ((threadIdx.x & 63) == 0) sh4[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) A.part[blockIdx.x] = ((sh4[0] + sh4[1]) + sh4[2]) + sh4[3];
}

hipError_t launch_adjoint(const psm_field &f, const AdjArgs &A, hipStream_t st) {
  const dim3 g((unsigned)((f.N + 255) / 256)), b(256);
  const int q = f.cfg.q, sto = f.cfg.storage;
  if (q == 19 && sto == PSM_F64) hipLaunchKernelGGL((k_adjoint<19, double>), g, b, 0, st, A);
  else if (q == 19 && sto == PSM_F32) hipLaunchKernelGGL((k_adjoint<19, float>), g, b, 0, st, A);
  else if (q == 19) hipLaunchKernelGGL((k_adjoint<19, _Float16>), g, b, 0, st, A);
  else if (sto == PSM_F64) hipLaunchKernelGGL((k_adjoint<27, double>), g, b, 0, st, A);
  else if (sto == PSM_F32) hipLaunchKernelGGL((k_adjoint<27, float>), g, b, 0, st, A);
  else hipLaunchKernelGGL((k_adjoint<27, _Float16>), g, b, 0, st, A);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_sum_accumulate(const double *p, uint32_t n, double *out) {
  double acc = 0.0;
  for (uint32_t i = threadIdx.x; i < n; i += 256) acc += p[i];
  __shared__ double sh[4];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[0] += ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

hipError_t launch_sum_accumulate(const double *p, uint32_t n, double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_accumulate, dim3(1), dim3(256), 0, st, p, n, out);
  return hipGetLastError();
}

}  // namespace psm
