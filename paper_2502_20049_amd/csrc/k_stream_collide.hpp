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

// Per-cell collision: TRT + Guo fluid collision blended with NS solid slots.
// f holds deviations delta f; on return f holds the post-collision deviations.
template <int Q, int SC, int NS, typename R>
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
  const R inv = R(1) / rho;
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

  // rest direction
  {
    const R w = (R)wt<Q>(0);
    const R E = w * (dr - R(1.5) * rho * usq);
    R om = -le * (f[0] - E);
    if (hf) om += ge * (R(-3) * w * uF);
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
    const R fp = R(0.5) * (av + bv), fm = R(0.5) * (av - bv);
    R rp = -le * (fp - E), rm = -lo * (fm - O);
    if (hf) {
      const R cF = R(ex) * Fx + R(ey) * Fy + R(ez) * Fz;
      rp += ge * (w * (R(9) * cu * cF - R(3) * uF));
      rm += go * (R(3) * w * cF);
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

template <int Q, typename T, int PAR, int SC, bool PSM, bool BIG>
__global__ __launch_bounds__(256) void k_stream_collide(const SCArgs a) {
  using R = typename Comp<T>::type;
  using Off = typename std::conditional<BIG, uint64_t, uint32_t>::type;
  constexpr Off S = sizeof(T);
  constexpr int H = Lat<Q>::H;
  (void)H;

  const uint32_t tile = a.xcd_remap ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
  const int tid = threadIdx.x;
  const int txi = (int)(tile % (uint32_t)a.ntx);
  const uint32_t rr = tile / (uint32_t)a.ntx;
  const int tyi = (int)(rr % (uint32_t)a.nty);
  const int z = (int)(rr / (uint32_t)a.nty);
  const int x = txi * a.TX + (tid & (a.TX - 1));
  const int y = tyi * a.TY + (tid >> a.lTX);
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const bool active = (x < nx) && (y < ny);
  const Off n = (Off)x + (Off)nx * ((Off)y + (Off)ny * (Off)z);
  char *const A = a.pdf;

  // face classification of every incoming direction (source x - c_k)
  uint32_t bcm = 0, outm = 0, inm = 0;
  sfor<Q>([&](auto K) {
    constexpr int k = K;
    constexpr int ex = cx<Q>(k), ey = cy<Q>(k), ez = cz<Q>(k);
    int kd = K_NONE;
    if constexpr (ex == 1) if (x == 0 && !a.periodic[0]) kd = face_merge(kd, a.bc[0]);
    if constexpr (ex == -1) if (x == nx - 1 && !a.periodic[0]) kd = face_merge(kd, a.bc[1]);
    if constexpr (ey == 1) if (y == 0 && !a.periodic[1]) kd = face_merge(kd, a.bc[2]);
    if constexpr (ey == -1) if (y == ny - 1 && !a.periodic[1]) kd = face_merge(kd, a.bc[3]);
    if constexpr (ez == 1) if (z == 0 && !a.periodic[2]) kd = face_merge(kd, a.bc[4]);
    if constexpr (ez == -1) if (z == nz - 1 && !a.periodic[2]) kd = face_merge(kd, a.bc[5]);
    if (kd != K_NONE) bcm |= 1u << k;
    if (kd == K_OUTLET) outm |= 1u << k;
    if (kd == K_INLET) inm |= 1u << k;
  });

  // odd-parity source offsets: interior rows need only the x wrap
  const bool general = a.force_general || y == 0 || y == ny - 1 || z == 0 || z == nz - 1;
  const Off rb = n - (Off)x;
  int xm, xp;
  if (a.periodic[0]) {
    xm = x == 0 ? nx - 1 : x - 1;
    xp = x == nx - 1 ? 0 : x + 1;
  } else {
    xm = x == 0 ? 0 : x - 1;
    xp = x == nx - 1 ? nx - 1 : x + 1;
  }
  auto src_of = [&](auto K) -> Off {
    constexpr int k = K;
    constexpr int ex = cx<Q>(k), ey = cy<Q>(k), ez = cz<Q>(k);
    const Off xs = (Off)(ex == 1 ? xm : (ex == -1 ? xp : x));
    if (!general) {
      return rb + xs - (Off)((long long)ey * nx) - (Off)((long long)ez * nx * ny);
    }
    int sy = y - ey, sz = z - ez;
    if (sy < 0) sy += ny;
    if (sy >= ny) sy -= ny;
    if (sz < 0) sz += nz;
    if (sz >= nz) sz -= nz;
    return xs + (Off)nx * ((Off)sy + (Off)ny * (Off)sz);
  };
  // direction base (uniform, 64-bit) + in-direction byte offset (32-bit unless
  // a direction array exceeds 4 GiB)
  const size_t NS = (size_t)a.N * S;
  auto addr = [&](auto K) -> char * {
    constexpr int k = K;
    if constexpr (PAR == 0) {
      return A + (size_t)k * NS + (size_t)(Off)(n * S);
    } else {
      if ((bcm >> k) & 1u) return A + (size_t)k * NS + (size_t)(Off)(n * S);
      return A + (size_t)opp<Q>(k) * NS + (size_t)(Off)(src_of(K) * S);
    }
  };
  auto inlet_term = [&](auto K) -> R {
    constexpr int k = K;
    return R(6.0 * wt<Q>(k)) *
           (R(cx<Q>(k)) * (R)a.u_in_d[0] + R(cy<Q>(k)) * (R)a.u_in_d[1] + R(cz<Q>(k)) * (R)a.u_in_d[2]);
  };

  R f[Q];
  if (active) {
    sfor<Q>([&](auto K) {
      constexpr int k = K;
      R v = ldv<T, R>(addr(K));
      if constexpr (PAR == 1) {
        if ((inm >> k) & 1u) v += inlet_term(K);
      }
      f[k] = v;
    });
  } else {
    sfor<Q>([&](auto K) { f[K] = R(0); });
  }

  // body slots of this cell
  R B0 = 0, B1 = 0;
  int b0 = 0, b1 = 0;
  bool two = false;
  if constexpr (PSM) {
    if (active) {
      B0 = (R)a.B0[n];
      if (B0 > R(0)) {
        const uint8_t m = a.meta[n];
        b0 = m & 15;
        if (b0 >= a.nb) b0 = 0;  // ids come from the mapping; never index past the body table
        if (a.slots == 2 && (m >> 4)) {
          b1 = (m >> 4) - 1;
          if (b1 >= a.nb) b1 = 0;
          B1 = (R)a.B1[n];
          two = true;
        }
      }
    }
  }
  R us0[3] = {0, 0, 0}, us1[3] = {0, 0, 0};
  R mom0[3] = {0, 0, 0}, mom1[3] = {0, 0, 0};
  const double xc = x + 0.5, yc = y + 0.5, zc = z + 0.5;
  bool solid_wave = false;
  if constexpr (PSM) solid_wave = __any(B0 > R(0));
  if (solid_wave) {
    auto usolid = [&](int b, R(&us)[3]) {
      const BodyK &bd = a.body[b];
      const R rx = (R)(xc - bd.X[0]), ry = (R)(yc - bd.X[1]), rz = (R)(zc - bd.X[2]);
      const R wx = (R)bd.W[0], wy = (R)bd.W[1], wz = (R)bd.W[2];
      us[0] = (R)bd.V[0] + (wy * rz - wz * ry);
      us[1] = (R)bd.V[1] + (wz * rx - wx * rz);
      us[2] = (R)bd.V[2] + (wx * ry - wy * rx);
    };
    if (B0 > R(0)) usolid(b0, us0);
    if (two) usolid(b1, us1);
    if (__any(two)) {
      collide<Q, SC, 2, R>(f, a, B0, us0, B1, us1, mom0, mom1);
    } else {
      collide<Q, SC, 1, R>(f, a, B0, us0, B1, us1, mom0, mom1);
    }
  } else {
    collide<Q, SC, 0, R>(f, a, B0, us0, B1, us1, mom0, mom1);
  }

  if (active) {
    sfor<Q>([&](auto K) {
      constexpr int k = K;
      R v = ((outm >> k) & 1u) ? f[k] : f[opp<Q>(k)];
      if constexpr (PAR == 1) {
        if ((inm >> k) & 1u) v += inlet_term(K);
      }
      stv<T, R>(addr(K), v);
    });
  }

  // force / torque partials of tiles inside a body's swept box (eqs. (10)-(11))
  if constexpr (PSM) {
    __shared__ double red[4][6];
    const int wid = tid >> 6, lane = tid & 63;
    for (int b = 0; b < a.nb; ++b) {
      const BodyK &bd = a.body[b];
      const bool inbox = txi >= bd.tlo[0] && txi <= bd.thi[0] && tyi >= bd.tlo[1] && tyi <= bd.thi[1] &&
                         z >= bd.tlo[2] && z <= bd.thi[2];
      if (!inbox) continue;  // uniform over the workgroup
      double v[6] = {0, 0, 0, 0, 0, 0};
      auto add = [&](const R(&m)[3]) {
        const double dx = (double)m[0], dy = (double)m[1], dz = (double)m[2];
        const double rx = xc - bd.X[0], ry = yc - bd.X[1], rz = zc - bd.X[2];
        v[0] += dx;
        v[1] += dy;
        v[2] += dz;
        v[3] += ry * dz - rz * dy;
        v[4] += rz * dx - rx * dz;
        v[5] += rx * dy - ry * dx;
      };
      if (B0 > R(0) && b0 == b) add(mom0);
      if (two && b1 == b) add(mom1);
      if (__any(B0 > R(0))) {
#pragma unroll
        for (int c = 0; c < 6; ++c) v[c] = wave_sum(v[c]);
      }
      if (lane == 0) {
#pragma unroll
        for (int c = 0; c < 6; ++c) red[wid][c] = v[c];
      }
      __syncthreads();
      if (tid < 6) {
        const double s = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
        a.ftp[((size_t)tile * a.max_bodies + b) * 6 + tid] = s;
      }
      __syncthreads();
    }
  }
}

}  // namespace psm
