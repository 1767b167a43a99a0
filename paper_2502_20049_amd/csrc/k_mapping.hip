// Geometry field -> solid fraction mapping (section III) for gfx950.
//
// The rotation/translation is folded into the lookup: each lab cell's centre
// is taken to the body frame once (FP64, fixed fma order), each of its
// (2^s)^3 sub-sample offsets is rotated once per launch into an LDS table,
// and sub-sample k of the cell lands in geometry lattice cell
//   m = floor((rint(p * 2^(s+32)) + rint((R^T delta_k) * 2^(s+32))) / 2^32)
// (signed 64-bit fixed point, 32 fraction bits, sub-cell units).
//
// The other reading of the section III average (per-body flag `block`, s >= 1):
// only the centre is taken to the body frame, and the cell averages the
// axis-aligned block of (2^s)^3 geometry cells whose lower corner is
//   j0 = floor((P - 2^(s+31) + 2^31) / 2^32)
// per axis (P the centre in the same fixed point); identical to the above at
// theta = 0 and for s = 0.
//
// Cost control: a coarse map (one byte per 2^s-cube block of the geometry
// lattice: all out / all in / mixed) classifies most cells exactly from the
// <= 3x3x3 blocks their sub-samples can touch; only surface cells are sampled:
// for s >= 2 a wave64 takes several of its surface cells per round, every lane
// taking sub-samples of each, and a ballot/popcount gives each count.
#include "psm_internal.hpp"

#pragma clang fp contract(off)

namespace psm {

__device__ __forceinline__ double rt_comp(const double *R, int a, double v0, double v1, double v2) {
  return __builtin_fma(R[a], v0, __builtin_fma(R[3 + a], v1, R[6 + a] * v2));
}

__device__ __forceinline__ void sub_offset(const MapBodyK &g, int k, long long D[3]) {
  const int s = g.s, n = 1 << s;
  const int kx = k & (n - 1), ky = (k >> s) & (n - 1), kz = k >> (2 * s);
  const double h2 = 1.0 / (double)(2 << s);  // 2^-(s+1), exact
  const double d0 = (2.0 * kx + 1.0) * h2 - 0.5;
  const double d1 = (2.0 * ky + 1.0) * h2 - 0.5;
  const double d2 = (2.0 * kz + 1.0) * h2 - 0.5;
  const double sc = (double)(1ull << (s + 32));
#pragma unroll
  for (int c = 0; c < 3; ++c) D[c] = __double2ll_rn(rt_comp(g.R, c, d0, d1, d2) * sc);
}

__device__ __forceinline__ int geo_bit(const MapBodyK &g, long long mx, long long my, long long mz) {
  const long long jx = mx - g.mmin[0], jy = my - g.mmin[1], jz = mz - g.mmin[2];
  if ((unsigned long long)jx >= (unsigned long long)g.dims[0] || (unsigned long long)jy >= (unsigned long long)g.dims[1] ||
      (unsigned long long)jz >= (unsigned long long)g.dims[2])
    return 0;
  const uint32_t w = g.bits[((size_t)jz * g.dims[1] + (size_t)jy) * g.wx + (size_t)(jx >> 5)];
  return (w >> (jx & 31)) & 1;
}

__device__ __forceinline__ int coarse_state(const MapBodyK &g, long long bx, long long by, long long bz) {
  const long long jx = bx - g.cmin[0], jy = by - g.cmin[1], jz = bz - g.cmin[2];
  if ((unsigned long long)jx >= (unsigned long long)g.cdims[0] || (unsigned long long)jy >= (unsigned long long)g.cdims[1] ||
      (unsigned long long)jz >= (unsigned long long)g.cdims[2])
    return 0;
  return g.coarse[((size_t)jz * g.cdims[1] + (size_t)jy) * g.cdims[0] + (size_t)jx] & 3;
}

// The cell decided from the block of its centre alone: every sub-sample lies
// within one block of the centre, so a centre two or more blocks outside the
// box is all out, and a block marked uniform with its 26 neighbours (bit 2)
// gives its state.  -1: undecided (look at every block the sub-samples span).
__device__ __forceinline__ int coarse_centre(const MapBodyK &g, const long long P[3]) {
  const long long jx = (P[0] >> (32 + g.s)) - g.cmin[0], jy = (P[1] >> (32 + g.s)) - g.cmin[1],
                  jz = (P[2] >> (32 + g.s)) - g.cmin[2];
  if (jx < -1 || jy < -1 || jz < -1 || jx > g.cdims[0] || jy > g.cdims[1] || jz > g.cdims[2]) return 0;
  if (jx < 0 || jy < 0 || jz < 0 || jx >= g.cdims[0] || jy >= g.cdims[1] || jz >= g.cdims[2]) return -1;
  const int v = g.coarse[((size_t)jz * g.cdims[1] + (size_t)jy) * g.cdims[0] + (size_t)jx];
  return (v & 4) ? (v & 3) : -1;
}

// Wave-cooperative sampling of the surface cells of a wave (s >= 2): the
// (2^s)^3 = 64*NIT sub-samples of a cell are spread over the 64 lanes (NIT per
// lane); NC cells are taken per round so that NC*NIT word loads per lane are
// in flight before the ballots.  `mask` holds the lanes whose cell needs
// sampling (wave-uniform); each such lane gets its count back.
__device__ __forceinline__ long long lane_ll(long long v, int l) {
  const int lo = __builtin_amdgcn_readlane((int)(unsigned long long)v, l);
  const int hi = __builtin_amdgcn_readlane((int)((unsigned long long)v >> 32), l);
  return (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

template <int NIT, int NC>
__device__ __forceinline__ int sample_cells(const MapBodyK &g, bool own_tab, const long long (*tab)[512],
                                            unsigned long long mask, const long long P[3], int lane, int count) {
  // This lane's rotated sub-sample offsets, fixed for the launch, split into
  // a signed high word and an unsigned low word: with P = Ph 2^32 + Pl, the
  // lattice index floor((P + D) / 2^32) is Ph + Dh + carry(Pl + Dl), exact in
  // 32-bit arithmetic (indices are far below 2^31).
  int Dh[NIT][3];
  uint32_t Dl[NIT][3];
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int k = it * 64 + lane;
    long long D[3];
    if (own_tab) {
      D[0] = tab[0][k];
      D[1] = tab[1][k];
      D[2] = tab[2][k];
    } else {
      sub_offset(g, k, D);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Dh[it][c] = (int)(D[c] >> 32);
      Dl[it][c] = (uint32_t)(unsigned long long)D[c];
    }
  }
  const int m0 = (int)g.mmin[0], m1 = (int)g.mmin[1], m2 = (int)g.mmin[2];
  const uint32_t d0 = (uint32_t)g.dims[0], d1 = (uint32_t)g.dims[1], d2 = (uint32_t)g.dims[2];
  while (mask) {
    int ls[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      ls[c] = mask ? __ffsll((long long)mask) - 1 : -1;
      mask &= mask - 1;
    }
    uint32_t word[NC][NIT];
    uint32_t bit[NC][NIT];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int l = ls[c] < 0 ? 0 : ls[c];
      // the cell's centre in the body frame (wave-uniform)
      const long long Px = lane_ll(P[0], l), Py = lane_ll(P[1], l), Pz = lane_ll(P[2], l);
      const int ph0 = (int)(Px >> 32) - m0, ph1 = (int)(Py >> 32) - m1, ph2 = (int)(Pz >> 32) - m2;
      const uint32_t pl0 = (uint32_t)(unsigned long long)Px, pl1 = (uint32_t)(unsigned long long)Py,
                     pl2 = (uint32_t)(unsigned long long)Pz;
#pragma unroll
      for (int it = 0; it < NIT; ++it) {
        const uint32_t jx = (uint32_t)(ph0 + Dh[it][0] + (int)(pl0 + Dl[it][0] < pl0));
        const uint32_t jy = (uint32_t)(ph1 + Dh[it][1] + (int)(pl1 + Dl[it][1] < pl1));
        const uint32_t jz = (uint32_t)(ph2 + Dh[it][2] + (int)(pl2 + Dl[it][2] < pl2));
        word[c][it] = 0;
        bit[c][it] = jx & 31u;
        if (ls[c] >= 0 && jx < d0 && jy < d1 && jz < d2)
          word[c][it] = g.bits[((size_t)jz * d1 + jy) * (size_t)g.wx + (jx >> 5)];
      }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      int n = 0;
#pragma unroll
      for (int it = 0; it < NIT; ++it) n += __popcll(__ballot((word[c][it] >> bit[c][it]) & 1u));
      if (lane == ls[c]) count = n;
    }
  }
  return count;
}

// Block reading, surface cells of a wave: each of a cell's (2^s)^2 rows of
// 2^s geometry cells along x is one lane's (at most two word loads), so a
// round takes 64 / 4^s cells (s = 1: 16, s = 2: 4, s = 3: 1).  A row holds at
// most 8 inside flags; the four bit planes of the row counts are ballotted
// and each group's lanes popcounted.  J: the block's lower corner relative
// to the stored box; `mask`: the lanes whose cell needs counting.
__device__ __forceinline__ int block_cells(const MapBodyK &g, unsigned long long mask, const int J[3], int lane,
                                           int count) {
  const int s = g.s, n = 1 << s;
  const int rows = 1 << (2 * s);
  const int cpr = 64 >> (2 * s);  // cells per round
  const int grp = lane >> (2 * s), r = lane & (rows - 1);
  const int dy = r & (n - 1), dz = r >> s;
  const int d0 = g.dims[0], d1 = g.dims[1], d2 = g.dims[2];
  while (mask) {
    // this lane's group takes the grp-th remaining cell of the mask
    unsigned long long mm = mask;
    int src = -1;
    for (int c = 0; c < cpr && mm; ++c) {
      const int l = __ffsll((long long)mm) - 1;
      mm &= mm - 1;
      if (c == grp) src = l;
    }
    const int sl = src < 0 ? 0 : src;
    const int jx = __shfl(J[0], sl), jy = __shfl(J[1], sl) + dy, jz = __shfl(J[2], sl) + dz;
    const int xa = max(jx, 0), xb = min(jx + n, d0);
    uint32_t c = 0;
    if (src >= 0 && jy >= 0 && jy < d1 && jz >= 0 && jz < d2 && xa < xb) {
      const uint32_t *row = g.bits + ((size_t)jz * d1 + jy) * (size_t)g.wx;
      const int w0 = xa >> 5, w1 = (xb - 1) >> 5;
      const uint64_t v = (uint64_t)row[w0] | (w1 != w0 ? (uint64_t)row[w1] << 32 : 0ull);
      c = (uint32_t)__popcll((v >> (xa & 31)) & ((1ull << (xb - xa)) - 1ull));
    }
    const unsigned long long b0 = __ballot(c & 1u), b1 = __ballot(c & 2u), b2 = __ballot(c & 4u),
                             b3 = __ballot(c & 8u);
    mm = mask;
    for (int cc = 0; cc < cpr && mm; ++cc) {
      const int l = __ffsll((long long)mm) - 1;
      mm &= mm - 1;
      const unsigned long long gm = (rows == 64 ? ~0ull : ((1ull << rows) - 1ull)) << (cc * rows);
      const int tot = __popcll(b0 & gm) + 2 * __popcll(b1 & gm) + 4 * __popcll(b2 & gm) + 8 * __popcll(b3 & gm);
      if (lane == l) count = tot;
    }
    mask = mm;
  }
  return count;
}

// Solid fraction from the inside count: eq. (5) (B = eps) or eq. (6).
__device__ __forceinline__ float fraction_of(const MapArgs &a, int count, int ns) {
  const double eps = (double)count / (double)ns;
  if (a.b_form == 0) return (float)eps;
  const double th = a.tau - 0.5;
  const double num = eps * th;
  const double den = (1.0 - eps) + th;
  return (float)(num / den);
}

// The cell centre in the body frame, fixed point (same operations in both
// mapping kernels, so both see the same P).
__device__ __forceinline__ void body_point(const MapBodyK &g, int x, int y, int z, long long P[3]) {
  const double d0 = (x + 0.5) - g.X[0], d1 = (y + 0.5) - g.X[1], d2 = (z + 0.5) - g.X[2];
  const double sc = (double)(1ull << (g.s + 32));
#pragma unroll
  for (int c = 0; c < 3; ++c) P[c] = __double2ll_rn(rt_comp(g.R, c, d0, d1, d2) * sc);
}

__device__ __forceinline__ void fill_table(const MapBodyK &G, long long (*tab)[512]) {
  const int nsr = 1 << (3 * G.s);
  for (int k = threadIdx.x; k < nsr; k += 256) {
    long long D[3];
    sub_offset(G, k, D);
    tab[0][k] = D[0];
    tab[1][k] = D[1];
    tab[2][k] = D[2];
  }
  __syncthreads();
}

__device__ __forceinline__ bool in_box(const IBox &b, int x, int y, int z) {
  return x >= b.lo[0] && x <= b.hi[0] && y >= b.lo[1] && y <= b.hi[1] && z >= b.lo[2] && z <= b.hi[2];
}

__global__ __launch_bounds__(256) void k_map(const MapArgs a) {
  const int rb = blockIdx.y;
  const MapBodyK &G = a.body[rb];
  if (blockIdx.x * 256u >= G.region_cells) return;  // whole workgroup idle
  __shared__ long long tab[3][512];
  fill_table(G, tab);

  const int lane = threadIdx.x & 63;
  const uint32_t idx = blockIdx.x * 256u + threadIdx.x;
  bool active = idx < G.region_cells;
  const int rx = G.region.hi[0] - G.region.lo[0] + 1, ry = G.region.hi[1] - G.region.lo[1] + 1;
  const int x = G.region.lo[0] + (int)(idx % (uint32_t)rx);
  const int y = G.region.lo[1] + (int)((idx / (uint32_t)rx) % (uint32_t)ry);
  const int z = G.region.lo[2] + (int)(idx / ((uint32_t)rx * (uint32_t)ry));
  for (int b = 0; b < rb; ++b)
    if (in_box(a.body[b].region, x, y, z)) active = false;  // written by an earlier region
  const size_t n = (size_t)x + (size_t)a.nx * ((size_t)y + (size_t)a.ny * (size_t)z);
  // bodies that can touch the cell: a surface cell of a single body may be
  // left to the sampling kernel (its B does not combine with another body's)
  int nin = 0;
  for (int bb = 0; bb < a.nb; ++bb) nin += (active && in_box(a.body[bb].active, x, y, z)) ? 1 : 0;

  float Bv[2] = {0.f, 0.f};
  int id[2] = {0, 0};
  int used = 0;
  bool overflow = false;
  __shared__ uint32_t lcnt[4], lbase;  // list appends: per-wave counts, the workgroup's base
  const int wid = threadIdx.x >> 6;
  for (int bb = 0; bb < a.nb; ++bb) {
    const MapBodyK &g = a.body[bb];
    const bool inb = active && in_box(g.active, x, y, z);
    const bool listing = a.list && g.s == 3 && !g.block;  // workgroup-uniform: every wave reaches its barriers
    if (!__any(inb) && !listing) continue;
    const int s = g.s;
    const int ns = 1 << (3 * s);
    long long P[3] = {0, 0, 0};
    int state = 0;  // 0 all out, 1 all in, 2 sample
    if (g.block) {
      // block reading (s >= 1): the block lies within one coarse block of the
      // centre's, and spans at most two coarse blocks per axis
      int J[3] = {0, 0, 0};
      if (inb) {
        body_point(g, x, y, z, P);
        const long long off = (1ll << 31) - (1ll << (s + 31));
#pragma unroll
        for (int c = 0; c < 3; ++c) J[c] = (int)((P[c] + off) >> 32);
        if ((state = coarse_centre(g, P)) < 0) {
          int vals[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const int bx = (J[0] + ((j & 1) ? (1 << s) - 1 : 0)) >> s;
            const int by = (J[1] + ((j & 2) ? (1 << s) - 1 : 0)) >> s;
            const int bz = (J[2] + ((j & 4) ? (1 << s) - 1 : 0)) >> s;
            vals[j] = coarse_state(g, bx, by, bz);
          }
          int st = vals[0];
#pragma unroll
          for (int j = 1; j < 8; ++j) st = (st == vals[j]) ? st : 2;
          state = st;
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) J[c] -= g.mmin[c];
      }
      int count = block_cells(g, __ballot(state == 2), J, lane, state == 1 ? ns : 0);
      if (inb && count > 0) {
        const float B = fraction_of(a, count, ns);
        if (used < a.slots) {
          Bv[used] = B;
          id[used] = bb;
          ++used;
        } else {
          overflow = true;
        }
      }
      continue;
    }
    if (inb) {
      body_point(g, x, y, z, P);
      if (s == 0) {
        state = 2;
      } else if ((state = coarse_centre(g, P)) < 0) {
        long long lo[3], hi[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          lo[c] = (P[c] - g.dabs[c]) >> (32 + s);
          hi[c] = (P[c] + g.dabs[c]) >> (32 + s);
        }
        // the sub-samples span at most 3 coarse blocks per axis: issue all
        // (up to 27) byte loads, then combine
        int vals[27];
#pragma unroll
        for (int j = 0; j < 27; ++j) {
          const long long bx = lo[0] + j % 3, by = lo[1] + (j / 3) % 3, bz = lo[2] + j / 9;
          vals[j] = (bx <= hi[0] && by <= hi[1] && bz <= hi[2]) ? coarse_state(g, bx, by, bz) : -1;
        }
        int st = vals[0];
#pragma unroll
        for (int j = 1; j < 27; ++j)
          if (vals[j] >= 0) st = (st == vals[j]) ? st : 2;
        state = st;
      }
    }
    int count = state == 1 ? ns : 0;
    const bool own_tab = (bb == rb);
    if (s <= 1) {
      if (state == 2) {
        int c = 0;
        for (int k = 0; k < ns; ++k) {
          long long D[3];
          if (own_tab) {
            D[0] = tab[0][k];
            D[1] = tab[1][k];
            D[2] = tab[2][k];
          } else {
            sub_offset(g, k, D);
          }
          c += geo_bit(g, (P[0] + D[0]) >> 32, (P[1] + D[1]) >> 32, (P[2] + D[2]) >> 32);
        }
        count = c;
      }
    } else {
      // at s = 3 (512 sub-samples) surface cells of a single body go to the
      // sampling list (three cells per wave and round there); the rest, and any beyond the
      // list's capacity, are sampled here.  At s = 2 (64 sub-samples, one
      // per lane) sampling here, several cells per round, is faster.
      bool listed = false;
      if (listing) {
        // one counter atomic per workgroup (the counter is shared by every
        // workgroup of the launch): wave counts, then the workgroup's base
        const bool cand = inb && state == 2 && nin == 1;
        const unsigned long long cm = __ballot(cand);
        if (lane == 0) lcnt[wid] = (uint32_t)__popcll(cm);
        __syncthreads();
        if (threadIdx.x == 0) {
          const uint32_t t = (lcnt[0] + lcnt[1]) + (lcnt[2] + lcnt[3]);
          lbase = t ? atomicAdd(&a.count[bb], t) : 0u;
        }
        __syncthreads();
        uint32_t pos = lbase + (uint32_t)__popcll(cm & ((1ull << lane) - 1ull));
        for (int w = 0; w < wid; ++w) pos += lcnt[w];
        if (cand && pos < a.cap) {
          a.list[(size_t)bb * a.cap + pos] = (uint32_t)n;
          listed = true;
        }
        __syncthreads();  // lcnt and lbase are reused for the next body
      }
      const unsigned long long sm = __ballot(state == 2 && !listed);
      if (s == 2)
        count = sample_cells<1, 4>(g, own_tab, tab, sm, P, lane, count);
      else
        count = sample_cells<8, 2>(g, own_tab, tab, sm, P, lane, count);
    }
    if (inb && count > 0) {
      const float B = fraction_of(a, count, ns);
      if (used < a.slots) {
        Bv[used] = B;
        id[used] = bb;
        ++used;
      } else {
        overflow = true;
      }
    }
  }
  if (active) {
    a.B0[n] = Bv[0];
    uint8_t m = (uint8_t)(id[0] & 15);
    if (a.slots == 2) {
      a.B1[n] = Bv[1];
      if (used == 2) m |= (uint8_t)((id[1] + 1) << 4);
    }
    a.meta[n] = m;
    if (overflow) atomicOr(a.err, 1);
  }
}

// Listed surface cells (s = 3): a wave samples three cells per round, 8
// sub-samples of each per lane (all gathers issued before the ballots), B
// and the body id written for cells with a nonzero count (the classification
// kernel already wrote zeros).  Also clears the counters the
// next mapping call appends to.
__global__ __launch_bounds__(256) void k_map_sample(const MapArgs a) {
  const int bb = blockIdx.y;
  const MapBodyK &G = a.body[bb];
  if (blockIdx.x == 0 && threadIdx.x == 0) a.count_next[bb] = 0u;
  if (G.s != 3 || G.block) return;
  const uint32_t total = min(a.count[bb], a.cap);
  constexpr int NCS = 3;  // cells per wave and round: their gathers are in flight together
  if (blockIdx.x * 4u * NCS >= total) return;  // whole workgroup idle
  __shared__ long long tab[3][512];
  fill_table(G, tab);
  const int lane = threadIdx.x & 63;
  const int ns = 1 << (3 * G.s);
  const uint32_t stride = gridDim.x * 4u * NCS;
  for (uint32_t e0 = (blockIdx.x * 4u + (threadIdx.x >> 6)) * NCS; e0 < total; e0 += stride) {
    // lanes 0 .. NCS-1 hold the entries e0 .. e0+NCS-1
    const uint32_t e = e0 + (uint32_t)lane;
    const bool mine = lane < NCS && e < total;
    uint32_t n = 0;
    long long P[3] = {0, 0, 0};
    if (mine) {
      n = a.list[(size_t)bb * a.cap + e];
      const int x = (int)(n % (uint32_t)a.nx);
      const int y = (int)((n / (uint32_t)a.nx) % (uint32_t)a.ny);
      const int z = (int)(n / ((uint32_t)a.nx * (uint32_t)a.ny));
      body_point(G, x, y, z, P);
    }
    const int c = sample_cells<8, NCS>(G, true, tab, __ballot(mine), P, lane, 0);
    if (mine && c > 0) {
      a.B0[n] = fraction_of(a, c, ns);
      a.meta[n] = (uint8_t)(bb & 15);
    }
  }
}

hipError_t launch_map(const MapArgs &a, uint32_t max_region_cells, int any_s_max, hipStream_t st) {
  (void)any_s_max;
  if (a.nb == 0 || max_region_cells == 0) return hipSuccess;
  dim3 grid((max_region_cells + 255) / 256, a.nb), block(256);
  hipLaunchKernelGGL(k_map, grid, block, 0, st, a);
  if (a.list) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_map_sample, dim3(MAP_SAMPLE_BLOCKS, a.nb), block, 0, st, a);
  }
  return hipGetLastError();
}

}  // namespace psm
