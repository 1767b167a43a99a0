// Reductions and utility kernels: per-body force/torque sum (FP64, fixed
// order), parity-aware macroscopic fields and FP64 mass, zero fill, copy probe.
#include "k_stream_collide.hpp"

namespace psm {

// One workgroup per body (the same sum also runs as an extra workgroup of the
// interior fluid launch when a whole step is one call).
__global__ __launch_bounds__(256) void k_ft_reduce(const double *ftp, int max_bodies, int nblocks, double *ft) {
  __shared__ double sh[4];
  ft_body_sum(ftp, max_bodies, nblocks, (int)blockIdx.x, ft, sh);
}

hipError_t launch_ft_reduce(const psm_field &f, int nb, double *ft, hipStream_t st) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ft_reduce, dim3(nb), dim3(256), 0, st, (const double *)f.ftp, f.cfg.max_bodies,
                     f.solid_blocks, ft);
  return hipGetLastError();
}

// Parity-aware read of f_k at cell (x,y,z): the standard slot at even parity;
// at odd parity the slot (x - c_k, kbar), or the cell's own slot (plus the
// inlet term) when the source is outside the domain.
template <int Q, typename T>
__device__ double read_f(const SCArgs &a, int parity, int k, int x, int y, int z, uint64_t n) {
  const uint64_t N = a.dS;  // direction stride
  const T *A = (const T *)a.pdf;
  const uint64_t e = pdf_row(a, (uint32_t)y + (uint32_t)a.ny * (uint32_t)z) + (uint64_t)x;  // the cell's element
  if (parity == 0) return (double)A[(uint64_t)k * N + e];
  // obstacle cells are never updated: their own slots hold their values
  if (a.ocls && a.ocls[n] == 2) return (double)A[(uint64_t)k * N + e];
  const int ex = cx<Q>(k), ey = cy<Q>(k), ez = cz<Q>(k);
  int sx = x - ex, sy = y - ey, sz = z - ez;
  int kd = K_NONE;
  const int nn[3] = {a.nx, a.ny, a.nz};
  int *sp[3] = {&sx, &sy, &sz};
  for (int d = 0; d < 3; ++d) {
    int &v = *sp[d];
    if (v < 0) {
      if (a.periodic[d]) v += nn[d];
      else kd = face_merge(kd, a.bc[2 * d]);
    } else if (v >= nn[d]) {
      if (a.periodic[d]) v -= nn[d];
      else kd = face_merge(kd, a.bc[2 * d + 1]);
    }
  }
  if (kd == K_NONE) {
    const uint64_t src = (uint64_t)sx + (uint64_t)a.nx * ((uint64_t)sy + (uint64_t)a.ny * (uint64_t)sz);
    const uint64_t es = pdf_row(a, (uint32_t)sy + (uint32_t)a.ny * (uint32_t)sz) + (uint64_t)sx;
    if (!(a.ocls && a.ocls[src] == 2)) return (double)A[(uint64_t)opp<Q>(k) * N + es];
    kd = K_WALL;  // link into an obstacle cell: bounce-back, the wall rule
  }
  double v = (double)A[(uint64_t)k * N + e];
  if (kd == K_INLET) v += 6.0 * wt<Q>(k) * (ex * a.u_in_d[0] + ey * a.u_in_d[1] + ez * a.u_in_d[2]);
  return v;
}

template <int Q, typename T>
__global__ __launch_bounds__(256) void k_macro(const SCArgs a, int parity, double *rho, double *u,
                                               double *partial, int want_field) {
  const uint64_t n = (uint64_t)blockIdx.x * 256u + threadIdx.x;
  const uint64_t N = a.N;
  double r = 0.0;
  if (n < N) {
    const int x = (int)(n % (uint64_t)a.nx);
    const int y = (int)((n / (uint64_t)a.nx) % (uint64_t)a.ny);
    const int z = (int)(n / ((uint64_t)a.nx * (uint64_t)a.ny));
    double dr = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
    for (int k = 0; k < Q; ++k) {
      const double v = read_f<Q, T>(a, parity, k, x, y, z, n);
      dr += v;
      jx += cx<Q>(k) * v;
      jy += cy<Q>(k) * v;
      jz += cz<Q>(k) * v;
    }
    r = 1.0 + dr;
    if (want_field) {
      rho[n] = r;
      u[3 * n + 0] = (jx + 0.5 * a.force[0]) / r;
      u[3 * n + 1] = (jy + 0.5 * a.force[1]) / r;
      u[3 * n + 2] = (jz + 0.5 * a.force[2]) / r;
    }
  }
  __shared__ double sh[4];
  const double s = block_sum256(r, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_sum_final(const double *p, uint32_t n, double *out) {
  double acc = 0.0;
  for (uint32_t i = threadIdx.x; i < n; i += 256) acc += p[i];
  __shared__ double sh[4];
  const double s = block_sum256(acc, sh);
  if (threadIdx.x == 0) out[0] = s;
}

uint32_t macro_blocks(const psm_field &f) { return (uint32_t)((f.N + 255) / 256); }


hipError_t launch_macro(const psm_field &f, int parity, double *rho, double *u, double *mass_partials,
                        int want_field, hipStream_t st) {
  const SCArgs a = make_sc_args(f);
  const dim3 grid(macro_blocks(f)), block(256);
  const int q = f.cfg.q, sto = f.cfg.storage;
#define PSM_MACRO(QQ, TT) \
  hipLaunchKernelGGL((k_macro<QQ, TT>), grid, block, 0, st, a, parity, rho, u, mass_partials, want_field)
  if (q == 19 && sto == PSM_F64) PSM_MACRO(19, double);
  else if (q == 19 && sto == PSM_F32) PSM_MACRO(19, float);
  else if (q == 19 && sto == PSM_F16) PSM_MACRO(19, _Float16);
  else if (q == 27 && sto == PSM_F64) PSM_MACRO(27, double);
  else if (q == 27 && sto == PSM_F32) PSM_MACRO(27, float);
  else PSM_MACRO(27, _Float16);
#undef PSM_MACRO
  return hipGetLastError();
}

hipError_t launch_mass_final(const double *partials, uint32_t n, double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, st, partials, n, out);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_fill_zero(uint4 *p, size_t n16, unsigned char *tail, size_t ntail) {
  const size_t stride = (size_t)gridDim.x * 256u;
  for (size_t i = (size_t)blockIdx.x * 256u + threadIdx.x; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
  if (blockIdx.x == 0 && threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  // callers pass 16-byte aligned buffers (device allocations, internal offsets)
  const size_t n16 = bytes / 16, ntail = bytes % 16;
  size_t blocks = (n16 + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, st, (uint4 *)p, n16,
                     (unsigned char *)p + n16 * 16, ntail);
  return hipGetLastError();
}

// The PDF buffer to (to_std) or from the standard layout [q][N]: thread t of
// direction blockIdx.y takes the t-th run of V cells of a slab of rows (row
// t / (nx/V)), so both sides are contiguous along the rows; V elements per
// access (16 bytes when every row start is 16-byte aligned).
template <typename T, int V>
__global__ __launch_bounds__(256) void k_pdf_convert(const SCArgs a, uint32_t total, T *dst, const T *src, int to_std) {
  typedef T vec __attribute__((ext_vector_type(V)));
  const uint32_t k = blockIdx.y;
  const uint32_t nx = (uint32_t)a.nx, nxv = nx / V;
  const uint32_t stride = gridDim.x * 256u;
  for (uint32_t t = blockIdx.x * 256u + threadIdx.x; t < total; t += stride) {
    const uint32_t r = t / nxv;  // row y + ny z within the slab
    const uint32_t x = (t - r * nxv) * V;
    const uint64_t i = (uint64_t)k * a.N + (uint64_t)r * nx + x;
    const uint64_t e = (uint64_t)k * a.dS + pdf_row(a, r) + x;
    if (to_std) *(vec *)(dst + i) = *(const vec *)(src + e);
    else *(vec *)(dst + e) = *(const vec *)(src + i);
  }
}

template <typename T>
static hipError_t convert_slab(const SCArgs &a, int q, uint64_t nr, T *d, const T *s, int to_std, hipStream_t st) {
  // 16-byte accesses when a row is a whole number of them (every row start,
  // in either layout and in the standard array, is a multiple of nx elements
  // from a 256-byte aligned base)
  constexpr int V = 16 / (int)sizeof(T);
  const bool vec = ((size_t)a.nx * sizeof(T)) % 16 == 0 && ((uintptr_t)d % 16) == 0 && ((uintptr_t)s % 16) == 0;
  const uint32_t total = (uint32_t)(nr * (uint64_t)(a.nx / (vec ? V : 1)));
  const uint32_t blocks = (total + 255) / 256;
  const dim3 g(blocks < 4096u ? blocks : 4096u, (unsigned)q);
  if (vec) hipLaunchKernelGGL((k_pdf_convert<T, V>), g, dim3(256), 0, st, a, total, d, s, to_std);
  else hipLaunchKernelGGL((k_pdf_convert<T, 1>), g, dim3(256), 0, st, a, total, d, s, to_std);
  return hipGetLastError();
}

hipError_t launch_pdf_gather(const psm_field &f, void *dst, const void *src, int to_std, size_t sz, hipStream_t st) {
  const SCArgs a = make_sc_args(f);
  const uint64_t rows = (uint64_t)f.cfg.ny * (uint64_t)f.cfg.nz;
  // slabs of rows whose thread count fits 32 bits, starting on block boundaries
  uint64_t per = ((1ull << 31) - 1) / (uint64_t)f.cfg.nx;
  if (a.bst != 0) per &= ~((1ull << a.lrb) - 1ull);
  for (uint64_t r0 = 0; r0 < rows; r0 += per) {
    const uint64_t nr = rows - r0 < per ? rows - r0 : per;
    // rows r0 .. r0 + nr - 1: shift the pointers so the kernel's row index starts at 0
    const uint64_t std_off = r0 * (uint64_t)f.cfg.nx;
    const uint64_t lay_off = pdf_row(a, (uint32_t)r0);
    const char *s = (const char *)src + (to_std ? lay_off : std_off) * sz;
    char *d = (char *)dst + (to_std ? std_off : lay_off) * sz;
    hipError_t e;
    switch (sz) {
      case 8: e = convert_slab<double>(a, f.cfg.q, nr, (double *)d, (const double *)s, to_std, st); break;
      case 4: e = convert_slab<float>(a, f.cfg.q, nr, (float *)d, (const float *)s, to_std, st); break;
      default: e = convert_slab<_Float16>(a, f.cfg.q, nr, (_Float16 *)d, (const _Float16 *)s, to_std, st);
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

__global__ __launch_bounds__(256) void k_copy(const uint4 *__restrict__ s, uint4 *__restrict__ d, size_t n16) {
  const size_t stride = (size_t)gridDim.x * 256u;
  for (size_t i = (size_t)blockIdx.x * 256u + threadIdx.x; i < n16; i += stride) d[i] = s[i];
}

__global__ void k_copy_tail(const unsigned char *s, unsigned char *d, size_t n) {
  if (threadIdx.x < n) d[threadIdx.x] = s[threadIdx.x];
}

hipError_t launch_copy(const void *src, void *dst, size_t bytes, hipStream_t st) {
  const size_t n16 = bytes / 16, tail = bytes % 16;
  if (n16) {
    size_t blocks = (n16 + 255) / 256;
    if (blocks > 1u << 20) blocks = 1u << 20;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, st, (const uint4 *)src, (uint4 *)dst, n16);
  }
  if (tail)
    hipLaunchKernelGGL(k_copy_tail, dim3(1), dim3(16), 0, st, (const unsigned char *)src + n16 * 16,
                       (unsigned char *)dst + n16 * 16, tail);
  return hipGetLastError();
}

__global__ void k_flags_copy(const int32_t *s, int32_t *d) {
  if (threadIdx.x < 4) d[threadIdx.x] = s[threadIdx.x];
}

hipError_t launch_flags_copy(const int32_t *src, int32_t *dst, hipStream_t st) {
  hipLaunchKernelGGL(k_flags_copy, dim3(1), dim3(64), 0, st, src, dst);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Static obstacle of a plain-LBM field (set-up, once): per cell the class
// (0 bulk fluid, 1 fluid with a link into an obstacle cell, 2 obstacle), the
// list of class-1 cells as (cell, link mask) pairs, and the bounding box of
// the cells of class 1 and 2.  Bit k of a link mask is set when the source
// x - c_k of direction k is an obstacle cell (periodic wrap; a source beyond a
// non-periodic face belongs to the face rules).
// ---------------------------------------------------------------------------
__global__ void k_obst_init(ObstHdr *h) {
  if (threadIdx.x == 0) {
    h->count = 0;
    for (int d = 0; d < 3; ++d) {
      h->lo[d] = 0x7fffffff;
      h->hi[d] = -1;
    }
  }
}

__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

template <int Q>
__global__ __launch_bounds__(256) void k_obst_build(const SCArgs a, const uint8_t *solid, uint8_t *cls,
                                                    uint32_t *list, uint32_t cap, ObstHdr *h) {
  const uint64_t n64 = (uint64_t)blockIdx.x * 256u + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const bool act = n64 < (uint64_t)a.N;
  const uint32_t n = act ? (uint32_t)n64 : 0u;
  const uint32_t nx = (uint32_t)a.nx, nxy = nx * (uint32_t)a.ny;
  const int z = (int)(n / nxy), y = (int)((n - (uint32_t)z * nxy) / nx), x = (int)(n - (uint32_t)z * nxy - (uint32_t)y * nx);
  uint32_t mask = 0;
  int c = 0;
  if (act) {
    if (solid[n]) {
      c = 2;
    } else {
      sfor<Q>([&](auto K) {
        constexpr int k = K;
        if constexpr (k != 0) {
          int s[3] = {x - cx<Q>(k), y - cy<Q>(k), z - cz<Q>(k)};
          const int nn[3] = {a.nx, a.ny, a.nz};
          bool out = false;
          for (int d = 0; d < 3; ++d) {
            if (s[d] < 0 || s[d] >= nn[d]) {
              if (a.periodic[d]) s[d] = s[d] < 0 ? s[d] + nn[d] : s[d] - nn[d];
              else out = true;
            }
          }
          if (!out) {
            const uint32_t src = (uint32_t)s[0] + nx * (uint32_t)s[1] + nxy * (uint32_t)s[2];
            if (solid[src]) mask |= 1u << k;
          }
        }
      });
      c = mask ? 1 : 0;
    }
    cls[n] = (uint8_t)c;
  }
  const bool near = act && c == 1;
  const unsigned long long bm = __ballot(near);
  if (bm) {
    const int leader = __ffsll((long long)bm) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(&h->count, (uint32_t)__popcll(bm));
    base = __shfl(base, leader);
    const uint32_t pos = base + (uint32_t)__popcll(bm & ((1ull << lane) - 1ull));
    if (near && pos < cap) {
      list[2 * (size_t)pos] = n;
      list[2 * (size_t)pos + 1] = mask;
    }
  }
  const bool in = act && c != 0;
  if (__ballot(in)) {
    const int lx = wave_min_i(in ? x : 0x7fffffff), ly = wave_min_i(in ? y : 0x7fffffff),
              lz = wave_min_i(in ? z : 0x7fffffff);
    const int hx = wave_max_i(in ? x : -1), hy = wave_max_i(in ? y : -1), hz = wave_max_i(in ? z : -1);
    if (lane == 0) {
      atomicMin(&h->lo[0], lx);
      atomicMin(&h->lo[1], ly);
      atomicMin(&h->lo[2], lz);
      atomicMax(&h->hi[0], hx);
      atomicMax(&h->hi[1], hy);
      atomicMax(&h->hi[2], hz);
    }
  }
}

hipError_t launch_obst_build(const psm_field &f, const uint8_t *solid, uint8_t *cls, uint32_t *list, uint32_t cap,
                             ObstHdr *h, hipStream_t st) {
  const SCArgs a = make_sc_args(f);
  hipLaunchKernelGGL(k_obst_init, dim3(1), dim3(64), 0, st, h);
  const dim3 g((unsigned)((f.N + 255) / 256));
  if (f.cfg.q == 19)
    hipLaunchKernelGGL((k_obst_build<19>), g, dim3(256), 0, st, a, solid, cls, list, cap, h);
  else
    hipLaunchKernelGGL((k_obst_build<27>), g, dim3(256), 0, st, a, solid, cls, list, cap, h);
  return hipGetLastError();
}

}  // namespace psm
