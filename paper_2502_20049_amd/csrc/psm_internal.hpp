// Internal definitions of the PSM library: lattice tables, handle layouts and
// kernel argument blocks.  Host and device code include this file.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "psm.h"

namespace psm {

// ---------------------------------------------------------------------------
// Velocity sets.  Order: 0 = rest, 1..H = half set, H+k = -(k) (so the
// opposite of i is i +- H).  D3Q19 half set: 3 axis + 6 face diagonals; D3Q27
// adds the 4 body diagonals.  Weights by |c|^2: D3Q19 1/3, 1/18, 1/36;
// D3Q27 8/27, 2/27, 1/54, 1/216.
// ---------------------------------------------------------------------------
template <int Q>
struct Lat;

template <>
struct Lat<19> {
  static constexpr int H = 9;
  static constexpr int hx[9] = {1, 0, 0, 1, 1, 1, 1, 0, 0};
  static constexpr int hy[9] = {0, 1, 0, 1, -1, 0, 0, 1, 1};
  static constexpr int hz[9] = {0, 0, 1, 0, 0, 1, -1, 1, -1};
  static constexpr double w0 = 1.0 / 3.0;
  static constexpr double wn(int m) { return m == 1 ? 1.0 / 18.0 : 1.0 / 36.0; }
};

template <>
struct Lat<27> {
  static constexpr int H = 13;
  static constexpr int hx[13] = {1, 0, 0, 1, 1, 1, 1, 0, 0, 1, 1, 1, 1};
  static constexpr int hy[13] = {0, 1, 0, 1, -1, 0, 0, 1, 1, 1, 1, -1, -1};
  static constexpr int hz[13] = {0, 0, 1, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
  static constexpr double w0 = 8.0 / 27.0;
  static constexpr double wn(int m) { return m == 1 ? 2.0 / 27.0 : (m == 2 ? 1.0 / 54.0 : 1.0 / 216.0); }
};

// full-set accessors (k in [0, Q))
template <int Q>
__host__ __device__ constexpr int cx(int k) {
  return k == 0 ? 0 : (k <= Lat<Q>::H ? Lat<Q>::hx[k - 1] : -Lat<Q>::hx[k - 1 - Lat<Q>::H]);
}
template <int Q>
__host__ __device__ constexpr int cy(int k) {
  return k == 0 ? 0 : (k <= Lat<Q>::H ? Lat<Q>::hy[k - 1] : -Lat<Q>::hy[k - 1 - Lat<Q>::H]);
}
template <int Q>
__host__ __device__ constexpr int cz(int k) {
  return k == 0 ? 0 : (k <= Lat<Q>::H ? Lat<Q>::hz[k - 1] : -Lat<Q>::hz[k - 1 - Lat<Q>::H]);
}
template <int Q>
__host__ __device__ constexpr int opp(int k) {
  return k == 0 ? 0 : (k <= Lat<Q>::H ? k + Lat<Q>::H : k - Lat<Q>::H);
}
template <int Q>
__host__ __device__ constexpr double wt(int k) {
  return k == 0 ? Lat<Q>::w0 : Lat<Q>::wn(cx<Q>(k) * cx<Q>(k) + cy<Q>(k) * cy<Q>(k) + cz<Q>(k) * cz<Q>(k));
}

// ---------------------------------------------------------------------------
// Face kinds and their precedence (wall > inlet > outlet).
// ---------------------------------------------------------------------------
enum : int { K_NONE = 0, K_WALL = PSM_WALL, K_INLET = PSM_INLET, K_OUTLET = PSM_OUTLET };

__host__ __device__ inline int face_rank(int kind) {
  return kind == K_WALL ? 3 : (kind == K_INLET ? 2 : (kind == K_OUTLET ? 1 : 0));
}
__host__ __device__ inline int face_merge(int a, int b) { return face_rank(b) > face_rank(a) ? b : a; }

struct IBox {
  int lo[3];
  int hi[3];  // inclusive; empty when any hi < lo
};

// per-body data of the stream-collide kernels
struct BodyK {
  double X[3];
  double V[3];
  double W[3];
};

// workgroups of the solid-cell kernel (fixed: its per-body partial sums are
// independent of the grid size)
constexpr int SOLID_BLOCKS = 4096;
// at most this many 256-cell chunks per workgroup group of the solid kernel
constexpr int SOLID_MAX_CPW = 8;

struct SCArgs {
  char *pdf;
  const float *B0;
  const float *B1;
  const uint8_t *meta;
  const float *dB;  // optional offset added to the slot-0 fraction (whole-domain mode)
  double *ftp;      // [solid workgroup][max_bodies][6]
  int nx, ny, nz;
  uint32_t N;
  uint64_t dS;  // elements between consecutive direction arrays of the PDF buffer (within a block)
  // PDF layout: row r = y + ny z starts at element (r >> lrb) * bst + (r & rbm) * nx
  // of direction array 0 (SoA: lrb = 31, rbm = all ones, bst = 0)
  int lrb;
  uint32_t rbm;
  uint64_t bst;
  int TX, TY, lTX;  // tile shape of the interior kernel, log2(TX)
  int ntx;
  int nty_i;          // tile rows over the interior rows 1..ny-2
  uint32_t ntiles_i;  // ntx * nty_i * (nz - 2): blocks of the interior kernel
  int nfrows;         // rows with y or z on a face
  uint32_t ntiles_e;  // ntx * ceil(nfrows / TY): blocks of the edge kernel
  int general;        // PSM_OPT_GENERAL_PATH: every cell through the general kernel
  int bc[6];
  int periodic[3];
  double u_in_d[3];
  double force[3];
  int has_force;
  double lam_e, lam_o;
  int nb;
  int max_bodies;
  int slots;
  int xcd_remap;  // PSM_OPT_XCD_REMAP: contiguous tile ranges per XCD
  int solid_grid;  // most workgroups of the solid kernel (PSM_OPT_SOLID_GRID), 1..SOLID_BLOCKS
  int nbox;       // boxes outside which every B is zero (one per body)
  IBox box[PSM_MAX_BODIES];
  uint32_t cprefix[PSM_MAX_BODIES + 1];  // 256-cell chunk offsets of the boxes
  uint32_t nchunks;
  int cpw;  // chunks per group of the solid kernel, 1..SOLID_MAX_CPW
  // non-null: the interior launch has one extra workgroup (index ft_block)
  // that sums the F/T of ft_nb bodies from ft_nblocks solid partials into it
  double *ft_out;
  int ft_nb, ft_nblocks;
  uint32_t ft_block;
  BodyK body[PSM_MAX_BODIES];
  // static obstacle of a plain-LBM field (ocls null: none)
  const uint8_t *ocls;    // per cell: 0 bulk fluid, 1 fluid next to the obstacle, 2 obstacle
  const uint32_t *olist;  // class-1 cells as (cell, link mask) pairs
  uint32_t ocount;
  IBox obox;              // bounding box of the class-1 and class-2 cells
};

// workgroups of the adjoint step: four waves of 64 cells of one row each
__host__ __device__ __forceinline__ uint32_t adjoint_blocks(int nx, int ny, int nz) {
  const uint64_t units = (uint64_t)ny * (uint64_t)nz * (uint64_t)((nx + 63) / 64);
  return (uint32_t)((units + 3) / 4);
}

// element offset of row r (= y + ny z) in direction array 0 of the PDF buffer
__host__ __device__ __forceinline__ uint64_t pdf_row(const SCArgs &a, uint32_t r) {
  return (uint64_t)(r >> a.lrb) * a.bst + (uint64_t)(r & a.rbm) * (uint64_t)(uint32_t)a.nx;
}

// header of the obstacle buffer (set-up counters)
struct ObstHdr {
  uint32_t count;
  int32_t lo[3];
  int32_t hi[3];
};

// arguments of the adjoint step kernel
struct AdjArgs {
  SCArgs s;           // field geometry, faces, rates, B pointers
  const char *fwd;    // forward state before step t (storage type, parity t&1), the PDF buffer's layout
  int parity;
  int o32;            // the PDF copy and both adjoint arrays each span < 2^32 bytes
  const void *ain;    // fhat(t+1): the PDF buffer's layout, adjoint precision
  void *aout;         // fhat(t)
  void *dJdB;         // accumulated, [N], adjoint precision
  double X[3], V[3], W[3], axis[3];
  double wt;
  double *part;       // per-workgroup dJ/dOmega partial sums
};

// per-body data of the mapping kernel
struct MapBodyK {
  double R[9];
  double X[3];
  const uint32_t *bits;
  const uint8_t *coarse;
  int mmin[3], dims[3], wx;
  int cmin[3], cdims[3];
  int s;
  int block;          // 1: the cell's centre only is rotated and the axis-aligned block averaged
  long long dabs[3];  // bound on |fixed-point sub-sample offset| per axis
  IBox region;        // cells rewritten this step (swept box now and before)
  IBox active;        // cells that can touch the body this step
  uint32_t region_cells;
};

// capacity of a body's list of surface cells left to the sampling kernel
constexpr uint32_t MAP_LIST_CAP = 1u << 21;
constexpr uint32_t MAP_SAMPLE_BLOCKS = 1024;

struct MapArgs {
  float *B0;
  float *B1;
  uint8_t *meta;
  int32_t *err;
  uint32_t *list;        // [body][cap] cell indices, or null (no list)
  uint32_t *count;       // [body] appended this call
  uint32_t *count_next;  // [body] cleared for the next call
  uint32_t cap;
  int nx, ny, nz;
  int nb;
  int slots;
  int b_form;
  double tau;
  MapBodyK body[PSM_MAX_BODIES];
};

}  // namespace psm

// ---------------------------------------------------------------------------
// Host handles
// ---------------------------------------------------------------------------
struct psm_field {
  psm_config cfg;
  void *pdf;
  size_t pdf_bytes;
  float *B0;
  float *B1;
  uint8_t *meta;
  size_t b_bytes;
  char *work;
  size_t work_bytes;
  int32_t *err;
  double *ftp;
  double *red;  // reduction scratch
  uint32_t *map_list;   // surface-cell lists of the mapping (null: none)
  uint32_t *map_count;  // two sets of per-body counters, used in turn
  int map_parity;
  int map_list_cap;     // entries per body actually used (PSM_OPT_MAP_LIST)
  int map_list_max;     // entries per body the work area holds
  bool static_work;     // work area: the library's static array (pdf_field_create_noalloc)
  size_t red_count;
  int64_t N;
  int64_t dstride;  // direction stride of the PDF buffer, elements (within a block)
  int lrb;          // PDF layout: log2 rows per block (SoA: 31), row mask, block stride
  uint32_t rbm;
  int64_t bstride;
  int TX, TY, lTX, ntx, nty;
  int64_t ntiles;
  int nb_mapped;
  int solid_blocks;  // workgroups of the last solid-cell launch (partials written)
  bool have_prev[PSM_MAX_BODIES];
  psm::IBox active[PSM_MAX_BODIES];
  int device;
  int opt_general_path;
  int opt_xcd_remap;
  int opt_solid_grid;
  int opt_whole_domain;  // B may be nonzero anywhere (offset field set)
  int opt_concurrent;    // PSM_OPT_CONCURRENT
  // second stream of the field (null for fields on the static work area): the
  // solid-cell and face-row launches of a step run on it beside the interior
  // launch, forked from and joined back into the caller's stream by events
  hipStream_t side;
  hipEvent_t ev_fork, ev_join;
  void *bbase;  // start of the fractions buffer (both sets with map_ahead)
  // map_ahead: the other set of fractions and its mapping state (swapped with
  // the current one by psm_step_ahead), the stream that maps into it, and
  // the step it holds when ahead_valid
  float *B0x, *B1x;
  uint8_t *metax;
  psm::IBox activex[PSM_MAX_BODIES];
  bool have_prevx[PSM_MAX_BODIES];
  int nb_mappedx;
  bool ahead_valid;
  int64_t ahead_step;
  int ahead_nb;
  hipStream_t mstream;
  hipEvent_t ev_mfork, ev_mjoin;
  const float *dB;       // caller-owned offset added to the slot-0 fraction
  // static obstacle (plain-LBM fields; null: none)
  uint8_t *ocls;
  uint32_t *olist;
  uint32_t ocount;
  psm::IBox obox;
};

struct psm_geom {
  int s;
  int32_t mmin[3], dims[3];
  int wx;
  int32_t cmin[3], cdims[3];
  double r_bound;  // every inside lattice centre lies within r_bound of the body origin
  uint32_t *dev_bits;
  uint8_t *dev_coarse;
  size_t bytes;
  uint32_t *host_bits;   // kept until destroy (source of the async upload)
  uint8_t *host_coarse;
};

namespace psm {
void set_error(const std::string &msg);
int hip_fail(hipError_t e, const char *what);

// launchers (defined in the .hip translation units)
hipError_t launch_map(const MapArgs &a, uint32_t max_region_cells, int any_s_max, hipStream_t st);
hipError_t launch_ft_reduce(const psm_field &f, int nb, double *ft, hipStream_t st);
SCArgs make_sc_args(const psm_field &f);
hipError_t launch_macro(const psm_field &f, int parity, double *rho, double *u, double *mass_partials,
                        int want_field, hipStream_t st);
hipError_t launch_mass_final(const double *partials, uint32_t n, double *out, hipStream_t st);
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t st);
hipError_t launch_copy(const void *src, void *dst, size_t bytes, hipStream_t st);
// a buffer in the PDF buffer's layout to (to_std) or from [q][N], elements of sz bytes
hipError_t launch_pdf_gather(const psm_field &f, void *dst, const void *src, int to_std, size_t sz, hipStream_t st);
hipError_t launch_flags_copy(const int32_t *src, int32_t *dst, hipStream_t st);
uint32_t macro_blocks(const psm_field &f);
hipError_t launch_sum_accumulate(const double *p, uint32_t n, double *out, hipStream_t st);
hipError_t launch_obst_build(const psm_field &f, const uint8_t *solid, uint8_t *cls, uint32_t *list, uint32_t cap,
                             ObstHdr *h, hipStream_t st);

// host geometry
int geom_box(int kind, const double *params, const double *verts, int64_t nv, int s, int32_t mmin[3],
             int32_t dims[3]);
void voxelize_rows(const double *verts, const int32_t *tris, int64_t nt, int s, const int32_t mmin[3],
                   const int32_t dims[3], uint32_t *bits);
void analytic_rows(int kind, const double *params, int s, const int32_t mmin[3], const int32_t dims[3],
                   uint32_t *bits);
void coarse_map(int s, const int32_t mmin[3], const int32_t dims[3], const uint32_t *bits, int32_t cmin[3],
                int32_t cdims[3], uint8_t *out);
void coarse_extent(int s, const int32_t mmin[3], const int32_t dims[3], int32_t cmin[3], int32_t cdims[3]);
}  // namespace psm
