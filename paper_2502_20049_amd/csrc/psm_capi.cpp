// C ABI of the PSM library: argument validation, host kinematics, handle
// bookkeeping and kernel launches.  All device memory is caller-owned.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <utility>
#include <atomic>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "psm_internal.hpp"

namespace psm {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

int hip_fail(hipError_t e, const char *what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return PSM_EHIP;
}

hipError_t launch_adjoint(const psm_field &f, const AdjArgs &A, hipStream_t st);
hipError_t launch_sc_f64(const psm_config &, const SCArgs &, int, hipStream_t, hipStream_t, int *, int *);
hipError_t launch_sc_f32(const psm_config &, const SCArgs &, int, hipStream_t, hipStream_t, int *, int *);
hipError_t launch_sc_f16(const psm_config &, const SCArgs &, int, hipStream_t, hipStream_t, int *, int *);

static size_t storage_size(int st) { return st == PSM_F64 ? 8 : (st == PSM_F32 ? 4 : 2); }

static void tile_shape(int nx, int &TX, int &lTX) {
  // the smallest padded row length; ties go to the wider tile
  int best = 256, bestpad = ((nx + 255) / 256) * 256;
  for (int t : {128, 64}) {
    const int pad = ((nx + t - 1) / t) * t;
    if (pad < bestpad) {
      best = t;
      bestpad = pad;
    }
  }
  TX = best;
  lTX = best == 256 ? 8 : (best == 128 ? 7 : 6);
}

struct Layout {
  int TX, TY, lTX, ntx, nty;
  int64_t ntiles, N;
  size_t off_ftp, off_red, off_list, work_bytes;
  uint32_t red_count;
};

// work buffer: [0, 256) error flags (offset 0) and the mapping's per-body
// list counters (offset 64, two sets); then F/T partials, reduction scratch
// and the mapping's surface-cell lists
constexpr size_t OFF_MAP_COUNT = 64;

// Direction arrays of the PDF buffer: N elements each, padded so that
// consecutive arrays start 4 KiB past a 4 KiB multiple apart (the 19 or 27
// streams of a step then do not all fall at the same offset modulo a large
// power of two: measured 1-4% faster on 256^3 than back-to-back arrays).
//
// Blocked layout: rows (r = y + ny z) in blocks of RB = 2^m rows (by default
// the largest power of two with RB nx sizeof(storage) <= 16 KiB, at least
// one row); each block holds its q direction arrays of RB nx cells back to
// back.
struct PdfLayout {
  int lrb;           // log2 RB (SoA: 31)
  uint32_t rbm;      // RB - 1 (SoA: all ones)
  int64_t rb;        // rows per block (SoA: ny nz)
  int64_t dstride;   // elements between direction arrays (within a block)
  int64_t bstride;   // elements between blocks (SoA: 0)
  int64_t elems;     // elements of the whole buffer
};

static PdfLayout pdf_layout_of(const psm_config &c) {
  PdfLayout L{};
  const int64_t N = (int64_t)c.nx * c.ny * c.nz;
  const int64_t rows = (int64_t)c.ny * c.nz;
  const int64_t sz = (int64_t)storage_size(c.storage);
  if (c.layout == PSM_LAYOUT_BLOCKED) {
    int m = 0;
    if (c.block_rows > 0) {
      while ((1 << m) < c.block_rows) ++m;
    } else {
      while (((int64_t)c.nx << (m + 1)) * sz <= 16384 && (1ll << (m + 1)) <= rows) ++m;
    }
    L.lrb = m;
    L.rbm = (1u << m) - 1u;
    L.rb = 1ll << m;
    L.dstride = L.rb * c.nx;
    L.bstride = L.dstride * c.q;
    L.elems = ((rows + L.rb - 1) >> m) * L.bstride;
  } else {
    const int64_t bytes = ((N * sz + 4095) / 4096) * 4096 + 4096;
    L.lrb = 31;
    L.rbm = 0xffffffffu;
    L.rb = rows;
    L.dstride = bytes / sz;
    L.bstride = 0;
    L.elems = L.dstride * c.q;
  }
  return L;
}

static int64_t pdf_stride_elems(const psm_config &c) { return pdf_layout_of(c).dstride; }

// One set of solid fractions: slot 0, slot 1 (two slots), body ids; with
// map_ahead the second set starts at this size rounded up to 256 bytes.
static size_t b_set_bytes(const psm_config &c) {
  const size_t N = (size_t)c.nx * (size_t)c.ny * (size_t)c.nz;
  const size_t one = N * 4 * (size_t)c.slots + N;
  return c.map_ahead ? (one + 255) / 256 * 256 : one;
}

// Adjoint arrays: the PDF buffer's layout (in elements) in the adjoint precision.
static size_t adjoint_elem_size(const psm_config &c) { return c.storage == PSM_F64 ? 8 : 4; }

static Layout layout_of(const psm_config &c) {
  Layout L{};
  L.N = (int64_t)c.nx * c.ny * c.nz;
  tile_shape(c.nx, L.TX, L.lTX);
  L.TY = 256 / L.TX;
  L.ntx = (c.nx + L.TX - 1) / L.TX;
  L.nty = (c.ny + L.TY - 1) / L.TY;
  L.ntiles = (int64_t)L.ntx * L.nty * c.nz;
  const int mb = c.psm ? std::max(1, c.max_bodies) : 0;
  L.off_ftp = 256;
  L.off_red = L.off_ftp + (size_t)SOLID_BLOCKS * mb * 6 * sizeof(double);
  L.red_count = (uint32_t)((L.N + 255) / 256);
  // the slots also hold the adjoint step's per-workgroup partials
  const size_t red_slots = std::max<size_t>(L.red_count, adjoint_blocks(c.nx, c.ny, c.nz));
  L.off_list = ((L.off_red + red_slots * sizeof(double) + 64 + 255) / 256) * 256;
  L.work_bytes = L.off_list + (size_t)mb * MAP_LIST_CAP * sizeof(uint32_t);
  return L;
}

static int check_config(const psm_config *c) {
  if (!c) return set_error("null config"), PSM_EINVAL;
  if (c->nx < 1 || c->ny < 1 || c->nz < 1) return set_error("grid dimensions must be >= 1"), PSM_EINVAL;
  const int64_t N = (int64_t)c->nx * c->ny * c->nz;
  if (N >= (int64_t)1 << 32) return set_error("more than 2^32 - 1 cells"), PSM_EUNSUP;
  if (c->q != 19 && c->q != 27) return set_error("q must be 19 or 27"), PSM_EINVAL;
  if (c->storage < PSM_F64 || c->storage > PSM_F16) return set_error("bad storage"), PSM_EINVAL;
  if (c->psm != 0 && c->psm != 1) return set_error("psm must be 0 or 1"), PSM_EINVAL;
  if (c->sc < 1 || c->sc > 3) return set_error("sc must be 1, 2 or 3"), PSM_EINVAL;
  if (c->b_form != 0 && c->b_form != 1) return set_error("b_form must be 0 or 1"), PSM_EINVAL;
  if (c->map_reading != PSM_MAP_SUBSAMPLES && c->map_reading != PSM_MAP_BLOCK)
    return set_error("map_reading must be PSM_MAP_SUBSAMPLES or PSM_MAP_BLOCK"), PSM_EINVAL;
  if (c->layout != PSM_LAYOUT_SOA && c->layout != PSM_LAYOUT_BLOCKED)
    return set_error("layout must be PSM_LAYOUT_SOA or PSM_LAYOUT_BLOCKED"), PSM_EINVAL;
  if (c->block_rows != 0) {
    if (c->layout != PSM_LAYOUT_BLOCKED) return set_error("block_rows needs PSM_LAYOUT_BLOCKED"), PSM_EINVAL;
    const int64_t rows = (int64_t)c->ny * c->nz;
    if (c->block_rows < 0 || (c->block_rows & (c->block_rows - 1)) != 0 || c->block_rows > 2 * rows ||
        (int64_t)c->block_rows * c->nx * c->q > ((int64_t)1 << 32))
      return set_error("block_rows must be a power of two, at most twice the row count"), PSM_EINVAL;
  }
  if (c->slots != 1 && c->slots != 2) return set_error("slots must be 1 or 2"), PSM_EINVAL;
  if (c->map_ahead != 0 && c->map_ahead != 1) return set_error("map_ahead must be 0 or 1"), PSM_EINVAL;
  if (c->map_ahead && !c->psm) return set_error("map_ahead needs psm = 1"), PSM_EINVAL;
  if (c->psm && (c->max_bodies < 1 || c->max_bodies > PSM_MAX_BODIES))
    return set_error("max_bodies must be in 1..8"), PSM_EINVAL;
  if (!(c->tau > 0.5) || !isfinite(c->tau)) return set_error("tau must be > 1/2"), PSM_EINVAL;
  if (!isfinite(c->magic) || !(c->magic > 0)) return set_error("magic must be > 0"), PSM_EINVAL;
  for (int f = 0; f < 6; ++f)
    if (c->bc[f] < PSM_PERIODIC || c->bc[f] > PSM_OUTLET) return set_error("bad face kind"), PSM_EINVAL;
  for (int a = 0; a < 3; ++a)
    if ((c->bc[2 * a] == PSM_PERIODIC) != (c->bc[2 * a + 1] == PSM_PERIODIC))
      return set_error("periodic faces must come in pairs"), PSM_EINVAL;
  if (c->collision != PSM_COLL_TRT && c->collision != PSM_COLL_CUMULANT)
    return set_error("collision must be PSM_COLL_TRT or PSM_COLL_CUMULANT"), PSM_EINVAL;
  if (c->collision == PSM_COLL_CUMULANT &&
      (c->q != 27 || c->force[0] != 0.0 || c->force[1] != 0.0 || c->force[2] != 0.0))
    return set_error("the cumulant collision is D3Q27 without body force"), PSM_EUNSUP;
  return PSM_OK;
}

SCArgs make_sc_args(const psm_field &f) {
  SCArgs a;
  memset(&a, 0, sizeof(a));
  const psm_config &c = f.cfg;
  a.pdf = (char *)f.pdf;
  a.B0 = f.B0;
  a.B1 = f.B1;
  a.meta = f.meta;
  a.ftp = f.ftp;
  a.nx = c.nx;
  a.ny = c.ny;
  a.nz = c.nz;
  a.N = (uint32_t)f.N;
  a.dS = (uint64_t)f.dstride;
  a.lrb = f.lrb;
  a.rbm = f.rbm;
  a.bst = (uint64_t)f.bstride;
  a.TX = f.TX;
  a.TY = f.TY;
  a.lTX = f.lTX;
  a.ntx = f.ntx;
  const bool interior = c.ny >= 3 && c.nz >= 3;
  a.nty_i = interior ? (c.ny - 2 + f.TY - 1) / f.TY : 0;
  a.ntiles_i = interior ? (uint32_t)((int64_t)f.ntx * a.nty_i * (c.nz - 2)) : 0u;
  const int nzp = c.nz >= 2 ? 2 : 1, nyp = c.ny >= 2 ? 2 : 1;
  a.nfrows = nzp * c.ny + (c.nz > 2 ? (c.nz - 2) * nyp : 0);
  a.ntiles_e = (uint32_t)((int64_t)f.ntx * ((a.nfrows + f.TY - 1) / f.TY));
  a.general = f.opt_general_path;
  for (int i = 0; i < 6; ++i) a.bc[i] = c.bc[i];
  for (int d = 0; d < 3; ++d) {
    a.periodic[d] = c.bc[2 * d] == PSM_PERIODIC;
    a.u_in_d[d] = c.u_in[d];
    a.force[d] = c.force[d];
  }
  a.has_force = (c.force[0] != 0.0 || c.force[1] != 0.0 || c.force[2] != 0.0);
  a.lam_e = 1.0 / c.tau;
  a.lam_o = 1.0 / (0.5 + c.magic / (c.tau - 0.5));
  a.max_bodies = std::max(1, c.max_bodies);
  a.slots = c.slots;
  a.dB = f.opt_whole_domain ? f.dB : nullptr;
  a.cpw = 1;
  a.solid_grid = f.opt_solid_grid;
  a.ft_out = nullptr;
  a.ft_nb = 0;
  a.ft_nblocks = 0;
  a.ft_block = 0;
  a.ocls = f.ocls;
  a.olist = f.olist;
  a.ocount = f.ocount;
  a.obox = f.obox;
  return a;
}

static IBox empty_box() {
  IBox b;
  for (int a = 0; a < 3; ++a) {
    b.lo[a] = 1;
    b.hi[a] = 0;
  }
  return b;
}

static bool box_empty(const IBox &b) { return b.hi[0] < b.lo[0] || b.hi[1] < b.lo[1] || b.hi[2] < b.lo[2]; }

static IBox box_union(const IBox &a, const IBox &b) {
  if (box_empty(a)) return b;
  if (box_empty(b)) return a;
  IBox r;
  for (int d = 0; d < 3; ++d) {
    r.lo[d] = std::min(a.lo[d], b.lo[d]);
    r.hi[d] = std::max(a.hi[d], b.hi[d]);
  }
  return r;
}

// ---- library-owned work area of pdf_field_create_noalloc ---------------------
// A file-scope device array: every GPU the library runs on holds its own copy
// until the process ends.  On the host the name is only a stand-in symbol, so
// host code never passes it to a kernel or copy: each device's address is
// looked up once (hipGetSymbolAddress, with that device current) and kept.
static __device__ __align__(256) unsigned char scratch[PSM_STATIC_WORK_BYTES];

constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[MAX_DEVICES];
// the field created (or reset) last on each device with the static work area;
// only that field may use it
static std::atomic<const psm_field *> g_scratch_owner[MAX_DEVICES];

static int scratch_address(int dev, void **out) {
  if (dev < 0 || dev >= MAX_DEVICES) return set_error("device ordinal out of range for the static work area"), PSM_EUNSUP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "static work area: hipGetSymbolAddress");
    if (!p) return set_error("static work area: null symbol address"), PSM_EHIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return PSM_OK;
}

// Entry points that touch the work area call this: a field on the static work
// area must be the one that last claimed it on its device.
static int work_usable(const psm_field *f) {
  if (!f->static_work) return PSM_OK;
  if (f->device < 0 || f->device >= MAX_DEVICES || g_scratch_owner[f->device].load() != f)
    return set_error("another field has claimed the library's static work area on this device since this field "
                     "was created or reset (psm_field_reset claims it back)"),
           PSM_EINVAL;
  return PSM_OK;
}

}  // namespace psm

using namespace psm;

extern "C" {

const char *psm_last_error(void) { return g_err.c_str(); }

// obstacle buffer: header (256 B), class bytes (N, padded to 256 B), list
static size_t obst_list_offset(int64_t N) { return 256 + (((size_t)N + 255) & ~(size_t)255); }

int psm_required_bytes(const psm_config *cfg, int which, size_t *out) {
  int r = check_config(cfg);
  if (r) return r;
  if (!out) return set_error("null output"), PSM_EINVAL;
  const Layout L = layout_of(*cfg);
  switch (which) {
    case PSM_BUF_PDF:
      *out = (size_t)pdf_layout_of(*cfg).elems * storage_size(cfg->storage);
      return PSM_OK;
    case PSM_BUF_B:
      *out = cfg->psm ? b_set_bytes(*cfg) * (cfg->map_ahead ? 2 : 1) : 0;
      return PSM_OK;
    case PSM_BUF_WORK:
      *out = L.work_bytes;
      return PSM_OK;
    case PSM_BUF_ADJOINT:
      *out = (size_t)pdf_layout_of(*cfg).elems * adjoint_elem_size(*cfg);
      return PSM_OK;
    case PSM_BUF_GRAD_B:
      *out = (size_t)L.N * (cfg->storage == PSM_F64 ? 8 : 4);
      return PSM_OK;
    case PSM_BUF_OBSTACLE:
      *out = cfg->psm ? 0 : obst_list_offset(L.N) + 8 * (size_t)L.N;
      return PSM_OK;
  }
  return set_error("bad buffer id"), PSM_EINVAL;
}

int psm_pdf_stride(const psm_config *cfg, int64_t *elems) {
  int r = check_config(cfg);
  if (r) return r;
  if (!elems) return set_error("null output"), PSM_EINVAL;
  *elems = pdf_stride_elems(*cfg);
  return PSM_OK;
}

int psm_pdf_layout(const psm_config *cfg, int32_t *rows_per_block, int64_t *dir_stride, int64_t *block_stride) {
  int r = check_config(cfg);
  if (r) return r;
  const PdfLayout L = pdf_layout_of(*cfg);
  if (rows_per_block) *rows_per_block = (int32_t)L.rb;
  if (dir_stride) *dir_stride = L.dstride;
  if (block_stride) *block_stride = L.bstride;
  return PSM_OK;
}

int psm_lattice(int q, int32_t *c, double *w, int32_t *o) {
  if ((q != 19 && q != 27) || !c || !w || !o) return set_error("psm_lattice: bad arguments"), PSM_EINVAL;
  for (int k = 0; k < q; ++k) {
    if (q == 19) {
      c[3 * k] = cx<19>(k);
      c[3 * k + 1] = cy<19>(k);
      c[3 * k + 2] = cz<19>(k);
      w[k] = wt<19>(k);
      o[k] = opp<19>(k);
    } else {
      c[3 * k] = cx<27>(k);
      c[3 * k + 1] = cy<27>(k);
      c[3 * k + 2] = cz<27>(k);
      w[k] = wt<27>(k);
      o[k] = opp<27>(k);
    }
  }
  return PSM_OK;
}

int psm_body_pose(const psm_motion *m, int64_t step, psm_body *out) {
  if (!m || !out) return set_error("psm_body_pose: null argument"), PSM_EINVAL;
  const double t = (double)step;
  const double theta = m->theta0 + m->omega * t;
  const double c = cos(theta), s = sin(theta), omc = 1.0 - c;
  const double *a = m->axis;
  const double K[9] = {0.0, -a[2], a[1], a[2], 0.0, -a[0], -a[1], a[0], 0.0};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const double d = (i == j) ? c : 0.0;
      out->R[3 * i + j] = (d + (omc * a[i]) * a[j]) + s * K[3 * i + j];
    }
  for (int i = 0; i < 3; ++i) {
    out->X[i] = m->x0[i] + m->v[i] * t;
    out->V[i] = m->v[i];
    out->W[i] = m->omega * a[i];
  }
  return PSM_OK;
}

// Shared by pdf_field_create and pdf_field_create_noalloc: `work` is the
// caller's buffer, or the device's static work area with the surface-cell
// lists cut to `list_cap` entries per body.
static int field_create(const psm_config *cfg, void *pdf, size_t pdf_bytes, void *b, size_t b_bytes, void *work,
                        size_t work_bytes, uint32_t list_cap, bool static_work, int device, void *stream,
                        psm_field **out) {
  size_t need_pdf, need_b;
  psm_required_bytes(cfg, PSM_BUF_PDF, &need_pdf);
  psm_required_bytes(cfg, PSM_BUF_B, &need_b);
  if (!pdf || !work || (cfg->psm && !b)) return set_error("null device buffer"), PSM_EINVAL;
  if (pdf_bytes < need_pdf) return set_error("pdf buffer too small"), PSM_ESIZE;
  if (b_bytes < need_b) return set_error("B buffer too small"), PSM_ESIZE;
  if (((uintptr_t)pdf | (uintptr_t)work | (uintptr_t)b) & 15u)
    return set_error("device buffers must be 16-byte aligned"), PSM_EINVAL;
  psm_field *f = new (std::nothrow) psm_field;
  if (!f) return set_error("out of host memory"), PSM_EINVAL;
  memset(f, 0, sizeof(*f));
  f->cfg = *cfg;
  if (!cfg->psm) f->cfg.max_bodies = 0;
  const Layout L = layout_of(*cfg);
  f->pdf = pdf;
  f->pdf_bytes = pdf_bytes;
  f->N = L.N;
  {
    const PdfLayout PL = pdf_layout_of(*cfg);
    f->dstride = PL.dstride;
    f->lrb = PL.lrb;
    f->rbm = PL.rbm;
    f->bstride = PL.bstride;
  }
  if (cfg->psm) {
    f->bbase = b;
    f->B0 = (float *)b;
    f->B1 = cfg->slots == 2 ? (float *)b + L.N : nullptr;
    f->meta = (uint8_t *)((float *)b + L.N * cfg->slots);
    f->b_bytes = b_bytes;
    if (cfg->map_ahead) {
      char *bx = (char *)b + b_set_bytes(*cfg);
      f->B0x = (float *)bx;
      f->B1x = cfg->slots == 2 ? (float *)bx + L.N : nullptr;
      f->metax = (uint8_t *)((float *)bx + L.N * cfg->slots);
    }
  }
  f->work = (char *)work;
  f->work_bytes = work_bytes;
  f->static_work = static_work;
  f->err = (int32_t *)work;
  f->ftp = (double *)((char *)work + L.off_ftp);
  f->red = (double *)((char *)work + L.off_red);
  f->red_count = L.red_count;
  if (cfg->psm) {
    f->map_list = (uint32_t *)((char *)work + L.off_list);
    f->map_count = (uint32_t *)((char *)work + OFF_MAP_COUNT);
  }
  f->TX = L.TX;
  f->TY = L.TY;
  f->lTX = L.lTX;
  f->ntx = L.ntx;
  f->nty = L.nty;
  f->ntiles = L.ntiles;
  for (int i = 0; i < PSM_MAX_BODIES; ++i) f->active[i] = f->activex[i] = empty_box();
  f->opt_xcd_remap = 0;
  f->opt_solid_grid = SOLID_BLOCKS;
  f->opt_concurrent = 1;
  if (!static_work) {
    // the second stream (default priority) and its fork / join events; the
    // field runs sequentially on the caller's stream if they cannot be made
    if (hipStreamCreateWithFlags(&f->side, hipStreamNonBlocking) == hipSuccess) {
      if (hipEventCreateWithFlags(&f->ev_fork, hipEventDisableTiming) != hipSuccess ||
          hipEventCreateWithFlags(&f->ev_join, hipEventDisableTiming) != hipSuccess) {
        if (f->ev_fork) hipEventDestroy(f->ev_fork);
        hipStreamDestroy(f->side);
        f->side = nullptr;
        f->ev_fork = nullptr;
      }
    } else {
      f->side = nullptr;
    }
    // the mapping stream of map_ahead fields, likewise optional
    if (cfg->map_ahead && hipStreamCreateWithFlags(&f->mstream, hipStreamNonBlocking) == hipSuccess) {
      if (hipEventCreateWithFlags(&f->ev_mfork, hipEventDisableTiming) != hipSuccess ||
          hipEventCreateWithFlags(&f->ev_mjoin, hipEventDisableTiming) != hipSuccess) {
        if (f->ev_mfork) hipEventDestroy(f->ev_mfork);
        hipStreamDestroy(f->mstream);
        f->mstream = nullptr;
        f->ev_mfork = nullptr;
      }
    } else {
      f->mstream = nullptr;
    }
    (void)hipGetLastError();
  }
  f->map_list_max = cfg->psm ? (int)list_cap : 0;
  f->map_list_cap = f->map_list_max;
  f->device = device;
  {
    // error flags and mapping counters start at zero
    hipError_t e = launch_fill_zero(work, 256, (hipStream_t)stream);
    if (e != hipSuccess) {
      delete f;
      return hip_fail(e, "pdf_field_create: clear");
    }
  }
  if (static_work) g_scratch_owner[device].store(f);
  *out = f;
  return PSM_OK;
}

int pdf_field_create(const psm_config *cfg, void *pdf, size_t pdf_bytes, void *b, size_t b_bytes, void *work,
                     size_t work_bytes, void *stream, psm_field **out) {
  int r = check_config(cfg);
  if (r) return r;
  if (!out) return set_error("null output handle"), PSM_EINVAL;
  size_t need_w;
  psm_required_bytes(cfg, PSM_BUF_WORK, &need_w);
  if (work && work_bytes < need_w) return set_error("work buffer too small"), PSM_ESIZE;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) dev = -1;
  return field_create(cfg, pdf, pdf_bytes, b, b_bytes, work, work_bytes, MAP_LIST_CAP, false, dev, stream, out);
}

int pdf_field_create_noalloc(const psm_config *cfg, void *pdf, size_t pdf_bytes, void *b, size_t b_bytes,
                             void *stream, psm_field **out) {
  int r = check_config(cfg);
  if (r) return r;
  if (!out) return set_error("null output handle"), PSM_EINVAL;
  const Layout L = layout_of(*cfg);
  if (L.off_list > (size_t)PSM_STATIC_WORK_BYTES)
    return set_error("pdf_field_create_noalloc: this lattice and body count need " + std::to_string(L.off_list) +
                     " bytes of work area, more than the static " + std::to_string((size_t)PSM_STATIC_WORK_BYTES)),
           PSM_ESIZE;
  const int mb = cfg->psm ? std::max(1, cfg->max_bodies) : 1;
  const size_t fit = ((size_t)PSM_STATIC_WORK_BYTES - L.off_list) / ((size_t)mb * sizeof(uint32_t));
  const uint32_t cap = (uint32_t)std::min<size_t>(fit, MAP_LIST_CAP);
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "pdf_field_create_noalloc: hipGetDevice");
  void *work = nullptr;
  r = scratch_address(dev, &work);
  if (r) return r;
  return field_create(cfg, pdf, pdf_bytes, b, b_bytes, work, PSM_STATIC_WORK_BYTES, cap, true, dev, stream, out);
}

int pdf_field_destroy(psm_field *f) {
  if (!f) return set_error("null handle"), PSM_EINVAL;
  if (f->static_work && f->device >= 0 && f->device < MAX_DEVICES) {
    const psm_field *mine = f;
    g_scratch_owner[f->device].compare_exchange_strong(mine, nullptr);
  }
  if (f->side) {
    hipStreamSynchronize(f->side);
    hipEventDestroy(f->ev_fork);
    hipEventDestroy(f->ev_join);
    hipStreamDestroy(f->side);
  }
  if (f->mstream) {
    hipStreamSynchronize(f->mstream);
    hipEventDestroy(f->ev_mfork);
    hipEventDestroy(f->ev_mjoin);
    hipStreamDestroy(f->mstream);
  }
  delete f;
  return PSM_OK;
}

int psm_field_reset(psm_field *f, void *stream) {
  if (!f) return set_error("null handle"), PSM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  size_t need;
  psm_required_bytes(&f->cfg, PSM_BUF_PDF, &need);
  hipError_t e = launch_fill_zero(f->pdf, need, st);
  if (e == hipSuccess && f->cfg.psm) {
    // the whole buffer from its start: with map_ahead, B0 may be the second set
    psm_required_bytes(&f->cfg, PSM_BUF_B, &need);
    e = launch_fill_zero(f->bbase, need, st);
  }
  if (e == hipSuccess) e = launch_fill_zero(f->work, 256, st);
  if (e != hipSuccess) return hip_fail(e, "psm_field_reset");
  if (f->static_work) g_scratch_owner[f->device].store(f);
  f->nb_mapped = f->nb_mappedx = 0;
  f->map_parity = 0;
  f->ahead_valid = false;
  if (f->cfg.map_ahead && (void *)f->B0 != f->bbase) {  // back to the first set as the current one
    std::swap(f->B0, f->B0x);
    std::swap(f->B1, f->B1x);
    std::swap(f->meta, f->metax);
  }
  for (int i = 0; i < PSM_MAX_BODIES; ++i) {
    f->have_prev[i] = f->have_prevx[i] = false;
    f->active[i] = f->activex[i] = empty_box();
  }
  return PSM_OK;
}

// ---- geometry ----------------------------------------------------------------
static size_t geom_bytes(int s, const int32_t mmin[3], const int32_t dims[3], size_t *coarse_off) {
  const size_t wx = ((size_t)dims[0] + 31) / 32;
  const size_t bits = wx * (size_t)dims[1] * (size_t)dims[2] * 4;
  int32_t cmin[3], cd[3];
  coarse_extent(s, mmin, dims, cmin, cd);
  const size_t off = (bits + 255) & ~(size_t)255;
  *coarse_off = off;
  return off + (size_t)cd[0] * cd[1] * cd[2];
}

int psm_geometry_box(int kind, const double *params, const double *verts, int64_t nv, int s, int32_t mmin[3],
                     int32_t dims[3], size_t *dev_bytes) {
  if (s < 0 || s > 3) return set_error("supersampling depth s must be 0..3"), PSM_EUNSUP;
  if (!mmin || !dims || !dev_bytes || (!verts && !params)) return set_error("null argument"), PSM_EINVAL;
  const int r = geom_box(kind, params, verts, nv, s, mmin, dims);
  if (r) return set_error("bad geometry description"), r;
  size_t off;
  *dev_bytes = geom_bytes(s, mmin, dims, &off);
  return PSM_OK;
}

int psm_voxelize_host(const double *verts, int64_t nv, const int32_t *tris, int64_t nt, int s,
                      const int32_t mmin[3], const int32_t dims[3], uint32_t *bits) {
  if (!verts || !tris || !mmin || !dims || !bits || nv <= 0 || nt <= 0 || s < 0 || s > 3)
    return set_error("psm_voxelize_host: bad arguments"), PSM_EINVAL;
  for (int64_t i = 0; i < 3 * nt; ++i)
    if (tris[i] < 0 || tris[i] >= nv) return set_error("triangle index out of range"), PSM_EINVAL;
  voxelize_rows(verts, tris, nt, s, mmin, dims, bits);
  return PSM_OK;
}

int psm_analytic_host(int kind, const double *params, int s, const int32_t mmin[3], const int32_t dims[3],
                      uint32_t *bits) {
  if (!params || !mmin || !dims || !bits || s < 0 || s > 3 || (kind != PSM_SHAPE_ELLIPSOID && kind != PSM_SHAPE_CUBE))
    return set_error("psm_analytic_host: bad arguments"), PSM_EINVAL;
  analytic_rows(kind, params, s, mmin, dims, bits);
  return PSM_OK;
}

static int geom_finish(psm_geom *g, void *dev, size_t bytes, hipStream_t st, psm_geom **out) {
  size_t coff;
  const size_t need = geom_bytes(g->s, g->mmin, g->dims, &coff);
  if (bytes < need) {
    delete[] g->host_bits;
    delete g;
    return set_error("geometry device buffer too small"), PSM_ESIZE;
  }
  int32_t cmin[3], cd[3];
  coarse_extent(g->s, g->mmin, g->dims, cmin, cd);
  const size_t nco = (size_t)cd[0] * cd[1] * cd[2];
  g->host_coarse = new (std::nothrow) uint8_t[nco];
  if (!g->host_coarse) {
    delete[] g->host_bits;
    delete g;
    return set_error("out of host memory"), PSM_EINVAL;
  }
  coarse_map(g->s, g->mmin, g->dims, g->host_bits, g->cmin, g->cdims, g->host_coarse);
  g->dev_bits = (uint32_t *)dev;
  g->dev_coarse = (uint8_t *)dev + coff;
  g->bytes = need;
  double rb = 0.0;
  const double h = ldexp(1.0, -g->s);
  for (int a = 0; a < 3; ++a) {
    const double m = std::max(fabs(g->mmin[a] * h), fabs((g->mmin[a] + g->dims[a]) * h));
    rb += m * m;
  }
  g->r_bound = sqrt(rb);
  const size_t wx = ((size_t)g->dims[0] + 31) / 32;
  hipError_t e = hipMemcpyAsync(g->dev_bits, g->host_bits, wx * g->dims[1] * g->dims[2] * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(g->dev_coarse, g->host_coarse, nco, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) {
    delete[] g->host_bits;
    delete[] g->host_coarse;
    delete g;
    return hip_fail(e, "geometry upload");
  }
  *out = g;
  return PSM_OK;
}

int geometry_field_create(const double *verts, int64_t nv, const int32_t *tris, int64_t nt, int s, void *dev,
                          size_t bytes, void *stream, psm_geom **out) {
  if (!out || !dev) return set_error("null argument"), PSM_EINVAL;
  psm_geom *g = new (std::nothrow) psm_geom;
  if (!g) return set_error("out of host memory"), PSM_EINVAL;
  memset(g, 0, sizeof(*g));
  g->s = s;
  size_t b;
  int r = psm_geometry_box(-1, nullptr, verts, nv, s, g->mmin, g->dims, &b);
  if (r) {
    delete g;
    return r;
  }
  g->wx = (g->dims[0] + 31) / 32;
  g->host_bits = new (std::nothrow) uint32_t[(size_t)g->wx * g->dims[1] * g->dims[2]];
  if (!g->host_bits) {
    delete g;
    return set_error("out of host memory"), PSM_EINVAL;
  }
  r = psm_voxelize_host(verts, nv, tris, nt, s, g->mmin, g->dims, g->host_bits);
  if (r) {
    delete[] g->host_bits;
    delete g;
    return r;
  }
  return geom_finish(g, dev, bytes, (hipStream_t)stream, out);
}

int geometry_field_create_analytic(int kind, const double *params, int s, void *dev, size_t bytes, void *stream,
                                   psm_geom **out) {
  if (!out || !dev || !params) return set_error("null argument"), PSM_EINVAL;
  psm_geom *g = new (std::nothrow) psm_geom;
  if (!g) return set_error("out of host memory"), PSM_EINVAL;
  memset(g, 0, sizeof(*g));
  g->s = s;
  size_t b;
  int r = psm_geometry_box(kind, params, nullptr, 0, s, g->mmin, g->dims, &b);
  if (r) {
    delete g;
    return r;
  }
  g->wx = (g->dims[0] + 31) / 32;
  g->host_bits = new (std::nothrow) uint32_t[(size_t)g->wx * g->dims[1] * g->dims[2]];
  if (!g->host_bits) {
    delete g;
    return set_error("out of host memory"), PSM_EINVAL;
  }
  analytic_rows(kind, params, s, g->mmin, g->dims, g->host_bits);
  return geom_finish(g, dev, bytes, (hipStream_t)stream, out);
}

int geometry_field_destroy(psm_geom *g) {
  if (!g) return set_error("null handle"), PSM_EINVAL;
  delete[] g->host_bits;
  delete[] g->host_coarse;
  delete g;
  return PSM_OK;
}

// ---- per-step path -----------------------------------------------------------
static int check_bodies(const psm_field *f, const psm_body *bodies, int nb) {
  if (!f) return set_error("null handle"), PSM_EINVAL;
  if (int r = work_usable(f)) return r;
  if (nb < 0 || nb > f->cfg.max_bodies) return set_error("n_bodies exceeds max_bodies"), PSM_EINVAL;
  if (nb > 0 && !bodies) return set_error("null bodies"), PSM_EINVAL;
  for (int b = 0; b < nb; ++b)
    for (int i = 0; i < 9; ++i)
      if (!isfinite(bodies[b].R[i])) return set_error("non-finite pose"), PSM_EINVAL;
  return PSM_OK;
}

// Host side of the mapping: the swept region of every body at its pose (a
// cell [i, i+1] meets [lo, hi] iff floor(lo) <= i < hi; one cell of margin)
// and the kernel arguments.
struct MapPlan {
  MapArgs a;
  uint32_t maxcells;
  IBox now[PSM_MAX_BODIES];
  int nb;
};

static int map_plan(psm_field *f, const psm_body *bodies, const psm_geom *const *geoms, int nb, MapPlan &P) {
  int r = check_bodies(f, bodies, nb);
  if (r) return r;
  if (!f->cfg.psm) return set_error("geometry_map_step on a plain-LBM field"), PSM_EINVAL;
  if (nb > 0 && !geoms) return set_error("null geometry list"), PSM_EINVAL;
  if (f->nb_mapped && nb != f->nb_mapped)
    return set_error("the number of bodies changed; reset the field first"), PSM_EINVAL;
  MapArgs &a = P.a;
  memset(&a, 0, sizeof(a));
  a.list = f->map_list_cap > 0 ? f->map_list : nullptr;
  a.count = f->map_count + (size_t)f->map_parity * PSM_MAX_BODIES;
  a.count_next = f->map_count + (size_t)(f->map_parity ^ 1) * PSM_MAX_BODIES;
  a.cap = (uint32_t)f->map_list_cap;
  a.B0 = f->B0;
  a.B1 = f->B1;
  a.meta = f->meta;
  a.err = f->err;
  a.nx = f->cfg.nx;
  a.ny = f->cfg.ny;
  a.nz = f->cfg.nz;
  a.nb = nb;
  a.slots = f->cfg.slots;
  a.b_form = f->cfg.b_form;
  a.tau = f->cfg.tau;
  uint32_t maxcells = 0;
  IBox *now = P.now;
  const int n3[3] = {f->cfg.nx, f->cfg.ny, f->cfg.nz};
  for (int b = 0; b < nb; ++b) {
    const psm_geom *g = geoms[b];
    if (!g) return set_error("null geometry"), PSM_EINVAL;
    MapBodyK &m = a.body[b];
    memcpy(m.R, bodies[b].R, sizeof(m.R));
    memcpy(m.X, bodies[b].X, sizeof(m.X));
    m.bits = g->dev_bits;
    m.coarse = g->dev_coarse;
    m.s = g->s;
    m.block = (f->cfg.map_reading == PSM_MAP_BLOCK && g->s >= 1) ? 1 : 0;
    m.wx = g->wx;
    for (int d = 0; d < 3; ++d) {
      m.mmin[d] = g->mmin[d];
      m.dims[d] = g->dims[d];
      m.cmin[d] = g->cmin[d];
      m.cdims[d] = g->cdims[d];
      // |(R^T delta)_d| <= sum_j |R_jd| (1 - h)/2; plus two fixed-point units
      const double sum = fabs(m.R[d]) + fabs(m.R[3 + d]) + fabs(m.R[6 + d]);
      m.dabs[d] = (long long)ceil(sum * (1.0 - ldexp(1.0, -g->s)) * 0.5 * ldexp(1.0, g->s + 32)) + 2;
    }
    // cells the body can touch at this pose: lab AABB of the rotated
    // geometry box (a cell [i, i+1] meets [lo, hi] iff floor(lo) <= i < hi),
    // one cell of margin; two below and one above for the block reading,
    // whose block reaches 1/2 + h/2 <= 3/4 per body axis from the centre
    // (<= 3/4 sqrt(3) in the lab)
    double blo[3], bhi[3];
    {
      const double h = ldexp(1.0, -g->s);
      for (int d = 0; d < 3; ++d) {
        blo[d] = 1e300;
        bhi[d] = -1e300;
      }
      for (int c = 0; c < 8; ++c) {
        double p[3];
        for (int d = 0; d < 3; ++d) p[d] = (((c >> d) & 1) ? (double)(g->mmin[d] + g->dims[d]) : (double)g->mmin[d]) * h;
        for (int d = 0; d < 3; ++d) {
          const double v = m.R[3 * d] * p[0] + m.R[3 * d + 1] * p[1] + m.R[3 * d + 2] * p[2] + m.X[d];
          blo[d] = std::min(blo[d], v);
          bhi[d] = std::max(bhi[d], v);
        }
      }
    }
    IBox A;
    bool empty = false;
    for (int d = 0; d < 3; ++d) {
      const double lo = floor(blo[d]) - (m.block ? 2.0 : 1.0), hi = ceil(bhi[d]) + (m.block ? 1.0 : 0.0);
      A.lo[d] = (int)std::max(0.0, std::min((double)n3[d], lo));
      A.hi[d] = (int)std::min((double)n3[d] - 1, std::max(-1.0, hi));
      if (A.hi[d] < A.lo[d]) empty = true;
    }
    if (empty) A = empty_box();
    now[b] = A;
    m.active = A;
    m.region = f->have_prev[b] ? box_union(A, f->active[b]) : A;
    if (box_empty(m.region)) {
      m.region_cells = 0;
    } else {
      const uint64_t cells = (uint64_t)(m.region.hi[0] - m.region.lo[0] + 1) *
                             (uint64_t)(m.region.hi[1] - m.region.lo[1] + 1) *
                             (uint64_t)(m.region.hi[2] - m.region.lo[2] + 1);
      if (cells >= (1ull << 32) - 256) return set_error("swept box too large"), PSM_EUNSUP;
      m.region_cells = (uint32_t)cells;
    }
    maxcells = std::max(maxcells, m.region_cells);
  }
  P.maxcells = maxcells;
  P.nb = nb;
  // the surface-cell list serves s = 3 bodies only
  bool any3 = false;
  for (int b = 0; b < nb; ++b) any3 = any3 || (geoms[b]->s == 3 && !a.body[b].block);
  if (!any3) a.list = nullptr;
  return PSM_OK;
}

static void map_commit(psm_field *f, const MapPlan &P) {
  if (P.a.list && P.maxcells > 0 && P.nb > 0) f->map_parity ^= 1;  // one counter set used, the other cleared
  for (int b = 0; b < P.nb; ++b) {
    f->active[b] = P.now[b];
    f->have_prev[b] = true;
  }
  f->nb_mapped = P.nb;
}

// Host side of a stream-collide step: per-body kinematics, the boxes outside
// which B is zero and the solid kernel's chunk offsets over them.
static int sc_plan(psm_field *f, const psm_body *bodies, int nb, int64_t step, const IBox *boxes, SCArgs &a) {
  int r = check_bodies(f, bodies, nb);
  if (r) return r;
  if (step < 0) return set_error("negative step"), PSM_EINVAL;
  a = make_sc_args(*f);
  a.nb = f->cfg.psm ? nb : 0;
  uint32_t chunks = 0;
  for (int b = 0; b < a.nb; ++b) {
    BodyK &k = a.body[b];
    for (int d = 0; d < 3; ++d) {
      k.X[d] = bodies[b].X[d];
      k.V[d] = bodies[b].V[d];
      k.W[d] = bodies[b].W[d];
    }
    // B is zero outside the mapped boxes; the solid kernel walks them
    const IBox &B = boxes[b];
    a.box[b] = B;
    a.cprefix[b] = chunks;
    if (!box_empty(B)) {
      const uint64_t cells = (uint64_t)(B.hi[0] - B.lo[0] + 1) * (uint64_t)(B.hi[1] - B.lo[1] + 1) *
                             (uint64_t)(B.hi[2] - B.lo[2] + 1);
      chunks += (uint32_t)((cells + 255) / 256);
    }
  }
  a.nbox = a.nb;
  a.cprefix[a.nb] = chunks;
  a.nchunks = chunks;
  if (f->opt_whole_domain && a.nb > 0) {
    // the offset field can make B nonzero anywhere: one box, the whole domain
    IBox W;
    W.lo[0] = W.lo[1] = W.lo[2] = 0;
    W.hi[0] = f->cfg.nx - 1;
    W.hi[1] = f->cfg.ny - 1;
    W.hi[2] = f->cfg.nz - 1;
    a.box[0] = W;
    for (int b = 1; b < a.nb; ++b) a.box[b] = empty_box();
    a.cprefix[0] = 0;
    const uint32_t whole = (uint32_t)((f->N + 255) / 256);
    for (int b = 1; b <= a.nb; ++b) a.cprefix[b] = whole;
    a.nchunks = whole;
  }
  // chunks per workgroup group: enough groups for the fixed grid, at most
  // SOLID_MAX_CPW chunks listed at once
  const uint32_t grid = (uint32_t)a.solid_grid;
  a.cpw = (int)std::min<uint32_t>((uint32_t)SOLID_MAX_CPW, std::max<uint32_t>(1u, (a.nchunks + grid - 1) / grid));
  a.xcd_remap = f->opt_xcd_remap;
  return PSM_OK;
}

// ft_done (may be null): set when the step's launches also summed the F/T
// into a.ft_out.  ss: stream of the solid-cell and face-row launches.
static int sc_launch(psm_field *f, const SCArgs &a, int64_t step, hipStream_t st, hipStream_t ss,
                     int *ft_done = nullptr) {
  const int parity = (int)(step & 1);
  hipError_t e;
  int sb = 0, fd = 0;
  switch (f->cfg.storage) {
    case PSM_F64: e = launch_sc_f64(f->cfg, a, parity, st, ss, &sb, &fd); break;
    case PSM_F32: e = launch_sc_f32(f->cfg, a, parity, st, ss, &sb, &fd); break;
    default: e = launch_sc_f16(f->cfg, a, parity, st, ss, &sb, &fd); break;
  }
  if (e != hipSuccess) return hip_fail(e, "psm_stream_collide launch");
  f->solid_blocks = sb;
  if (ft_done) *ft_done = fd;
  return PSM_OK;
}

int geometry_map_step(psm_field *f, const psm_body *bodies, const psm_geom *const *geoms, int nb, void *stream) {
  MapPlan P;
  int r = map_plan(f, bodies, geoms, nb, P);
  if (r) return r;
  f->ahead_valid = false;
  hipError_t e = launch_map(P.a, P.maxcells, 0, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "geometry_map_step launch");
  map_commit(f, P);
  return PSM_OK;
}

// ft_dev (may be null): the F/T of the step too, summed by an extra workgroup
// of the interior launch, else by the separate reduction kernel.  With the
// field's second stream (PSM_OPT_CONCURRENT, steps with a face-row launch)
// the solid-cell launch, the F/T sum and the face-row launch run there, beside
// the interior launch on the caller's stream, which then waits for them.
static int stream_collide(psm_field *f, const psm_body *bodies, int nb, int64_t step, void *stream,
                          double *ft_dev) {
  if (!f) return set_error("null handle"), PSM_EINVAL;
  if (f->cfg.psm && nb > 0 && nb != f->nb_mapped)
    return set_error("psm_stream_collide: bodies do not match the mapped field"), PSM_EINVAL;
  SCArgs a;
  int r = sc_plan(f, bodies, nb, step, f->active, a);
  if (r) return r;
  hipStream_t st = (hipStream_t)stream;
  // the second stream pays for its two cross-stream waits only where the step
  // has a face-row launch to move off the critical path (odd steps, D3Q27);
  // even D3Q19 steps take their face rows as extra blocks of the interior launch
  const bool edge_launch = a.ntiles_e > 0 && !((step & 1) == 0 && f->cfg.q == 19);
  const bool conc = f->side && f->opt_concurrent && !a.general && edge_launch;
  if (conc) {
    hipError_t e = hipEventRecord(f->ev_fork, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(f->side, f->ev_fork, 0);
    if (e != hipSuccess) return hip_fail(e, "psm_stream_collide: fork");
  }
  a.ft_out = (!conc && ft_dev && a.nb > 0) ? ft_dev : nullptr;
  int done = 0;
  r = sc_launch(f, a, step, st, conc ? f->side : st, &done);
  if (conc) {
    if (!r && ft_dev) r = body_force_torque(f, nb, ft_dev, f->side);
    // join even after a failed launch, so that no work stays behind on the side stream
    hipError_t e = hipEventRecord(f->ev_join, f->side);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, f->ev_join, 0);
    if (!r && e != hipSuccess) r = hip_fail(e, "psm_stream_collide: join");
  } else if (!r && ft_dev && !done) {
    r = body_force_torque(f, nb, ft_dev, stream);
  }
  return r;
}

int psm_stream_collide(psm_field *f, const psm_body *bodies, int nb, int64_t step, void *stream) {
  return stream_collide(f, bodies, nb, step, stream, nullptr);
}

int psm_step(psm_field *f, const psm_body *map_poses, const psm_body *bodies, const psm_geom *const *geoms, int nb,
             int64_t step, double *ft_dev, void *stream) {
  if (!f) return set_error("null handle"), PSM_EINVAL;
  if (!f->cfg.psm || nb == 0) {
    if (ft_dev) return set_error("psm_step: force/torque needs bodies"), PSM_EINVAL;
    return psm_stream_collide(f, bodies, nb, step, stream);
  }
  if (!map_poses) map_poses = bodies;
  int r = geometry_map_step(f, map_poses, geoms, nb, stream);
  if (!r) r = stream_collide(f, bodies, nb, step, stream, ft_dev);
  return r;
}

// Exchange the current set of fractions (and its mapping state) with the other.
static void swap_fraction_sets(psm_field *f) {
  std::swap(f->B0, f->B0x);
  std::swap(f->B1, f->B1x);
  std::swap(f->meta, f->metax);
  for (int b = 0; b < PSM_MAX_BODIES; ++b) {
    std::swap(f->active[b], f->activex[b]);
    std::swap(f->have_prev[b], f->have_prevx[b]);
  }
  std::swap(f->nb_mapped, f->nb_mappedx);
}

int psm_step_ahead(psm_field *f, const psm_body *map_poses, const psm_body *bodies, const psm_body *next_map_poses,
                   const psm_geom *const *geoms, int nb, int64_t step, double *ft_dev, void *stream) {
  if (!f) return set_error("null handle"), PSM_EINVAL;
  if (!f->cfg.map_ahead) return set_error("psm_step_ahead needs a field made with map_ahead = 1"), PSM_EUNSUP;
  if (nb == 0) return psm_step(f, map_poses, bodies, geoms, nb, step, ft_dev, stream);
  if (!next_map_poses) return set_error("null next_map_poses"), PSM_EINVAL;
  if (int r = check_bodies(f, next_map_poses, nb)) return r;
  if (!map_poses) map_poses = bodies;
  hipStream_t st = (hipStream_t)stream;
  // this step's fractions: mapped by the previous call, else now
  int r = PSM_OK;
  if (f->ahead_valid && f->ahead_step == step && f->ahead_nb == nb) {
    swap_fraction_sets(f);
  } else {
    r = geometry_map_step(f, map_poses, geoms, nb, stream);
    if (r) return r;
  }
  f->ahead_valid = false;
  // the next step's mapping, planned on the host for the other set
  MapPlan P;
  swap_fraction_sets(f);
  r = map_plan(f, next_map_poses, geoms, nb, P);
  swap_fraction_sets(f);
  if (r) return r;
  // the mapping stream starts after everything before this point on `stream`
  // (every earlier read of the other set included) and runs beside this
  // step's launches (starting it after the solid-cell launch measured 0.7%
  // slower on the rotor box)
  hipStream_t ms = f->mstream ? f->mstream : st;
  hipError_t e = f->mstream ? hipEventRecord(f->ev_mfork, st) : hipSuccess;
  if (e != hipSuccess) return hip_fail(e, "psm_step_ahead: fork");
  r = stream_collide(f, bodies, nb, step, stream, ft_dev);
  if (r) return r;
  if (f->mstream) e = hipStreamWaitEvent(ms, f->ev_mfork, 0);
  if (e == hipSuccess) e = launch_map(P.a, P.maxcells, 0, ms);
  if (e == hipSuccess) {
    swap_fraction_sets(f);
    map_commit(f, P);
    swap_fraction_sets(f);
  } else {
    r = hip_fail(e, "psm_step_ahead: mapping launch");
  }
  if (f->mstream) {
    e = hipEventRecord(f->ev_mjoin, ms);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, f->ev_mjoin, 0);
    if (!r && e != hipSuccess) r = hip_fail(e, "psm_step_ahead: join");
  }
  if (!r) {
    f->ahead_valid = true;
    f->ahead_step = step + 1;
    f->ahead_nb = nb;
  }
  return r;
}

int psm_fractions(psm_field *f, const float **b0, const float **b1, const uint8_t **meta) {
  if (!f) return set_error("null handle"), PSM_EINVAL;
  if (b0) *b0 = f->B0;
  if (b1) *b1 = f->B1;
  if (meta) *meta = f->meta;
  return PSM_OK;
}

int psm_rigid_body(const psm_rigid *s, psm_body *out) {
  if (!s || !out) return set_error("psm_rigid_body: null argument"), PSM_EINVAL;
  for (int i = 0; i < 9; ++i) out->R[i] = s->R[i];
  for (int d = 0; d < 3; ++d) {
    out->X[d] = s->X[d];
    out->V[d] = s->V[d];
    out->W[d] = s->W[d];
  }
  return PSM_OK;
}

int psm_rigid_advance(psm_rigid *s, const double ft_step[6], double dt) {
  if (!s || !ft_step) return set_error("psm_rigid_advance: null argument"), PSM_EINVAL;
  if (!(s->m > 0.0) || !(s->I[0] > 0.0) || !(s->I[1] > 0.0) || !(s->I[2] > 0.0) || !isfinite(dt))
    return set_error("psm_rigid_advance: mass and moments of inertia must be positive, dt finite"), PSM_EINVAL;
  double ft[6];
  for (int i = 0; i < 6; ++i) {
    ft[i] = s->average ? 0.5 * (ft_step[i] + s->ft_prev[i]) : ft_step[i];
    s->ft_prev[i] = ft_step[i];
  }
  // translation
  for (int d = 0; d < 3; ++d) {
    s->V[d] += dt * ((ft[d] + s->F_ext[d]) / s->m);
    s->X[d] += dt * s->V[d];
  }
  // rotation: body-frame components through R^T, inertia diagonal there
  const double *R = s->R;
  double wb[3], lb[3], L[3];
  for (int i = 0; i < 3; ++i) wb[i] = R[i] * s->W[0] + R[3 + i] * s->W[1] + R[6 + i] * s->W[2];
  for (int i = 0; i < 3; ++i) lb[i] = s->I[i] * wb[i];
  for (int i = 0; i < 3; ++i) L[i] = R[3 * i] * lb[0] + R[3 * i + 1] * lb[1] + R[3 * i + 2] * lb[2];
  const double rhs[3] = {ft[3] - (s->W[1] * L[2] - s->W[2] * L[1]), ft[4] - (s->W[2] * L[0] - s->W[0] * L[2]),
                         ft[5] - (s->W[0] * L[1] - s->W[1] * L[0])};
  double ab[3];
  for (int i = 0; i < 3; ++i) ab[i] = (R[i] * rhs[0] + R[3 + i] * rhs[1] + R[6 + i] * rhs[2]) / s->I[i];
  for (int i = 0; i < 3; ++i) s->W[i] += dt * (R[3 * i] * ab[0] + R[3 * i + 1] * ab[1] + R[3 * i + 2] * ab[2]);
  // orientation: rotate by the angle dt |W| about W
  const double om[3] = {dt * s->W[0], dt * s->W[1], dt * s->W[2]};
  const double th = sqrt(om[0] * om[0] + om[1] * om[1] + om[2] * om[2]);
  if (th > 0.0) {
    const double a[3] = {om[0] / th, om[1] / th, om[2] / th};
    const double c = cos(th), sn = sin(th), omc = 1.0 - c;
    const double K[9] = {0.0, -a[2], a[1], a[2], 0.0, -a[0], -a[1], a[0], 0.0};
    double Q[9], Rn[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Q[3 * i + j] = ((i == j ? c : 0.0) + (omc * a[i]) * a[j]) + sn * K[3 * i + j];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Rn[3 * i + j] = Q[3 * i] * R[j] + Q[3 * i + 1] * R[3 + j] + Q[3 * i + 2] * R[6 + j];
    for (int i = 0; i < 9; ++i) s->R[i] = Rn[i];
  }
  return PSM_OK;
}

int psm_coupled_step(psm_field *f, psm_rigid *states, const psm_geom *const *geoms, int nb, int64_t step,
                     double *ft_dev, double *ft_host, void *stream) {
  if (!f || !states || !geoms || !ft_dev || !ft_host) return set_error("psm_coupled_step: null argument"), PSM_EINVAL;
  if (nb < 1 || nb > PSM_MAX_BODIES) return set_error("psm_coupled_step: 1 .. PSM_MAX_BODIES bodies"), PSM_EINVAL;
  psm_body P[PSM_MAX_BODIES];
  for (int b = 0; b < nb; ++b) psm_rigid_body(&states[b], &P[b]);
  int r = psm_step(f, P, P, geoms, nb, step, ft_dev, stream);
  if (r) return r;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(ft_host, ft_dev, (size_t)nb * 6 * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "psm_coupled_step force/torque read-back");
  for (int b = 0; b < nb; ++b) {
    r = psm_rigid_advance(&states[b], ft_host + 6 * b, 1.0);
    if (r) return r;
  }
  return PSM_OK;
}

int body_force_torque(psm_field *f, int nb, double *ft, void *stream) {
  if (!f || !ft) return set_error("null argument"), PSM_EINVAL;
  if (!f->cfg.psm) return set_error("body_force_torque on a plain-LBM field"), PSM_EINVAL;
  if (int r = work_usable(f)) return r;
  if (nb < 1 || nb > f->nb_mapped) return set_error("n_bodies does not match the mapped bodies"), PSM_EINVAL;
  hipError_t e = launch_ft_reduce(*f, nb, ft, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "body_force_torque launch");
  return PSM_OK;
}

int psm_mass_fp64(psm_field *f, int64_t step, double *out, void *stream) {
  if (!f || !out) return set_error("null argument"), PSM_EINVAL;
  if (int r = work_usable(f)) return r;
  hipError_t e = launch_macro(*f, (int)(step & 1), nullptr, nullptr, f->red, 0, (hipStream_t)stream);
  if (e == hipSuccess) e = launch_mass_final(f->red, f->red_count, out, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "psm_mass_fp64 launch");
  return PSM_OK;
}

int psm_macroscopic(psm_field *f, int64_t step, double *rho, double *u, void *stream) {
  if (!f || !rho || !u) return set_error("null argument"), PSM_EINVAL;
  if (int r = work_usable(f)) return r;
  hipError_t e = launch_macro(*f, (int)(step & 1), rho, u, f->red, 1, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "psm_macroscopic launch");
  return PSM_OK;
}

int psm_set_option(psm_field *f, int option, int value) {
  if (!f) return set_error("null handle"), PSM_EINVAL;
  switch (option) {
    case PSM_OPT_GENERAL_PATH: f->opt_general_path = value ? 1 : 0; return PSM_OK;
    case PSM_OPT_XCD_REMAP: f->opt_xcd_remap = value ? 1 : 0; return PSM_OK;
    case PSM_OPT_CONCURRENT: f->opt_concurrent = value ? 1 : 0; return PSM_OK;
    case PSM_OPT_SOLID_GRID:
      if (value < 0 || value > SOLID_BLOCKS) return set_error("PSM_OPT_SOLID_GRID takes 0 .. 4096"), PSM_EINVAL;
      f->opt_solid_grid = value ? value : SOLID_BLOCKS;
      return PSM_OK;
    case PSM_OPT_MAP_LIST:
      if (value < 0 || value > f->map_list_max)
        return set_error("PSM_OPT_MAP_LIST takes 0 .. the list capacity"), PSM_EINVAL;
      f->map_list_cap = value;
      return PSM_OK;
  }
  return set_error("unknown option"), PSM_EINVAL;
}

int psm_set_fraction_offset(psm_field *f, const float *dB) {
  if (!f) return set_error("null handle"), PSM_EINVAL;
  if (!f->cfg.psm) return set_error("fraction offset on a plain-LBM field"), PSM_EINVAL;
  if (((uintptr_t)dB) & 3u) return set_error("offset field must be 4-byte aligned"), PSM_EINVAL;
  f->dB = dB;
  f->opt_whole_domain = dB != nullptr;
  return PSM_OK;
}

int lbm_set_obstacle(psm_field *f, const uint8_t *solid_dev, void *obst_dev, size_t obst_bytes, int64_t *n_near,
                     void *stream) {
  if (!f) return set_error("null handle"), PSM_EINVAL;
  f->ocls = nullptr;
  f->olist = nullptr;
  f->ocount = 0;
  f->obox = empty_box();
  if (n_near) *n_near = 0;
  if (!solid_dev) return PSM_OK;
  if (f->cfg.psm) return set_error("a static obstacle needs a plain-LBM field (psm = 0)"), PSM_EUNSUP;
  if (!obst_dev) return set_error("null obstacle buffer"), PSM_EINVAL;
  if (((uintptr_t)obst_dev) & 255u) return set_error("obstacle buffer must be 256-byte aligned"), PSM_EINVAL;
  const size_t off = obst_list_offset(f->N);
  if (obst_bytes < off) return set_error("obstacle buffer smaller than its header and class map"), PSM_ESIZE;
  const size_t cap64 = (obst_bytes - off) / 8;
  const uint32_t cap = (uint32_t)std::min<size_t>(cap64, (size_t)f->N);
  char *base = (char *)obst_dev;
  ObstHdr *h = (ObstHdr *)base;
  uint8_t *cls = (uint8_t *)(base + 256);
  uint32_t *list = (uint32_t *)(base + off);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = launch_obst_build(*f, solid_dev, cls, list, cap, h, st);
  if (e != hipSuccess) return hip_fail(e, "lbm_set_obstacle build");
  ObstHdr hh;
  e = hipMemcpyAsync(&hh, h, sizeof(hh), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "lbm_set_obstacle read-back");
  if (n_near) *n_near = hh.count;
  if (hh.count > cap)
    return set_error("obstacle list needs " + std::to_string(hh.count) + " entries, the buffer holds " +
                     std::to_string(cap)),
           PSM_ESIZE;
  if (hh.count > 1) {
    // the kernel appends in arrival order: sort by cell index once, so that
    // neighbouring lanes of the list kernel update neighbouring cells
    std::vector<uint64_t> v((size_t)hh.count);
    e = hipMemcpyAsync(v.data(), list, v.size() * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "lbm_set_obstacle list read-back");
    for (uint64_t &x : v) x = (x << 32) | (x >> 32);  // (cell, mask) pairs -> key cell
    std::sort(v.begin(), v.end());
    for (uint64_t &x : v) x = (x << 32) | (x >> 32);
    e = hipMemcpyAsync(list, v.data(), v.size() * 8, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "lbm_set_obstacle list upload");
  }
  f->ocls = cls;
  f->olist = list;
  f->ocount = hh.count;
  for (int d = 0; d < 3; ++d) {
    f->obox.lo[d] = hh.lo[d];
    f->obox.hi[d] = hh.hi[d];
  }
  return PSM_OK;
}

int psm_adjoint_step(psm_field *f, const void *fwd, int64_t step, const void *ain, void *aout, void *dJdB,
                     const psm_body *body, const double axis[3], double wt, void *stream) {
  if (!f || !fwd || !ain || !aout || !dJdB || !body || !axis) return set_error("null argument"), PSM_EINVAL;
  if (int r = work_usable(f)) return r;
  if (step < 0) return set_error("negative step"), PSM_EINVAL;
  if (!f->cfg.psm || f->cfg.sc != 1 || f->cfg.slots != 1 || f->cfg.collision != PSM_COLL_TRT)
    return set_error("psm_adjoint_step supports PSM fields with TRT, SC1 and one body slot"), PSM_EUNSUP;
  if (f->nb_mapped != 1) return set_error("psm_adjoint_step needs the single body mapped for this step"), PSM_EINVAL;
  if (ain == aout) return set_error("adjoint input and output must differ"), PSM_EINVAL;
  const double an = axis[0] * axis[0] + axis[1] * axis[1] + axis[2] * axis[2];
  if (!(fabs(an - 1.0) < 1e-12) || !isfinite(wt)) return set_error("axis must be a unit vector, wt finite"), PSM_EINVAL;
  AdjArgs A;
  memset(&A, 0, sizeof(A));
  A.s = make_sc_args(*f);
  A.fwd = (const char *)fwd;
  A.parity = (int)(step & 1);
  size_t pb = 0, ab = 0;
  psm_required_bytes(&f->cfg, PSM_BUF_PDF, &pb);
  psm_required_bytes(&f->cfg, PSM_BUF_ADJOINT, &ab);
  A.o32 = pb < (1ull << 32) && ab < (1ull << 32);
  A.ain = ain;
  A.aout = aout;
  A.dJdB = dJdB;
  for (int d = 0; d < 3; ++d) {
    A.X[d] = body->X[d];
    A.V[d] = body->V[d];
    A.W[d] = body->W[d];
    A.axis[d] = axis[d];
  }
  A.wt = wt;
  A.part = f->red;
  hipError_t e = launch_adjoint(*f, A, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "psm_adjoint_step launch");
  return PSM_OK;
}

int psm_adjoint_omega(psm_field *f, double *out, void *stream) {
  if (!f || !out) return set_error("null argument"), PSM_EINVAL;
  if (int r = work_usable(f)) return r;
  hipError_t e = launch_sum_accumulate(f->red, adjoint_blocks(f->cfg.nx, f->cfg.ny, f->cfg.nz), out,
                                       (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "psm_adjoint_omega launch");
  return PSM_OK;
}

// `lay` (a buffer in the PDF buffer's layout, `lay_bytes` long) to or from the
// standard [q][N] array `std_arr`, elements of sz bytes
static int layout_convert(psm_field *f, void *lay, size_t lay_bytes, void *std_arr, int to_std, size_t sz,
                          void *stream) {
  const size_t bytes = (size_t)f->cfg.q * (size_t)f->N * sz;
  const char *p = (const char *)lay, *o = (const char *)std_arr;
  if (o < p + lay_bytes && p < o + bytes) return set_error("the standard-layout array overlaps the buffer"), PSM_EINVAL;
  hipError_t e = to_std ? launch_pdf_gather(*f, std_arr, lay, 1, sz, (hipStream_t)stream)
                        : launch_pdf_gather(*f, lay, std_arr, 0, sz, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "layout conversion launch");
  return PSM_OK;
}

static int pdf_convert(psm_field *f, void *dst, const void *src, int to_std, void *stream) {
  if (!f || !dst || !src) return set_error("null argument"), PSM_EINVAL;
  size_t pb;
  psm_required_bytes(&f->cfg, PSM_BUF_PDF, &pb);
  return layout_convert(f, f->pdf, pb, to_std ? dst : const_cast<void *>(src), to_std, storage_size(f->cfg.storage),
                        stream);
}

int psm_adjoint_gather(psm_field *f, const void *adj, void *dst, void *stream) {
  if (!f || !adj || !dst) return set_error("null argument"), PSM_EINVAL;
  size_t ab;
  psm_required_bytes(&f->cfg, PSM_BUF_ADJOINT, &ab);
  return layout_convert(f, const_cast<void *>(adj), ab, dst, 1, adjoint_elem_size(f->cfg), stream);
}

int psm_pdf_gather(psm_field *f, void *dst, void *stream) {
  return pdf_convert(f, dst, f ? f->pdf : nullptr, 1, stream);
}

int psm_pdf_scatter(psm_field *f, const void *src, void *stream) {
  return pdf_convert(f, f ? f->pdf : nullptr, src, 0, stream);
}

int psm_error_flags(psm_field *f, int32_t *out, void *stream) {
  if (!f || !out) return set_error("null argument"), PSM_EINVAL;
  if (int r = work_usable(f)) return r;
  hipError_t e = launch_flags_copy(f->err, out, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "psm_error_flags launch");
  return PSM_OK;
}

int psm_stream_copy(const void *src, void *dst, size_t bytes, void *stream) {
  if (!src || !dst) return set_error("null argument"), PSM_EINVAL;
  if (((uintptr_t)src | (uintptr_t)dst) & 15u) return set_error("copy buffers must be 16-byte aligned"), PSM_EINVAL;
  hipError_t e = launch_copy(src, dst, bytes, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "psm_stream_copy launch");
  return PSM_OK;
}

}  // extern "C"
