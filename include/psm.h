/*
 * psm.h -- C ABI of the MI355X (gfx950) PSM hot path.
 *
 * Method: lattice Boltzmann with the Partially Saturated Cells method (PSM)
 * for complex moving geometries, after Suffa, Kemmler, Koestler, Ruede,
 * "Large-Scale Simulations of Fully Resolved Complex Moving Geometries with
 * Partially Saturated Cells" (arXiv 2502.20049).
 *
 * One time step of the hot path is, on the caller's HIP stream:
 *   geometry_map_step   solid fractions B(x,t) from body-frame geometry fields
 *                       under each body's current rotation/translation (sec. III)
 *   psm_stream_collide  fused in-place (AA pattern) stream + TRT (or cumulant) collision
 *                       blended with the solid collision, eq. (4), summed over
 *                       up to two overlapping bodies per cell; writes per-tile
 *                       force/torque partials (eqs. (10)-(11))
 *   body_force_torque   FP64 fixed-order sum of those partials per body
 *
 * Conventions shared by every entry point
 *   - Memory ownership: every device buffer is allocated and freed by the
 *     caller (e.g. torch tensors) and passed as pointer + byte count.  Handles
 *     own host-side metadata only.  No per-step call allocates anything.
 *   - Streams: `stream` is a hipStream_t (NULL = default stream).  Calls are
 *     asynchronous on it; results are valid after the stream is synchronised.
 *   - Errors: 0 on success, a negative PSM_E* code otherwise; psm_last_error()
 *     returns a thread-local message for the last failure.  Kernel launch
 *     failures are reported as PSM_EHIP.  No C++ exception crosses the ABI.
 *   - Lattice units: dx = dt = 1, rest density 1, cell (i,j,k) has its centre
 *     at (i+1/2, j+1/2, k+1/2).  Linear cell index n = x + nx*(y + ny*z).
 *   - PDF layout: structure of arrays, slot (k, n) at element k*S + n (N =
 *     nx*ny*nz cells, x fastest; S = psm_pdf_stride() >= N, the direction
 *     arrays padded apart).  Stored values are deviations
 *     delta f_k = f_k - w_k from the lattice weights, in the storage type.
 *     Direction order is this library's own (psm_lattice()).  The in-place
 *     AA pattern leaves the buffer in the standard layout (slot (k,n) holds
 *     f_k at cell n) after every even number of steps; psm_macroscopic and
 *     psm_mass_fp64 read either parity.
 */
#ifndef PSM_H
#define PSM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes --------------------------------------------------------- */
#define PSM_OK 0
#define PSM_EINVAL (-1)  /* invalid argument (null handle, bad enum, bad size) */
#define PSM_ESIZE (-2)   /* a caller buffer is smaller than required         */
#define PSM_EUNSUP (-3)  /* valid but unsupported request                    */
#define PSM_EHIP (-4)    /* HIP runtime / launch failure                      */

/* ---- enums --------------------------------------------------------------- */
enum { PSM_F64 = 0, PSM_F32 = 1, PSM_F16 = 2 };                 /* PDF storage */
enum { PSM_PERIODIC = 0, PSM_WALL = 1, PSM_INLET = 2, PSM_OUTLET = 3 }; /* faces */
enum { PSM_BUF_PDF = 0, PSM_BUF_B = 1, PSM_BUF_WORK = 2, PSM_BUF_ADJOINT = 3, PSM_BUF_GRAD_B = 4,
       PSM_BUF_OBSTACLE = 5 };
enum { PSM_SHAPE_ELLIPSOID = 0, PSM_SHAPE_CUBE = 1 };
enum { PSM_COLL_TRT = 0, PSM_COLL_CUMULANT = 1 };               /* fluid collision */
enum { PSM_MAP_SUBSAMPLES = 0, PSM_MAP_BLOCK = 1 };             /* mapping reading */
enum { PSM_LAYOUT_SOA = 0, PSM_LAYOUT_BLOCKED = 1 };            /* PDF buffer layout */
#define PSM_MAX_BODIES 8

/* Simulation configuration (section II.A; readings of unstated details in the
 * design notes).
 *   q        19 (D3Q19) or 27 (D3Q27)
 *   storage  PSM_F64 (FP64 arithmetic) / PSM_F32 / PSM_F16 (FP32 arithmetic)
 *   psm      1: PSM blend of eq. (4); 0: plain LBM (no B access at all)
 *   sc       solid collision operator 1, 2 or 3 (eqs. (7)-(9))
 *   b_form   0: B = eps (eq. (5)); 1: tau-weighted B (eq. (6))
 *   slots    body slots per cell, 1 or 2 (sum over overlapping bodies)
 *   max_bodies  1..PSM_MAX_BODIES (sizes the force/torque partials)
 *   bc       face kinds for -x,+x,-y,+y,-z,+z: PSM_PERIODIC (both faces of
 *            an axis), PSM_WALL (halfway bounce-back), PSM_INLET (moving-wall
 *            bounce-back with u_in, rest density 1), PSM_OUTLET (zero
 *            gradient: an incoming PDF equals the cell's own post-collision
 *            PDF of the same direction).  Precedence wall > inlet > outlet.
 *   tau      relaxation time of the even (viscous) moments, > 1/2
 *   magic    TRT parameter Lambda; odd rate 1/(1/2 + Lambda/(tau - 1/2))
 *   force    body-force density (Guo forcing, part of the fluid collision)
 *   collision  PSM_COLL_TRT (the above) or PSM_COLL_CUMULANT: the cumulant
 *            operator the paper's performance runs use (section V, listed in
 *            section II.B), D3Q27 only and without body force: shear rate
 *            1/tau, every other rate one (second-order trace to 3 c_s^2,
 *            cumulants of orders 3..6 to zero); magic is unused
 *   map_reading  how geometry_map_step reads section III's average over the
 *            super-sampled geometry cells that correspond to a lab cell:
 *            PSM_MAP_SUBSAMPLES: each of the cell's (2^s)^3 sub-sample points
 *            is rotated to the body frame and looked up; PSM_MAP_BLOCK: the
 *            cell centre alone is rotated and the axis-aligned (2^s)^3 block
 *            of geometry cells nearest to the cell's extent is averaged
 *            (cheaper; larger per-cell error under rotation).  The two agree
 *            at zero rotation and for s = 0.
 *   layout   PDF buffer layout (psm_pdf_layout gives the numbers):
 *            PSM_LAYOUT_SOA: one array per direction (cell n = x + nx*(y +
 *            ny*z) of direction k at k*S + n, S = psm_pdf_stride);
 *            PSM_LAYOUT_BLOCKED: the rows of the lattice (row r = y + ny*z)
 *            in blocks of RB = 2^m consecutive rows, RB*nx <= 4096 cells (m
 *            as large as that allows), each block holding its q direction
 *            arrays one after another: cell (x, r) of direction k at
 *            (r / RB)*q*RB*nx + k*RB*nx + (r mod RB)*nx + x (RB from
 *            block_rows).  The blocked
 *            form keeps the 2q streams of a step within a few hundred KiB
 *            (the in-place step's memory pattern runs ~9% faster on 256^3).
 *   block_rows  rows per block of the blocked layout: a power of two, or 0
 *            for the library's choice (the largest RB with RB*nx*sizeof
 *            (storage) <= 16 KiB, at least one row); 0 for PSM_LAYOUT_SOA
 *   map_ahead  1: the field keeps two sets of solid fractions, so that
 *            psm_step_ahead can map the next step into one while this step
 *            reads the other (PSM_BUF_B twice as large); 0: one set.  psm = 1
 */
typedef struct psm_config {
  int32_t nx, ny, nz;
  int32_t q;
  int32_t storage;
  int32_t psm;
  int32_t sc;
  int32_t b_form;
  int32_t slots;
  int32_t max_bodies;
  int32_t bc[6];
  double tau;
  double magic;
  double force[3];
  double u_in[3];
  int32_t collision;
  int32_t map_reading;
  int32_t layout;
  int32_t block_rows;
  int32_t map_ahead;
} psm_config;

/* Pose and velocity of one rigid body at one step: a body-frame point p is at
 * x = R p + X in the lab; the solid velocity is u_s(x) = V + W x (x - X).
 * R is row-major.  W is the angular-velocity vector (rate times unit axis). */
typedef struct psm_body {
  double R[9];
  double X[3];
  double V[3];
  double W[3];
} psm_body;

/* Prescribed motion (one-way coupling, section V.A): rotation by
 * theta(t) = theta0 + omega*t about the unit `axis` through x0 + v*t. */
typedef struct psm_motion {
  double axis[3];
  double theta0;
  double omega;
  double x0[3];
  double v[3];
} psm_motion;

typedef struct psm_field psm_field; /* opaque: lattice + B + partial buffers  */
typedef struct psm_geom psm_geom;   /* opaque: body-frame geometry field      */

/* ---- errors, sizes, tables ---------------------------------------------- */
const char *psm_last_error(void);

/* Bytes the caller must provide for buffer `which` (PSM_BUF_*):
 *   PDF  SoA: q*S*sizeof(storage): direction k occupies elements
 *        [k*S, k*S + N) with S = psm_pdf_stride(cfg) >= N (cell n = x +
 *        nx*(y + ny*z)); blocked: ceil(ny*nz / RB) blocks of q*RB*nx
 *        elements (psm_pdf_layout)
 *   B    psm ? N*4*slots + N (FP32 fraction per slot + one body-id byte) : 0;
 *        map_ahead: two such sets, the second at the first's size rounded up
 *        to 256 bytes
 *   WORK flags + force/torque partials (max_bodies*6 doubles per solid-kernel
 *        workgroup, 4096 of them) + reduction scratch + the mapping's lists
 *        of surface cells (psm ? max_bodies * 2^21 * 4 bytes : 0)
 *   ADJOINT  one adjoint PDF buffer of psm_adjoint_step: the PDF buffer's
 *        layout (psm_pdf_layout, in elements) with adjoint-precision
 *        elements (FP64 for PSM_F64 fields, else FP32)
 *   GRAD_B   the dJ/dB accumulator of psm_adjoint_step: N adjoint-precision
 *        values
 *   OBSTACLE  lbm_set_obstacle's buffer (plain-LBM fields; 0 for psm = 1):
 *        256 B header + N class bytes (padded to 256 B) + 8 B per listed
 *        cell, sized here for the worst case of N listed cells              */
int psm_required_bytes(const psm_config *cfg, int which, size_t *out_bytes);

/* Elements between the starts of consecutive direction arrays of the PDF
 * buffer.  PSM_LAYOUT_SOA: N rounded up to a 4 KiB multiple in bytes, plus
 * 4 KiB (so the arrays do not all start at the same offset modulo a large
 * power of two).  PSM_LAYOUT_BLOCKED: RB*nx, within a block. */
int psm_pdf_stride(const psm_config *cfg, int64_t *elems);

/* The PDF buffer layout of cfg (see psm_config.layout): rows per block RB
 * (SoA: ny*nz, one block), the direction stride in elements (as
 * psm_pdf_stride) and the block stride in elements (SoA: 0).  The element
 * of direction k, cell x of row r = y + ny*z is at
 *   (r / RB)*block_stride + k*dir_stride + (r mod RB)*nx + x.
 * Any output pointer may be NULL. */
int psm_pdf_layout(const psm_config *cfg, int32_t *rows_per_block, int64_t *dir_stride, int64_t *block_stride);

/* This library's lattice: velocities c[q][3], weights w[q], opposite opp[q]
 * (host arrays of at least q entries). */
int psm_lattice(int q, int32_t *c, double *w, int32_t *opp);

/* ---- host kinematics (section III: rotation folded into the lookup) ------ */
/* Body pose at `step`: theta = theta0 + omega*step (never accumulated), R by
 * Rodrigues' formula evaluated entry-wise as
 *   R_ij = ((c*delta_ij + ((1-c)*a_i)*a_j) + s*K_ij),  K = [a]_x,
 * X = x0 + v*step, V = v, W = omega*axis.  `axis` must be a unit vector. */
int psm_body_pose(const psm_motion *m, int64_t step, psm_body *out);

/* ---- field lifetime -------------------------------------------------------- */
/* Validates cfg and the caller buffers (sizes from psm_required_bytes; the
 * B buffer may be NULL when cfg->psm == 0) and records them.  Clears the
 * first 256 bytes of the work buffer (flags, counters) on `stream`; the PDFs
 * and B are not touched: call psm_field_reset before the first step.  Also
 * makes the field's own streams (default priority, non-blocking; they are
 * synchronised and destroyed by pdf_field_destroy): one for the solid-cell
 * and face-row launches (PSM_OPT_CONCURRENT) and, with map_ahead, one for
 * the mapping; if they cannot be made the field runs on the caller's
 * stream. */
int pdf_field_create(const psm_config *cfg, void *pdf_dev, size_t pdf_bytes, void *b_dev,
                     size_t b_bytes, void *work_dev, size_t work_bytes, void *stream,
                     psm_field **out);
int pdf_field_destroy(psm_field *f);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * pdf_field_create without the work buffer.  The field's work area (error
 * flags, mapping counters, force/torque partials, reduction scratch and the
 * mapping's surface-cell lists) is instead a static device array of the
 * library, PSM_STATIC_WORK_BYTES (16 MiB), of which each GPU the library runs
 * on holds one copy until the process ends.  The caller still passes the PDF
 * and B buffers (sizes and alignment as for pdf_field_create).  This call and
 * every later call on the field allocate nothing (no hipMalloc / hipFree).
 * Results are bitwise those of a field made by pdf_field_create: the
 * surface-cell lists are cut to what fits (PSM_OPT_MAP_LIST's upper limit
 * shrinks accordingly), and cells beyond a list are sampled by the
 * classification kernel, which gives the same fractions.
 * Sharing: all such fields on one GPU share its array.  Creating one (or
 * psm_field_reset of one) claims the array and clears its flags and counters
 * on `stream`; calls on an earlier such field of that GPU then fail with
 * PSM_EINVAL until it is reset.  Calls on the owning field that overlap in
 * time (several host threads, or several streams) race on the array.
 * Errors: as pdf_field_create; PSM_ESIZE when the lattice and max_bodies need
 * more than PSM_STATIC_WORK_BYTES before any list entry (the reduction scratch
 * takes N/32 bytes: about 5e8 cells at most); PSM_EHIP when the array's
 * device address cannot be looked up. */
#define PSM_STATIC_WORK_BYTES (16u << 20)
int pdf_field_create_noalloc(const psm_config *cfg, void *pdf_dev, size_t pdf_bytes, void *b_dev, size_t b_bytes,
                             void *stream, psm_field **out);

/* Rest equilibrium (delta f = 0, rho = 1, u = 0), B = 0, body ids 0, flags 0. */
int psm_field_reset(psm_field *f, void *stream);

/* ---- geometry field (section III; voxelised once on the host) ---------- */
/* Body-frame geometry lattice: spacing h = 2^-s LBM cells, cell centres at
 * (m + 1/2) h for integer m.  A bit is set when its centre is inside the
 * object.  The field is stored only over the object's body-frame bounding box
 * plus one LBM cell of padding, bit-packed along body x (32-bit words, row
 * length ceil(dims[0]/32) words), followed by a coarse map of one byte per
 * 2^s x 2^s x 2^s block (0 all outside, 1 all inside, 2 mixed).
 *
 * psm_geometry_box: box (mmin, dims) and device bytes for a mesh (verts != NULL)
 * or an analytic shape (kind PSM_SHAPE_*, params: ellipsoid semi-axes a,b,c;
 * cube half side).  Meshes: verts[nv][3] doubles (body frame), tris[nt][3]
 * int32 indices, closed and consistently oriented; inside = nonzero winding
 * number along +x rays. */
int psm_geometry_box(int kind, const double *params, const double *verts, int64_t nv, int s,
                     int32_t mmin[3], int32_t dims[3], size_t *dev_bytes);
/* Host voxelisation into a caller host buffer of dims[2]*dims[1]*ceil(dims[0]/32)
 * uint32 words (exported for host-side checks). */
int psm_voxelize_host(const double *verts, int64_t nv, const int32_t *tris, int64_t nt, int s,
                      const int32_t mmin[3], const int32_t dims[3], uint32_t *bits);
int psm_analytic_host(int kind, const double *params, int s, const int32_t mmin[3],
                      const int32_t dims[3], uint32_t *bits);
/* Voxelise on the host, then copy to the caller's device buffer (async on
 * stream; the host copy is kept by the handle until destroy). */
int geometry_field_create(const double *verts, int64_t nv, const int32_t *tris, int64_t nt, int s,
                          void *dev_buf, size_t bytes, void *stream, psm_geom **out);
int geometry_field_create_analytic(int kind, const double *params, int s, void *dev_buf,
                                   size_t bytes, void *stream, psm_geom **out);
int geometry_field_destroy(psm_geom *g);

/* ---- per-step hot path ----------------------------------------------------- */
/* Section III mapping, reading "transform each sub-sample": for each lab cell
 * in the swept box of each body and each of its (2^s)^3 sub-sample points at
 * offsets delta_k = (k + 1/2) h - 1/2 from the cell centre, the body-frame
 * point p_k = R^T (x_c - X) + R^T delta_k is looked up in the geometry lattice
 * cell that contains it; eps = (#inside)/8^s; B = eps or eq. (6).  FP64
 * arithmetic p_a = fma(R[0][a], d0, fma(R[1][a], d1, R[2][a]*d2)) for both
 * terms, then signed 64-bit fixed point with 32 fraction bits in sub-cell
 * units: m = floor((rint(p*2^(s+32)) + rint((R^T delta_k)*2^(s+32))) / 2^32).
 * Swept box of a body: cells within its geometry's bounding sphere around X,
 * this step and the previous mapped step (cells a body has left are reset).
 * Bodies are assigned to the cell's slots in body order; a cell touched by
 * more bodies than cfg->slots raises error flag bit 0 (psm_error_flags).
 * `geoms[b]` is the geometry of body b.  n_bodies <= cfg->max_bodies. */
int geometry_map_step(psm_field *f, const psm_body *bodies, const psm_geom *const *geoms,
                      int n_bodies, void *stream);

/* One in-place time step (eqs. (1), (3), (4), (7)-(9)) with parity step&1.
 * Per cell: rho = 1 + sum df, u = (sum c df + F/2)/rho; TRT + Guo fluid
 * collision Omega^F; for each body slot k with B_k > 0 the solid collision
 * Omega^S_k with u_s = V + W x (x_c - X); f* = f + (1 - sum B)Omega^F +
 * sum B_k Omega^S_k (B scaled to sum 1 when it exceeds 1); streaming by the
 * AA pattern with the face rules of cfg->bc.  Writes per-tile FP64 partials of
 * the force -B_k sum_i c_i Omega^S_{k,i} on each body and its torque about X
 * (eqs. (10)-(11), force on the body).  `bodies` must be the poses used by
 * the last geometry_map_step (B(t) and u_s(t) of the same step). */
int psm_stream_collide(psm_field *f, const psm_body *bodies, int n_bodies, int64_t step,
                       void *stream);

/* Sum the partials of the last psm_stream_collide in fixed order: ft_dev is a
 * device array double[n_bodies][6] = (Fx,Fy,Fz,Tx,Ty,Tz) on each body, lattice
 * units. */
int body_force_torque(psm_field *f, int n_bodies, double *ft_dev, void *stream);

/* One whole step in one call: geometry_map_step(map_poses) +
 * psm_stream_collide(bodies, step) + (ft_dev != NULL) body_force_torque, in
 * that order on `stream`.  map_poses may be NULL (= bodies); it differs from
 * bodies only when the velocity used by the solid collision differs from the
 * motion that places the geometry (sensitivity runs).  A plain-LBM field (or
 * n_bodies = 0) takes one psm_stream_collide.  With ft_dev the per-body sum is
 * taken by one extra workgroup of the step's last fluid launch (one launch fewer;
 * same order as body_force_torque, so the same bits); the partials stay
 * readable by a later body_force_torque. */
int psm_step(psm_field *f, const psm_body *map_poses, const psm_body *bodies, const psm_geom *const *geoms,
             int n_bodies, int64_t step, double *ft_dev, void *stream);

/* psm_step with the mapping one step ahead (section III's per-step mapping,
 * overlapped with the update), for fields made with map_ahead = 1 and motion
 * known a step in advance.  Step `step` uses the fractions that the previous
 * call mapped from its next_map_poses when that call was for step - 1 with the
 * same n_bodies, else (the first call, or after geometry_map_step,
 * psm_field_reset or another step) it maps them from map_poses (NULL =
 * bodies) first.  It then runs psm_stream_collide(bodies, step) (+ the F/T
 * sum into ft_dev) and maps step + 1 from next_map_poses into the field's
 * other set of fractions on a mapping stream of the field (made at
 * pdf_field_create, default priority), forked from `stream` at the start of
 * the step and joined back into it before the call's later work: the mapping
 * overlaps the step's launches.
 * The results equal psm_step(map_poses, bodies, step) bit for bit, provided
 * next_map_poses are the map poses of the next call.  PSM_EUNSUP without
 * map_ahead; fields from pdf_field_create_noalloc map on `stream`.  Which set
 * a call reads is host state, so a captured graph would replay one call's
 * choice every time: capture psm_step instead. */
int psm_step_ahead(psm_field *f, const psm_body *map_poses, const psm_body *bodies, const psm_body *next_map_poses,
                   const psm_geom *const *geoms, int n_bodies, int64_t step, double *ft_dev, void *stream);

/* Device pointers of the fractions the last step used (map_ahead fields swap
 * between two sets): slot 0, slot 1 (NULL with one slot) and the body-id
 * bytes.  Any output pointer may be NULL. */
int psm_fractions(psm_field *f, const float **b0, const float **b1, const uint8_t **meta);

/* ---- sensitivities (adjoint) ------------------------------------------------ */
/* Optional time-invariant offset field dB (device, N floats, caller-owned,
 * NULL to clear): every later step uses B_eff = B + dB in slot 0 (body 0).
 * The offset can make B nonzero anywhere, so the field then treats the whole
 * domain as possibly solid (slower; meant for sensitivity runs). */
int psm_set_fraction_offset(psm_field *f, const float *dB_dev);

/* ---- two-way coupling: rigid bodies driven by the hydrodynamic force ------ */
/* State of a freely moving rigid body (the settling-sphere validation of
 * section IV: the body moves under gravity, buoyancy and the force / torque of
 * eqs. (10)-(11)).  Lattice units.
 *   m      mass
 *   I      principal moments of inertia (body frame axes, about X)
 *   F_ext  constant external force on the body (gravity minus buoyancy), lab
 *   X, V   reference point (body-frame origin) and its velocity, lab
 *   R      orientation (body -> lab, row-major), W angular velocity, lab
 *   ft_prev   hydrodynamic F/T of the previous step (zero at rest)
 *   average   1: advance with the mean of this step's and the previous
 *             step's hydrodynamic F/T (keeps the explicit coupling of bodies
 *             not much denser than the fluid stable: the solid collision
 *             hands the body the change of its inner fluid's momentum one
 *             step late, up to 1/tau times over with SC2); 0: this step's */
typedef struct psm_rigid {
  double m;
  double I[3];
  double F_ext[3];
  double X[3];
  double V[3];
  double R[9];
  double W[3];
  double ft_prev[6];
  int32_t average;
  int32_t reserved;
} psm_rigid;

/* Pose and velocity of a rigid-body state, for the mapping and the solid
 * collision of the next step. */
int psm_rigid_body(const psm_rigid *s, psm_body *out);

/* Advance a rigid-body state by dt with the hydrodynamic force / torque
 * ft = (F, T) of the step just taken (force on the body, torque about X;
 * with `average`, (ft + ft_prev) / 2 in its place; ft_prev = ft after):
 * semi-implicit Euler,
 *   V += dt (F + F_ext) / m,  X += dt V,
 *   W += dt I_lab^-1 (T - W x (I_lab W)),  I_lab = R diag(I) R^T,
 *   R <- Rot(dt W) R,  Rot by Rodrigues' formula about W / |W| (identity
 *   when W = 0).  Host arithmetic, FP64.  m and every I must be > 0. */
int psm_rigid_advance(psm_rigid *s, const double ft[6], double dt);

/* One two-way coupled step of n_bodies free bodies: psm_step with the poses
 * and velocities of states (map, stream-collide, F/T into ft_dev, device
 * double[n_bodies][6]), then the F/T are copied to ft_host (host
 * double[n_bodies][6], may be pinned), `stream` is synchronised, and every
 * state advances by one step (dt = 1).  The states of step `step` in, those
 * of step + 1 out. */
int psm_coupled_step(psm_field *f, psm_rigid *states, const psm_geom *const *geoms, int n_bodies, int64_t step,
                     double *ft_dev, double *ft_host, void *stream);

/* ---- static no-slip obstacle (plain LBM) ----------------------------------- */
/* The LBM variant of the paper's node-level benchmark (section V: an LBM
 * kernel plus the no-slip treatment of a stationary geometry).  For a field
 * with psm = 0: cells with solid_dev[n] != 0 (device, N bytes, read during
 * this call only) become obstacle cells, never updated; every link from a
 * fluid cell whose source x - c_k is an obstacle cell takes halfway
 * bounce-back, the wall rule (ahead of inlet / outlet faces).  Builds, on
 * `stream`, the cell classes, the list of fluid cells next to the obstacle
 * (with their link masks) and the obstacle's bounding box in obst_dev
 * (caller-owned, 256-byte aligned, kept until the obstacle is replaced;
 * obst_bytes from psm_required_bytes(PSM_BUF_OBSTACLE) always suffices, a
 * smaller buffer holds (obst_bytes - 256 - N rounded up to 256) / 8 list
 * entries), then synchronises `stream` to read the list length back
 * (*n_near, may be NULL).  Later psm_stream_collide / psm_step calls skip the
 * obstacle and its neighbours in the bulk kernels and update the neighbours
 * in a kernel of their own.  solid_dev = NULL removes the obstacle.
 * psm_field_reset keeps it.  Errors: PSM_EUNSUP on a PSM field, PSM_ESIZE
 * when the list does not fit (the field is then left without obstacle). */
int lbm_set_obstacle(psm_field *f, const uint8_t *solid_dev, void *obst_dev, size_t obst_bytes, int64_t *n_near,
                     void *stream);

/* The field's PDF buffer to or from the standard layout: q arrays of N
 * values, element k*N + n (cell n = x + nx*(y + ny*z)), in the field's
 * storage type, device memory, on `stream`.  The slots are copied as they
 * are (no parity handling: after an even number of steps they hold f_k - w_k
 * of each cell in its own slot).  For either layout; dst / src must not
 * overlap the PDF buffer. */
int psm_pdf_gather(psm_field *f, void *dst, void *stream);
int psm_pdf_scatter(psm_field *f, const void *src, void *stream);

/* Reverse-mode (adjoint) of step `step` for the torque objective
 *   J = sum_t wt(t) * axis . T(t)
 * of body 0 (eq. (11), force on the body, about X), under the frozen-B
 * convention: the fractions B(t) are inputs (call geometry_map_step for this
 * step first); the rotation rate enters through u_s = V + W x (x - X) only.
 * Needs a PSM field with TRT collision, sc = 1, slots = 1 and one mapped body.
 *   fwd_pdf   the forward state before step `step` (parity step&1): a copy
 *             of the field's PDF buffer (psm_required_bytes PSM_BUF_PDF
 *             bytes, the field's layout and storage type), e.g. made by
 *             psm_stream_copy before the step
 *   ahat_in   adjoint of f(step+1), direction k of cell x at the PDF
 *             buffer's element of direction k, cell x (psm_pdf_layout), in
 *             the adjoint precision (PSM_BUF_ADJOINT bytes); elements outside
 *             the lattice are not read
 *   ahat_out  adjoint of f(step) (written; must not alias ahat_in)
 *   dJdB      accumulated: dJdB[n] += dJ/dB(n, step)
 *   body      the pose/velocity of body 0 used by the forward step (W may
 *             differ from the rotation that produced B)
 *   axis      unit vector a; wt the weight of this step's torque in J
 * The dJ/dW-along-axis contribution of this step is kept in the field's work
 * buffer until the next psm_adjoint_step; psm_adjoint_omega adds it (FP64,
 * fixed order) to out_dev[0]. */
int psm_adjoint_step(psm_field *f, const void *fwd_pdf, int64_t step, const void *ahat_in, void *ahat_out,
                     void *dJdB, const psm_body *body, const double axis[3], double wt, void *stream);
int psm_adjoint_omega(psm_field *f, double *out_dev, void *stream);
/* An adjoint buffer (PSM_BUF_ADJOINT, the PDF buffer's layout) to the
 * standard layout: q arrays of N adjoint-precision values, element k*N + n,
 * on `stream`; dst must not overlap adj. */
int psm_adjoint_gather(psm_field *f, const void *adj, void *dst, void *stream);

/* ---- diagnostics ------------------------------------------------------------ */
/* Total mass sum_x rho(x) in FP64 (fixed-order tree) into out_dev[0];
 * `step` is the number of steps taken (selects the AA parity). */
int psm_mass_fp64(psm_field *f, int64_t step, double *out_dev, void *stream);
/* rho[N] and u[N][3] (u = (sum c f + F/2)/rho) in FP64 after `step` steps. */
int psm_macroscopic(psm_field *f, int64_t step, double *rho_dev, double *u_dev, void *stream);
/* Copy the field's int32 error flags (bit 0: too many bodies in a cell). */
int psm_error_flags(psm_field *f, int32_t *out_dev, void *stream);
/* Per-field options (defaults in brackets):
 *   PSM_OPT_GENERAL_PATH [0]  1: every row of psm_stream_collide takes the
 *                             general (face-row) addressing path; results are
 *                             bitwise identical, used to cross-check the fast path
 *   PSM_OPT_XCD_REMAP    [0]  1: workgroup ids are remapped so each of the 8
 *                             XCDs walks a contiguous range of tiles
 *   PSM_OPT_MAP_LIST  [2^21]  entries per body of the list of surface cells
 *                             (s = 3 bodies) that geometry_map_step samples in
 *                             a second kernel (three cells per wave); cells beyond it,
 *                             and every cell with 0, are sampled in the
 *                             classification kernel.  Results are identical.
 *   PSM_OPT_SOLID_GRID [4096] most workgroups of the solid-cell kernel (1 ..
 *                             4096, 0 = default); fewer make each workgroup walk
 *                             more groups of chunks.  PDFs are identical; the
 *                             F/T partials are grouped differently (FP64
 *                             rounding only).  Meant for tests.
 *   PSM_OPT_CONCURRENT   [1]  1: in steps with a separate face-row launch
 *                             (odd steps, and every D3Q27 step),
 *                             psm_stream_collide / psm_step run the solid-cell
 *                             launch, the F/T sum and the face-row launch on a
 *                             second stream of the field (default priority,
 *                             made at pdf_field_create), beside the interior
 *                             launch on the caller's stream, which waits for
 *                             them before any later work on it;
 *                             0: all on the caller's stream.  Results are
 *                             bitwise identical.  Fields made by
 *                             pdf_field_create_noalloc have no second stream
 *                             and always run on the caller's stream. */
enum { PSM_OPT_GENERAL_PATH = 1, PSM_OPT_XCD_REMAP = 2, PSM_OPT_MAP_LIST = 4, PSM_OPT_SOLID_GRID = 8,
       PSM_OPT_CONCURRENT = 16 };
int psm_set_option(psm_field *f, int option, int value);
/* Device-to-device copy kernel (measured-bandwidth probe); 16-byte aligned
 * src and dst. */
int psm_stream_copy(const void *src, void *dst, size_t bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* PSM_H */
