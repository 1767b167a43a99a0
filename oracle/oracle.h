/*
 * FP64 CPU oracle for the PSM hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline
 * leg of the benchmark may load or call this library.  The product (HIP)
 * path never does, and this tree shares no code, header, table or constant
 * generator with it.
 *
 * It is a plain, slow, scalar implementation of what the paper defines, in
 * full distribution functions f (not deviations), with a two-buffer pull
 * streaming scheme (deliberately unlike the in-place scheme of the GPU path):
 *   - lattice Boltzmann update, section II.A eq. (1)
 *   - equilibrium eq. (3) with the sign of the u^2 term corrected to "-"
 *   - SRT eq. (2) as the special case of TRT (lbmpy's TRT, section II.B)
 *   - PSM rule eq. (4), B = eps eq. (5) or the tau-weighted form eq. (6)
 *   - solid collision operators SC1/SC2/SC3, eqs. (7)-(9)
 *   - hydrodynamic force / torque, eqs. (10)-(11), reported as the force ON
 *     the body (minus the printed fluid-side sum)
 *   - geometry field -> solid fraction mapping with rotation/translation,
 *     section III (supersampled body-frame lookup of every sub-sample; the
 *     other reading, centre transform + axis-aligned block average)
 *   - generalised winding number voxelisation, divergence-theorem volume
 *   - FP64 discrete adjoint of one step (explicit per-cell Jacobian)
 *   - cumulant fluid collision (D3Q27; shear rate 1/tau, every other rate
 *     one), through set-partition moment / cumulant relations and a linear
 *     solve for the populations
 *   - plain LBM with halfway bounce-back on static obstacle cells (the LBM
 *     variant of the node-level benchmark, section V)
 *
 * Readings of ambiguous passages are listed in the design notes of the
 * repository; each function below names the equation it follows.
 */
#ifndef PSM_ORACLE_H
#define PSM_ORACLE_H
#ifdef __cplusplus
extern "C" {
#endif

#define OR_MAXQ 27

/* face boundary kinds (faces ordered -x,+x,-y,+y,-z,+z) */
enum { OR_PERIODIC = 0, OR_WALL = 1, OR_INLET = 2, OR_OUTLET = 3 };

typedef struct {
  int nx, ny, nz, q;
  double tau;     /* relaxation time of the even moments (viscosity) */
  double magic;   /* TRT parameter Lambda */
  double force[3];/* body-force density (Guo forcing), lattice units */
  int bc[6];
  double u_in[3]; /* inlet velocity (moving-wall bounce-back) */
  int sc;         /* 1, 2 or 3 */
  int psm;        /* 0: plain LBM (solid fraction ignored), 1: PSM */
  int collision;  /* OR_TRT or OR_CUMULANT (D3Q27, no body force) */
} or_config;

/* fluid collision operators */
enum { OR_TRT = 0, OR_CUMULANT = 1 };

/* Pose of a body at one step: lab = R * body + X; solid velocity
 * u_s(x) = V + W x (x - X). R row-major. */
typedef struct {
  double R[9];
  double X[3];
  double V[3];
  double W[3];
} or_pose;

/* Geometry: kind 0 = analytic ellipsoid (p = semi-axes), 1 = analytic cube
 * (p[0] = half side), 2 = stored inside flags over the box mmin..mmin+dims,
 * 3 = mesh evaluated on demand (winding number at each queried centre). */
typedef struct {
  int kind;
  double p[3];
  int s;
  int mmin[3];
  int dims[3];
  const unsigned char *inside;
  double r_bound;  /* every inside lattice centre is within r_bound of the origin */
  const double *verts;
  const int *tris;
  long long nt;
} or_geom;

int or_lattice(int q, int *c, double *w, int *opp);
void or_feq(int q, double rho, const double u[3], double *feq);

void or_pose_at(const double axis[3], double theta0, double omega, const double x0[3],
                const double v[3], long long t, or_pose *out);

int or_collide_cell(const or_config *cfg, const double *fin, int nslot, const double *B,
                    const double *us, double *fout, double *dF);

int or_step(const or_config *cfg, double *f, double *fpost, int nb, const double *B,
            const or_pose *poses, double *ft);
/* plain LBM (cfg->psm == 0) with static no-slip obstacle cells solid[n] != 0 */
int or_step_obstacle(const or_config *cfg, double *f, double *fpost, const unsigned char *solid);

void or_macro(const or_config *cfg, const double *f, double *rho, double *u);
double or_mass(const or_config *cfg, const double *f);

int or_geom_inside(const or_geom *g, long long mx, long long my, long long mz);
double or_map_cell(const or_geom *g, const or_pose *pose, int ix, int iy, int iz);
double or_map_cell_block(const or_geom *g, const or_pose *pose, int ix, int iy, int iz);
int or_map(const or_config *cfg, const or_geom *g, const or_pose *pose, int b_form, int reading,
           double *B_out);
float or_b_from_eps(double eps, double tau, int b_form);

int or_update_cell(const or_config *cfg, int x, int y, int z, const double *nbr, int nb, const double *Bn,
                   const or_pose *poses, double *out);

int or_adjoint_step(const or_config *cfg, const double *f, const double *ghat_next, double *ghat, const double *B,
                    const or_pose *pose, const double *axis, double wt, double *dJdB, double *dJdW);

double or_winding(const double *v, const int *t, long long nt, const double p[3]);
int or_voxelize(const double *v, const int *t, long long nt, int s, const int mmin[3],
                const int dims[3], unsigned char *out);
double or_mesh_volume(const double *v, const int *t, long long nt);

void or_set_threads(int n);
int or_threads(void);

#ifdef __cplusplus
}
#endif
#endif
