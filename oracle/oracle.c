/*
 * FP64 CPU oracle for the PSM hot path -- TEST INFRASTRUCTURE ONLY.
 * (Only tests/, the smoke check and the benchmark's CPU-baseline leg may use
 * it; the product path never does.)  See oracle.h for the list of equations.
 *
 * Everything is plain scalar FP64 on full distribution functions.  Build with
 * -ffp-contract=off: the geometry lookup (section III) must evaluate exactly
 * the FP64 operation sequence its definition states.
 */
#include "oracle.h"

#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------------------
 * Lattice (section II.B names D3Q19 and D3Q27).  Velocities are enumerated in
 * lexicographic order over {-1,0,1}^3 (x fastest) and kept if |c|^2 <= 2
 * (D3Q19) or <= 3 (D3Q27).  Weights: D3Q19 1/3, 1/18, 1/36; D3Q27 8/27,
 * 2/27, 1/54, 1/216 by |c|^2 = 0, 1, 2, 3.  The opposite direction is found by
 * search.
 * ------------------------------------------------------------------------- */
int or_lattice(int q, int *c, double *w, int *opp) {
  int maxn;
  double wq[4];
  if (q == 19) {
    maxn = 2;
    wq[0] = 1.0 / 3.0; wq[1] = 1.0 / 18.0; wq[2] = 1.0 / 36.0; wq[3] = 0.0;
  } else if (q == 27) {
    maxn = 3;
    wq[0] = 8.0 / 27.0; wq[1] = 2.0 / 27.0; wq[2] = 1.0 / 54.0; wq[3] = 1.0 / 216.0;
  } else {
    return -1;
  }
  int n = 0;
  for (int z = -1; z <= 1; ++z)
    for (int y = -1; y <= 1; ++y)
      for (int x = -1; x <= 1; ++x) {
        int m = x * x + y * y + z * z;
        if (m > maxn) continue;
        c[3 * n + 0] = x; c[3 * n + 1] = y; c[3 * n + 2] = z;
        w[n] = wq[m];
        ++n;
      }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      if (c[3 * j] == -c[3 * i] && c[3 * j + 1] == -c[3 * i + 1] && c[3 * j + 2] == -c[3 * i + 2])
        opp[i] = j;
  return n == q ? 0 : -1;
}

typedef struct {
  int q;
  int c[OR_MAXQ * 3];
  double w[OR_MAXQ];
  int opp[OR_MAXQ];
} lat_t;

static int lat_get(int q, lat_t *L) {
  L->q = q;
  return or_lattice(q, L->c, L->w, L->opp);
}

/* Equilibrium, eq. (3) with "- u^2/(2 c_s^2)" (the printed "+" breaks
 * sum_i f^eq = rho), c_s^2 = 1/3:
 *   f^eq_i = w_i rho [1 + c.u/cs2 + (c.u)^2/(2 cs2^2) - u.u/(2 cs2)] */
static void feq_lat(const lat_t *L, double rho, const double u[3], double *feq) {
  const double cs2 = 1.0 / 3.0;
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < L->q; ++i) {
    double cu = L->c[3 * i] * u[0] + L->c[3 * i + 1] * u[1] + L->c[3 * i + 2] * u[2];
    feq[i] = L->w[i] * rho * (1.0 + cu / cs2 + cu * cu / (2.0 * cs2 * cs2) - uu / (2.0 * cs2));
  }
}

void or_feq(int q, double rho, const double u[3], double *feq) {
  lat_t L;
  if (lat_get(q, &L) != 0) return;
  feq_lat(&L, rho, u, feq);
}

/* ---------------------------------------------------------------------------
 * Prescribed rigid motion (one-way coupling, section V.A): angle
 * theta = theta0 + omega t (never accumulated), Rodrigues rotation about the
 * unit axis a: R = c I + (1-c) a a^T + s [a]_x, evaluated entry-wise as
 * ((c*delta_ij + ((1-c)*a_i)*a_j) + s*K_ij); X = x0 + v t; W = omega a.
 * ------------------------------------------------------------------------- */
void or_pose_at(const double axis[3], double theta0, double omega, const double x0[3],
                const double v[3], long long t, or_pose *out) {
  double tt = (double)t;
  double theta = theta0 + omega * tt;
  double c = cos(theta), s = sin(theta), omc = 1.0 - c;
  const double *a = axis;
  double K[9] = {0.0, -a[2], a[1], a[2], 0.0, -a[0], -a[1], a[0], 0.0};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double d = (i == j) ? c : 0.0;
      out->R[3 * i + j] = (d + (omc * a[i]) * a[j]) + s * K[3 * i + j];
    }
  for (int i = 0; i < 3; ++i) {
    out->X[i] = x0[i] + v[i] * tt;
    out->V[i] = v[i];
    out->W[i] = omega * a[i];
  }
}

/* ---------------------------------------------------------------------------
 * One collision at one cell, eq. (4) with TRT fluid collision and SC1/2/3.
 *   rho = sum f, u = (sum c f + F/2)/rho                       (Guo shift)
 *   Omega^F_i = -le (f+_i - feq+_i) - lo (f-_i - feq-_i)
 *               + (1 - le/2) S+_i + (1 - lo/2) S-_i            (TRT + Guo)
 *   S_i = w_i [ (c_i - u)/cs2 + (c_i.u) c_i / cs2^2 ] . F
 *   le = 1/tau, 1/lo = 1/2 + Lambda/(tau - 1/2)
 *   f*_i = f_i + (1 - sum_k B_k) Omega^F_i + sum_k B_k Omega^S_{k,i}
 * with the B_k scaled by 1/sum B when the sum exceeds one.  The force on the
 * body in slot k is dF_k = -B_k sum_i c_i Omega^S_{k,i} (eq. (10), body side).
 * ------------------------------------------------------------------------- */
/* ---- cumulant fluid collision (section II.B lists it; section V runs with it) ----
 * D3Q27 without body force.  The shear rate is omega = 1/tau, every other rate
 * is one (the trace of the second-order cumulants and all cumulants of orders
 * 3 to 6).  Steps, for one cell:
 *   1. u = j / rho; central moments M_abc = sum_i (c_ix-u_x)^a (c_iy-u_y)^b
 *      (c_iz-u_z)^c f_i / rho for a, b, c in {0, 1, 2};
 *   2. cumulants K_abc of that normalised distribution from the moments: a
 *      multi-index is a list of n = a+b+c axis labels, and
 *      K = sum over set partitions P of the list of (-1)^(|P|-1) (|P|-1)!
 *          times the product over the blocks of the blocks' moments;
 *   3. relaxation: K_110, K_101, K_011 and the deviators K_200 - K_020,
 *      K_200 - K_002 are multiplied by (1 - omega), the trace K_200 + K_020 +
 *      K_002 is set to 3 c_s^2 = 1, every cumulant of order >= 3 to zero;
 *   4. moments from cumulants: M = sum over set partitions of the product of
 *      the blocks' cumulants;
 *   5. the 27 populations solve sum_i (c_i - u)^abc f_i = rho M_abc. */
static int midx(int a, int b, int c) { return 9 * a + 3 * b + c; }

/* sum over the set partitions of the n labelled positions (n <= 6) of
 * weight(#blocks) * prod over blocks of T[multi-index of the block] */
static double partition_sum(int n, const int *lab, const double *T, int signed_weights) {
  int rgs[6] = {0, 0, 0, 0, 0, 0};
  double total = 0.0;
  for (;;) {
    int nb = 0;
    for (int i = 0; i < n; ++i)
      if (rgs[i] + 1 > nb) nb = rgs[i] + 1;
    double prod = 1.0;
    for (int b = 0; b < nb; ++b) {
      int cnt[3] = {0, 0, 0};
      for (int i = 0; i < n; ++i)
        if (rgs[i] == b) cnt[lab[i]]++;
      prod *= T[midx(cnt[0], cnt[1], cnt[2])];
    }
    double wgt = 1.0;
    if (signed_weights) {
      for (int k = 2; k < nb; ++k) wgt *= k; /* (nb - 1)! */
      if ((nb - 1) & 1) wgt = -wgt;
    }
    total += wgt * prod;
    /* next restricted growth string: rgs[i] <= 1 + max(rgs[0..i-1]) */
    int i = n - 1;
    for (; i > 0; --i) {
      int mx = 0;
      for (int k = 0; k < i; ++k)
        if (rgs[k] > mx) mx = rgs[k];
      if (rgs[i] <= mx) break;
    }
    if (i <= 0) break;
    rgs[i]++;
    for (int k = i + 1; k < n; ++k) rgs[k] = 0;
  }
  return total;
}

static int labels_of(int a, int b, int c, int *lab) {
  int n = 0;
  for (int k = 0; k < a; ++k) lab[n++] = 0;
  for (int k = 0; k < b; ++k) lab[n++] = 1;
  for (int k = 0; k < c; ++k) lab[n++] = 2;
  return n;
}

static int solve_dense(int n, double *A, double *x) { /* A[n][n] x = b (x holds b), partial pivoting */
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int r = k + 1; r < n; ++r)
      if (fabs(A[r * n + k]) > fabs(A[p * n + k])) p = r;
    if (A[p * n + k] == 0.0) return -1;
    if (p != k) {
      for (int cc = 0; cc < n; ++cc) {
        double t = A[k * n + cc];
        A[k * n + cc] = A[p * n + cc];
        A[p * n + cc] = t;
      }
      double t = x[k];
      x[k] = x[p];
      x[p] = t;
    }
    for (int r = k + 1; r < n; ++r) {
      double m = A[r * n + k] / A[k * n + k];
      for (int cc = k; cc < n; ++cc) A[r * n + cc] -= m * A[k * n + cc];
      x[r] -= m * x[k];
    }
  }
  for (int k = n - 1; k >= 0; --k) {
    double s = x[k];
    for (int cc = k + 1; cc < n; ++cc) s -= A[k * n + cc] * x[cc];
    x[k] = s / A[k * n + k];
  }
  return 0;
}

static void cumulant_collide(const or_config *cfg, const lat_t *L, const double *fin, double *fout) {
  double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < 27; ++i) {
    rho += fin[i];
    for (int a = 0; a < 3; ++a) j[a] += L->c[3 * i + a] * fin[i];
  }
  const double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
  double M[27], K[27], Kp[27], Mp[27];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      for (int c = 0; c < 3; ++c) {
        double s = 0.0;
        for (int i = 0; i < 27; ++i)
          s += pow(L->c[3 * i] - u[0], a) * pow(L->c[3 * i + 1] - u[1], b) * pow(L->c[3 * i + 2] - u[2], c) * fin[i];
        M[midx(a, b, c)] = s / rho;
      }
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      for (int c = 0; c < 3; ++c) {
        int lab[6];
        const int n = labels_of(a, b, c, lab);
        K[midx(a, b, c)] = n == 0 ? 0.0 : partition_sum(n, lab, M, 1);
      }
  const double om = 1.0 / cfg->tau;
  for (int k = 0; k < 27; ++k) Kp[k] = 0.0;
  Kp[midx(1, 1, 0)] = (1.0 - om) * K[midx(1, 1, 0)];
  Kp[midx(1, 0, 1)] = (1.0 - om) * K[midx(1, 0, 1)];
  Kp[midx(0, 1, 1)] = (1.0 - om) * K[midx(0, 1, 1)];
  const double dxy = (1.0 - om) * (K[midx(2, 0, 0)] - K[midx(0, 2, 0)]);
  const double dxz = (1.0 - om) * (K[midx(2, 0, 0)] - K[midx(0, 0, 2)]);
  const double tr = 1.0; /* 3 c_s^2 */
  Kp[midx(2, 0, 0)] = (tr + dxy + dxz) / 3.0;
  Kp[midx(0, 2, 0)] = Kp[midx(2, 0, 0)] - dxy;
  Kp[midx(0, 0, 2)] = Kp[midx(2, 0, 0)] - dxz;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      for (int c = 0; c < 3; ++c) {
        int lab[6];
        const int n = labels_of(a, b, c, lab);
        Mp[midx(a, b, c)] = n == 0 ? 1.0 : partition_sum(n, lab, Kp, 0);
      }
  double A[27 * 27], x[27];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      for (int c = 0; c < 3; ++c) {
        const int r = midx(a, b, c);
        for (int i = 0; i < 27; ++i)
          A[r * 27 + i] = pow(L->c[3 * i] - u[0], a) * pow(L->c[3 * i + 1] - u[1], b) * pow(L->c[3 * i + 2] - u[2], c);
        x[r] = rho * Mp[r];
      }
  solve_dense(27, A, x);
  for (int i = 0; i < 27; ++i) fout[i] = x[i];
}

static void collide_lat(const or_config *cfg, const lat_t *L, const double *fin, int nslot,
                        const double *Bin, const double *us, double *fout, double *dF) {
  const int q = L->q;
  const double cs2 = 1.0 / 3.0;
  double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < q; ++i) {
    rho += fin[i];
    for (int a = 0; a < 3; ++a) j[a] += L->c[3 * i + a] * fin[i];
  }
  double u[3];
  for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * cfg->force[a]) / rho;
  double feq[OR_MAXQ], S[OR_MAXQ], OmF[OR_MAXQ];
  feq_lat(L, rho, u, feq);
  for (int i = 0; i < q; ++i) {
    double cu = 0.0, cF = 0.0, uF = 0.0;
    for (int a = 0; a < 3; ++a) {
      cu += L->c[3 * i + a] * u[a];
      cF += L->c[3 * i + a] * cfg->force[a];
      uF += u[a] * cfg->force[a];
    }
    S[i] = L->w[i] * ((cF - uF) / cs2 + cu * cF / (cs2 * cs2));
  }
  double le = 1.0 / cfg->tau;
  double lo = 1.0 / (0.5 + cfg->magic / (cfg->tau - 0.5));
  if (cfg->collision == OR_CUMULANT) {
    double fc[OR_MAXQ];
    cumulant_collide(cfg, L, fin, fc);
    for (int i = 0; i < q; ++i) OmF[i] = fc[i] - fin[i];
  } else {
    for (int i = 0; i < q; ++i) {
      int k = L->opp[i];
      double fp = 0.5 * (fin[i] + fin[k]), fm = 0.5 * (fin[i] - fin[k]);
      double ep = 0.5 * (feq[i] + feq[k]), em = 0.5 * (feq[i] - feq[k]);
      double sp = 0.5 * (S[i] + S[k]), sm = 0.5 * (S[i] - S[k]);
      OmF[i] = -le * (fp - ep) - lo * (fm - em) + (1.0 - 0.5 * le) * sp + (1.0 - 0.5 * lo) * sm;
    }
  }
  if (!cfg->psm || nslot == 0) {
    for (int i = 0; i < q; ++i) fout[i] = fin[i] + OmF[i];
    return;
  }
  /* several bodies in one cell: fractions summing past one are scaled to one */
  double B[2], Bsum = 0.0;
  for (int k = 0; k < nslot; ++k) Bsum += Bin[k];
  const int scale = nslot == 2 && Bsum > 1.0;
  for (int k = 0; k < nslot; ++k) B[k] = scale ? Bin[k] / Bsum : Bin[k];
  double fluid = scale ? 0.0 : 1.0 - Bsum;
  for (int i = 0; i < q; ++i) fout[i] = fin[i] + fluid * OmF[i];
  for (int k = 0; k < nslot; ++k) {
    double feqs[OR_MAXQ];
    feq_lat(L, rho, us + 3 * k, feqs);
    double mom[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < q; ++i) {
      int ib = L->opp[i];
      double om;
      if (cfg->sc == 1)        /* eq. (7) */
        om = (fin[ib] - feq[ib]) - (fin[i] - feqs[i]);
      else if (cfg->sc == 2)   /* eq. (8) */
        om = (feqs[i] - fin[i]) + (1.0 - 1.0 / cfg->tau) * (fin[i] - feqs[i]);
      else                     /* eq. (9) */
        om = (fin[ib] - feqs[ib]) - (fin[i] - feqs[i]);
      fout[i] += B[k] * om;
      for (int a = 0; a < 3; ++a) mom[a] += L->c[3 * i + a] * om;
    }
    for (int a = 0; a < 3; ++a) dF[3 * k + a] = -B[k] * mom[a];
  }
}

int or_collide_cell(const or_config *cfg, const double *fin, int nslot, const double *B,
                    const double *us, double *fout, double *dF) {
  lat_t L;
  if (lat_get(cfg->q, &L) != 0 || nslot < 0 || nslot > 2) return -1;
  if (cfg->collision == OR_CUMULANT && (cfg->q != 27 || cfg->force[0] != 0.0 || cfg->force[1] != 0.0 ||
                                        cfg->force[2] != 0.0))
    return -5;
  collide_lat(cfg, &L, fin, nslot, B, us, fout, dF);
  return 0;
}

/* Classification of the source cell y - c_k of an incoming direction: periodic
 * axes wrap; a source outside a non-periodic face takes that face's kind, with
 * precedence wall > inlet > outlet (when it leaves through several faces). */
static int classify(const or_config *cfg, int x, int y, int z, const int *c, int *src) {
  int p[3] = {x - c[0], y - c[1], z - c[2]};
  int n[3] = {cfg->nx, cfg->ny, cfg->nz};
  int kind = 0;
  for (int a = 0; a < 3; ++a) {
    int face = -1;
    if (p[a] < 0) face = 2 * a;
    else if (p[a] >= n[a]) face = 2 * a + 1;
    if (face < 0) continue;
    int b = cfg->bc[face];
    if (b == OR_PERIODIC) {
      p[a] = (p[a] + n[a]) % n[a];
      continue;
    }
    int rank_new = b == OR_WALL ? 3 : (b == OR_INLET ? 2 : 1);
    int rank_old = kind == OR_WALL ? 3 : (kind == OR_INLET ? 2 : (kind == OR_OUTLET ? 1 : 0));
    if (rank_new > rank_old) kind = b;
  }
  *src = p[0] + n[0] * (p[1] + n[1] * p[2]);
  return kind;
}

/* One full time step: collide every cell (reading f), then pull-stream the
 * post-collision values back into f.  Domain faces (named, not specified, in
 * the paper) for an incoming direction k whose source is outside:
 *   wall   : f_k(y) = f*_{kbar}(y)                         (halfway bounce-back)
 *   inlet  : f_k(y) = f*_{kbar}(y) + 2 w_k (c_k . u_in)/cs2 (moving wall, rho0=1)
 *   outlet : f_k(y) = f*_k(y)                              (zero gradient)
 * B is dense per body, B[b*N + n].  ft[b*6..] = (F, T) on body b, summed per
 * z-slab then over slabs in z order. */
static int step_impl(const or_config *cfg, double *f, double *fpost, int nb, const double *B,
                     const or_pose *poses, double *ft, const unsigned char *solid) {
  lat_t L;
  if (lat_get(cfg->q, &L) != 0) return -1;
  if (cfg->collision == OR_CUMULANT &&
      (cfg->q != 27 || cfg->force[0] != 0.0 || cfg->force[1] != 0.0 || cfg->force[2] != 0.0))
    return -5;
  for (int a = 0; a < 3; ++a)
    if ((cfg->bc[2 * a] == OR_PERIODIC) != (cfg->bc[2 * a + 1] == OR_PERIODIC)) return -2;
  const int q = L.q, nx = cfg->nx, ny = cfg->ny, nz = cfg->nz;
  const long long N = (long long)nx * ny * nz;
  double *slab = (double *)calloc((size_t)nz * (nb > 0 ? nb : 1) * 6, sizeof(double));
  int err = 0;
#pragma omp parallel for schedule(static) reduction(| : err)
  for (int z = 0; z < nz; ++z) {
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        long long n = x + (long long)nx * (y + (long long)ny * z);
        double fin[OR_MAXQ], fo[OR_MAXQ], Bs[2], us[6], dF[6];
        int bid[2], ns = 0;
        if (solid && solid[n]) { /* obstacle cell: not updated */
          for (int i = 0; i < q; ++i) fpost[i * N + n] = f[i * N + n];
          continue;
        }
        for (int i = 0; i < q; ++i) fin[i] = f[i * N + n];
        if (cfg->psm)
          for (int b = 0; b < nb; ++b) {
            double v = B[b * N + n];
            if (v != 0.0) {
              if (ns == 2) { err |= 1; continue; }
              bid[ns] = b;
              Bs[ns] = v;
              ++ns;
            }
          }
        double xc[3] = {x + 0.5, y + 0.5, z + 0.5};
        for (int k = 0; k < ns; ++k) {
          const or_pose *P = &poses[bid[k]];
          double r[3] = {xc[0] - P->X[0], xc[1] - P->X[1], xc[2] - P->X[2]};
          us[3 * k + 0] = P->V[0] + (P->W[1] * r[2] - P->W[2] * r[1]);
          us[3 * k + 1] = P->V[1] + (P->W[2] * r[0] - P->W[0] * r[2]);
          us[3 * k + 2] = P->V[2] + (P->W[0] * r[1] - P->W[1] * r[0]);
        }
        collide_lat(cfg, &L, fin, ns, Bs, us, fo, dF);
        for (int i = 0; i < q; ++i) fpost[i * N + n] = fo[i];
        for (int k = 0; k < ns; ++k) {
          const or_pose *P = &poses[bid[k]];
          double r[3] = {xc[0] - P->X[0], xc[1] - P->X[1], xc[2] - P->X[2]};
          double *acc = &slab[((size_t)z * nb + bid[k]) * 6];
          const double *d = &dF[3 * k];
          acc[0] += d[0]; acc[1] += d[1]; acc[2] += d[2];
          acc[3] += r[1] * d[2] - r[2] * d[1];
          acc[4] += r[2] * d[0] - r[0] * d[2];
          acc[5] += r[0] * d[1] - r[1] * d[0];
        }
      }
  }
  if (ft) {
    for (int b = 0; b < nb * 6; ++b) ft[b] = 0.0;
    for (int z = 0; z < nz; ++z)
      for (int b = 0; b < nb; ++b)
        for (int m = 0; m < 6; ++m) ft[b * 6 + m] += slab[((size_t)z * nb + b) * 6 + m];
  }
  free(slab);
  if (err) return -3;
  const double cs2 = 1.0 / 3.0;
#pragma omp parallel for schedule(static)
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        long long n = x + (long long)nx * (y + (long long)ny * z);
        if (solid && solid[n]) continue;
        for (int k = 0; k < q; ++k) {
          long long src;
          {
            int s32;
            int kind = classify(cfg, x, y, z, &L.c[3 * k], &s32);
            src = s32;
            /* a source inside an obstacle cell: halfway bounce-back, the wall rule */
            if (kind == 0 && solid && solid[src]) kind = OR_WALL;
            double v;
            if (kind == 0) {
              v = fpost[k * N + src];
            } else if (kind == OR_WALL) {
              v = fpost[L.opp[k] * N + n];
            } else if (kind == OR_INLET) {
              double cu = L.c[3 * k] * cfg->u_in[0] + L.c[3 * k + 1] * cfg->u_in[1] + L.c[3 * k + 2] * cfg->u_in[2];
              v = fpost[L.opp[k] * N + n] + 2.0 * L.w[k] * cu / cs2;
            } else {
              v = fpost[k * N + n];
            }
            f[k * N + n] = v;
          }
        }
      }
  return 0;
}

int or_step(const or_config *cfg, double *f, double *fpost, int nb, const double *B,
            const or_pose *poses, double *ft) {
  return step_impl(cfg, f, fpost, nb, B, poses, ft, NULL);
}

/* Plain LBM with a static no-slip obstacle: the LBM variant of the paper's
 * node-level benchmark (section V, an LBM kernel plus the no-slip treatment of
 * a stationary geometry).  solid[n] != 0 marks obstacle cells; every link from
 * a fluid cell whose source is an obstacle cell takes halfway bounce-back,
 * f_k(y) = f*_{kbar}(y), the wall rule above; obstacle cells are not updated.
 * Needs cfg->psm == 0. */
int or_step_obstacle(const or_config *cfg, double *f, double *fpost, const unsigned char *solid) {
  if (cfg->psm) return -4;
  return step_impl(cfg, f, fpost, 0, NULL, NULL, NULL, solid);
}

/* density and (Guo-shifted) velocity u = (sum c f + F/2)/rho per cell */
void or_macro(const or_config *cfg, const double *f, double *rho, double *u) {
  lat_t L;
  if (lat_get(cfg->q, &L) != 0) return;
  const long long N = (long long)cfg->nx * cfg->ny * cfg->nz;
#pragma omp parallel for schedule(static)
  for (long long n = 0; n < N; ++n) {
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < L.q; ++i) {
      double v = f[i * N + n];
      r += v;
      for (int a = 0; a < 3; ++a) j[a] += L.c[3 * i + a] * v;
    }
    rho[n] = r;
    for (int a = 0; a < 3; ++a) u[3 * n + a] = (j[a] + 0.5 * cfg->force[a]) / r;
  }
}

/* total mass sum_x sum_i f_i, summed per z-slab then in z order */
double or_mass(const or_config *cfg, const double *f) {
  const long long N = (long long)cfg->nx * cfg->ny * cfg->nz;
  const long long plane = (long long)cfg->nx * cfg->ny;
  double *part = (double *)calloc((size_t)cfg->nz, sizeof(double));
#pragma omp parallel for schedule(static)
  for (int z = 0; z < cfg->nz; ++z) {
    double s = 0.0;
    for (int i = 0; i < cfg->q; ++i)
      for (long long n = z * plane; n < (z + 1) * plane; ++n) s += f[i * N + n];
    part[z] = s;
  }
  double m = 0.0;
  for (int z = 0; z < cfg->nz; ++z) m += part[z];
  free(part);
  return m;
}

/* ---------------------------------------------------------------------------
 * Geometry field and mapping (section III).
 *
 * The body-frame geometry lattice has spacing h = 2^-s LBM cells and cell
 * centres at (m + 1/2) h, m integer.  A geometry cell is "inside" when its
 * centre is inside the object.  Analytic shapes are tested exactly in
 * integer-valued FP64 arithmetic:
 *   ellipsoid (a,b,c): with C = 2m+1 (centre = C h/2),
 *     (Cx^2 b^2 c^2 + Cy^2 a^2 c^2) + Cz^2 a^2 b^2 < 4^(s+1) a^2 b^2 c^2
 *   cube (half side L): |C| < 2^(s+1) L on every axis.
 * ------------------------------------------------------------------------- */
int or_geom_inside(const or_geom *g, long long mx, long long my, long long mz) {
  if (g->kind == 0) {
    double Cx = (double)(2 * mx + 1), Cy = (double)(2 * my + 1), Cz = (double)(2 * mz + 1);
    double a2 = g->p[0] * g->p[0], b2 = g->p[1] * g->p[1], c2 = g->p[2] * g->p[2];
    double lhs = (Cx * Cx * (b2 * c2) + Cy * Cy * (a2 * c2)) + Cz * Cz * (a2 * b2);
    double rhs = ldexp(1.0, 2 * (g->s + 1)) * (a2 * b2 * c2);
    return lhs < rhs;
  }
  if (g->kind == 1) {
    double lim = ldexp(g->p[0], g->s + 1);
    return fabs((double)(2 * mx + 1)) < lim && fabs((double)(2 * my + 1)) < lim &&
           fabs((double)(2 * mz + 1)) < lim;
  }
  if (g->kind == 3) {
    const double h = ldexp(1.0, -g->s);
    double p[3] = {((double)mx + 0.5) * h, ((double)my + 0.5) * h, ((double)mz + 0.5) * h};
    if (p[0] * p[0] + p[1] * p[1] + p[2] * p[2] > g->r_bound * g->r_bound) return 0;
    return or_winding(g->verts, g->tris, g->nt, p) > 0.5;
  }
  long long jx = mx - g->mmin[0], jy = my - g->mmin[1], jz = mz - g->mmin[2];
  if (jx < 0 || jy < 0 || jz < 0 || jx >= g->dims[0] || jy >= g->dims[1] || jz >= g->dims[2]) return 0;
  return g->inside[jx + (long long)g->dims[0] * (jy + (long long)g->dims[1] * jz)] != 0;
}

/* floor(v / 2^32) for a signed 64-bit value */
static long long floor_div32(long long v) {
  const long long d = 4294967296LL;
  long long qv = v / d;
  if (v % d != 0 && v < 0) qv -= 1;
  return qv;
}

/* body-frame vector R^T v with the fixed FP64 order
 * p_a = fma(R[0][a], v0, fma(R[1][a], v1, R[2][a] * v2)) */
static void rt_mul(const double *R, const double *v, double *p) {
  for (int a = 0; a < 3; ++a) p[a] = fma(R[0 * 3 + a], v[0], fma(R[1 * 3 + a], v[1], R[2 * 3 + a] * v[2]));
}

/* Solid fraction eps of lab cell (ix,iy,iz) for one body (section III: the
 * cell's value is the mean over the geometry cells its sub-samples land in,
 * with the rotation folded into the lookup): each of the (2^s)^3 sub-sample points of the cell,
 * at offsets delta_k = (k + 1/2) h - 1/2 from the cell centre, is taken to the
 * body frame, p_k = R^T (x_c - X) + R^T delta_k, and looked up in the
 * geometry lattice cell that contains it.  Coordinates are measured in
 * sub-cell units in signed 64-bit fixed point with 32 fraction bits:
 *   P = rint(p * 2^(s+32)),  D_k = rint((R^T delta_k) * 2^(s+32)),
 *   m = floor((P + D_k) / 2^32).
 * eps = (#inside) / 8^s. */
double or_map_cell(const or_geom *g, const or_pose *pose, int ix, int iy, int iz) {
  const int s = g->s, n = 1 << s;
  double d[3] = {(ix + 0.5) - pose->X[0], (iy + 0.5) - pose->X[1], (iz + 0.5) - pose->X[2]};
  double p[3];
  rt_mul(pose->R, d, p);
  long long P[3];
  for (int a = 0; a < 3; ++a) P[a] = llrint(ldexp(p[a], s + 32));
  long long count = 0;
  for (int kz = 0; kz < n; ++kz)
    for (int ky = 0; ky < n; ++ky)
      for (int kx = 0; kx < n; ++kx) {
        double del[3] = {ldexp(2.0 * kx + 1.0, -(s + 1)) - 0.5, ldexp(2.0 * ky + 1.0, -(s + 1)) - 0.5,
                         ldexp(2.0 * kz + 1.0, -(s + 1)) - 0.5};
        double r[3];
        rt_mul(pose->R, del, r);
        long long m[3];
        for (int a = 0; a < 3; ++a) m[a] = floor_div32(P[a] + llrint(ldexp(r[a], s + 32)));
        count += or_geom_inside(g, m[0], m[1], m[2]);
      }
  return (double)count / (double)((long long)n * n * n);
}

/* Solid fraction eps of lab cell (ix,iy,iz) for one body, the other reading
 * of section III's mapping paragraph: only the cell centre is taken to the
 * body frame, and eps is the mean of the inside flags of the axis-aligned
 * (2^s)^3 block of geometry lattice cells nearest to the cell's extent there,
 * i.e. the block whose lower corner is the multiple of the sub-cell size
 * nearest to q - 2^(s-1) (q = the centre in sub-cell units):
 *   j0 = floor(q - 2^(s-1) + 1/2),  cells j0 .. j0 + 2^s - 1 per axis.
 * Same fixed point as or_map_cell: Q = rint(q * 2^32), so
 *   j0 = floor((Q - 2^(s+31) + 2^31) / 2^32).
 * At theta = 0 and for s = 0 this selects exactly the geometry cells of
 * or_map_cell's sub-samples; under rotation the block is a cube rotated
 * against the lab cell (larger per-cell error than or_map_cell). */
double or_map_cell_block(const or_geom *g, const or_pose *pose, int ix, int iy, int iz) {
  const int s = g->s, n = 1 << s;
  double d[3] = {(ix + 0.5) - pose->X[0], (iy + 0.5) - pose->X[1], (iz + 0.5) - pose->X[2]};
  double p[3];
  rt_mul(pose->R, d, p);
  long long j0[3];
  const long long half = 2147483648LL; /* 2^31 */
  const long long corner = (long long)1 << (s + 31);
  for (int a = 0; a < 3; ++a) j0[a] = floor_div32(llrint(ldexp(p[a], s + 32)) - corner + half);
  long long count = 0;
  for (int kz = 0; kz < n; ++kz)
    for (int ky = 0; ky < n; ++ky)
      for (int kx = 0; kx < n; ++kx) count += or_geom_inside(g, j0[0] + kx, j0[1] + ky, j0[2] + kz);
  return (double)count / (double)((long long)n * n * n);
}

/* B from eps: eq. (5) (b_form 0) or eq. (6) (b_form 1); stored as binary32 */
float or_b_from_eps(double eps, double tau, int b_form) {
  if (b_form == 0) return (float)eps;
  double th = tau - 0.5;
  double num = eps * th;
  double den = (1.0 - eps) + th;
  return (float)(num / den);
}

/* Dense B of one body; reading 0: or_map_cell (every sub-sample rotated),
 * reading 1: or_map_cell_block (centre rotated, axis-aligned block).  Cells
 * farther than r_bound + 2 from the body centre cannot see an inside geometry
 * cell (sub-samples lie within sqrt(3)/2 of the cell centre and a lattice
 * centre within sqrt(3)/2 h of the sample; a block's lattice centres lie
 * within sqrt(3) (1/2 + h/2) <= sqrt(3) of it for s >= 1) and get 0. */
int or_map(const or_config *cfg, const or_geom *g, const or_pose *pose, int b_form, int reading,
           double *B_out) {
  if (reading != 0 && reading != 1) return -1;
  const int nx = cfg->nx, ny = cfg->ny, nz = cfg->nz;
  const double rb = g->r_bound + 2.0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        long long n = x + (long long)nx * (y + (long long)ny * z);
        double dx = x + 0.5 - pose->X[0], dy = y + 0.5 - pose->X[1], dz = z + 0.5 - pose->X[2];
        if (dx * dx + dy * dy + dz * dz > rb * rb) {
          B_out[n] = 0.0;
          continue;
        }
        double eps = reading ? or_map_cell_block(g, pose, x, y, z) : or_map_cell(g, pose, x, y, z);
        B_out[n] = (double)or_b_from_eps(eps, cfg->tau, b_form);
      }
  return 0;
}

/* ---------------------------------------------------------------------------
 * Meshes: generalised winding number (sum of signed solid angles / 4 pi,
 * van Oosterom-Strackee formula per triangle), inside iff w > 1/2; volume by
 * the divergence theorem, V = 1/6 sum a.(b x c).
 * ------------------------------------------------------------------------- */
double or_winding(const double *v, const int *t, long long nt, const double p[3]) {
  double sum = 0.0;
  for (long long i = 0; i < nt; ++i) {
    double a[3], b[3], c[3];
    for (int k = 0; k < 3; ++k) {
      a[k] = v[3 * t[3 * i + 0] + k] - p[k];
      b[k] = v[3 * t[3 * i + 1] + k] - p[k];
      c[k] = v[3 * t[3 * i + 2] + k] - p[k];
    }
    double la = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    double lb = sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
    double lc = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    double det = a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
                 a[2] * (b[0] * c[1] - b[1] * c[0]);
    double ab = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
    double bc = b[0] * c[0] + b[1] * c[1] + b[2] * c[2];
    double ca = c[0] * a[0] + c[1] * a[1] + c[2] * a[2];
    double den = la * lb * lc + ab * lc + bc * la + ca * lb;
    sum += 2.0 * atan2(det, den);
  }
  return sum / (4.0 * M_PI);
}

int or_voxelize(const double *v, const int *t, long long nt, int s, const int mmin[3],
                const int dims[3], unsigned char *out) {
  const double h = ldexp(1.0, -s);
  const long long total = (long long)dims[0] * dims[1] * dims[2];
#pragma omp parallel for schedule(dynamic, 64)
  for (long long idx = 0; idx < total; ++idx) {
    long long jx = idx % dims[0], jy = (idx / dims[0]) % dims[1], jz = idx / ((long long)dims[0] * dims[1]);
    double p[3] = {((double)(mmin[0] + jx) + 0.5) * h, ((double)(mmin[1] + jy) + 0.5) * h,
                   ((double)(mmin[2] + jz) + 0.5) * h};
    out[idx] = or_winding(v, t, nt, p) > 0.5 ? 1 : 0;
  }
  return 0;
}

double or_mesh_volume(const double *v, const int *t, long long nt) {
  double s = 0.0;
  for (long long i = 0; i < nt; ++i) {
    const double *a = &v[3 * t[3 * i]], *b = &v[3 * t[3 * i + 1]], *c = &v[3 * t[3 * i + 2]];
    s += a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
         a[2] * (b[0] * c[1] - b[1] * c[0]);
  }
  return s / 6.0;
}

/* ---------------------------------------------------------------------------
 * One step of one cell, for sampled checks on domains too large for or_step:
 * the same update as or_step restricted to the cell (x,y,z).  nbr holds the
 * pre-step f of the 3x3x3 neighbourhood, nbr[(((dz+1)*3 + (dy+1))*3 + (dx+1))*q
 * + i] for the cell at (x+dx, y+dy, z+dz) (periodic axes wrapped); entries of
 * cells outside the domain are not read.  Bn[j*nb + b] is B of body b at
 * neighbour j (same order).  out[i] = f_i(x, t+1).
 * ------------------------------------------------------------------------- */
int or_update_cell(const or_config *cfg, int x, int y, int z, const double *nbr, int nb, const double *Bn,
                   const or_pose *poses, double *out) {
  lat_t L;
  if (lat_get(cfg->q, &L) != 0) return -1;
  const int q = L.q;
  const int n3[3] = {cfg->nx, cfg->ny, cfg->nz};
  double post[27][OR_MAXQ];
  int done[27] = {0};
  const double cs2 = 1.0 / 3.0;
  for (int k = 0; k < q; ++k) {
    int s32;
    int kind = classify(cfg, x, y, z, &L.c[3 * k], &s32);
    int j, dir;
    if (kind == 0) {
      j = ((-L.c[3 * k + 2] + 1) * 3 + (-L.c[3 * k + 1] + 1)) * 3 + (-L.c[3 * k] + 1);
      dir = k;
    } else {
      j = 13;
      dir = (kind == OR_OUTLET) ? k : L.opp[k];
    }
    if (!done[j]) {
      int d[3] = {j % 3 - 1, (j / 3) % 3 - 1, j / 9 - 1};
      int p[3] = {x + d[0], y + d[1], z + d[2]};
      for (int a = 0; a < 3; ++a) p[a] = (p[a] + n3[a]) % n3[a];
      double Bs[2], us[6], dF[6];
      int ns = 0;
      if (cfg->psm)
        for (int b = 0; b < nb; ++b) {
          double v = Bn[j * nb + b];
          if (v != 0.0) {
            if (ns == 2) return -3;
            const or_pose *P = &poses[b];
            double r[3] = {p[0] + 0.5 - P->X[0], p[1] + 0.5 - P->X[1], p[2] + 0.5 - P->X[2]};
            us[3 * ns + 0] = P->V[0] + (P->W[1] * r[2] - P->W[2] * r[1]);
            us[3 * ns + 1] = P->V[1] + (P->W[2] * r[0] - P->W[0] * r[2]);
            us[3 * ns + 2] = P->V[2] + (P->W[0] * r[1] - P->W[1] * r[0]);
            Bs[ns++] = v;
          }
        }
      collide_lat(cfg, &L, nbr + (size_t)j * q, ns, Bs, us, post[j], dF);
      done[j] = 1;
    }
    double v = post[j][dir];
    if (kind == OR_INLET) {
      double cu = L.c[3 * k] * cfg->u_in[0] + L.c[3 * k + 1] * cfg->u_in[1] + L.c[3 * k + 2] * cfg->u_in[2];
      v += 2.0 * L.w[k] * cu / cs2;
    }
    out[k] = v;
  }
  return 0;
}

/* ---------------------------------------------------------------------------
 * Discrete adjoint of one step for the torque objective
 *   J_t = wt * a . T_0(t)  (torque of body 0 about X, eq. (11), body side)
 * with frozen solid fractions.  Independent of any hand-derived Jacobian:
 * every per-cell derivative is obtained by complex-step differentiation of the
 * collision above, re-evaluated in complex arithmetic (step 1e-30, exact to
 * rounding), and the transposed streaming is the literal scatter of the pull
 * rules of or_step.
 * ------------------------------------------------------------------------- */
typedef double complex zc;

static void feq_z(const lat_t *L, zc rho, const zc u[3], zc *feq) {
  const double cs2 = 1.0 / 3.0;
  zc uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < L->q; ++i) {
    zc cu = L->c[3 * i] * u[0] + L->c[3 * i + 1] * u[1] + L->c[3 * i + 2] * u[2];
    feq[i] = L->w[i] * rho * (1.0 + cu / cs2 + cu * cu / (2.0 * cs2 * cs2) - uu / (2.0 * cs2));
  }
}

/* the collision of collide_lat for one body slot, in complex arithmetic */
static void collide_z(const or_config *cfg, const lat_t *L, const zc *fin, zc B, const zc us[3], zc *fout,
                      zc dF[3]) {
  const int q = L->q;
  const double cs2 = 1.0 / 3.0;
  zc rho = 0.0, j[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < q; ++i) {
    rho += fin[i];
    for (int a = 0; a < 3; ++a) j[a] += L->c[3 * i + a] * fin[i];
  }
  zc u[3];
  for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * cfg->force[a]) / rho;
  zc feq[OR_MAXQ], S[OR_MAXQ], OmF[OR_MAXQ], feqs[OR_MAXQ];
  feq_z(L, rho, u, feq);
  for (int i = 0; i < q; ++i) {
    zc cu = 0.0, uF = 0.0;
    double cF = 0.0;
    for (int a = 0; a < 3; ++a) {
      cu += L->c[3 * i + a] * u[a];
      cF += L->c[3 * i + a] * cfg->force[a];
      uF += u[a] * cfg->force[a];
    }
    S[i] = L->w[i] * ((cF - uF) / cs2 + cu * cF / (cs2 * cs2));
  }
  double le = 1.0 / cfg->tau;
  double lo = 1.0 / (0.5 + cfg->magic / (cfg->tau - 0.5));
  for (int i = 0; i < q; ++i) {
    int k = L->opp[i];
    zc fp = 0.5 * (fin[i] + fin[k]), fm = 0.5 * (fin[i] - fin[k]);
    zc ep = 0.5 * (feq[i] + feq[k]), em = 0.5 * (feq[i] - feq[k]);
    zc sp = 0.5 * (S[i] + S[k]), sm = 0.5 * (S[i] - S[k]);
    OmF[i] = -le * (fp - ep) - lo * (fm - em) + (1.0 - 0.5 * le) * sp + (1.0 - 0.5 * lo) * sm;
  }
  feq_z(L, rho, us, feqs);
  zc mom[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < q; ++i) {
    int ib = L->opp[i];
    zc om;
    if (cfg->sc == 1)
      om = (fin[ib] - feq[ib]) - (fin[i] - feqs[i]);
    else if (cfg->sc == 2)
      om = (feqs[i] - fin[i]) + (1.0 - 1.0 / cfg->tau) * (fin[i] - feqs[i]);
    else
      om = (fin[ib] - feqs[ib]) - (fin[i] - feqs[i]);
    fout[i] = fin[i] + (1.0 - B) * OmF[i] + B * om;
    for (int a = 0; a < 3; ++a) mom[a] += L->c[3 * i + a] * om;
  }
  for (int a = 0; a < 3; ++a) dF[a] = -B * mom[a];
}

int or_adjoint_step(const or_config *cfg, const double *f, const double *ghat_next, double *ghat, const double *B,
                    const or_pose *pose, const double *axis, double wt, double *dJdB, double *dJdW) {
  lat_t L;
  if (lat_get(cfg->q, &L) != 0) return -1;
  const int q = L.q, nx = cfg->nx, ny = cfg->ny, nz = cfg->nz;
  const long long N = (long long)nx * ny * nz;
  /* adjoint of the post-collision values: scatter of the pull rules */
  double *gpost = (double *)calloc((size_t)q * N, sizeof(double));
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        long long n = x + (long long)nx * (y + (long long)ny * z);
        for (int k = 0; k < q; ++k) {
          int s32;
          int kind = classify(cfg, x, y, z, &L.c[3 * k], &s32);
          double g = ghat_next[k * N + n];
          if (kind == 0) gpost[k * N + s32] += g;
          else if (kind == OR_WALL || kind == OR_INLET) gpost[L.opp[k] * N + n] += g;
          else gpost[k * N + n] += g;
        }
      }
  const double h = 1e-30;
  double *slab = (double *)calloc((size_t)nz, sizeof(double));
#pragma omp parallel for schedule(static)
  for (int z = 0; z < nz; ++z) {
    double acc = 0.0;
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        long long n = x + (long long)nx * (y + (long long)ny * z);
        double r[3] = {x + 0.5 - pose->X[0], y + 0.5 - pose->X[1], z + 0.5 - pose->X[2]};
        double us[3] = {pose->V[0] + (pose->W[1] * r[2] - pose->W[2] * r[1]),
                        pose->V[1] + (pose->W[2] * r[0] - pose->W[0] * r[2]),
                        pose->V[2] + (pose->W[0] * r[1] - pose->W[1] * r[0])};
        double axr[3] = {axis[1] * r[2] - axis[2] * r[1], axis[2] * r[0] - axis[0] * r[2],
                         axis[0] * r[1] - axis[1] * r[0]};
        zc fin[OR_MAXQ], fo[OR_MAXQ], usz[3], dF[3];
        /* d(objective contribution)/d(parameter) for a perturbed evaluation:
         * sum_i gpost_i Im(f*_i)/h + wt * Im(a . (r x dF))/h */
        for (int j = -2; j < q; ++j) {
          for (int i = 0; i < q; ++i) fin[i] = f[i * N + n];
          for (int a = 0; a < 3; ++a) usz[a] = us[a];
          zc Bz = B[n];
          if (j >= 0) fin[j] += I * h;
          else if (j == -1) Bz += I * h;
          else
            for (int a = 0; a < 3; ++a) usz[a] += I * h * axr[a];
          collide_z(cfg, &L, fin, Bz, usz, fo, dF);
          double d = 0.0;
          for (int i = 0; i < q; ++i) d += gpost[i * N + n] * cimag(fo[i]) / h;
          zc tq = axis[0] * (r[1] * dF[2] - r[2] * dF[1]) + axis[1] * (r[2] * dF[0] - r[0] * dF[2]) +
                  axis[2] * (r[0] * dF[1] - r[1] * dF[0]);
          d += wt * cimag(tq) / h;
          if (j >= 0) ghat[j * N + n] = d;
          else if (j == -1) dJdB[n] += d;
          else acc += d;
        }
      }
    slab[z] = acc;
  }
  for (int z = 0; z < nz; ++z) *dJdW += slab[z];
  free(slab);
  free(gpost);
  return 0;
}

/* Thread count of the parallel loops (for timing the oracle on one core or
 * on all of them); or_threads returns the count the loops will use. */
void or_set_threads(int n) {
  if (n > 0) omp_set_num_threads(n);
}

int or_threads(void) { return omp_get_max_threads(); }
