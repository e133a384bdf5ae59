/*
 * dmr_oracle.c -- FP64 CPU oracle (test infrastructure only; see oracle.h).
 *
 * Plain loops, one array per quantity, no blocking or fusion.  Every
 * function names the part of the paper it follows.  Where the paper is
 * silent the reading used is stated at the function.  Loops whose
 * iterations update distinct entities from values no iteration writes are
 * marked for OpenMP worker threads; each entity is computed by the same
 * operations whatever the thread count, so results are bit-identical.
 *
 * Storage (private to this file): column-major in the sense a[i][j] with j
 * fastest; Hz[nx][ny], Ex[nx][ny+1], Ey[nx+1][ny], nodes [nx+1][ny+1].
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* CODATA 2018 SI constants (the paper prints none). */
static const double Q_E = 1.602176634e-19;
static const double M_E = 9.1093837015e-31;
static const double K_B = 1.380649e-23; /* J/K */
static const double EPS_0 = 8.8541878128e-12;
static const double C_0 = 299792458.0;
static const double PI_ = 3.14159265358979323846;

#define NRING 8 /* blocks per period in the E_rms window */

typedef struct {
  int nx, ny;
  double dx, dt;
  int spp, spb; /* steps per period, steps per window block */
  /* update coefficients */
  double ch, ce, a, b, kn, cmur;
  double *hz, *ex, *ey, *jx, *jy, *n, *acc, *ring;
} level_t;

struct orc_sim {
  orc_params p;
  double omega, lambda, nu_m, n_c, eeff_fac, e0, d_e, d_a, n_amb, ktil, eta0;
  double nu_att; /* nu_m*A*(E_cr/p)^beta */
  level_t L0, L1;
  int has_patch;
  int ext[4]; /* I0, J0, I1, J1 base cells */
  int64_t step;
  int64_t blocks; /* window blocks closed so far */
  /* hz_lo, hz_hi: fine Hz after substeps r/2 and r/2 + 1, the two half
   * levels that bracket coarse n+1/2 (for r = 2, hz_hi is the final Hz) */
  double *ex_old, *ey_old, *hz_prev, *hz_lo, *hz_hi;
  int NBx, NBy;
  uint8_t *bflag;
  int32_t *bscan, *blist, bcount;
  /* ORC_RULE_UNION: active blocks [NBy][NBx]; the fine level L1 then spans
   * the whole domain at r times the resolution */
  uint8_t *act;
};

/* ---- indexing ---------------------------------------------------------- */
#define HZ(L, i, j) ((L)->hz[(size_t)(i) * (L)->ny + (j)])
#define EX(L, i, j) ((L)->ex[(size_t)(i) * ((L)->ny + 1) + (j)])
#define JX(L, i, j) ((L)->jx[(size_t)(i) * ((L)->ny + 1) + (j)])
#define EY(L, i, j) ((L)->ey[(size_t)(i) * (L)->ny + (j)])
#define JY(L, i, j) ((L)->jy[(size_t)(i) * (L)->ny + (j)])
#define NODE(L, arr, i, j) ((L)->arr[(size_t)(i) * ((L)->ny + 1) + (j)])
#define RING(L, s, i, j)                                                       \
  ((L)->ring[(size_t)(s) * ((L)->nx + 1) * ((L)->ny + 1) +                    \
             (size_t)(i) * ((L)->ny + 1) + (j)])

static size_t n_hz(const level_t *L) { return (size_t)L->nx * L->ny; }
static size_t n_ex(const level_t *L) { return (size_t)L->nx * (L->ny + 1); }
static size_t n_ey(const level_t *L) { return (size_t)(L->nx + 1) * L->ny; }
static size_t n_nd(const level_t *L) { return (size_t)(L->nx + 1) * (L->ny + 1); }

/* ---- derived scalars (Sec. II.A, Sec. III.A, Sec. IV.D) ---------------- */
static double mu0(void) { return 1.0 / (EPS_0 * C_0 * C_0); }

static void derive(orc_sim *s) {
  const orc_params *p = &s->p;
  s->omega = 2.0 * PI_ * p->freq_hz;
  s->lambda = C_0 / p->freq_hz;
  /* collision frequency for air, Sec. II.A: nu_m = 5.3e9 p[Torr] */
  s->nu_m = 5.3e9 * p->p_torr;
  /* critical density m eps0 omega^2 / e^2 (Sec. III.A prints it without
   * the square; the cutoff value of Sec. IV.D fixes the square) */
  s->n_c = M_E * EPS_0 * s->omega * s->omega / (Q_E * Q_E);
  /* effective field: E_eff^2 = E_rms^2 / (1 + omega^2/nu_m^2) */
  s->eeff_fac = 1.0 / (1.0 + (s->omega * s->omega) / (s->nu_m * s->nu_m));
  /* breakdown: incident rms field at which E_eff equals E_cr(p) */
  {
    double e_cr = p->ecr_over_p * 100.0 * p->p_torr; /* V/m */
    double e_bd = e_cr / sqrt(s->eeff_fac);
    double e_rms = p->erms_over_ebd * e_bd;
    s->e0 = sqrt(2.0) * e_rms; /* peak amplitude */
  }
  /* free diffusion D_e = e T_e / (m nu_m); ambipolar D_a = mu_i (T_e+T_i) */
  s->d_e = Q_E * p->te_ev / (M_E * s->nu_m);
  s->d_a = p->mu_i_760 * (760.0 / p->p_torr) * (p->te_ev + p->ti_ev);
  /* alpha = (L / lambda_D)^2 = n / n_amb */
  s->n_amb = EPS_0 * p->te_ev / (Q_E * p->L_amb * p->L_amb);
  s->nu_att = s->nu_m * p->A_ion * pow(p->ecr_over_p, p->beta_ion);
  s->eta0 = mu0() * C_0;
}

static int level_init(level_t *L, int nx, int ny, double dx, double dt,
                      int spp, double nu_m, double S) {
  memset(L, 0, sizeof(*L));
  L->nx = nx;
  L->ny = ny;
  L->dx = dx;
  L->dt = dt;
  L->spp = spp;
  L->spb = spp / NRING;
  L->ch = dt / (mu0() * dx);
  L->ce = dt / EPS_0;
  /* exponential integrator of dJ/dt = -nu_m J + (e^2 n / m) E over one step
   * with E taken as the mean of its end values */
  L->a = exp(-nu_m * dt);
  L->b = Q_E * Q_E * (1.0 - L->a) / (M_E * nu_m);
  L->kn = dt * L->b / (4.0 * EPS_0);
  /* first-order Mur coefficient */
  L->cmur = (S - 1.0) / (S + 1.0);
  L->hz = calloc(n_hz(L), sizeof(double));
  L->ex = calloc(n_ex(L), sizeof(double));
  L->jx = calloc(n_ex(L), sizeof(double));
  L->ey = calloc(n_ey(L), sizeof(double));
  L->jy = calloc(n_ey(L), sizeof(double));
  L->n = calloc(n_nd(L), sizeof(double));
  L->acc = calloc(n_nd(L), sizeof(double));
  L->ring = calloc(n_nd(L) * NRING, sizeof(double));
  if (!L->hz || !L->ex || !L->jx || !L->ey || !L->jy || !L->n || !L->acc ||
      !L->ring)
    return -2;
  return 0;
}

static void level_free(level_t *L) {
  free(L->hz);
  free(L->ex);
  free(L->jx);
  free(L->ey);
  free(L->jy);
  free(L->n);
  free(L->acc);
  free(L->ring);
  memset(L, 0, sizeof(*L));
}

/* ---- incident plane wave (Sec. II.B: Ey-polarised, k along x, from the
 * left), as an exact 1-D Yee solution after a sin^2 ramp ------------------ */
static double ramp(const orc_sim *s, double tau) {
  double tr = s->p.ramp_periods / s->p.freq_hz;
  if (tau <= 0.0) return 0.0;
  if (tau >= tr) return 1.0;
  double sn = sin(0.5 * PI_ * tau / tr);
  return sn * sn;
}

static double ey_inc(const orc_sim *s, double x, double t) {
  return s->e0 * ramp(s, t - x / C_0) * sin(s->omega * t - s->ktil * x);
}

static double hz_inc(const orc_sim *s, double x, double t) {
  return ey_inc(s, x, t) / s->eta0;
}

/* ---- Eqs. (1) and (3): one edge of the coupled E-J update -------------- */
/* E^{n+1}(1+k) = (1-k)E^n + (dt/eps0)(curl H - (1+a)J^n/2),
 * J^{n+1} = a J^n + (b n_e / 2)(E^n + E^{n+1}),  k = dt b n_e / (4 eps0).   */
static void ej_edge(const level_t *L, double *e, double *j, double curl,
                    double ne) {
  double kap = L->kn * ne;
  double en = ((1.0 - kap) * (*e) + L->ce * (curl - 0.5 * (1.0 + L->a) * (*j))) /
              (1.0 + kap);
  *j = L->a * (*j) + 0.5 * L->b * ne * (*e + en);
  *e = en;
}

static void j_only(const level_t *L, double *j, double eo, double en,
                   double ne) {
  *j = L->a * (*j) + 0.5 * L->b * ne * (eo + en);
}

/* squared field at a node: mean of the squares of the edges that exist on
 * each axis (the one-period average of Sec. II.A is taken of these) */
static double node_e2(const level_t *L, int i, int j, int perx, int pery) {
  double sx = 0.0, sy = 0.0;
  int cx = 0, cy = 0;
  if (i > 0) {
    sx += EX(L, i - 1, j) * EX(L, i - 1, j);
    cx++;
  } else if (perx) {
    sx += EX(L, L->nx - 1, j) * EX(L, L->nx - 1, j);
    cx++;
  }
  if (i < L->nx) {
    sx += EX(L, i, j) * EX(L, i, j);
    cx++;
  }
  if (j > 0) {
    sy += EY(L, i, j - 1) * EY(L, i, j - 1);
    cy++;
  } else if (pery) {
    sy += EY(L, i, L->ny - 1) * EY(L, i, L->ny - 1);
    cy++;
  }
  if (j < L->ny) {
    sy += EY(L, i, j) * EY(L, i, j);
    cy++;
  }
  return (cx ? sx / cx : 0.0) + (cy ? sy / cy : 0.0);
}

static void accumulate(level_t *L, int perx, int pery) {
  #pragma omp parallel for schedule(static)
  for (int i = 0; i <= L->nx; i++)
    for (int j = 0; j <= L->ny; j++) {
      if ((perx && i == L->nx) || (pery && j == L->ny)) continue;
      NODE(L, acc, i, j) += node_e2(L, i, j, perx, pery);
    }
  if (perx)
    for (int j = 0; j <= L->ny; j++) NODE(L, acc, L->nx, j) = NODE(L, acc, 0, j);
  if (pery)
    for (int i = 0; i <= L->nx; i++) NODE(L, acc, i, L->ny) = NODE(L, acc, i, 0);
}

/* ---- one EM step of the base (coarse or uniform) level, Eqs. (1)-(3),
 * total-field/scattered-field source, outer boundary ---------------------- */
static void em_step_base(orc_sim *s) {
  level_t *L = &s->L0;
  const int nx = L->nx, ny = L->ny;
  const int perx = s->p.bc_x == ORC_BC_PERIODIC;
  const int pery = s->p.bc_y == ORC_BC_PERIODIC;
  const int is = s->p.tfsf_i;
  const double t = (double)s->step * L->dt;
  const double xs = is * L->dx;

  /* E^n and Hz^{n-1/2} are kept: Mur needs E^n, the coarse/fine transfer
   * needs the old coarse E, a regrid extrapolates Hz in time */
  memcpy(s->ex_old, L->ex, n_ex(L) * sizeof(double));
  memcpy(s->ey_old, L->ey, n_ey(L) * sizeof(double));
  memcpy(s->hz_prev, L->hz, n_hz(L) * sizeof(double));

  /* Faraday, Eq. (2): dHz/dt = -(dEy/dx - dEx/dy)/mu0 */
  #pragma omp parallel for schedule(static)
  for (int i = 0; i < nx; i++)
    for (int j = 0; j < ny; j++)
      HZ(L, i, j) -= L->ch * ((EY(L, i + 1, j) - EY(L, i, j)) -
                              (EX(L, i, j + 1) - EX(L, i, j)));
  if (is > 0) /* scattered-field cells left of the source line */
    for (int j = 0; j < ny; j++) HZ(L, is - 1, j) += L->ch * ey_inc(s, xs, t);

  /* Ampere with current, Eq. (1), and Drude current, Eq. (3) */
  #pragma omp parallel for schedule(static)
  for (int i = 0; i < nx; i++)
    for (int j = (pery ? 0 : 1); j < ny; j++) {
      int jm = j > 0 ? j - 1 : ny - 1;
      double curl = (HZ(L, i, j) - HZ(L, i, jm)) / L->dx;
      double ne = 0.5 * (NODE(L, n, i, j) + NODE(L, n, i + 1, j));
      ej_edge(L, &EX(L, i, j), &JX(L, i, j), curl, ne);
    }
  #pragma omp parallel for schedule(static)
  for (int i = (perx ? 0 : 1); i < nx; i++)
    for (int j = 0; j < ny; j++) {
      int im = i > 0 ? i - 1 : nx - 1;
      double curl = -(HZ(L, i, j) - HZ(L, im, j)) / L->dx;
      if (is > 0 && i == is) /* total-field edge next to the source line */
        curl += hz_inc(s, xs - 0.5 * L->dx, t + 0.5 * L->dt) / L->dx;
      double ne = 0.5 * (NODE(L, n, i, j) + NODE(L, n, i, j + 1));
      ej_edge(L, &EY(L, i, j), &JY(L, i, j), curl, ne);
    }

  /* outer boundary on the tangential edges */
  if (perx) {
    for (int j = 0; j < ny; j++) {
      EY(L, nx, j) = EY(L, 0, j);
      JY(L, nx, j) = JY(L, 0, j);
    }
  } else {
    for (int j = 0; j < ny; j++) {
      const int ib[2] = {0, nx}, in[2] = {1, nx - 1};
      for (int k = 0; k < 2; k++) {
        int i = ib[k];
        double eo = s->ey_old[(size_t)i * ny + j];
        double en = 0.0;
        if (s->p.bc_x == ORC_BC_MUR) /* first-order Mur */
          en = s->ey_old[(size_t)in[k] * ny + j] +
               L->cmur * (EY(L, in[k], j) - eo);
        double ne = 0.5 * (NODE(L, n, i, j) + NODE(L, n, i, j + 1));
        j_only(L, &JY(L, i, j), eo, en, ne);
        EY(L, i, j) = en;
      }
    }
  }
  if (pery) {
    for (int i = 0; i < nx; i++) {
      EX(L, i, ny) = EX(L, i, 0);
      JX(L, i, ny) = JX(L, i, 0);
    }
  } else {
    for (int i = 0; i < nx; i++) {
      const int jb[2] = {0, ny}, jn[2] = {1, ny - 1};
      for (int k = 0; k < 2; k++) {
        int j = jb[k];
        double eo = s->ex_old[(size_t)i * (ny + 1) + j];
        double en = 0.0;
        if (s->p.bc_y == ORC_BC_MUR)
          en = s->ex_old[(size_t)i * (ny + 1) + jn[k]] +
               L->cmur * (EX(L, i, jn[k]) - eo);
        double ne = 0.5 * (NODE(L, n, i, j) + NODE(L, n, i + 1, j));
        j_only(L, &JX(L, i, j), eo, en, ne);
        EX(L, i, j) = en;
      }
    }
  }
  accumulate(L, perx, pery);
}

/* ---- coarse -> fine transfer on the coarse/fine boundary, Eq. (5b) ------ */
/* linear in time between the old and new coarse values (frac), linear in
 * space along the boundary line; coarse Ey lies at j+1/2, coarse Ex at i+1/2.
 * A fine y-edge at global fine row Q sits at coarse y-index (Q+1/2)/r - 1/2
 * (r = 2: Q/2 - 1/4; the offsets 1/(2r) of Fig. 5(c)). */
static double cfb_ey(const orc_sim *s, int I, int Q, double frac) {
  const level_t *C = &s->L0;
  double v = (Q + 0.5) / s->p.r - 0.5;
  int j = (int)floor(v);
  double xp = v - j;
  double o = (1.0 - xp) * s->ey_old[(size_t)I * C->ny + j] +
             xp * s->ey_old[(size_t)I * C->ny + j + 1];
  double nw = (1.0 - xp) * EY(C, I, j) + xp * EY(C, I, j + 1);
  return (1.0 - frac) * o + frac * nw;
}

static double cfb_ex(const orc_sim *s, int P, int J, double frac) {
  const level_t *C = &s->L0;
  double u = (P + 0.5) / s->p.r - 0.5;
  int i = (int)floor(u);
  double xp = u - i;
  double o = (1.0 - xp) * s->ex_old[(size_t)i * (C->ny + 1) + J] +
             xp * s->ex_old[(size_t)(i + 1) * (C->ny + 1) + J];
  double nw = (1.0 - xp) * EX(C, i, J) + xp * EX(C, i + 1, J);
  return (1.0 - frac) * o + frac * nw;
}

/* ---- Eq. (5b) on every coarse/fine boundary edge of the fine level ------
 * The tangential fine E on the boundary comes from the coarse mesh (cfb_ey,
 * cfb_ex); the boundary current follows Eq. (3) with that field.  Boundary
 * edges: the patch sides (Ey on its left and right columns, Ex on its bottom
 * and top rows); for the union of blocks, every level edge with an active
 * cell on one side only (these lie on block lines, so on coarse lines).
 * out_ex == NULL drives the edges; otherwise the Eq. (5b) values are only
 * stored into out_ex / out_ey (level-1 internal layout) and nothing changes. */
static int ex_has(const orc_sim *s, int P, int Q);
static int ey_has(const orc_sim *s, int P, int Q);
static int ex_inner(const orc_sim *s, int P, int Q);
static int ey_inner(const orc_sim *s, int P, int Q);

static void cfb_edge(level_t *F, double *e, double *j, double en, double ne,
                     double *out) {
  if (out) {
    *out = en;
    return;
  }
  j_only(F, j, *e, en, ne);
  *e = en;
}

static void cfb_edges(orc_sim *s, double frac, double *out_ex, double *out_ey) {
  level_t *F = &s->L1;
  const int fw = F->nx, fh = F->ny, r = s->p.r;
  if (s->act) {
    #pragma omp parallel for schedule(static)
    for (int i = 0; i <= fw; i++)
      for (int j = 0; j < fh; j++) {
        if (!ey_has(s, i, j) || ey_inner(s, i, j)) continue;
        double ne = 0.5 * (NODE(F, n, i, j) + NODE(F, n, i, j + 1));
        cfb_edge(F, &EY(F, i, j), &JY(F, i, j), cfb_ey(s, i / r, j, frac), ne,
                 out_ey ? &out_ey[(size_t)i * fh + j] : NULL);
      }
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < fw; i++)
      for (int j = 0; j <= fh; j++) {
        if (!ex_has(s, i, j) || ex_inner(s, i, j)) continue;
        double ne = 0.5 * (NODE(F, n, i, j) + NODE(F, n, i + 1, j));
        cfb_edge(F, &EX(F, i, j), &JX(F, i, j), cfb_ex(s, i, j / r, frac), ne,
                 out_ex ? &out_ex[(size_t)i * (fh + 1) + j] : NULL);
      }
    return;
  }
  const int P0 = s->ext[0] * r, Q0 = s->ext[1] * r;
  for (int j = 0; j < fh; j++) {
    const int ib[2] = {0, fw}, Ic[2] = {s->ext[0], s->ext[2]};
    for (int k = 0; k < 2; k++) {
      int i = ib[k];
      double ne = 0.5 * (NODE(F, n, i, j) + NODE(F, n, i, j + 1));
      cfb_edge(F, &EY(F, i, j), &JY(F, i, j), cfb_ey(s, Ic[k], Q0 + j, frac), ne,
               out_ey ? &out_ey[(size_t)i * fh + j] : NULL);
    }
  }
  for (int i = 0; i < fw; i++) {
    const int jb[2] = {0, fh}, Jc[2] = {s->ext[1], s->ext[3]};
    for (int k = 0; k < 2; k++) {
      int j = jb[k];
      double ne = 0.5 * (NODE(F, n, i, j) + NODE(F, n, i + 1, j));
      cfb_edge(F, &EX(F, i, j), &JX(F, i, j), cfb_ex(s, P0 + i, Jc[k], frac), ne,
               out_ex ? &out_ex[(size_t)i * (fh + 1) + j] : NULL);
    }
  }
}

/* ---- weak fourth-order hyper-diffusion of the fine interior E ----------
 * E <- E - gamma L(L(E)), L the 5-point Laplacian of each component on its
 * own grid, entries outside the patch replaced by the entry itself (zero
 * normal difference).  Boundary (coarse-driven) edges are not changed.
 * The paper does not describe how its interface is stabilised; without this
 * term modes finer than the coarse grid can resolve grow slowly inside the
 * patch (doubling every few tens of periods).  gamma = 1e-3 keeps every
 * patch shape tried stable (1e-4 is not enough for patches 16 coarse cells
 * across: the growth returns after some hundred periods) and damps a
 * wavelength of 64 fine cells by ~1e-7 per substep. */
static void lap_grid(const double *a, double *out, int ni, int nj) {
  #pragma omp parallel for schedule(static)
  for (int i = 0; i < ni; i++)
    for (int j = 0; j < nj; j++) {
      double c = a[(size_t)i * nj + j];
      double l = i > 0 ? a[(size_t)(i - 1) * nj + j] : c;
      double r = i < ni - 1 ? a[(size_t)(i + 1) * nj + j] : c;
      double d = j > 0 ? a[(size_t)i * nj + j - 1] : c;
      double u = j < nj - 1 ? a[(size_t)i * nj + j + 1] : c;
      out[(size_t)i * nj + j] = l + r + d + u - 4.0 * c;
    }
}

static void fine_filter(orc_sim *s) {
  level_t *F = &s->L1;
  const double g = s->p.fine_filter;
  if (g <= 0.0) return;
  const int fw = F->nx, fh = F->ny;
  size_t nx_ = n_ex(F), ny_ = n_ey(F);
  size_t nmax = nx_ > ny_ ? nx_ : ny_;
  double *t1 = malloc(nmax * sizeof(double)), *t2 = malloc(nmax * sizeof(double));
  /* Ex grid: fw x (fh+1), interior rows 1..fh-1 */
  lap_grid(F->ex, t1, fw, fh + 1);
  lap_grid(t1, t2, fw, fh + 1);
  #pragma omp parallel for schedule(static)
  for (int i = 0; i < fw; i++)
    for (int j = 1; j < fh; j++) EX(F, i, j) -= g * t2[(size_t)i * (fh + 1) + j];
  /* Ey grid: (fw+1) x fh, interior columns 1..fw-1 */
  lap_grid(F->ey, t1, fw + 1, fh);
  lap_grid(t1, t2, fw + 1, fh);
  #pragma omp parallel for schedule(static)
  for (int i = 1; i < fw; i++)
    for (int j = 0; j < fh; j++) EY(F, i, j) -= g * t2[(size_t)i * fh + j];
  free(t1);
  free(t2);
}

/* ---- one fine substep m (1..r) on the patch, Sec. III.C ---------------- */
static void em_step_fine(orc_sim *s, int m) {
  level_t *F = &s->L1;
  const int fw = F->nx, fh = F->ny;
  const double frac = (double)m / s->p.r;

  fine_filter(s);

  #pragma omp parallel for schedule(static)
  for (int i = 0; i < fw; i++)
    for (int j = 0; j < fh; j++)
      HZ(F, i, j) -= F->ch * ((EY(F, i + 1, j) - EY(F, i, j)) -
                              (EX(F, i, j + 1) - EX(F, i, j)));
  if (m == s->p.r / 2) memcpy(s->hz_lo, F->hz, n_hz(F) * sizeof(double));
  if (m == s->p.r / 2 + 1 && m < s->p.r)
    memcpy(s->hz_hi, F->hz, n_hz(F) * sizeof(double));

  #pragma omp parallel for schedule(static)
  for (int i = 0; i < fw; i++)
    for (int j = 1; j < fh; j++) {
      double curl = (HZ(F, i, j) - HZ(F, i, j - 1)) / F->dx;
      double ne = 0.5 * (NODE(F, n, i, j) + NODE(F, n, i + 1, j));
      ej_edge(F, &EX(F, i, j), &JX(F, i, j), curl, ne);
    }
  #pragma omp parallel for schedule(static)
  for (int i = 1; i < fw; i++)
    for (int j = 0; j < fh; j++) {
      double curl = -(HZ(F, i, j) - HZ(F, i - 1, j)) / F->dx;
      double ne = 0.5 * (NODE(F, n, i, j) + NODE(F, n, i, j + 1));
      ej_edge(F, &EY(F, i, j), &JY(F, i, j), curl, ne);
    }
  cfb_edges(s, frac, NULL, NULL);
  accumulate(F, 0, 0);
}

/* ---- fine -> coarse transfer after the last substep (Sec. III.C: the
 * updated fine values go back to the coarse mesh): edge means for E and J,
 * cell and half-level mean for Hz (coarse n+1/2 lies midway between the two
 * fine H levels of the interval) ---------------------------------------- */
static void restrict_patch(orc_sim *s) {
  level_t *C = &s->L0, *F = &s->L1;
  const int r = s->p.r;
  const int I0 = s->ext[0], J0 = s->ext[1], I1 = s->ext[2], J1 = s->ext[3];
  const int fh = F->ny;
  const double *hi = r == 2 ? F->hz : s->hz_hi;
  #pragma omp parallel for schedule(static)
  for (int i = I0; i < I1; i++)
    for (int j = J0; j < J1; j++) {
      int p = r * (i - I0), q = r * (j - J0);
      double sum = 0.0;
      for (int a = 0; a < r; a++)
        for (int b = 0; b < r; b++)
          sum += 0.5 * (s->hz_lo[(size_t)(p + a) * fh + q + b] +
                        hi[(size_t)(p + a) * fh + q + b]);
      HZ(C, i, j) = sum / (r * r);
    }
  #pragma omp parallel for schedule(static)
  for (int i = I0; i < I1; i++)
    for (int j = J0 + 1; j < J1; j++) {
      int p = r * (i - I0), q = r * (j - J0);
      double se = 0.0, sj = 0.0;
      for (int a = 0; a < r; a++) {
        se += EX(F, p + a, q);
        sj += JX(F, p + a, q);
      }
      EX(C, i, j) = se / r;
      JX(C, i, j) = sj / r;
    }
  #pragma omp parallel for schedule(static)
  for (int i = I0 + 1; i < I1; i++)
    for (int j = J0; j < J1; j++) {
      int p = r * (i - I0), q = r * (j - J0);
      double se = 0.0, sj = 0.0;
      for (int b = 0; b < r; b++) {
        se += EY(F, p, q + b);
        sj += JY(F, p, q + b);
      }
      EY(C, i, j) = se / r;
      JY(C, i, j) = sj / r;
    }
}

/* ---- continuity, Eq. (4) ----------------------------------------------- */
double orc_nu_net(const orc_params *p, double erms2) {
  double omega = 2.0 * PI_ * p->freq_hz;
  double nu_m = 5.3e9 * p->p_torr;
  double eeff2 = erms2 / (1.0 + (omega * omega) / (nu_m * nu_m));
  if (p->source_model == ORC_SOURCE_TOWNSEND) {
    /* Eq. (4) with nu_i - nu_a = gamma v_d: Townsend's first coefficient
     * gamma = A p exp(-B p / E_eff) (per cm, E in V/cm), the drift velocity
     * of the collisional electron fluid v_d = mu_e E_eff, mu_e = e/(m nu_m);
     * attachment as a separate constant rate */
    double eeff = sqrt(eeff2);                 /* V/m */
    if (eeff <= 0.0) return -p->nu_att;
    double e_cm = eeff / 100.0;                /* V/cm */
    double gamma_cm = p->A_town * p->p_torr * exp(-p->B_town * p->p_torr / e_cm);
    double v_d = Q_E / (M_E * nu_m) * eeff;    /* m/s */
    return 100.0 * gamma_cm * v_d - p->nu_att;
  }
  /* (E_eff / p)^beta with E_eff/p in V/(cm Torr), via the square */
  double x = eeff2 / (1.0e4 * p->p_torr * p->p_torr);
  return nu_m * p->A_ion *
         (pow(x, 0.5 * p->beta_ion) - pow(p->ecr_over_p, p->beta_ion));
}

double orc_r_ei(const orc_params *p) {
  if (!(p->beta_rec > 0.0)) return 0.0;
  double te_kelvin = p->te_ev * Q_E / K_B;
  return p->beta_rec * 1e-13 * sqrt(300.0 / te_kelvin);
}

double orc_d_eff(const orc_params *p, double n) {
  if (p->d_mode == ORC_D_CONST) return p->d_const;
  double nu_m = 5.3e9 * p->p_torr;
  double d_e = Q_E * p->te_ev / (M_E * nu_m);
  double d_a = p->mu_i_760 * (760.0 / p->p_torr) * (p->te_ev + p->ti_ev);
  double n_amb = EPS_0 * p->te_ev / (Q_E * p->L_amb * p->L_amb);
  double alpha = n / n_amb;
  return (alpha * d_a + d_e) / (1.0 + alpha);
}

/* close one window block: its mean square field goes into the ring */
static void close_block(level_t *L, int slot) {
  #pragma omp parallel for schedule(static)
  for (int i = 0; i <= L->nx; i++)
    for (int j = 0; j <= L->ny; j++) {
      RING(L, slot, i, j) = NODE(L, acc, i, j) / L->spp;
      NODE(L, acc, i, j) = 0.0;
    }
}

static double erms2_at(const level_t *L, int i, int j) {
  double e2 = 0.0;
  for (int k = 0; k < NRING; k++) e2 += RING(L, k, i, j);
  return e2;
}

/* forward Euler, flux form with face D = mean of the two node values,
 * zero flux through the outer faces (or periodic wrap).  Arrays are node
 * arrays [nx+1][ny+1] (j fastest); nodes in [ilo,ihi]x[jlo,jhi] (and, when
 * mask is given, with a non-zero mask entry) are updated, the rest copied. */
static void continuity_core(const orc_params *p, int nx, int ny, double dx,
                            double dtn, int ilo, int ihi, int jlo, int jhi,
                            int perx, int pery, const double *nold,
                            const double *e2, double *nout,
                            const uint8_t *mask) {
#define AT(arr, i, j) arr[(size_t)(i) * (ny + 1) + (j)]
  const double r_ei = orc_r_ei(p);
  memcpy(nout, nold, (size_t)(nx + 1) * (ny + 1) * sizeof(double));
  #pragma omp parallel for schedule(static)
  for (int i = ilo; i <= ihi; i++)
    for (int j = jlo; j <= jhi; j++) {
      if ((perx && i == nx) || (pery && j == ny)) continue;
      if (mask && !AT(mask, i, j)) continue;
      double ni = AT(nold, i, j);
      double di = orc_d_eff(p, ni);
      double flux = 0.0;
      int nb[4][2] = {{i - 1, j}, {i + 1, j}, {i, j - 1}, {i, j + 1}};
      for (int k = 0; k < 4; k++) {
        int a = nb[k][0], b = nb[k][1];
        if (a < 0 || a > nx) {
          if (!perx) continue;
          a = (a + nx) % nx;
        }
        if (b < 0 || b > ny) {
          if (!pery) continue;
          b = (b + ny) % ny;
        }
        double nn = AT(nold, a, b);
        flux += 0.5 * (di + orc_d_eff(p, nn)) * (nn - ni);
      }
      double nu = orc_nu_net(p, AT(e2, i, j));
      double nnew = ni + dtn * (flux / (dx * dx) + nu * ni - r_ei * ni * ni);
      AT(nout, i, j) = nnew > 0.0 ? nnew : 0.0;
    }
  if (perx)
    for (int j = 0; j <= ny; j++) AT(nout, nx, j) = AT(nout, 0, j);
  if (pery)
    for (int i = 0; i <= nx; i++) AT(nout, i, ny) = AT(nout, i, 0);
#undef AT
}

/* interior_only leaves the patch boundary nodes (they carry coarse values)
 * untouched; mask (node array) restricts the update further */
static void continuity(orc_sim *s, level_t *L, int interior_only, int perx,
                       int pery, const uint8_t *mask) {
  const int nx = L->nx, ny = L->ny;
  const double dtn = L->spb * L->dt;
  double *nold = malloc(n_nd(L) * sizeof(double));
  double *e2 = malloc(n_nd(L) * sizeof(double));
  memcpy(nold, L->n, n_nd(L) * sizeof(double));
  #pragma omp parallel for schedule(static)
  for (int i = 0; i <= nx; i++)
    for (int j = 0; j <= ny; j++) e2[(size_t)i * (ny + 1) + j] = erms2_at(L, i, j);
  if (interior_only)
    continuity_core(&s->p, nx, ny, L->dx, dtn, 1, nx - 1, 1, ny - 1, 0, 0,
                    nold, e2, L->n, mask);
  else
    continuity_core(&s->p, nx, ny, L->dx, dtn, 0, nx, 0, ny, perx, pery, nold,
                    e2, L->n, mask);
  free(nold);
  free(e2);
}

int orc_continuity_apply(const orc_params *p, int nx, int ny, double dx,
                         double dtn, int perx, int pery, const double *n_in,
                         const double *erms2, double *n_out) {
  size_t nn = (size_t)(nx + 1) * (ny + 1);
  double *a = calloc(nn, sizeof(double)), *e = calloc(nn, sizeof(double)),
         *o = calloc(nn, sizeof(double));
  if (!a || !e || !o) {
    free(a); free(e); free(o);
    return -2;
  }
  for (int j = 0; j <= ny; j++)
    for (int i = 0; i <= nx; i++) {
      a[(size_t)i * (ny + 1) + j] = n_in[(size_t)j * (nx + 1) + i];
      e[(size_t)i * (ny + 1) + j] = erms2[(size_t)j * (nx + 1) + i];
    }
  continuity_core(p, nx, ny, dx, dtn, 0, nx, 0, ny, perx, pery, a, e, o, NULL);
  for (int j = 0; j <= ny; j++)
    for (int i = 0; i <= nx; i++)
      n_out[(size_t)j * (nx + 1) + i] = o[(size_t)i * (ny + 1) + j];
  free(a); free(e); free(o);
  return 0;
}

/* ---- bilinear sampling of a coarse array, Eq. (5a) area weights -------- */
/* arr has (ni x nj) entries with j fastest; (u, v) in that array's index
 * space; only entries with non-zero weight are touched */
static double bilin(const double *arr, int nj, double u, double v) {
  int i = (int)floor(u), j = (int)floor(v);
  double fu = u - i, fv = v - j, val = 0.0;
  for (int di = 0; di < 2; di++) {
    double wu = di ? fu : 1.0 - fu;
    if (wu == 0.0) continue;
    for (int dj = 0; dj < 2; dj++) {
      double wv = dj ? fv : 1.0 - fv;
      if (wv == 0.0) continue;
      val += wu * wv * arr[(size_t)(i + di) * nj + (j + dj)];
    }
  }
  return val;
}

/* coarse n -> fine patch boundary nodes, then fine -> coarse injection at
 * the coarse nodes strictly inside the patch (Sec. III.C transfers) */
static void transfer_density(orc_sim *s) {
  level_t *C = &s->L0, *F = &s->L1;
  const int r = s->p.r;
  const int P0 = r * s->ext[0], Q0 = r * s->ext[1];
  const int fw = F->nx, fh = F->ny;
  #pragma omp parallel for schedule(static)
  for (int i = 0; i <= fw; i++)
    for (int j = 0; j <= fh; j++) {
      if (i != 0 && i != fw && j != 0 && j != fh) continue;
      NODE(F, n, i, j) = bilin(C->n, C->ny + 1, (double)(P0 + i) / r, (double)(Q0 + j) / r);
    }
  for (int i = s->ext[0] + 1; i < s->ext[2]; i++)
    for (int j = s->ext[1] + 1; j < s->ext[3]; j++)
      NODE(C, n, i, j) = NODE(F, n, r * (i - s->ext[0]), r * (j - s->ext[1]));
}

/* ---- self-aware expansion, Sec. III.A/B/D ------------------------------ */
/* node flag: threshold density, or (above a floor) a density gradient
 * length n/|grad n| below dx/grad_thr.  Decided in binary32 on
 * n * 2^-60 (an exact scaling that keeps n^2 in range):
 *   n > n_thr  or  (n > n_floor and gx*gx + gy*gy > g2 * (n*n)),
 * g = central difference in cell units, zero on the domain boundary. */
static int node_flag(const orc_sim *s, int i, int j, float thr, float flo,
                     float g2) {
  const level_t *L = &s->L0;
  float nv = (float)NODE(L, n, i, j);
  if (nv > thr) return 1;
  if (!(nv > flo)) return 0;
  float ns = ldexpf(nv, -60);
  float gx = 0.0f, gy = 0.0f;
  if (i > 0 && i < L->nx) {
    float r = ldexpf((float)NODE(L, n, i + 1, j), -60);
    float l = ldexpf((float)NODE(L, n, i - 1, j), -60);
    gx = (r - l) * 0.5f;
  }
  if (j > 0 && j < L->ny) {
    float u = ldexpf((float)NODE(L, n, i, j + 1), -60);
    float d = ldexpf((float)NODE(L, n, i, j - 1), -60);
    gy = (u - d) * 0.5f;
  }
  float gx2 = gx * gx;
  float gy2 = gy * gy;
  float lhs = gx2 + gy2;
  float n2 = ns * ns;
  float rhs = g2 * n2;
  return lhs > rhs;
}

/* flags -> block flags -> exclusive prefix sum -> compacted block list */
static void flag_blocks(orc_sim *s) {
  const level_t *L = &s->L0;
  const int B = s->p.block, NBx = s->NBx, NBy = s->NBy;
  const float thr = (float)(s->p.n_thr_over_nc * s->n_c);
  const float flo = (float)(s->p.n_floor_over_nc * s->n_c);
  const float g2 = (float)(s->p.grad_thr * s->p.grad_thr);
  memset(s->bflag, 0, (size_t)NBx * NBy);
  for (int i = 0; i <= L->nx; i++)
    for (int j = 0; j <= L->ny; j++) {
      int bx = i / B < NBx - 1 ? i / B : NBx - 1;
      int by = j / B < NBy - 1 ? j / B : NBy - 1;
      if (node_flag(s, i, j, thr, flo, g2)) s->bflag[by * NBx + bx] = 1;
    }
  int32_t run = 0;
  for (int b = 0; b < NBx * NBy; b++) {
    s->bscan[b] = run;
    if (s->bflag[b]) s->blist[run] = b;
    run += s->bflag[b];
  }
  s->bcount = run;
}

/* first block column a patch may use: one block clear of the outer boundary
 * and of the source line */
static int block_xmin(const orc_sim *s) {
  const int B = s->p.block;
  int xmin = 1;
  if (s->p.tfsf_i > 0) {
    int m = (s->p.tfsf_i + 2 * B - 1) / B;
    if (m > xmin) xmin = m;
  }
  return xmin;
}

/* bounding box of old patch and flagged blocks, clipped to the margins */
static void regrid_test(orc_sim *s, int newext[4]) {
  const int B = s->p.block, NBx = s->NBx, NBy = s->NBy;
  flag_blocks(s);
  int bx0 = NBx, by0 = NBy, bx1 = 0, by1 = 0;
  for (int k = 0; k < s->bcount; k++) {
    int bx = s->blist[k] % NBx, by = s->blist[k] / NBx;
    if (bx < bx0) bx0 = bx;
    if (by < by0) by0 = by;
    if (bx + 1 > bx1) bx1 = bx + 1;
    if (by + 1 > by1) by1 = by + 1;
  }
  if (s->has_patch) { /* the patch only grows (Sec. III.D) */
    int o0 = s->ext[0] / B, o1 = s->ext[1] / B, o2 = s->ext[2] / B,
        o3 = s->ext[3] / B;
    if (o0 < bx0) bx0 = o0;
    if (o1 < by0) by0 = o1;
    if (o2 > bx1) bx1 = o2;
    if (o3 > by1) by1 = o3;
  }
  /* keep one block clear of the outer boundary and of the source line */
  const int xmin = block_xmin(s);
  if (bx0 < xmin) bx0 = xmin;
  if (by0 < 1) by0 = 1;
  if (bx1 > NBx - 1) bx1 = NBx - 1;
  if (by1 > NBy - 1) by1 = NBy - 1;
  if (bx0 >= bx1 || by0 >= by1) {
    newext[0] = newext[1] = newext[2] = newext[3] = 0;
  } else {
    newext[0] = bx0 * B;
    newext[1] = by0 * B;
    newext[2] = bx1 * B;
    newext[3] = by1 * B;
  }
}

/* Build the fine patch for new extents: data of the old patch is copied
 * where it exists, the rest is interpolated from the coarse mesh
 * (Sec. III.D), bilinearly with the area weights of Eq. (5a).  E, J, n and
 * the window use the current coarse values (frac = 1); fine Hz must sit at
 * coarse time n+3/4, so Eq. (5a) is applied with frac = 5/4 between coarse
 * Hz^{n-1/2} and Hz^{n+1/2}. */
static int build_patch(orc_sim *s, const int ne[4], const double *seed_fine) {
  const level_t *C = &s->L0;
  const int r = s->p.r;
  level_t F;
  int rc = level_init(&F, r * (ne[2] - ne[0]), r * (ne[3] - ne[1]), C->dx / r,
                      C->dt / r, C->spp * r, s->nu_m, s->p.courant);
  if (rc) {
    level_free(&F);
    return rc;
  }
  const int P0 = r * ne[0], Q0 = r * ne[1];
  const level_t *O = s->has_patch ? &s->L1 : NULL;
  const int oP0 = O ? r * s->ext[0] : 0, oQ0 = O ? r * s->ext[1] : 0;
  const int oP1 = O ? r * s->ext[2] : 0, oQ1 = O ? r * s->ext[3] : 0;
  /* fine Hz after a coarse step sits at coarse n + 1 - 1/(2r): Eq. (5a)
   * in time with frac 3/2 - 1/(2r) between Hz^{n-1/2} and Hz^{n+1/2}
   * (5/4 for r = 2) */
  const double fr = 1.5 - 0.5 / r;
  const int fgx = r * s->p.nx + 1;

  for (int i = 0; i < F.nx; i++)
    for (int j = 0; j < F.ny; j++) {
      int P = P0 + i, Q = Q0 + j;
      if (O && P >= oP0 && P < oP1 && Q >= oQ0 && Q < oQ1) {
        HZ(&F, i, j) = HZ(O, P - oP0, Q - oQ0);
      } else {
        double u = (P + 0.5) / r - 0.5, v = (Q + 0.5) / r - 0.5;
        HZ(&F, i, j) = (1.0 - fr) * bilin(s->hz_prev, C->ny, u, v) +
                       fr * bilin(C->hz, C->ny, u, v);
      }
    }
  for (int i = 0; i < F.nx; i++)
    for (int j = 0; j <= F.ny; j++) {
      int P = P0 + i, Q = Q0 + j;
      if (O && P >= oP0 && P < oP1 && Q >= oQ0 && Q <= oQ1) {
        EX(&F, i, j) = EX(O, P - oP0, Q - oQ0);
        JX(&F, i, j) = JX(O, P - oP0, Q - oQ0);
      } else {
        double u = (P + 0.5) / r - 0.5, v = (double)Q / r;
        EX(&F, i, j) = bilin(C->ex, C->ny + 1, u, v);
        JX(&F, i, j) = bilin(C->jx, C->ny + 1, u, v);
      }
    }
  for (int i = 0; i <= F.nx; i++)
    for (int j = 0; j < F.ny; j++) {
      int P = P0 + i, Q = Q0 + j;
      if (O && P >= oP0 && P <= oP1 && Q >= oQ0 && Q < oQ1) {
        EY(&F, i, j) = EY(O, P - oP0, Q - oQ0);
        JY(&F, i, j) = JY(O, P - oP0, Q - oQ0);
      } else {
        double u = (double)P / r, v = (Q + 0.5) / r - 0.5;
        EY(&F, i, j) = bilin(C->ey, C->ny, u, v);
        JY(&F, i, j) = bilin(C->jy, C->ny, u, v);
      }
    }
  for (int i = 0; i <= F.nx; i++)
    for (int j = 0; j <= F.ny; j++) {
      int P = P0 + i, Q = Q0 + j;
      if (O && P >= oP0 && P <= oP1 && Q >= oQ0 && Q <= oQ1) {
        int a = P - oP0, b = Q - oQ0;
        NODE(&F, n, i, j) = NODE(O, n, a, b);
        NODE(&F, acc, i, j) = NODE(O, acc, a, b);
        for (int k = 0; k < NRING; k++) RING(&F, k, i, j) = RING(O, k, a, b);
      } else {
        double u = (double)P / r, v = (double)Q / r;
        NODE(&F, n, i, j) = seed_fine ? seed_fine[(size_t)Q * fgx + P]
                                      : bilin(C->n, C->ny + 1, u, v);
        NODE(&F, acc, i, j) = bilin(C->acc, C->ny + 1, u, v);
        for (int k = 0; k < NRING; k++)
          RING(&F, k, i, j) = bilin(C->ring + (size_t)k * n_nd(C), C->ny + 1, u, v);
      }
    }
  if (s->has_patch) level_free(&s->L1);
  free(s->hz_lo);
  free(s->hz_hi);
  s->L1 = F;
  s->hz_lo = calloc(n_hz(&F), sizeof(double));
  s->hz_hi = calloc(n_hz(&F), sizeof(double));
  memcpy(s->ext, ne, sizeof(s->ext));
  s->has_patch = 1;
  return s->hz_lo && s->hz_hi ? 0 : -2;
}

/* The threshold lines of Sec. III.D.  The lines coincide with the sides of
 * the patch (the coarse-fine boundary).  A side whose line carries a base
 * node with n above the threshold density moves outward: by m_ex for the
 * two sides crossing x (left, right), by m_ey for the two crossing y (bottom,
 * top).  Before any patch exists, the first one is m_lx x m_ly cells centred
 * on the peak of the density (its first maximum, rows from the bottom).  The
 * same margins as the block rule apply; the patch only grows.  The density is
 * compared in binary32, as the flags of the block rule. */
static void line_rule(orc_sim *s, int ne[4]) {
  const orc_params *p = &s->p;
  const level_t *L = &s->L0;
  const int B = p->block;
  int xmin = 1;
  if (p->tfsf_i > 0) {
    int m = (p->tfsf_i + 2 * B - 1) / B;
    if (m > xmin) xmin = m;
  }
  if (!s->has_patch) {
    int pi = 0, pj = 0;
    double best = NODE(L, n, 0, 0);
    for (int j = 0; j <= L->ny; j++)
      for (int i = 0; i <= L->nx; i++)
        if (NODE(L, n, i, j) > best) {
          best = NODE(L, n, i, j);
          pi = i;
          pj = j;
        }
    ne[0] = pi - p->m_lx / 2;
    ne[1] = pj - p->m_ly / 2;
    ne[2] = ne[0] + p->m_lx;
    ne[3] = ne[1] + p->m_ly;
  } else {
    const float thr = (float)p->n_line;
    int left = 0, right = 0, bottom = 0, top = 0;
    for (int j = s->ext[1]; j <= s->ext[3]; j++) {
      if ((float)NODE(L, n, s->ext[0], j) > thr) left = 1;
      if ((float)NODE(L, n, s->ext[2], j) > thr) right = 1;
    }
    for (int i = s->ext[0]; i <= s->ext[2]; i++) {
      if ((float)NODE(L, n, i, s->ext[1]) > thr) bottom = 1;
      if ((float)NODE(L, n, i, s->ext[3]) > thr) top = 1;
    }
    ne[0] = s->ext[0] - (left ? p->m_ex : 0);
    ne[2] = s->ext[2] + (right ? p->m_ex : 0);
    ne[1] = s->ext[1] - (bottom ? p->m_ey : 0);
    ne[3] = s->ext[3] + (top ? p->m_ey : 0);
  }
  if (ne[0] < xmin * B) ne[0] = xmin * B;
  if (ne[1] < B) ne[1] = B;
  if (ne[2] > L->nx - B) ne[2] = L->nx - B;
  if (ne[3] > L->ny - B) ne[3] = L->ny - B;
  if (ne[0] >= ne[2] || ne[1] >= ne[3]) ne[0] = ne[1] = ne[2] = ne[3] = 0;
}

/* ---- the fine level as a union of blocks (ORC_RULE_UNION) --------------
 * The growth test of Sec. III.A/B flags blocks; here the fine level is the
 * union of the flagged blocks themselves instead of their bounding box, so
 * that several separate regions are refined without the space between them.
 * The fine arrays span the whole domain at r times the resolution.  A fine
 * cell belongs to the fine level when its block is active.  An edge belongs
 * to it when a cell beside it does: interior when both cells do, a
 * coarse/fine boundary edge (driven by Eq. (5b)) when exactly one does.  A
 * node belongs to it when a cell around it does, interior when all four do.
 * Every rule of the rectangular patch above is the special case of a
 * rectangle of blocks. */
static int cact_m(const orc_sim *s, const uint8_t *map, int P, int Q) {
  const int fb = s->p.r * s->p.block;
  if (P < 0 || Q < 0 || P >= s->p.r * s->p.nx || Q >= s->p.r * s->p.ny) return 0;
  return map[(size_t)(Q / fb) * s->NBx + P / fb];
}
static int cact(const orc_sim *s, int P, int Q) { return cact_m(s, s->act, P, Q); }
static int ex_has_m(const orc_sim *s, const uint8_t *m, int P, int Q) {
  return cact_m(s, m, P, Q) || cact_m(s, m, P, Q - 1);
}
static int ey_has_m(const orc_sim *s, const uint8_t *m, int P, int Q) {
  return cact_m(s, m, P, Q) || cact_m(s, m, P - 1, Q);
}
static int nd_has_m(const orc_sim *s, const uint8_t *m, int P, int Q) {
  return cact_m(s, m, P - 1, Q - 1) || cact_m(s, m, P, Q - 1) ||
         cact_m(s, m, P - 1, Q) || cact_m(s, m, P, Q);
}
static int ex_has(const orc_sim *s, int P, int Q) { return ex_has_m(s, s->act, P, Q); }
static int ey_has(const orc_sim *s, int P, int Q) { return ey_has_m(s, s->act, P, Q); }
static int nd_has(const orc_sim *s, int P, int Q) { return nd_has_m(s, s->act, P, Q); }
static int ex_inner(const orc_sim *s, int P, int Q) { return cact(s, P, Q) && cact(s, P, Q - 1); }
static int ey_inner(const orc_sim *s, int P, int Q) { return cact(s, P, Q) && cact(s, P - 1, Q); }
static int nd_inner(const orc_sim *s, int P, int Q) {
  return cact(s, P - 1, Q - 1) && cact(s, P, Q - 1) && cact(s, P - 1, Q) && cact(s, P, Q);
}
/* coarse cell (I, J) active */
static int coarse_act(const orc_sim *s, int I, int J) {
  const int B = s->p.block;
  if (I < 0 || J < 0 || I >= s->p.nx || J >= s->p.ny) return 0;
  return s->act[(size_t)(J / B) * s->NBx + I / B];
}

/* 5-point Laplacian on the fine level's own edges of one kind (0: Ex grid
 * [fw][fh+1], 1: Ey grid [fw+1][fh]); a neighbour outside the level counts
 * as the centre value, as for the rectangle */
static void lap_union(const orc_sim *s, const double *a, double *out, int ni,
                      int nj, int kind) {
#define HAS(i, j) (kind ? ey_has(s, i, j) : ex_has(s, i, j))
  #pragma omp parallel for schedule(static)
  for (int i = 0; i < ni; i++)
    for (int j = 0; j < nj; j++) {
      if (!HAS(i, j)) {
        out[(size_t)i * nj + j] = 0.0;
        continue;
      }
      double c = a[(size_t)i * nj + j];
      double l = HAS(i - 1, j) ? a[(size_t)(i - 1) * nj + j] : c;
      double r = HAS(i + 1, j) ? a[(size_t)(i + 1) * nj + j] : c;
      double d = HAS(i, j - 1) ? a[(size_t)i * nj + j - 1] : c;
      double u = HAS(i, j + 1) ? a[(size_t)i * nj + j + 1] : c;
      out[(size_t)i * nj + j] = l + r + d + u - 4.0 * c;
    }
#undef HAS
}

static void fine_filter_union(orc_sim *s) {
  level_t *F = &s->L1;
  const double g = s->p.fine_filter;
  if (g <= 0.0) return;
  const int fw = F->nx, fh = F->ny;
  size_t nx_ = n_ex(F), ny_ = n_ey(F);
  size_t nmax = nx_ > ny_ ? nx_ : ny_;
  double *t1 = malloc(nmax * sizeof(double)), *t2 = malloc(nmax * sizeof(double));
  lap_union(s, F->ex, t1, fw, fh + 1, 0);
  lap_union(s, t1, t2, fw, fh + 1, 0);
  #pragma omp parallel for schedule(static)
  for (int i = 0; i < fw; i++)
    for (int j = 1; j < fh; j++)
      if (ex_inner(s, i, j)) EX(F, i, j) -= g * t2[(size_t)i * (fh + 1) + j];
  lap_union(s, F->ey, t1, fw + 1, fh, 1);
  lap_union(s, t1, t2, fw + 1, fh, 1);
  #pragma omp parallel for schedule(static)
  for (int i = 1; i < fw; i++)
    for (int j = 0; j < fh; j++)
      if (ey_inner(s, i, j)) EY(F, i, j) -= g * t2[(size_t)i * fh + j];
  free(t1);
  free(t2);
}

/* node E^2 from the fine level's own edges (as node_e2) */
static double node_e2_union(const orc_sim *s, int i, int j) {
  const level_t *L = &s->L1;
  double sx = 0.0, sy = 0.0;
  int cx = 0, cy = 0;
  if (ex_has(s, i - 1, j)) {
    sx += EX(L, i - 1, j) * EX(L, i - 1, j);
    cx++;
  }
  if (ex_has(s, i, j)) {
    sx += EX(L, i, j) * EX(L, i, j);
    cx++;
  }
  if (ey_has(s, i, j - 1)) {
    sy += EY(L, i, j - 1) * EY(L, i, j - 1);
    cy++;
  }
  if (ey_has(s, i, j)) {
    sy += EY(L, i, j) * EY(L, i, j);
    cy++;
  }
  return (cx ? sx / cx : 0.0) + (cy ? sy / cy : 0.0);
}

/* one fine substep m (1..r) on the union of blocks, Sec. III.C */
static void em_step_fine_union(orc_sim *s, int m) {
  level_t *F = &s->L1;
  const int fw = F->nx, fh = F->ny, r = s->p.r;
  const double frac = (double)m / r;

  fine_filter_union(s);

  #pragma omp parallel for schedule(static)
  for (int i = 0; i < fw; i++)
    for (int j = 0; j < fh; j++)
      if (cact(s, i, j))
        HZ(F, i, j) -= F->ch * ((EY(F, i + 1, j) - EY(F, i, j)) -
                                (EX(F, i, j + 1) - EX(F, i, j)));
  if (m == r / 2) memcpy(s->hz_lo, F->hz, n_hz(F) * sizeof(double));
  if (m == r / 2 + 1 && m < r) memcpy(s->hz_hi, F->hz, n_hz(F) * sizeof(double));

  #pragma omp parallel for schedule(static)
  for (int i = 0; i < fw; i++)
    for (int j = 1; j < fh; j++) {
      if (!ex_inner(s, i, j)) continue;
      double curl = (HZ(F, i, j) - HZ(F, i, j - 1)) / F->dx;
      double ne = 0.5 * (NODE(F, n, i, j) + NODE(F, n, i + 1, j));
      ej_edge(F, &EX(F, i, j), &JX(F, i, j), curl, ne);
    }
  #pragma omp parallel for schedule(static)
  for (int i = 1; i < fw; i++)
    for (int j = 0; j < fh; j++) {
      if (!ey_inner(s, i, j)) continue;
      double curl = -(HZ(F, i, j) - HZ(F, i - 1, j)) / F->dx;
      double ne = 0.5 * (NODE(F, n, i, j) + NODE(F, n, i, j + 1));
      ej_edge(F, &EY(F, i, j), &JY(F, i, j), curl, ne);
    }
  cfb_edges(s, frac, NULL, NULL);
  #pragma omp parallel for schedule(static)
  for (int i = 0; i <= fw; i++)
    for (int j = 0; j <= fh; j++)
      if (nd_has(s, i, j)) NODE(F, acc, i, j) += node_e2_union(s, i, j);
}

/* fine -> coarse transfer over the coarse entities whose cells are all
 * active (as restrict_patch) */
static void restrict_union(orc_sim *s) {
  level_t *C = &s->L0, *F = &s->L1;
  const int r = s->p.r, fh = F->ny;
  const double *hi = r == 2 ? F->hz : s->hz_hi;
  #pragma omp parallel for schedule(static)
  for (int i = 0; i < C->nx; i++)
    for (int j = 0; j < C->ny; j++) {
      if (!coarse_act(s, i, j)) continue;
      int p = r * i, q = r * j;
      double sum = 0.0;
      for (int a = 0; a < r; a++)
        for (int b = 0; b < r; b++)
          sum += 0.5 * (s->hz_lo[(size_t)(p + a) * fh + q + b] +
                        hi[(size_t)(p + a) * fh + q + b]);
      HZ(C, i, j) = sum / (r * r);
    }
  #pragma omp parallel for schedule(static)
  for (int i = 0; i < C->nx; i++)
    for (int j = 1; j < C->ny; j++) {
      if (!coarse_act(s, i, j) || !coarse_act(s, i, j - 1)) continue;
      int p = r * i, q = r * j;
      double se = 0.0, sj = 0.0;
      for (int a = 0; a < r; a++) {
        se += EX(F, p + a, q);
        sj += JX(F, p + a, q);
      }
      EX(C, i, j) = se / r;
      JX(C, i, j) = sj / r;
    }
  #pragma omp parallel for schedule(static)
  for (int i = 1; i < C->nx; i++)
    for (int j = 0; j < C->ny; j++) {
      if (!coarse_act(s, i, j) || !coarse_act(s, i - 1, j)) continue;
      int p = r * i, q = r * j;
      double se = 0.0, sj = 0.0;
      for (int b = 0; b < r; b++) {
        se += EY(F, p, q + b);
        sj += JY(F, p, q + b);
      }
      EY(C, i, j) = se / r;
      JY(C, i, j) = sj / r;
    }
}

/* density transfers of the union (as transfer_density): the level's
 * boundary nodes take the coarse density (Eq. (5a) weights: copy at
 * coincident nodes, mean at mid nodes); coarse nodes with all four cells
 * active take the fine density */
static void transfer_density_union(orc_sim *s) {
  level_t *C = &s->L0, *F = &s->L1;
  const int r = s->p.r, fw = F->nx, fh = F->ny;
  #pragma omp parallel for schedule(static)
  for (int i = 0; i <= fw; i++)
    for (int j = 0; j <= fh; j++)
      if (nd_has(s, i, j) && !nd_inner(s, i, j))
        NODE(F, n, i, j) = bilin(C->n, C->ny + 1, (double)i / r, (double)j / r);
  #pragma omp parallel for schedule(static)
  for (int i = 1; i < C->nx; i++)
    for (int j = 1; j < C->ny; j++)
      if (coarse_act(s, i - 1, j - 1) && coarse_act(s, i, j - 1) &&
          coarse_act(s, i - 1, j) && coarse_act(s, i, j))
        NODE(C, n, i, j) = NODE(F, n, r * i, r * j);
}

/* continuity on the interior fine nodes, then the density transfers */
static void sync_union(orc_sim *s) {
  level_t *F = &s->L1;
  const int fw = F->nx, fh = F->ny;
  uint8_t *mask = malloc(n_nd(F));
  #pragma omp parallel for schedule(static)
  for (int i = 0; i <= fw; i++)
    for (int j = 0; j <= fh; j++)
      mask[(size_t)i * (fh + 1) + j] = (uint8_t)nd_inner(s, i, j);
  continuity(s, F, 1, 0, 0, mask);
  free(mask);
  transfer_density_union(s);
}

/* Add blocks to the fine level (growth only, Sec. III.D).  Entities new to
 * the level take Eq. (5a) values from the coarse mesh exactly as in
 * build_patch; the ones it already had keep theirs.  add: [NBy][NBx];
 * blocks outside the margins are an error. */
static int grow_union(orc_sim *s, const uint8_t *add, const double *seed_fine) {
  const level_t *C = &s->L0;
  level_t *F = &s->L1;
  const int r = s->p.r, NBx = s->NBx, NBy = s->NBy, xmin = block_xmin(s);
  size_t nb = (size_t)NBx * NBy;
  uint8_t *old = malloc(nb);
  if (!old) return -2;
  memcpy(old, s->act, nb);
  int changed = 0;
  for (int by = 0; by < NBy; by++)
    for (int bx = 0; bx < NBx; bx++)
      if (add[by * NBx + bx] && (bx < xmin || by < 1 || bx > NBx - 2 || by > NBy - 2)) {
        free(old);
        return -1;
      }
  for (size_t b = 0; b < nb; b++)
    if (add[b] && !s->act[b]) {
      s->act[b] = 1;
      changed = 1;
    }
  if (!changed) {
    free(old);
    return 0;
  }
  const double fr = 1.5 - 0.5 / r;
  const int fw = F->nx, fh = F->ny, fgx = fw + 1;
  for (int i = 0; i < fw; i++)
    for (int j = 0; j < fh; j++) {
      if (!cact(s, i, j) || cact_m(s, old, i, j)) continue;
      double u = (i + 0.5) / r - 0.5, v = (j + 0.5) / r - 0.5;
      HZ(F, i, j) = (1.0 - fr) * bilin(s->hz_prev, C->ny, u, v) +
                    fr * bilin(C->hz, C->ny, u, v);
    }
  for (int i = 0; i < fw; i++)
    for (int j = 0; j <= fh; j++) {
      if (!ex_has(s, i, j) || ex_has_m(s, old, i, j)) continue;
      double u = (i + 0.5) / r - 0.5, v = (double)j / r;
      EX(F, i, j) = bilin(C->ex, C->ny + 1, u, v);
      JX(F, i, j) = bilin(C->jx, C->ny + 1, u, v);
    }
  for (int i = 0; i <= fw; i++)
    for (int j = 0; j < fh; j++) {
      if (!ey_has(s, i, j) || ey_has_m(s, old, i, j)) continue;
      double u = (double)i / r, v = (j + 0.5) / r - 0.5;
      EY(F, i, j) = bilin(C->ey, C->ny, u, v);
      JY(F, i, j) = bilin(C->jy, C->ny, u, v);
    }
  for (int i = 0; i <= fw; i++)
    for (int j = 0; j <= fh; j++) {
      if (!nd_has(s, i, j) || nd_has_m(s, old, i, j)) continue;
      double u = (double)i / r, v = (double)j / r;
      NODE(F, n, i, j) = seed_fine ? seed_fine[(size_t)j * fgx + i]
                                   : bilin(C->n, C->ny + 1, u, v);
      NODE(F, acc, i, j) = bilin(C->acc, C->ny + 1, u, v);
      for (int k = 0; k < NRING; k++)
        RING(F, k, i, j) = bilin(C->ring + (size_t)k * n_nd(C), C->ny + 1, u, v);
    }
  free(old);
  /* extents reported for the union: its bounding box */
  int bx0 = NBx, by0 = NBy, bx1 = 0, by1 = 0;
  for (int by = 0; by < NBy; by++)
    for (int bx = 0; bx < NBx; bx++)
      if (s->act[by * NBx + bx]) {
        if (bx < bx0) bx0 = bx;
        if (by < by0) by0 = by;
        if (bx + 1 > bx1) bx1 = bx + 1;
        if (by + 1 > by1) by1 = by + 1;
      }
  const int B = s->p.block;
  s->ext[0] = bx0 * B;
  s->ext[1] = by0 * B;
  s->ext[2] = bx1 * B;
  s->ext[3] = by1 * B;
  s->has_patch = 1;
  return 0;
}

/* growth test of the union: the flagged blocks inside the margins join */
static int regrid_union(orc_sim *s, const double *seed_fine) {
  const int NBx = s->NBx, NBy = s->NBy, xmin = block_xmin(s);
  flag_blocks(s);
  uint8_t *add = calloc((size_t)NBx * NBy, 1);
  if (!add) return -2;
  for (int by = 1; by < NBy - 1; by++)
    for (int bx = xmin; bx < NBx - 1; bx++) add[by * NBx + bx] = s->bflag[by * NBx + bx];
  int rc = grow_union(s, add, seed_fine);
  free(add);
  return rc;
}

int orc_add_blocks(orc_sim *s, const uint8_t *mask) {
  if (!s || !mask || s->p.regrid_rule != ORC_RULE_UNION || s->p.mode == ORC_UNIFORM)
    return -1;
  return grow_union(s, mask, NULL);
}

int orc_get_blocks(const orc_sim *s, uint8_t *dst) {
  if (!s || !dst || s->p.regrid_rule != ORC_RULE_UNION || s->p.mode == ORC_UNIFORM)
    return -1;
  memcpy(dst, s->act, (size_t)s->NBx * s->NBy);
  return 0;
}

static int do_regrid(orc_sim *s, const double *seed_fine) {
  int ne[4];
  if (s->p.regrid_rule == ORC_RULE_UNION) return regrid_union(s, seed_fine);
  if (s->p.regrid_rule == ORC_RULE_LINES)
    line_rule(s, ne);
  else
    regrid_test(s, ne);
  if (ne[2] <= ne[0]) return 0; /* nothing to refine */
  if (s->has_patch && !memcmp(ne, s->ext, sizeof(ne))) return 0;
  return build_patch(s, ne, seed_fine);
}

int orc_regrid(orc_sim *s) {
  if (!s || s->p.mode == ORC_UNIFORM) return -1;
  return do_regrid(s, NULL);
}

/* ---- driver: one base step with subcycling, Sec. III.C ----------------- */
static void sync_point(orc_sim *s) {
  const int perx = s->p.bc_x == ORC_BC_PERIODIC;
  const int pery = s->p.bc_y == ORC_BC_PERIODIC;
  int slot = (int)(s->blocks % NRING);
  close_block(&s->L0, slot);
  if (s->has_patch) close_block(&s->L1, slot);
  s->blocks++;
  if (s->blocks < NRING) return; /* the first period only fills the window */
  continuity(s, &s->L0, 0, perx, pery, NULL);
  if (s->has_patch && s->act) {
    sync_union(s);
  } else if (s->has_patch) {
    continuity(s, &s->L1, 1, 0, 0, NULL);
    transfer_density(s);
  }
}

static int base_step(orc_sim *s) {
  em_step_base(s);
  if (s->has_patch && s->act) {
    for (int m = 1; m <= s->p.r; m++) em_step_fine_union(s, m);
    restrict_union(s);
  } else if (s->has_patch) {
    for (int m = 1; m <= s->p.r; m++) em_step_fine(s, m);
    restrict_patch(s);
  }
  s->step++;
  if (s->p.continuity_on && s->step % s->L0.spb == 0) sync_point(s);
  if (s->p.mode == ORC_DYNAMIC && s->step % s->p.regrid_every == 0)
    return do_regrid(s, NULL);
  return 0;
}

int orc_step(orc_sim *s, int64_t n) {
  if (!s || n < 0) return -1;
  for (int64_t k = 0; k < n; k++) {
    int rc = base_step(s);
    if (rc) return rc;
  }
  return 0;
}

/* ---- create / destroy --------------------------------------------------- */
int orc_create(const orc_params *p, const double *seed_base,
               const double *seed_fine, orc_sim **out) {
  *out = NULL;
  if (p->nx < 2 || p->ny < 2 || p->cells_per_lambda < 1 || p->courant <= 0.0)
    return -1;
  double sppd = p->cells_per_lambda / p->courant;
  int spp = (int)floor(sppd + 0.5);
  if (fabs(sppd - spp) > 1e-9 || spp % NRING) return -1;
  if (p->mode != ORC_UNIFORM) {
    if ((p->r != 2 && p->r != 4) || p->block < 1 || p->nx % p->block ||
        p->ny % p->block)
      return -1;
    if (p->bc_x == ORC_BC_PERIODIC || p->bc_y == ORC_BC_PERIODIC) return -1;
    if (p->mode == ORC_DYNAMIC && p->regrid_every % (spp / NRING)) return -1;
    if (p->regrid_rule < 0 || p->regrid_rule > 2) return -1;
    if (p->regrid_rule == ORC_RULE_LINES &&
        (p->m_lx < 1 || p->m_ly < 1 || p->m_ex < 1 || p->m_ey < 1 || !(p->n_line > 0.0)))
      return -1;
  }
  if (p->tfsf_i > 0 && (p->tfsf_i >= p->nx || p->bc_x == ORC_BC_PERIODIC))
    return -1;
  if (p->source_model < 0 || p->source_model > 1 || !(p->beta_rec >= 0.0) ||
      p->beta_rec > 2.0)
    return -1;
  orc_sim *s = calloc(1, sizeof(*s));
  if (!s) return -2;
  s->p = *p;
  derive(s);
  double dx = s->lambda / p->cells_per_lambda;
  double dt = p->courant * dx / C_0;
  /* numerical wavenumber of the 1-D Yee wave: sin(w dt/2)/(c dt) =
   * sin(k dx/2)/dx */
  s->ktil = 2.0 / dx * asin(sin(0.5 * s->omega * dt) / p->courant);
  int rc = level_init(&s->L0, p->nx, p->ny, dx, dt, spp, s->nu_m, p->courant);
  s->ex_old = calloc(n_ex(&s->L0), sizeof(double));
  s->ey_old = calloc(n_ey(&s->L0), sizeof(double));
  s->hz_prev = calloc(n_hz(&s->L0), sizeof(double));
  if (rc || !s->ex_old || !s->ey_old || !s->hz_prev) {
    orc_destroy(s);
    return -2;
  }
  if (seed_base)
    for (int j = 0; j <= p->ny; j++)
      for (int i = 0; i <= p->nx; i++)
        NODE(&s->L0, n, i, j) = seed_base[(size_t)j * (p->nx + 1) + i];
  if (p->mode != ORC_UNIFORM) {
    s->NBx = p->nx / p->block;
    s->NBy = p->ny / p->block;
    s->bflag = calloc((size_t)s->NBx * s->NBy, 1);
    s->bscan = calloc((size_t)s->NBx * s->NBy, sizeof(int32_t));
    s->blist = calloc((size_t)s->NBx * s->NBy, sizeof(int32_t));
    if (!s->bflag || !s->bscan || !s->blist) {
      orc_destroy(s);
      return -2;
    }
    if (p->regrid_rule == ORC_RULE_UNION) {
      s->act = calloc((size_t)s->NBx * s->NBy, 1);
      rc = level_init(&s->L1, p->r * p->nx, p->r * p->ny, dx / p->r, dt / p->r,
                      spp * p->r, s->nu_m, p->courant);
      s->hz_lo = calloc(n_hz(&s->L1), sizeof(double));
      s->hz_hi = calloc(n_hz(&s->L1), sizeof(double));
      if (rc || !s->act || !s->hz_lo || !s->hz_hi) {
        orc_destroy(s);
        return -2;
      }
    }
    if (p->mode == ORC_STATIC && p->regrid_rule == ORC_RULE_UNION) {
      /* the blocks covering static_ext (which must be whole blocks) */
      const int *e = p->static_ext, B = p->block;
      uint8_t *add = calloc((size_t)s->NBx * s->NBy, 1);
      rc = add ? 0 : -2;
      if (!rc && (e[0] % B || e[1] % B || e[2] % B || e[3] % B || e[0] >= e[2] ||
                  e[1] >= e[3]))
        rc = -1;
      for (int by = e[1] / B; !rc && by < e[3] / B; by++)
        for (int bx = e[0] / B; bx < e[2] / B; bx++) add[by * s->NBx + bx] = 1;
      if (!rc) rc = grow_union(s, add, seed_fine);
      free(add);
    } else if (p->mode == ORC_STATIC) {
      const int *e = p->static_ext;
      if (e[0] < 1 || e[1] < 1 || e[2] > p->nx - 1 || e[3] > p->ny - 1 ||
          e[0] >= e[2] || e[1] >= e[3] ||
          (p->tfsf_i > 0 && e[0] <= p->tfsf_i)) {
        orc_destroy(s);
        return -1;
      }
      rc = build_patch(s, e, seed_fine);
    } else {
      rc = do_regrid(s, seed_fine); /* the patch at t = 0 */
    }
    if (rc) {
      orc_destroy(s);
      return rc;
    }
  }
  *out = s;
  return 0;
}

void orc_destroy(orc_sim *s) {
  if (!s) return;
  level_free(&s->L0);
  if (s->has_patch || s->act) level_free(&s->L1);
  free(s->ex_old);
  free(s->ey_old);
  free(s->hz_prev);
  free(s->hz_lo);
  free(s->hz_hi);
  free(s->bflag);
  free(s->bscan);
  free(s->blist);
  free(s->act);
  free(s);
}

/* ---- field access ------------------------------------------------------- */
/* a level and the region of it that the field calls see: the whole base
 * level; the patch; for the union of blocks, the bounding box of the active
 * blocks on the full-domain fine arrays (entries outside the union are 0) */
typedef struct {
  const level_t *L;
  int i0, j0, nx, ny;
} view_t;

static int view_of(const orc_sim *s, int level, view_t *v) {
  if (level == 0) {
    *v = (view_t){&s->L0, 0, 0, s->L0.nx, s->L0.ny};
    return 0;
  }
  if (level == 1 && s->has_patch) {
    if (s->act) {
      const int r = s->p.r;
      *v = (view_t){&s->L1, r * s->ext[0], r * s->ext[1], r * (s->ext[2] - s->ext[0]),
                    r * (s->ext[3] - s->ext[1])};
    } else {
      *v = (view_t){&s->L1, 0, 0, s->L1.nx, s->L1.ny};
    }
    return 0;
  }
  return -1;
}

int orc_field_dims(const orc_sim *s, int field, int level, int32_t dims[2]) {
  view_t v;
  if (view_of(s, level, &v)) return -1;
  switch (field) {
  case ORC_HZ: dims[0] = v.ny; dims[1] = v.nx; break;
  case ORC_EX: case ORC_JX: dims[0] = v.ny + 1; dims[1] = v.nx; break;
  case ORC_EY: case ORC_JY: dims[0] = v.ny; dims[1] = v.nx + 1; break;
  case ORC_N: case ORC_ACC: case ORC_ERMS2:
    dims[0] = v.ny + 1; dims[1] = v.nx + 1; break;
  case ORC_RING: dims[0] = NRING * (v.ny + 1); dims[1] = v.nx + 1; break;
  default: return -1;
  }
  return 0;
}

/* visit every entry of a field in output order, handing out its address */
static double *field_ptr(const level_t *L, int field, int i, int j, int k) {
  switch (field) {
  case ORC_HZ: return &HZ(L, i, j);
  case ORC_EX: return &EX(L, i, j);
  case ORC_JX: return &JX(L, i, j);
  case ORC_EY: return &EY(L, i, j);
  case ORC_JY: return &JY(L, i, j);
  case ORC_N: return &NODE(L, n, i, j);
  case ORC_ACC: return &NODE(L, acc, i, j);
  case ORC_RING: return &RING(L, k, i, j);
  }
  return NULL;
}

int orc_get_field(const orc_sim *s, int field, int level, double *dst) {
  view_t v;
  int32_t d[2];
  if (view_of(s, level, &v) || orc_field_dims(s, field, level, d)) return -1;
  int planes = field == ORC_RING ? NRING : 1;
  int rows = d[0] / planes, cols = d[1];
  for (int k = 0; k < planes; k++)
    for (int j = 0; j < rows; j++)
      for (int i = 0; i < cols; i++) {
        int a = v.i0 + i, b = v.j0 + j;
        double val = field == ORC_ERMS2 ? erms2_at(v.L, a, b)
                                        : *field_ptr(v.L, field, a, b, k);
        dst[((size_t)k * rows + j) * cols + i] = val;
      }
  return 0;
}

int orc_set_field(orc_sim *s, int field, int level, const double *src) {
  view_t v;
  int32_t d[2];
  if (view_of(s, level, &v) || field == ORC_ERMS2 || orc_field_dims(s, field, level, d))
    return -1;
  int planes = field == ORC_RING ? NRING : 1;
  int rows = d[0] / planes, cols = d[1];
  for (int k = 0; k < planes; k++)
    for (int j = 0; j < rows; j++)
      for (int i = 0; i < cols; i++)
        *field_ptr(v.L, field, v.i0 + i, v.j0 + j, k) = src[((size_t)k * rows + j) * cols + i];
  return 0;
}

int orc_get_patch(const orc_sim *s, int32_t ext[4]) {
  for (int k = 0; k < 4; k++) ext[k] = s->has_patch ? s->ext[k] : 0;
  return 0;
}

int orc_get_regrid(const orc_sim *s, uint8_t *flags, int32_t *scan,
                   int32_t *list, int32_t *count) {
  if (s->p.mode == ORC_UNIFORM) return -1;
  size_t nb = (size_t)s->NBx * s->NBy;
  if (flags) memcpy(flags, s->bflag, nb);
  if (scan) memcpy(scan, s->bscan, nb * sizeof(int32_t));
  if (list) memcpy(list, s->blist, (size_t)s->bcount * sizeof(int32_t));
  if (count) *count = s->bcount;
  return 0;
}

int orc_time(const orc_sim *s, double *t, int64_t *step) {
  if (t) *t = (double)s->step * s->L0.dt;
  if (step) *step = s->step;
  return 0;
}

/* ---- test hooks: the coarse/fine transfers on the current layout -------
 * These expose the interface operators of Sec. III.C to the pins (exactness
 * on fields linear in space and time); the time stepping does not use them.
 * Arrays are in the public layout of the field calls. */

/* coarse E^n that Eq. (5b) interpolates from (base level, EX and EY) */
int orc_set_old_e(orc_sim *s, const double *ex, const double *ey) {
  if (!s || !ex || !ey) return -1;
  const level_t *C = &s->L0;
  for (int j = 0; j <= C->ny; j++)
    for (int i = 0; i < C->nx; i++)
      s->ex_old[(size_t)i * (C->ny + 1) + j] = ex[(size_t)j * C->nx + i];
  for (int j = 0; j < C->ny; j++)
    for (int i = 0; i <= C->nx; i++)
      s->ey_old[(size_t)i * C->ny + j] = ey[(size_t)j * (C->nx + 1) + i];
  return 0;
}

/* Eq. (5b) values at time fraction frac on every boundary edge of the fine
 * level (level-1 EX / EY layout); every other entry is set to NaN.  The
 * level's own fields are not changed. */
int orc_cfb_fill(orc_sim *s, double frac, double *ex, double *ey) {
  view_t v;
  if (!s || !ex || !ey || view_of(s, 1, &v)) return -1;
  const level_t *F = &s->L1;
  double *tx = malloc(n_ex(F) * sizeof(double)), *ty = malloc(n_ey(F) * sizeof(double));
  if (!tx || !ty) {
    free(tx);
    free(ty);
    return -2;
  }
  for (size_t k = 0; k < n_ex(F); k++) tx[k] = NAN;
  for (size_t k = 0; k < n_ey(F); k++) ty[k] = NAN;
  cfb_edges(s, frac, tx, ty);
  for (int j = 0; j <= v.ny; j++)
    for (int i = 0; i < v.nx; i++)
      ex[(size_t)j * v.nx + i] = tx[(size_t)(v.i0 + i) * (F->ny + 1) + v.j0 + j];
  for (int j = 0; j < v.ny; j++)
    for (int i = 0; i <= v.nx; i++)
      ey[(size_t)j * (v.nx + 1) + i] = ty[(size_t)(v.i0 + i) * F->ny + v.j0 + j];
  free(tx);
  free(ty);
  return 0;
}

/* the two fine Hz half levels the fine -> coarse transfer averages (level-1
 * HZ layout): lo after substep r/2; hi after substep r/2 + 1, which for
 * r = 2 is the level's own Hz (written there) */
int orc_set_hz_halves(orc_sim *s, const double *lo, const double *hi) {
  view_t v;
  if (!s || !lo || !hi || view_of(s, 1, &v)) return -1;
  level_t *F = &s->L1;
  double *dst_hi = s->p.r == 2 ? F->hz : s->hz_hi;
  for (int j = 0; j < v.ny; j++)
    for (int i = 0; i < v.nx; i++) {
      size_t a = (size_t)(v.i0 + i) * F->ny + v.j0 + j, b = (size_t)j * v.nx + i;
      s->hz_lo[a] = lo[b];
      dst_hi[a] = hi[b];
    }
  return 0;
}

/* the fine -> coarse transfer of the end of a base step */
int orc_restrict(orc_sim *s) {
  if (!s || !s->has_patch) return -1;
  if (s->act) restrict_union(s);
  else restrict_patch(s);
  return 0;
}

/* the density transfers of a sync point (without its continuity steps) */
int orc_transfer_density(orc_sim *s) {
  if (!s || !s->has_patch) return -1;
  if (s->act) transfer_density_union(s);
  else transfer_density(s);
  return 0;
}

/* out: omega, lambda, dx, dt, nu_m, n_c, eeff_fac, E_bd, E0, D_e, D_a, n_amb,
 * a, b, ktilde, nu_att, steps_per_period */
int orc_derived(const orc_params *p, double *out, int n_out) {
  orc_sim s;
  memset(&s, 0, sizeof(s));
  s.p = *p;
  derive(&s);
  double dx = s.lambda / p->cells_per_lambda;
  double dt = p->courant * dx / C_0;
  double a = exp(-s.nu_m * dt);
  double v[17] = {s.omega, s.lambda, dx, dt, s.nu_m, s.n_c, s.eeff_fac,
                  s.e0 / sqrt(2.0) / p->erms_over_ebd, s.e0, s.d_e, s.d_a,
                  s.n_amb, a, Q_E * Q_E * (1.0 - a) / (M_E * s.nu_m),
                  2.0 / dx * asin(sin(0.5 * s.omega * dt) / p->courant),
                  s.nu_att, p->cells_per_lambda / p->courant};
  for (int k = 0; k < n_out && k < 17; k++) out[k] = v[k];
  return 0;
}

/* worker threads of the marked loops; n <= 0: all processors */
int orc_set_threads(int n) {
#ifdef _OPENMP
  omp_set_num_threads(n > 0 ? n : omp_get_num_procs());
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

int orc_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
