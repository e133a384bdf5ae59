/*
 * oracle.h -- FP64 CPU oracle of the coupled EM / plasma-fluid update with
 * dynamic mesh refinement (Ghosh & Chaudhury, "Efficient Dynamic Mesh
 * Refinement Technique for Simulation of HPM Breakdown induced Plasma Pattern
 * Formation").
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against a plain, slow, obviously correct implementation.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header, table or constant with the GPU library.
 *
 * What it computes (paper section / equation in brackets):
 *   - Maxwell TE_z on a Yee grid, Eqs. (1)-(2) [Sec. II.B]
 *   - electron momentum in current form, J = -e n v, Eq. (3), with a
 *     semi-implicit exponential-trapezoid E-J coupling
 *   - a one-period sliding E_rms window and the continuity step, Eq. (4),
 *     with effective-field ionisation and an effective-diffusion blend
 *   - one r = 2 (or 4) fine patch with time subcycling, Eq. (5b) boundary
 *     transfer, restriction back to the coarse mesh, and the self-aware
 *     expansion of Sec. III.D (threshold + gradient-length flags on 16x16
 *     blocks, prefix sum compaction, bounding-box growth; or the threshold
 *     lines on the patch sides with steps m_ex, m_ey; Eq. (5a)
 *     prolongation); or, as a variant, a fine level that is the union of the
 *     flagged blocks themselves.
 * All floating-point state is double.  The regrid flag decision is taken in
 * binary32 (the precision of the GPU kernels) so that both sides decide on
 * identical inputs identically.
 *
 * Field layout returned by orc_get_field / taken by orc_set_field:
 * row-major, y rows, x fastest, no padding:
 *   HZ  [ny  ][nx  ]   cell centres (i+1/2, j+1/2)
 *   EX  [ny+1][nx  ]   x-edges      (i+1/2, j)      (JX likewise)
 *   EY  [ny  ][nx+1]   y-edges      (i, j+1/2)      (JY likewise)
 *   N, ACC, ERMS2 [ny+1][nx+1] nodes (i, j); RING = 8 node planes.
 * For level 1 (the fine patch) nx, ny are the patch size in fine cells; for
 * the union of blocks, the size of its bounding box (entries outside the
 * union read 0).
 * Units are SI.  Functions return 0 on success and a negative code on error.
 */
#ifndef DMR_ORACLE_H
#define DMR_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_BC_MUR = 0, ORC_BC_PEC = 1, ORC_BC_PERIODIC = 2 };
enum { ORC_UNIFORM = 0, ORC_STATIC = 1, ORC_DYNAMIC = 2 };
enum { ORC_D_BLEND = 0, ORC_D_CONST = 1 };
enum { ORC_RULE_BLOCKS = 0, ORC_RULE_LINES = 1, ORC_RULE_UNION = 2 };
enum { ORC_SOURCE_POWER = 0, ORC_SOURCE_TOWNSEND = 1 };
enum {
  ORC_HZ = 0, ORC_EX = 1, ORC_EY = 2, ORC_JX = 3, ORC_JY = 4,
  ORC_N = 5, ORC_ACC = 6, ORC_ERMS2 = 7, ORC_RING = 8
};

typedef struct orc_params {
  /* wave and gas */
  double freq_hz;          /* incident frequency f */
  double erms_over_ebd;    /* incident rms field / breakdown field */
  double p_torr;           /* gas pressure */
  /* ionisation fit: nu_net = nu_m*A*[(E_eff/p)^beta - (E_cr/p)^beta] */
  double A_ion, beta_ion, ecr_over_p; /* E/p in V/(cm Torr) */
  /* diffusion */
  double te_ev, ti_ev, mu_i_760, L_amb, d_const;
  /* refinement criteria */
  double n_thr_over_nc, grad_thr, n_floor_over_nc;
  double courant;          /* S = c dt / dx on every level */
  double fine_filter;      /* gamma of the fine-patch E hyper-diffusion */
  int32_t nx, ny;          /* base-level cells */
  int32_t cells_per_lambda;/* base-level N_lambda */
  int32_t r;               /* refinement factor (2) */
  int32_t block;           /* regrid block edge in base cells */
  int32_t regrid_every;    /* base steps between regrids */
  int32_t tfsf_i;          /* TF/SF node column on the base level; <=0: off */
  int32_t ramp_periods;    /* sin^2 ramp length */
  int32_t bc_x, bc_y;      /* ORC_BC_* */
  int32_t mode;            /* ORC_UNIFORM / ORC_STATIC / ORC_DYNAMIC */
  int32_t static_ext[4];   /* I0, J0, I1, J1 in base cells (ORC_STATIC) */
  int32_t d_mode;          /* ORC_D_* */
  int32_t continuity_on;   /* 0 freezes n (and skips the window) */
  /* growth rule of ORC_DYNAMIC: ORC_RULE_BLOCKS (flags, 16x16 blocks,
   * bounding box) or ORC_RULE_LINES (threshold lines on the patch sides,
   * Sec. III.D): initial m_lx x m_ly cells centred on the seed peak; a side
   * whose line has a node with n > n_line moves out by m_ex (x) / m_ey (y);
   * or ORC_RULE_UNION: the fine level is the union of the flagged blocks
   * themselves (with ORC_STATIC: the blocks of static_ext, whole blocks) */
  int32_t regrid_rule;
  int32_t m_lx, m_ly, m_ex, m_ey;
  double n_line;           /* m^-3 */
  /* source of Eq. (4): ORC_SOURCE_POWER (the net power law above) or
   * ORC_SOURCE_TOWNSEND: nu_i - nu_a = gamma v_d - nu_att with the Townsend
   * coefficient gamma = A_town p exp(-B_town p / E_eff) (A_town 1/(cm Torr),
   * B_town V/(cm Torr)) and the drift velocity v_d = e E_eff / (m nu_m);
   * recombination r_ei = beta_rec 1e-13 (300/T_e[K])^(1/2) m^3/s */
  int32_t source_model;
  double A_town, B_town, nu_att, beta_rec;
} orc_params;

typedef struct orc_sim orc_sim;

/* seed_base: node densities of the base level, [ny+1][nx+1] (NULL: zero).
 * seed_fine: node densities on the full-domain fine grid [r*ny+1][r*nx+1],
 * used for the fine patch built at t = 0 (NULL: prolong from seed_base). */
int orc_create(const orc_params *p, const double *seed_base,
               const double *seed_fine, orc_sim **out);
void orc_destroy(orc_sim *s);
int orc_step(orc_sim *s, int64_t n_base_steps);
int orc_regrid(orc_sim *s);
int orc_get_patch(const orc_sim *s, int32_t ext[4]);
int orc_field_dims(const orc_sim *s, int field, int level, int32_t dims[2]);
int orc_get_field(const orc_sim *s, int field, int level, double *dst);
int orc_set_field(orc_sim *s, int field, int level, const double *src);
/* block flags [NBy][NBx], exclusive scan, compacted list, count of the last
 * regrid test */
int orc_get_regrid(const orc_sim *s, uint8_t *flags, int32_t *scan,
                   int32_t *list, int32_t *count);
int orc_time(const orc_sim *s, double *t, int64_t *step);
/* ORC_RULE_UNION: add blocks (mask [NBy][NBx], growth only; a block outside
 * the margins is an error) / read the active blocks */
int orc_add_blocks(orc_sim *s, const uint8_t *mask);
int orc_get_blocks(const orc_sim *s, uint8_t *dst);
/* Test hooks: the coarse/fine transfers of Sec. III.C on the current layout,
 * for the pins (arrays in the field-call layout; see the source):
 * orc_set_old_e sets the coarse E^n that Eq. (5b) interpolates from;
 * orc_cfb_fill writes the Eq. (5b) values at time fraction frac on the fine
 * level's boundary edges (NaN elsewhere) without changing the level;
 * orc_set_hz_halves sets the two fine Hz half levels the fine -> coarse
 * transfer averages; orc_restrict runs that transfer; orc_transfer_density
 * runs the density transfers of a sync point. */
int orc_set_old_e(orc_sim *s, const double *ex, const double *ey);
int orc_cfb_fill(orc_sim *s, double frac, double *ex, double *ey);
int orc_set_hz_halves(orc_sim *s, const double *lo, const double *hi);
int orc_restrict(orc_sim *s);
int orc_transfer_density(orc_sim *s);
/* OpenMP worker threads of the loops over independent entities (results are
 * bit-identical for any count); n <= 0: all processors.  Both return the
 * count in use (1 in a build without OpenMP). */
int orc_set_threads(int n);
int orc_get_threads(void);
/* derived scalars, for pins: see orc_derived in the source */
int orc_derived(const orc_params *p, double *out, int n_out);
/* net ionisation rate for a given E_rms^2 (V^2/m^2) */
double orc_nu_net(const orc_params *p, double erms2);
/* recombination coefficient r_ei, m^3/s */
double orc_r_ei(const orc_params *p);
double orc_d_eff(const orc_params *p, double n);
/* one continuity step on given node arrays (layout as the fields above),
 * zero-flux or periodic outer faces */
int orc_continuity_apply(const orc_params *p, int nx, int ny, double dx,
                         double dtn, int perx, int pery, const double *n_in,
                         const double *erms2, double *n_out);

#ifdef __cplusplus
}
#endif
#endif
