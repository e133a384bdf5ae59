/*
 * sanitize_main.c -- a small driver of the FP64 oracle for sanitizer builds
 * (test infrastructure only): runs short uniform, static-patch, dynamic
 * (bounding box, threshold lines, union of blocks) and r = 4 cases through
 * every public call, so that an AddressSanitizer / UndefinedBehaviorSanitizer
 * build of the oracle sees all of its code paths.  Exit status 0 on success.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static void defaults(orc_params *p, int nx, int ny, int cpl, int mode) {
  memset(p, 0, sizeof(*p));
  p->freq_hz = 110e9;
  p->erms_over_ebd = 3.0;
  p->p_torr = 700.0;
  p->A_ion = 9.02e-14;
  p->beta_ion = 5.3;
  p->ecr_over_p = 2.5e6 / 760.0 / 100.0;
  p->te_ev = 2.0;
  p->ti_ev = 0.025;
  p->mu_i_760 = 2.0e-4;
  p->L_amb = 299792458.0 / 110e9 / 20.0;
  p->d_const = 0.05;
  p->n_thr_over_nc = 1e-3;
  p->grad_thr = 0.2;
  p->n_floor_over_nc = 1e-6;
  p->courant = 0.5;
  p->fine_filter = 1e-4;
  p->nx = nx;
  p->ny = ny;
  p->cells_per_lambda = cpl;
  p->r = 2;
  p->block = 8;
  p->regrid_every = 2 * (int)(cpl / p->courant);
  p->tfsf_i = cpl / 4;
  p->ramp_periods = 2;
  p->bc_x = ORC_BC_MUR;
  p->bc_y = ORC_BC_MUR;
  p->mode = mode;
  p->d_mode = ORC_D_BLEND;
  p->continuity_on = 1;
  p->m_lx = p->m_ly = 8;
  p->m_ex = 8;
  p->m_ey = 4;
  p->n_line = 1e15;
}

/* Gaussian seed, peak n0 at cell (cx, cy), sigma in cells */
static double *seed(int nx, int ny, double cx, double cy, double n0, double sig) {
  double *s = calloc((size_t)(nx + 1) * (ny + 1), sizeof(double));
  for (int j = 0; j <= ny; j++)
    for (int i = 0; i <= nx; i++)
      s[(size_t)j * (nx + 1) + i] =
          n0 * exp(-((i - cx) * (i - cx) + (j - cy) * (j - cy)) / (sig * sig));
  return s;
}

static int read_all(orc_sim *s) {
  const int fields[] = {ORC_HZ, ORC_EX, ORC_EY, ORC_JX, ORC_JY, ORC_N, ORC_ACC, ORC_ERMS2, ORC_RING};
  for (int lv = 0; lv < 2; lv++)
    for (int k = 0; k < 9; k++) {
      int32_t d[2];
      if (orc_field_dims(s, fields[k], lv, d)) {
        if (lv == 0) return 1;
        continue; /* no patch */
      }
      double *b = malloc((size_t)d[0] * d[1] * sizeof(double));
      if (orc_get_field(s, fields[k], lv, b)) { free(b); return 1; }
      if (fields[k] != ORC_ERMS2 && orc_set_field(s, fields[k], lv, b)) { free(b); return 1; }
      free(b);
    }
  return 0;
}

static int run(const orc_params *p, const double *sb, int steps, const char *tag) {
  orc_sim *s = NULL;
  int rc = orc_create(p, sb, NULL, &s);
  if (rc) { fprintf(stderr, "%s: create %d\n", tag, rc); return 1; }
  rc = orc_step(s, steps);
  if (!rc) rc = read_all(s);
  if (!rc && p->mode == ORC_DYNAMIC) rc = orc_regrid(s);
  int32_t ext[4];
  orc_get_patch(s, ext);
  if (!rc && p->mode != ORC_UNIFORM) {
    int nb = (p->nx / p->block) * (p->ny / p->block);
    uint8_t *f = calloc(nb, 1);
    int32_t *sc = calloc(nb, sizeof(int32_t)), *l = calloc(nb, sizeof(int32_t)), cnt;
    rc = orc_get_regrid(s, f, sc, l, &cnt);
    if (!rc && p->regrid_rule == ORC_RULE_UNION) {
      rc = orc_get_blocks(s, f);
      memset(f, 0, nb);
      f[(p->ny / p->block - 2) * (p->nx / p->block) + p->nx / p->block - 2] = 1;
      if (!rc) rc = orc_add_blocks(s, f);
      if (!rc) rc = orc_step(s, 4);
    }
    free(f); free(sc); free(l);
  }
  double t; int64_t st;
  orc_time(s, &t, &st);
  orc_destroy(s);
  if (rc) { fprintf(stderr, "%s: rc %d\n", tag, rc); return 1; }
  printf("%s: ok, %lld steps, patch %d %d %d %d\n", tag, (long long)st, ext[0], ext[1], ext[2], ext[3]);
  return 0;
}

int main(void) {
  orc_params p;
  int bad = 0;
  double *sb = seed(96, 48, 60.5, 24.0, 3e17, 1.6);
  defaults(&p, 96, 48, 32, ORC_UNIFORM);
  bad |= run(&p, sb, 200, "uniform");
  defaults(&p, 96, 48, 32, ORC_STATIC);
  p.static_ext[0] = 48; p.static_ext[1] = 16; p.static_ext[2] = 72; p.static_ext[3] = 32;
  bad |= run(&p, sb, 200, "static");
  defaults(&p, 96, 48, 32, ORC_DYNAMIC);
  bad |= run(&p, sb, 300, "dynamic-blocks");
  defaults(&p, 96, 48, 32, ORC_DYNAMIC);
  p.regrid_rule = ORC_RULE_LINES;
  bad |= run(&p, sb, 300, "dynamic-lines");
  defaults(&p, 96, 48, 32, ORC_DYNAMIC);
  p.regrid_rule = ORC_RULE_UNION;
  bad |= run(&p, sb, 300, "dynamic-union");
  defaults(&p, 96, 48, 32, ORC_DYNAMIC);
  p.source_model = ORC_SOURCE_TOWNSEND;
  p.A_town = 15.0; p.B_town = 365.0; p.nu_att = 3.7e7; p.beta_rec = 1.0;
  bad |= run(&p, sb, 200, "townsend");
  free(sb);
  sb = seed(48, 24, 30.25, 12.0, 3e17, 0.8);
  defaults(&p, 48, 24, 16, ORC_DYNAMIC);
  p.r = 4;
  bad |= run(&p, sb, 200, "r4");
  free(sb);
  double nin[9 * 9], e2[9 * 9], nout[9 * 9];
  for (int k = 0; k < 81; k++) { nin[k] = 1e16 * (1 + k % 3); e2[k] = 1e13; }
  defaults(&p, 8, 8, 32, ORC_UNIFORM);
  bad |= orc_continuity_apply(&p, 8, 8, 1e-4, 1e-9, 1, 0, nin, e2, nout) != 0;
  double out[17];
  orc_derived(&p, out, 17);
  return bad;
}
