/* oracle_drive.c -- runs the FP64 oracle through every code path (QED with
 * sub-cycling, tracked photons, conversion, injection, absorption, outflow,
 * merge, filter, periodic box, event record and replay, state loading) under
 * AddressSanitizer and UndefinedBehaviorSanitizer.  Test infrastructure. */
#include "../../oracle/oracle.c"

#include <stdio.h>

static orc_params tiny(void) {
  orc_params p;
  memset(&p, 0, sizeof p);
  p.n_cells = 256; p.init_kind = 1; p.ppc_init = 8; p.ppc_ref = 16;
  p.dx = 0.25; p.cfl = 0.45; p.alpha = 1.5; p.b = 0.1; p.r_curv_cm = 1e7; p.period_s = 1.0;
  p.lambda_c_scale = 1.7e5; p.r_curv_scale = 1.4e-5; p.h_gap_frac = 0.8;
  p.inj_rate = 0.1; p.inj_weight = 1.0; p.x_thr = 2.0; p.xc_floor = 1e-2; p.merge_frac = 0.5;
  p.seed = 3; p.cap_leptons = 5000; p.cap_photons = 1500; p.nsub_max = 64; p.merge_every = 8;
  return p;
}

int main(void) {
  int32_t err = 0;
  int64_t c[16];
  /* the tiny gap with QED, merging and recording */
  orc_params p = tiny();
  p.flags = ORC_MERGE_ON | ORC_RECORD;
  orc_sim* s = orc_create(&p, &err);
  if (!s) return 1;
  orc_step(s, 400);
  orc_counts(s, c);
  printf("tiny: leptons %lld photons %lld emissions %lld conversions %lld merged %lld events %lld\n",
         (long long)c[0], (long long)c[1], (long long)c[3], (long long)c[5], (long long)c[10], (long long)c[12]);
  if (c[5] == 0 || c[10] == 0 || c[12] == 0) { printf("a path was not reached\n"); return 2; }
  /* replay of the recorded realisation from the same start */
  int64_t n = c[12];
  int32_t* kind = malloc(sizeof(int32_t) * n); int32_t* sub = malloc(sizeof(int32_t) * n);
  int64_t* step = malloc(sizeof(int64_t) * n); uint64_t* id = malloc(sizeof(uint64_t) * n);
  double* x = malloc(sizeof(double) * n); int32_t* cell = malloc(sizeof(int32_t) * n);
  double* xi = malloc(sizeof(double) * n); double* w = malloc(sizeof(double) * n);
  orc_get_events(s, kind, sub, step, id, x, cell, xi, w);
  orc_params q = tiny();
  q.flags = ORC_REPLAY;
  orc_sim* r = orc_create(&q, &err);
  orc_set_replay(r, n, kind, sub, step, id, x, cell, xi, w);
  orc_set_replay(r, n, kind, sub, step, id, x, cell, xi, w);   /* installed twice: the first is released */
  orc_step(r, 100);
  free(kind); free(sub); free(step); free(id); free(x); free(cell); free(xi); free(w);
  double ret[ORC_RET_NB + 2];
  orc_return(s, ret);
  /* state loading and the merge hook */
  int32_t lc[3] = {1, 5, 250}; double lx[3] = {0.5, 0.25, 0.75}, lu[3] = {1e4, -3.0, 40.0}, lw[3] = {1, -1, 2};
  uint64_t lid[3] = {7, 8, 9};
  int32_t pc[2] = {3, 4}; double px[2] = {0.1, 0.2}, pxx[2] = {5e3, -8e3}, pw[2] = {1, 1};
  int64_t pn0[2] = {0, 0}; uint64_t pid[2] = {11, 12};
  orc_set_state(s, 3, lc, lx, lu, lw, lid, 2, pc, px, pxx, pw, pn0, pid, 0.5, 401);
  orc_merge_now(s);
  orc_step(s, 50);
  /* filtered periodic box and a frozen field */
  orc_params f = tiny();
  f.flags = ORC_FILTER | ORC_PERIODIC | ORC_QED_OFF;
  f.inj_rate = 0.0;
  orc_sim* t = orc_create(&f, &err);
  orc_step(t, 60);
  double E[256];
  orc_field(t, E);
  orc_params z = tiny();
  z.flags = ORC_FIELD_FROZEN | ORC_TRACK_ALL;
  orc_sim* u = orc_create(&z, &err);
  orc_set_field(u, E, 1.0);
  orc_step(u, 60);
  /* the physics entry points */
  double xs[4] = {1e-3, 0.3, 0.9, 0.999}, ys[4];
  orc_sync_inverse_many(xs, ys, 4);
  (void)orc_tsyn(0.5); (void)orc_tbw(2.0); (void)orc_sync_cdf(1.0);
  double buf[1024];
  orc_filter(buf, 0, 8, 0);
  for (int i = 0; i < 1024; ++i) buf[i] = i;
  orc_filter(buf, 1024, 8, 1);
  orc_free(s); orc_free(r); orc_free(t); orc_free(u);
  printf("ORACLE OK\n");
  return 0;
}
