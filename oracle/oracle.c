/*
 * oracle.c -- plain, slow FP64 CPU oracle of the 1D radiative PIC step of the
 * polar-cap pair discharge (Natttila & Salmi, "Pair Discharges and Radio
 * Emission from Pulsar Magnetospheres", Sects. 2-4 and 6.1).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant generator with the HIP path of the package.
 *
 * Every routine follows the passage named in its comment.  Normalised units:
 * lengths in the co-rotation skin depth d = c/omega_p,co, times in
 * 1/omega_p,co, c = 1, u = gamma*beta, E in m_e c omega_p,co / e, charge
 * density in e n_co (Sect. 2.2, eq. for n_co and omega_p,co^2 = Omega omega_B).
 *
 * Single-threaded on purpose: nothing here is blocked, fused or reordered.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Physical constants (CGS, CODATA values).                            */
/* ------------------------------------------------------------------ */
#define ORC_C_LIGHT   2.99792458e10      /* cm/s                       */
#define ORC_E_OVER_MC 1.75882001076e7    /* e/(m_e c), 1/(G s)          */
#define ORC_LAMBDA_C  3.8615926796e-11   /* reduced Compton wavelength  */
#define ORC_B_Q       4.41400e13         /* Schwinger field m^2c^3/(hbar e), G */
#define ORC_ALPHA_EM  (1.0 / 137.035999084)
#define ORC_PI        3.14159265358979323846

/* Fixed-point scale of the charge deposit: a unit-weight particle carries
 * 2^F integer charge units. */
#define ORC_FP_BITS 24
#define ORC_FP_ONE  16777216.0
#define ORC_RET_NB  64                 /* return-flux bins: 1/8 decade of gamma each */

/* Flags (bit values are part of the interface between the two sides). */
#define ORC_QED_OFF      1u
#define ORC_ETA_CO_OFF   2u
#define ORC_FIELD_FROZEN 4u
#define ORC_RECOIL_OFF   8u
#define ORC_PERIODIC     16u
#define ORC_MERGE_ON     32u
#define ORC_TRACK_ALL    64u
#define ORC_ANTI_ALIGNED 128u
#define ORC_RECORD       256u
#define ORC_REPLAY       512u
#define ORC_CONV_OFF     1024u
#define ORC_EMIT_OFF     2048u
#define ORC_INJ_FIXED    4096u   /* injection count independent of inj_weight */
#define ORC_FILTER       8192u   /* binomial current filter, ORC_FILTER_PASSES passes per step */
#define ORC_QUANTUM      16384u  /* quantum photon spectrum and pair split (Sect. 3.1, 3.2)    */
#define ORC_FILTER_PASSES 8

/* Random-stream tags (upper 16 bits of the fourth counter word). */
#define TAG_INIT  1u
#define TAG_EMIT  2u
#define TAG_CONV  3u
#define TAG_INJ   4u
#define TAG_MERGE 5u
#define TAG_CHILD 6u

#define INJ_ID_BASE (1ull << 62)
#define ATM_ID_BASE (3ull << 61)
#define TAG_ATM   7u
#define ORC_MASS_P 1836.0      /* proton to electron mass ratio (Sect. 6.1) */

/* error codes */
#define ORC_OK     0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_ECAP   (-3)

typedef struct {
  int32_t n_cells;
  int32_t init_kind;     /* 0 vacuum below H + e- above; 1 uniform e+-; 2 empty; 3 uniform e- */
  int32_t ppc_init;
  int32_t ppc_ref;
  double dx, cfl, alpha, b, r_curv_cm, period_s;
  double lambda_c_scale, r_curv_scale, h_gap_frac;
  double inj_rate;       /* charge injected per step, in units of n_co*dx */
  double inj_weight;     /* weight of one injected macro-electron (units w0) */
  double x_thr;          /* minimum stored photon energy (m_e c^2) */
  double xc_floor;       /* emission evaluated only if x_c(gamma) >= floor */
  double u_init;         /* initial momentum of init particles */
  double merge_frac;     /* merge when count > merge_frac * cap */
  uint64_t seed;
  int64_t cap_leptons, cap_photons;
  uint32_t flags;
  int32_t nsub_max;      /* sub-cycling cap */
  int32_t merge_every;   /* merge check period (steps) */
  int32_t pad_;
  double atm_temp;       /* atmosphere temperature k_B T / (m_e c^2) */
  int32_t atm_ppc;       /* atmosphere: electrons and protons kept in cell 0 (0: none) */
  int32_t pad2_;
} orc_params;

typedef struct { int32_t cell; double xi, u, w; uint64_t id; } olep;
typedef struct { int32_t cell; double xi, x, w; int64_t n0; uint64_t id; } opho;

/* A recorded QED event.  kind 0: emission by lepton `id` (x = signed photon
 * energy, dir * x); kind 1: conversion of photon `id`; kind 2: birth of the
 * tracked photon `id` at (cell, xi) with signed energy x and weight w. */
typedef struct { int32_t kind, sub; int64_t step; uint64_t id; double x; int32_t cell; double xi, w; } oevent;

typedef struct {
  orc_params p;
  /* derived */
  double d_cm, lam, rc, lr, dt, H, w0, s_co;
  int32_t N;
  /* state */
  olep* lep; int64_t nlep, lep_alloc;
  opho* pho; int64_t npho, pho_alloc;
  olep* pro; int64_t npro, pro_alloc;   /* protons (charge +1, mass ORC_MASS_P) */
  double* E;     /* E at cell centres k+1/2, k = 0..N-1 */
  double* E0;    /* filtered runs: the field when the state was last set */
  double* Eb;    /* node field, nodes 0..N */
  int64_t* rho;  /* node charge, fixed point, nodes 0..N */
  double Es;
  int64_t dq;    /* surface charge since the last field update (fixed point) */
  double dcur;   /* periodic mode: sum of charge x displacement (w0 * cells) this step */
  double inj_acc;
  uint64_t inj_count;
  int64_t step;
  int32_t err;
  /* counters */
  int64_t n_emit, n_pho_born, n_conv, n_absorbed, n_outflow, n_pho_exit, n_dropped, n_merged;
  int64_t n_emit_eval, n_conv_eval;
  int64_t n_pro_absorbed, n_pro_outflow, n_atm_e, n_atm_p;
  int64_t atm_prev[2];   /* electrons / protons in cell 0 after the last push */
  uint64_t atm_count;    /* atmosphere particles created (their ids) */
  double e_rad;  /* radiated energy (m_e c^2 units, weighted) */
  /* return flux (Sect. 5, Fig. 7): weight of the leptons absorbed at h = 0
   * per 1/8 decade of gamma in [1, 1e8), then total weight and weight x gamma */
  double ret[ORC_RET_NB + 2];
  /* event log */
  oevent* ev; int64_t nev, ev_alloc;
  /* replay cursor (events sorted by step when replaying) */
  const oevent* rep; int64_t nrep;
  /* synchrotron quadrature nodes */
  int32_t nq; double qh; double* q_cosh; double* q_g;
} orc_sim;

/* ------------------------------------------------------------------ */
/* Philox4x32-10, written from Salmon, Moraes, Dror & Shaw (SC'11):     */
/* ten rounds of two 32x32->64 multiplies with a Weyl-sequence key.     */
/* ------------------------------------------------------------------ */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    uint64_t pa = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t pb = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t y0 = (uint32_t)(pb >> 32) ^ x1 ^ k0;
    uint32_t y1 = (uint32_t)pb;
    uint32_t y2 = (uint32_t)(pa >> 32) ^ x3 ^ k1;
    uint32_t y3 = (uint32_t)pa;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static void draw(uint64_t seed, uint64_t id, int64_t step, uint32_t tag, uint32_t sub, uint32_t out[4]) {
  uint32_t c[4] = {(uint32_t)id, (uint32_t)(id >> 32), (uint32_t)step, (tag << 16) | (sub & 0xFFFFu)};
  uint32_t k[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  orc_philox(c, k, out);
}

/* 24-bit uniform on the open interval (0,1): midpoint of the k-th bin. */
static double u24(uint32_t r) { return ((double)(r >> 8) + 0.5) / 16777216.0; }

/* Positions drawn at random sit on the 2^-24 grid of a cell: xi = k 2^-24. */
static double xi24(uint32_t r) { return (double)(r >> 8) / 16777216.0; }

static uint64_t child_id(uint64_t seed, uint64_t parent, int64_t step, uint32_t j) {
  uint32_t r[4];
  draw(seed, parent, step, TAG_CHILD, j, r);
  return (uint64_t)r[0] | ((uint64_t)r[1] << 32);
}

/* ------------------------------------------------------------------ */
/* QED rate functions (Sect. 3).                                        */
/* ------------------------------------------------------------------ */
/* Emission-rate function T_syn, the fit quoted with eq. tau_syn. */
double orc_tsyn(double chi) {
  double s3 = sqrt(3.0);
  return 5.0 / (2.0 * s3) * pow(1.0 + 16.0 * s3 / 5.0 * chi + 1.1 * chi * chi, -1.0 / 6.0);
}

/* Pair-creation function T_BW, the fit quoted with eq. tau_bw. */
double orc_tbw(double chi) {
  if (!(chi > 0.0)) return 0.0;
  return 0.23 * exp(-8.0 / (3.0 * chi)) * pow(1.0 + 0.22 * chi, -1.0 / 3.0);
}

/* ------------------------------------------------------------------ */
/* Classical synchrotron photon-number spectrum (reading of S(gamma,x)): */
/*   dN/dxi ~ F1(xi) = int_xi^inf K_{5/3}(t) dt,  xi = x / x_c.          */
/* With K_nu(t) = int_0^inf exp(-t cosh s) cosh(nu s) ds the t-integrals */
/* are done in closed form:                                             */
/*   F1(xi)  = int_0^inf exp(-xi cosh s) cosh(5s/3) / cosh s  ds         */
/*   1-C(xi) = (3/5pi) int_0^inf exp(-xi cosh s) cosh(5s/3)/cosh^2 s ds  */
/* (normalisation int_0^inf cosh(5s/3)/cosh^2 s ds = 5pi/3).             */
/* The integrands are even and analytic in a strip of half-width pi/2,  */
/* so the trapezoidal rule on s in [0, S] converges geometrically.      */
/* ------------------------------------------------------------------ */
static void sync_nodes(orc_sim* s) {
  s->qh = 0.125;
  s->nq = (int32_t)(240.0 / s->qh) + 1;
  s->q_cosh = (double*)malloc(sizeof(double) * s->nq);
  s->q_g = (double*)malloc(sizeof(double) * s->nq);
  for (int i = 0; i < s->nq; ++i) {
    double x = i * s->qh;
    double ch = cosh(x);
    s->q_cosh[i] = ch;
    s->q_g[i] = cosh(5.0 * x / 3.0) / (ch * ch) * (i == 0 ? 0.5 : 1.0) * s->qh;
  }
}

/* tail(xi) = 1 - C(xi) and its derivative -dC/dxi = -(3/5pi) F1(xi). */
static void sync_tail(const orc_sim* s, double xi, double* tail, double* dens) {
  double t = 0.0, f = 0.0;
  for (int i = 0; i < s->nq; ++i) {
    double a = xi * s->q_cosh[i];
    if (a > 745.0) break;
    double e = exp(-a) * s->q_g[i];
    t += e;
    f += e * s->q_cosh[i];
  }
  *tail = t * 3.0 / (5.0 * ORC_PI);
  *dens = f * 3.0 / (5.0 * ORC_PI);
}

/* Newton on log(xi) with a bisection bracket: C(xi) = r. */
static double sync_inverse(const orc_sim* s, double r) {
  double lo = -80.0, hi = 5.0;           /* log(xi) bracket */
  double y;
  if (r < 0.5) y = 3.0 * log(r / 1.2316); /* C ~ 1.2316 xi^(1/3) as xi -> 0 */
  else y = log(-log(1.0 - r) + 1e-300);
  if (!(y > lo && y < hi)) y = 0.5 * (lo + hi);
  for (int it = 0; it < 200; ++it) {
    double xi = exp(y), tail, dens;
    sync_tail(s, xi, &tail, &dens);
    double c = 1.0 - tail;
    double g = c - r;
    if (g > 0) hi = y; else lo = y;
    double dy = -g / (dens * xi);
    double yn = y + dy;
    if (!(yn > lo && yn < hi) || !isfinite(yn)) yn = 0.5 * (lo + hi);
    if (fabs(yn - y) < 1e-14 || hi - lo < 1e-14) { y = yn; break; }
    y = yn;
  }
  return exp(y);
}

/* ------------------------------------------------------------------ */
/* Quantum-corrected spectra (optional, flag ORC_QUANTUM).  The paper    */
/* names the first-order QED rates it builds on (Sect. 3.1: the photon   */
/* spectrum S(gamma, x) and the Gaunt factor g_Q of P_syn; Sect. 3.2:    */
/* the one-photon pair creation rate) without printing the spectra.      */
/* Reading: the textbook first-order forms, in units where the rates of  */
/* eqs. tau_syn and tau_bw are alpha_em b sin(psi) / t_C times           */
/*   T_syn(chi) = 1/(sqrt3 pi chi) int_0^1 s(d) dd,                      */
/*   s(d) = (1 - d + 1/(1-d)) K_{2/3}(z) - Ki_{1/3}(z),                 */
/*   z = 2 d / (3 chi (1 - d)),  d = x / gamma (photon energy fraction); */
/*   T_BW(chi) = 1/(sqrt3 pi chi) int_0^1 p(v) dv,                       */
/*   p(v) = (v/(1-v) + (1-v)/v) K_{2/3}(e) + Ki_{1/3}(e),               */
/*   e = 2 / (3 chi v (1 - v)),  v = gamma_- / x (electron fraction);    */
/* with Ki_nu(z) = int_z^inf K_nu.  For chi -> 0, s dd reduces to the     */
/* classical number spectrum int_z^inf K_{5/3} dz of the classical      */
/* sampler above, and the Gaunt factor is                                */
/*   g_Q(chi) = sqrt3/(2 pi chi^2) int_0^1 d s(d) dd.                    */
/* ------------------------------------------------------------------ */

/* K_{2/3}(z) e^off and Ki_{1/3}(z) e^off from
 *   K_nu(z) = int_0^inf exp(-z cosh u) cosh(nu u) du,
 *   Ki_nu(z) = int_0^inf exp(-z cosh u) cosh(nu u) / cosh u du,
 * by the trapezoidal rule (step 1/16; the integrands are analytic in a strip
 * of half-width pi/2, so the rule converges geometrically). */
static void bessel_k23_ki13(double z, double off, double* k23, double* ki13) {
  const double h = 1.0 / 16.0;
  double a = 0.0, b = 0.0;
  for (int i = 0; i < 16 * 100; ++i) {      /* u < 100: z cosh u > 745 for every z > 1e-40 */
    double u = i * h, c = cosh(u);
    double ex = z * c - off;
    if (ex > 745.0) break;
    double e = exp(-ex) * (i == 0 ? 0.5 : 1.0);
    a += e * cosh(2.0 * u / 3.0);
    b += e * cosh(u / 3.0) / c;
  }
  *k23 = a * h;
  *ki13 = b * h;
}

/* 8-point Gauss-Legendre nodes and weights on [-1, 1]. */
static const double GL8_X[8] = {-0.9602898564975363, -0.7966664774136267, -0.5255324099163290,
                                -0.1834346424956498, 0.1834346424956498, 0.5255324099163290,
                                0.7966664774136267, 0.9602898564975363};
static const double GL8_W[8] = {0.1012285362903763, 0.2223810344533745, 0.3137066458778873,
                                0.3626837833783620, 0.3626837833783620, 0.3137066458778873,
                                0.2223810344533745, 0.1012285362903763};

/* Photon spectrum per unit t, z = t^3: s(d(z)) dd/dz dz/dt, with
 * d = 3 chi z / (2 + 3 chi z).  `moment` 1 multiplies by d. */
static double qsyn_dens_t(double chi, double t, int moment) {
  double z = t * t * t;
  double q = 2.0 + 3.0 * chi * z;
  double d = 3.0 * chi * z / q, omd = 2.0 / q;
  double k23, ki13;
  bessel_k23_ki13(z, 0.0, &k23, &ki13);
  double sd = (omd + 1.0 / omd) * k23 - ki13;
  double v = sd * (6.0 * chi / (q * q)) * 3.0 * t * t;
  return moment ? v * d : v;
}

#define QSYN_TMAX 3.915     /* z = 60: the spectrum there is below e^-60 of its peak */
#define QSYN_PANELS 80

static double gl8(double (*f)(double, double, int), double chi, int moment, double a, double b) {
  double m = 0.5 * (a + b), r = 0.5 * (b - a), acc = 0.0;
  for (int k = 0; k < 8; ++k) acc += GL8_W[k] * f(chi, m + r * GL8_X[k], moment);
  return acc * r;
}

/* int_0^1 s(d) dd (moment 0) or int_0^1 d s(d) dd (moment 1). */
static double qsyn_total(double chi, int moment) {
  const double dt = QSYN_TMAX / QSYN_PANELS;
  double acc = 0.0;
  for (int i = 0; i < QSYN_PANELS; ++i) acc += gl8(qsyn_dens_t, chi, moment, i * dt, (i + 1) * dt);
  return acc;
}

/* Emission rate function from the spectrum (compare the fit orc_tsyn). */
double orc_qsyn_T(double chi) { return qsyn_total(chi, 0) / (sqrt(3.0) * ORC_PI * chi); }

/* Gaunt factor g_Q = P_syn / P_classical. */
double orc_qsyn_g(double chi) { return sqrt(3.0) / (2.0 * ORC_PI * chi * chi) * qsyn_total(chi, 1); }

/* Fraction of emitted photons with energy fraction below d. */
double orc_qsyn_cdf(double chi, double d) {
  if (!(d > 0.0)) return 0.0;
  if (!(d < 1.0)) return 1.0;
  double t = cbrt(2.0 * d / (3.0 * chi * (1.0 - d)));
  const double dt = QSYN_TMAX / QSYN_PANELS;
  double acc = 0.0;
  for (int i = 0; i < QSYN_PANELS; ++i) {
    double a = i * dt, b = (i + 1) * dt;
    if (a >= t) break;
    acc += gl8(qsyn_dens_t, chi, 0, a, b < t ? b : t);
  }
  if (t > QSYN_TMAX) acc += 0.0;   /* beyond z = 60 nothing is left */
  return acc / qsyn_total(chi, 0);
}

/* Energy fraction d with cdf(d) = r: the panel holding r, then Newton on t
 * inside it (bisection bracket). */
double orc_qsyn_inverse(double chi, double r) {
  const double dt = QSYN_TMAX / QSYN_PANELS;
  double part[QSYN_PANELS], tot = 0.0;
  for (int i = 0; i < QSYN_PANELS; ++i) {
    part[i] = gl8(qsyn_dens_t, chi, 0, i * dt, (i + 1) * dt);
    tot += part[i];
  }
  double target = r * tot, acc = 0.0;
  int i = 0;
  while (i < QSYN_PANELS - 1 && acc + part[i] < target) acc += part[i++];
  double a = i * dt, b = (i + 1) * dt, need = target - acc;
  double lo = a, hi = b, t = a + (b - a) * (part[i] > 0.0 ? need / part[i] : 0.5);
  for (int it = 0; it < 60; ++it) {
    double g = gl8(qsyn_dens_t, chi, 0, a, t) - need;
    if (g > 0.0) hi = t; else lo = t;
    double dg = qsyn_dens_t(chi, t, 0);
    double tn = dg > 0.0 ? t - g / dg : 0.5 * (lo + hi);
    if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
    if (fabs(tn - t) <= 1e-15 * (t > 1e-300 ? t : 1e-300) || hi - lo <= 1e-15 * hi) { t = tn; break; }
    t = tn;
  }
  double z = t * t * t;
  return 3.0 * chi * z / (2.0 + 3.0 * chi * z);
}

/* Pair spectrum per unit w, v = 1/2 - w, scaled by exp(8/(3 chi)) (the
 * smallest e, at v = 1/2), so that small chi does not underflow. */
static double qbw_dens_w(double chi, double w, int unused) {
  (void)unused;
  double v = 0.5 - w, m = 0.5 + w;
  double e = 2.0 / (3.0 * chi * v * m);
  double k23, ki13;
  bessel_k23_ki13(e, 8.0 / (3.0 * chi), &k23, &ki13);
  return (v / m + m / v) * k23 + ki13;
}

#define QBW_PANELS 200

/* int_0^{1/2} p dw, scaled as qbw_dens_w. */
static double qbw_half(double chi) {
  const double dw = 0.5 / QBW_PANELS;
  double acc = 0.0;
  for (int i = 0; i < QBW_PANELS; ++i) acc += gl8(qbw_dens_w, chi, 0, i * dw, (i + 1) * dw);
  return acc;
}

/* Pair creation rate function from the spectrum (compare the fit orc_tbw). */
double orc_qbw_T(double chi) {
  return 2.0 * qbw_half(chi) * exp(-8.0 / (3.0 * chi)) / (sqrt(3.0) * ORC_PI * chi);
}

/* Fraction of pairs whose electron takes less than the fraction v. */
double orc_qbw_cdf(double chi, double v) {
  if (!(v > 0.0)) return 0.0;
  if (!(v < 1.0)) return 1.0;
  if (v > 0.5) return 1.0 - orc_qbw_cdf(chi, 1.0 - v);
  double w = 0.5 - v;                      /* mass between v and 1/2 */
  const double dw = 0.5 / QBW_PANELS;
  double acc = 0.0;
  for (int i = 0; i < QBW_PANELS; ++i) {
    double a = i * dw, b = (i + 1) * dw;
    if (a >= w) break;
    acc += gl8(qbw_dens_w, chi, 0, a, b < w ? b : w);
  }
  return 0.5 - 0.5 * acc / qbw_half(chi);
}

/* Electron fraction v with cdf(v) = r; the spectrum is symmetric, so
 * v(r) = 1 - v(1 - r) and only r < 1/2 is solved (w = 1/2 - v). */
double orc_qbw_inverse(double chi, double r) {
  if (r > 0.5) return 1.0 - orc_qbw_inverse(chi, 1.0 - r);
  const double dw = 0.5 / QBW_PANELS;
  double part[QBW_PANELS], half = 0.0;
  for (int i = 0; i < QBW_PANELS; ++i) {
    part[i] = gl8(qbw_dens_w, chi, 0, i * dw, (i + 1) * dw);
    half += part[i];
  }
  double target = (1.0 - 2.0 * r) * half, acc = 0.0;
  int i = 0;
  while (i < QBW_PANELS - 1 && acc + part[i] < target) acc += part[i++];
  double a = i * dw, b = (i + 1) * dw, need = target - acc;
  double lo = a, hi = b, w = a + (b - a) * (part[i] > 0.0 ? need / part[i] : 0.5);
  for (int it = 0; it < 60; ++it) {
    double g = gl8(qbw_dens_w, chi, 0, a, w) - need;
    if (g > 0.0) hi = w; else lo = w;
    double dg = qbw_dens_w(chi, w, 0);
    double wn = dg > 0.0 ? w - g / dg : 0.5 * (lo + hi);
    if (!(wn > lo && wn < hi)) wn = 0.5 * (lo + hi);
    if (fabs(wn - w) <= 1e-16 || hi - lo <= 1e-16) { w = wn; break; }
    w = wn;
  }
  return 0.5 - w;
}

/* ------------------------------------------------------------------ */
/* Parameters -> normalised units (Sect. 2.2; App. A).                  */
/* ------------------------------------------------------------------ */
static int derive(orc_sim* s) {
  const orc_params* p = &s->p;
  if (p->n_cells < 2 || !(p->dx > 0) || !(p->cfl > 0 && p->cfl < 1.0) || p->ppc_ref < 1) return ORC_EINVAL;
  if (!(p->b > 0) || !(p->r_curv_cm > 0) || !(p->period_s > 0)) return ORC_EINVAL;
  double omega = 2.0 * ORC_PI / p->period_s;
  double omega_b = ORC_E_OVER_MC * p->b * ORC_B_Q;
  double omega_p = sqrt(omega * omega_b);           /* omega_p,co^2 = Omega omega_B */
  s->d_cm = ORC_C_LIGHT / omega_p;
  s->lam = ORC_LAMBDA_C / s->d_cm * p->lambda_c_scale;
  s->rc = p->r_curv_cm / s->d_cm * p->r_curv_scale;
  s->lr = s->lam / s->rc;
  s->N = p->n_cells;
  s->dt = p->cfl * p->dx;
  s->H = p->h_gap_frac * p->n_cells * p->dx;
  s->w0 = p->dx / p->ppc_ref;
  s->s_co = (p->flags & ORC_ANTI_ALIGNED) ? 1.0 : -1.0;
  return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Containers.                                                          */
/* ------------------------------------------------------------------ */
static int push_lep(orc_sim* s, olep l) {
  if (s->nlep >= s->p.cap_leptons) { s->n_dropped++; s->err = ORC_ECAP; return 0; }
  if (s->nlep == s->lep_alloc) {
    s->lep_alloc = s->lep_alloc ? 2 * s->lep_alloc : 1024;
    s->lep = (olep*)realloc(s->lep, sizeof(olep) * s->lep_alloc);
  }
  s->lep[s->nlep++] = l;
  return 1;
}

static int push_pro(orc_sim* s, olep l) {
  if (s->npro >= s->p.cap_leptons) { s->n_dropped++; s->err = ORC_ECAP; return 0; }
  if (s->npro == s->pro_alloc) {
    s->pro_alloc = s->pro_alloc ? 2 * s->pro_alloc : 1024;
    s->pro = (olep*)realloc(s->pro, sizeof(olep) * s->pro_alloc);
  }
  s->pro[s->npro++] = l;
  return 1;
}

static int push_pho(orc_sim* s, opho g) {
  if (s->npho >= s->p.cap_photons) { s->n_dropped++; s->err = ORC_ECAP; return 0; }
  if (s->npho == s->pho_alloc) {
    s->pho_alloc = s->pho_alloc ? 2 * s->pho_alloc : 1024;
    s->pho = (opho*)realloc(s->pho, sizeof(opho) * s->pho_alloc);
  }
  s->pho[s->npho++] = g;
  return 1;
}

static void log_event(orc_sim* s, int32_t kind, int64_t step, uint64_t id, int32_t sub, double x,
                      int32_t cell, double xi, double w) {
  if (!(s->p.flags & ORC_RECORD)) return;
  if (s->nev == s->ev_alloc) {
    s->ev_alloc = s->ev_alloc ? 2 * s->ev_alloc : 4096;
    s->ev = (oevent*)realloc(s->ev, sizeof(oevent) * s->ev_alloc);
  }
  oevent e = {kind, sub, step, id, x, cell, xi, w};
  s->ev[s->nev++] = e;
}

/* ------------------------------------------------------------------ */
/* Deposit and field (Sect. 2.2 field equations; Sect. 6.1 solver).     */
/* Charge of a particle with weight w: split by the linear (CIC) shape  */
/* in integer units, T = round(|w| 2^F), A = round(T xi):               */
/*   node k gets s (T - A), node k+1 gets s A.                           */
/* ------------------------------------------------------------------ */
static int64_t wt_fixed(double w) { return (int64_t)llrint(fabs(w) * ORC_FP_ONE); }

static void deposit_one(orc_sim* s, int32_t k, double xi, double w) {
  int64_t T = wt_fixed(w);
  /* round(T xi), half up; long double keeps T xi exact when xi is on the
   * 2^-24 grid and |w| < 2^16 */
  int64_t A = (int64_t)floorl((long double)T * (long double)xi + 0.5L);
  int64_t sg = w < 0 ? -1 : 1;
  int32_t k1 = k + 1;
  if ((s->p.flags & ORC_PERIODIC) && k1 == s->N) k1 = 0;
  s->rho[k] += sg * (T - A);
  s->rho[k1] += sg * A;
}

static void deposit_all(orc_sim* s) {
  memset(s->rho, 0, sizeof(int64_t) * (s->N + 1));
  for (int64_t i = 0; i < s->nlep; ++i) deposit_one(s, s->lep[i].cell, s->lep[i].xi, s->lep[i].w);
  for (int64_t i = 0; i < s->npro; ++i) deposit_one(s, s->pro[i].cell, s->pro[i].xi, s->pro[i].w);
}

/* Gauss's law, dE/dh = rho - eta_co, integrated from the surface:
 *   E_{k+1/2} = E_s + w0/2^F * ( sum_{i<=k} rho_i  - s_co ppc_ref 2^F (k+1/2) ).
 * The background term is an exact integer. */
static void field_from_rho(orc_sim* s) {
  int N = s->N;
  int64_t acc = 0;
  int64_t bg_unit = (s->p.flags & ORC_ETA_CO_OFF) ? 0 : (int64_t)(-s->s_co) * s->p.ppc_ref * (int64_t)ORC_FP_ONE;
  double scale = s->w0 / ORC_FP_ONE;
  for (int k = 0; k < N; ++k) {
    acc += s->rho[k];
    int64_t eint = acc + bg_unit * k + bg_unit / 2;
    s->E[k] = (double)eint * scale;
  }
  if (s->p.flags & ORC_PERIODIC) {
    /* periodic: Gauss fixes E up to a constant; the mean field is the
     * state variable carried in Es and advanced by Ampere's law. */
    double m = 0;
    for (int k = 0; k < N; ++k) m += s->E[k];
    m /= N;
    for (int k = 0; k < N; ++k) s->E[k] += s->Es - m;
  } else {
    for (int k = 0; k < N; ++k) s->E[k] += s->Es;
  }
}

/* The digital filter of the current (Sect. 6.1: binomial 3-point shape,
 * several passes per step).  One pass replaces x_i by (x_{i-1} + 2 x_i +
 * x_{i+1}) / 4.  Ends: periodic boxes wrap; otherwise the missing neighbour
 * is the end value itself (x_{-1} = x_0, x_n = x_{n-1}), so a uniform array
 * is unchanged and the sum is kept. */
void orc_filter(double* x, int32_t n, int32_t passes, int32_t periodic) {
  double* y = (double*)malloc(sizeof(double) * (size_t)n);
  for (int32_t p = 0; p < passes; ++p) {
    for (int32_t i = 0; i < n; ++i) {
      double l = i > 0 ? x[i - 1] : (periodic ? x[n - 1] : x[0]);
      double r = i < n - 1 ? x[i + 1] : (periodic ? x[0] : x[n - 1]);
      y[i] = (l + 2.0 * x[i] + r) / 4.0;
    }
    memcpy(x, y, sizeof(double) * (size_t)n);
  }
  free(y);
}

/* Filtered Ampere update.  The field obeys E^{n+1} = E^n - dt (F[J] - j_m)
 * with F linear and time-independent and j_m uniform (F keeps uniform
 * arrays), so summed over steps E^n = E^0 + F[E_u^n - E^0], where E_u is the
 * unfiltered field that Gauss's law gives for the same particles and E_s,
 * and E^0 the field when the state was set. */
static void filter_field(orc_sim* s) {
  if (!(s->p.flags & ORC_FILTER)) return;
  int N = s->N;
  double* d = (double*)malloc(sizeof(double) * (size_t)N);
  for (int k = 0; k < N; ++k) d[k] = s->E[k] - s->E0[k];
  orc_filter(d, N, ORC_FILTER_PASSES, (s->p.flags & ORC_PERIODIC) != 0);
  for (int k = 0; k < N; ++k) s->E[k] = s->E0[k] + d[k];
  free(d);
}

/* Node field for the gather: average of the two adjacent cell fields.
 * Ghosts: E_{-1/2} = E_s (the surface value), E_{N+1/2} = E_{N-1/2}. */
static void node_field(orc_sim* s) {
  int N = s->N;
  if (s->p.flags & ORC_PERIODIC) {
    for (int i = 0; i < N; ++i) s->Eb[i] = 0.5 * (s->E[(i + N - 1) % N] + s->E[i]);
    s->Eb[N] = s->Eb[0];
  } else {
    s->Eb[0] = 0.5 * (s->Es + s->E[0]);
    for (int i = 1; i < N; ++i) s->Eb[i] = 0.5 * (s->E[i - 1] + s->E[i]);
    s->Eb[N] = s->E[N - 1];
  }
}

/* ------------------------------------------------------------------ */
/* Initial state (Sect. 6.1 initial condition; uniform-pair start).     */
/* ------------------------------------------------------------------ */
static void init_particles(orc_sim* s) {
  const orc_params* p = &s->p;
  int N = s->N;
  int k_lo = 0;
  int nspecies = 0;
  double sign[2] = {-1.0, 1.0};
  if (p->init_kind == 0) { k_lo = (int)ceil(s->H / p->dx - 1e-9); nspecies = 1; }
  else if (p->init_kind == 1) nspecies = 2;
  else if (p->init_kind == 3 || p->init_kind == 4) nspecies = 1;
  uint64_t id = 1;
  for (int sp = 0; sp < nspecies; ++sp)
    for (int k = k_lo; k < N; ++k)
      for (int j = 0; j < p->ppc_init; ++j, ++id) {
        uint32_t r[4];
        draw(p->seed, id, 0, TAG_INIT, 0, r);
        olep l = {k, xi24(r[0]), p->u_init, sign[sp], id};
        push_lep(s, l);
      }
  /* kind 4 (Sect. 6.1 initial condition with protons): electrons everywhere
   * and as many protons below H, so that eta = 0 below H and eta_co above */
  if (p->init_kind == 4) {
    int k_h = (int)ceil(s->H / p->dx - 1e-9);
    if (k_h > N) k_h = N;
    for (int k = 0; k < k_h; ++k)
      for (int j = 0; j < p->ppc_init; ++j, ++id) {
        uint32_t r[4];
        draw(p->seed, id, 0, TAG_INIT, 0, r);
        olep l = {k, xi24(r[0]), p->u_init, 1.0, id};
        push_pro(s, l);
      }
  }
}

/* ------------------------------------------------------------------ */
/* Thermal atmosphere (Sect. 2.3 atmospheric boundary; Sect. 6.1:        */
/* k_B T / m_e c^2 = 0.3, protons with m_p / m_e = 1836).                */
/* Reading: the atmosphere is a reservoir in cell 0 holding atm_ppc      */
/* electrons and atm_ppc protons (weight 1 each): every step, before     */
/* the push, each species is refilled to atm_ppc from the count left in  */
/* cell 0 by the previous push; new particles are uniform in the cell,   */
/* with momenta of the one-dimensional relativistic thermal distribution */
/* f(u) ~ exp(-gamma / Theta), Theta = k_B T / (m c^2) of the species.   */
/* The charge they bring leaves the star (surface field bookkeeping as   */
/* for the injected electrons).                                          */
/* ------------------------------------------------------------------ */
/* One momentum of f(u) ~ exp(-gamma/Theta) by rejection.  In the kinetic
 * energy e = gamma - 1 the density is exp(-e/Theta) h(e), h = (1+e) /
 * sqrt(e (2+e)) <= 1/sqrt(2e) + 1; the envelope exp(-e/Theta) (1/sqrt(2e)
 * + 1) is a mixture of e = Theta Z^2/2 (Z standard normal, Box-Muller) of
 * weight sqrt(pi Theta / 2) and e = -Theta ln U of weight Theta.  Attempt j
 * uses the words of draw(seed, id, step, TAG_ATM, j): u24 of word 0 picks
 * the component, words 1 and 2 make e, word 3 accepts with probability
 * h/(1/sqrt(2e) + 1), and bit 0 of word 0 gives the sign of u.  After 64
 * rejections (probability below 1e-30) u = 0. */
double orc_atm_momentum(uint64_t seed, uint64_t id, int64_t step, double theta) {
  const double wa = sqrt(ORC_PI * theta / 2.0), wb = theta;
  for (uint32_t j = 0; j < 64; ++j) {
    uint32_t r[4];
    draw(seed, id, step, TAG_ATM, j, r);
    double e;
    if (u24(r[0]) * (wa + wb) < wa) {
      double c = cos(2.0 * ORC_PI * u24(r[2]));
      e = -theta * log(u24(r[1])) * c * c;
    } else {
      e = -theta * log(u24(r[1]));
    }
    if (!(e > 0.0)) continue;
    double h = (1.0 + e) / sqrt(e * (2.0 + e));
    double bnd = 1.0 / sqrt(2.0 * e) + 1.0;
    if (u24(r[3]) * bnd < h) {
      double u = sqrt(e * (2.0 + e));
      return (r[0] & 1u) ? u : -u;
    }
  }
  return 0.0;
}

static void atmosphere_refill(orc_sim* s, int64_t n) {
  const orc_params* p = &s->p;
  for (int sp = 0; sp < 2; ++sp) {
    int64_t m = (int64_t)p->atm_ppc - s->atm_prev[sp];
    double theta = sp == 0 ? p->atm_temp : p->atm_temp / ORC_MASS_P;
    for (int64_t j = 0; j < m; ++j) {
      uint64_t id = ATM_ID_BASE + s->atm_count++;
      uint32_t r[4];
      draw(p->seed, id, n, TAG_ATM, 0xFFFFu, r);
      double u = orc_atm_momentum(p->seed, id, n, theta);
      if (sp == 0) {
        olep l = {0, xi24(r[0]), u, -1.0, id};
        if (push_lep(s, l)) { s->dq += wt_fixed(1.0); s->n_atm_e++; }
      } else {
        olep l = {0, xi24(r[0]), u, 1.0, id};
        if (push_pro(s, l)) { s->dq -= wt_fixed(1.0); s->n_atm_p++; }
      }
    }
  }
}

orc_sim* orc_create(const orc_params* p, int32_t* err) {
  orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
  s->p = *p;
  if (s->p.nsub_max < 1) s->p.nsub_max = 64;
  if (s->p.merge_every < 1) s->p.merge_every = 64;
  int e = derive(s);
  if (e) { free(s); if (err) *err = e; return NULL; }
  s->E = (double*)calloc(s->N, sizeof(double));
  s->E0 = (double*)calloc(s->N, sizeof(double));
  s->Eb = (double*)calloc(s->N + 1, sizeof(double));
  s->rho = (int64_t*)calloc(s->N + 1, sizeof(int64_t));
  sync_nodes(s);
  init_particles(s);
  s->atm_prev[0] = s->atm_prev[1] = s->p.atm_ppc;   /* no refill before the first push */
  s->Es = 0.0;
  deposit_all(s);
  field_from_rho(s);
  memcpy(s->E0, s->E, sizeof(double) * s->N);
  node_field(s);
  if (err) *err = s->err;
  return s;
}

void orc_free(orc_sim* s) {
  if (!s) return;
  free(s->lep); free(s->pho); free(s->pro); free(s->E); free(s->E0); free(s->Eb); free(s->rho); free(s->ev);
  free(s->q_cosh); free(s->q_g); free((void*)s->rep);
  free(s);
}

/* ------------------------------------------------------------------ */
/* Replay of a recorded QED realisation: events looked up by            */
/* (kind, step, id, sub) with a binary search over the sorted log.      */
/* ------------------------------------------------------------------ */
static int ev_cmp(const oevent* a, int32_t kind, int64_t step, uint64_t id, int32_t sub) {
  if (a->step != step) return a->step < step ? -1 : 1;
  if (a->kind != kind) return a->kind < kind ? -1 : 1;
  if (a->id != id) return a->id < id ? -1 : 1;
  if (a->sub != sub) return a->sub < sub ? -1 : 1;
  return 0;
}

static const oevent* ev_find(const orc_sim* s, int32_t kind, int64_t step, uint64_t id, int32_t sub) {
  int64_t lo = 0, hi = s->nrep;
  while (lo < hi) {
    int64_t mid = (lo + hi) / 2;
    int c = ev_cmp(&s->rep[mid], kind, step, id, sub);
    if (c == 0) return &s->rep[mid];
    if (c < 0) lo = mid + 1; else hi = mid;
  }
  return NULL;
}

/* First recorded event of (kind, step, id) in sub order, and the next one. */
static const oevent* ev_first(const orc_sim* s, int32_t kind, int64_t step, uint64_t id) {
  int64_t lo = 0, hi = s->nrep;
  while (lo < hi) {
    int64_t mid = (lo + hi) / 2;
    if (ev_cmp(&s->rep[mid], kind, step, id, INT32_MIN) < 0) lo = mid + 1; else hi = mid;
  }
  if (lo < s->nrep && s->rep[lo].kind == kind && s->rep[lo].step == step && s->rep[lo].id == id) return &s->rep[lo];
  return NULL;
}
static const oevent* ev_next(const orc_sim* s, const oevent* e) {
  const oevent* f = e + 1;
  if (f < s->rep + s->nrep && f->kind == e->kind && f->step == e->step && f->id == e->id) return f;
  return NULL;
}

/* All recorded events of one kind at one step. */
static const oevent* ev_kind_first(const orc_sim* s, int32_t kind, int64_t step) {
  int64_t lo = 0, hi = s->nrep;
  while (lo < hi) {
    int64_t mid = (lo + hi) / 2;
    if (ev_cmp(&s->rep[mid], kind, step, 0, INT32_MIN) < 0) lo = mid + 1; else hi = mid;
  }
  if (lo < s->nrep && s->rep[lo].kind == kind && s->rep[lo].step == step) return &s->rep[lo];
  return NULL;
}
static const oevent* ev_kind_next(const orc_sim* s, const oevent* e) {
  const oevent* f = e + 1;
  if (f < s->rep + s->nrep && f->kind == e->kind && f->step == e->step) return f;
  return NULL;
}

/* ------------------------------------------------------------------ */
/* Merge (weight doubling): per (cell, charge sign, direction,          */
/* floor(log2 gamma)) group, sorted by id, consecutive pairs fuse; the  */
/* survivor, picked by one random bit, takes the summed weight.         */
/* ------------------------------------------------------------------ */
typedef struct { int64_t key; uint64_t id; int64_t idx; } mkey;
static int mkey_cmp(const void* a, const void* b) {
  const mkey* x = (const mkey*)a; const mkey* y = (const mkey*)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  if (x->id != y->id) return x->id < y->id ? -1 : 1;
  return 0;
}

static int lg2bin(double v) {
  int e; frexp(v, &e);            /* v = m 2^e, m in [0.5,1) -> floor(log2 v) = e-1 */
  int b = e - 1;
  if (b < -64) b = -64;
  if (b > 63) b = 63;
  return b + 64;                  /* 0..127 */
}

static void merge_leptons(orc_sim* s) {
  int64_t n = s->nlep;
  mkey* m = (mkey*)malloc(sizeof(mkey) * (n ? n : 1));
  for (int64_t i = 0; i < n; ++i) {
    const olep* l = &s->lep[i];
    double g = sqrt(1.0 + l->u * l->u);
    int64_t key = ((int64_t)l->cell << 9) | ((int64_t)(l->w > 0) << 8) | ((int64_t)(l->u >= 0) << 7) | lg2bin(g);
    m[i].key = key; m[i].id = l->id; m[i].idx = i;
  }
  qsort(m, n, sizeof(mkey), mkey_cmp);
  for (int64_t i = 0; i + 1 < n; ) {
    if (m[i].key == m[i + 1].key) {
      olep* a = &s->lep[m[i].idx];
      olep* b = &s->lep[m[i + 1].idx];
      uint32_t r[4];
      draw(s->p.seed, a->id, s->step, TAG_MERGE, 0, r);
      olep* keep = (r[0] & 1u) ? b : a;
      olep* drop = (r[0] & 1u) ? a : b;
      keep->w += drop->w;
      drop->w = 0.0;
      s->n_merged++;
      i += 2;
    } else {
      i += 1;
    }
  }
  int64_t j = 0;
  for (int64_t i = 0; i < n; ++i) if (s->lep[i].w != 0.0) s->lep[j++] = s->lep[i];
  s->nlep = j;
  free(m);
}

static void merge_photons(orc_sim* s) {
  int64_t n = s->npho;
  mkey* m = (mkey*)malloc(sizeof(mkey) * (n ? n : 1));
  for (int64_t i = 0; i < n; ++i) {
    const opho* g = &s->pho[i];
    int64_t key = ((int64_t)g->cell << 9) | ((int64_t)(g->x >= 0) << 7) | lg2bin(fabs(g->x));
    m[i].key = key; m[i].id = g->id; m[i].idx = i;
  }
  qsort(m, n, sizeof(mkey), mkey_cmp);
  for (int64_t i = 0; i + 1 < n; ) {
    if (m[i].key == m[i + 1].key) {
      opho* a = &s->pho[m[i].idx];
      opho* b = &s->pho[m[i + 1].idx];
      uint32_t r[4];
      draw(s->p.seed, a->id, s->step, TAG_MERGE, 0, r);
      opho* keep = (r[0] & 1u) ? b : a;
      opho* drop = (r[0] & 1u) ? a : b;
      keep->w += drop->w;
      drop->w = 0.0;
      s->n_merged++;
      i += 2;
    } else {
      i += 1;
    }
  }
  int64_t j = 0;
  for (int64_t i = 0; i < n; ++i) if (s->pho[i].w != 0.0) s->pho[j++] = s->pho[i];
  s->npho = j;
  free(m);
}

/* ------------------------------------------------------------------ */
/* One step.                                                            */
/* ------------------------------------------------------------------ */
static void wrap_cell(const orc_sim* s, int32_t* k, double* xi) {
  if (*xi >= 1.0) { *k += 1; *xi -= 1.0; }
  else if (*xi < 0.0) {
    *k -= 1; *xi += 1.0;
    if (*xi >= 1.0) { *k += 1; *xi = 0.0; }
  }
  if (s->p.flags & ORC_PERIODIC) {
    if (*k < 0) *k += s->N;
    if (*k >= s->N) *k -= s->N;
  }
}

typedef struct { double x; uint64_t id; } pending_ph;

/* One emitted photon of energy x (m_e c^2): recoil along the motion with x
 * clamped to |u| (Sect. 4), energy bookkeeping, event log, and a pending
 * photon birth if it is tracked (x >= x_thr, Sect. 6.1). */
static void emit_apply(orc_sim* s, olep* l, int64_t n, int j, double x, pending_ph* pend, int* npend) {
  const orc_params* p = &s->p;
  double au = fabs(l->u);
  if (x > au) x = au;
  double dir = l->u >= 0 ? 1.0 : -1.0;
  if (!(p->flags & ORC_RECOIL_OFF)) l->u = dir * (au - x);
  s->n_emit++;
  s->e_rad += x * fabs(l->w);
  log_event(s, 0, n, l->id, j, dir * x, 0, 0.0, 0.0);
  if ((x >= p->x_thr || (p->flags & ORC_TRACK_ALL)) && *npend < 64) {
    pend[*npend].x = dir * x;
    pend[*npend].id = child_id(p->seed, l->id, n, 2u + (uint32_t)j);
    (*npend)++;
  }
}

static void step_once(orc_sim* s) {
  const orc_params* p = &s->p;
  const int64_t n = s->step;
  const int N = s->N;
  const int qed = !(p->flags & ORC_QED_OFF);
  const int periodic = (p->flags & ORC_PERIODIC) != 0;
  const int replay = (p->flags & ORC_REPLAY) != 0;

  /* (0) merge when above the cap threshold */
  if ((p->flags & ORC_MERGE_ON) && (n % p->merge_every) == 0) {
    if ((double)s->nlep > p->merge_frac * (double)p->cap_leptons) merge_leptons(s);
    if ((double)s->npho > p->merge_frac * (double)p->cap_photons) merge_photons(s);
  }

  /* (1a) the thermal atmosphere refills cell 0 */
  if (p->atm_ppc > 0 && !periodic) atmosphere_refill(s, n);

  /* (1) surface injection of cold electrons into cell 0 (Sect. 2.3: the
   * atmosphere supplies charges; here a deterministic accumulator). */
  if (p->inj_rate > 0.0 && !periodic) {
    s->inj_acc += p->inj_rate * p->ppc_ref / ((p->flags & ORC_INJ_FIXED) ? 1.0 : p->inj_weight);
    int64_t m = (int64_t)floor(s->inj_acc);
    s->inj_acc -= (double)m;
    for (int64_t j = 0; j < m; ++j) {
      uint64_t id = INJ_ID_BASE + s->inj_count++;
      uint32_t r[4];
      draw(p->seed, id, n, TAG_INJ, 0, r);
      olep l = {0, xi24(r[0]), 0.0, -p->inj_weight, id};
      if (push_lep(s, l)) s->dq += wt_fixed(p->inj_weight);   /* E_s -= Q_inj, Q_inj < 0 */
    }
  }

  /* (2) leptons: gather + kick, emission, drift, boundaries, deposit */
  memset(s->rho, 0, sizeof(int64_t) * (N + 1));
  s->atm_prev[0] = s->atm_prev[1] = 0;
  int64_t nl = s->nlep;
  int64_t npho0 = s->npho;
  pending_ph pend[64];
  for (int64_t i = 0; i < nl; ++i) {
    olep* l = &s->lep[i];
    double sg = l->w < 0 ? -1.0 : 1.0;
    /* gather (first-order interpolation of the node field) and kick:
     * du/dt = q E (beads-on-a-wire form of the Lorentz force, Sect. 4) */
    double Ep = (1.0 - l->xi) * s->Eb[l->cell] + l->xi * s->Eb[l->cell + 1];
    l->u += sg * Ep * s->dt;

    /* curvature emission by Monte Carlo (Sect. 3.1, eqs. tau_syn, P_curv,
     * x_curv; Sect. 6.1: QED only below H, sub-cycling when the step is long) */
    int npend = 0;
    double h = (l->cell + l->xi) * p->dx;
    if (replay) {
      /* frozen realisation: each recorded emission of this lepton at this
       * step is a constant recoil offset, whatever its current momentum */
      for (const oevent* e = ev_first(s, 0, n, l->id); e; e = ev_next(s, e)) {
        if (!(p->flags & ORC_RECOIL_OFF)) l->u -= e->x;
        s->n_emit++;
        s->e_rad += fabs(e->x) * fabs(l->w);
      }
    } else if (qed && !(p->flags & ORC_EMIT_OFF) && h < s->H) {
      double g = sqrt(1.0 + l->u * l->u);
      double chi = g * g * s->lr;          /* chi = gamma b sin(psi), sin(psi) = gamma r_g/R */
      double xc = 1.5 * g * chi;           /* x_curv = (3/2) b (r_g/R) gamma^3 */
      if (xc >= p->xc_floor) {
        double dtau = ORC_ALPHA_EM * g / s->rc * orc_tsyn(chi) * s->dt;
        int nsub = (int)ceil(dtau / 0.1);
        if (nsub < 1) nsub = 1;
        if (nsub > p->nsub_max) nsub = p->nsub_max;
        double pe = -expm1(-dtau / nsub);
        s->n_emit_eval++;
        for (int j = 0; j < nsub; ++j) {
          uint32_t r[4];
          draw(p->seed, l->id, n, TAG_EMIT, (uint32_t)j, r);
          if (u24(r[0]) < pe) {
            /* photon energy: classical x = xi x_c, or the quantum spectrum's
             * energy fraction of the emitter's gamma at its chi */
            double x = (p->flags & ORC_QUANTUM) ? orc_qsyn_inverse(chi, u24(r[1])) * g
                                                : sync_inverse(s, u24(r[1])) * xc;
            emit_apply(s, l, n, j, x, pend, &npend);
          }
        }
      }
    }

    /* drift: dh/dt = u / gamma */
    double g2 = sqrt(1.0 + l->u * l->u);
    double disp = l->u / g2 * p->cfl;
    l->xi += disp;
    s->dcur += sg * fabs(l->w) * disp;
    wrap_cell(s, &l->cell, &l->xi);
    if (!periodic && l->cell < 0) {            /* absorbed by the star */
      s->dq += (int64_t)sg * wt_fixed(l->w);
      s->n_absorbed++;
      {
        /* bin b holds gamma in [10^(b/8), 10^((b+1)/8)): the last b whose
         * lower edge in u^2 = gamma^2 - 1, 10^(b/4) - 1, u^2 reaches */
        double u2 = l->u * l->u;
        int b = 0;
        while (b + 1 < ORC_RET_NB && pow(10.0, (b + 1) / 4.0) - 1.0 <= u2) ++b;
        s->ret[b] += fabs(l->w);
        s->ret[ORC_RET_NB] += fabs(l->w);
        s->ret[ORC_RET_NB + 1] += fabs(l->w) * sqrt(1.0 + u2);
      }
      l->w = 0.0;
      continue;
    }
    if (!periodic && l->cell >= N) {           /* free outflow */
      s->n_outflow++;
      l->w = 0.0;
      continue;
    }
    if (l->w < 0.0 && l->cell == 0) s->atm_prev[0]++;
    double hn = (l->cell + l->xi) * p->dx;
    for (int j = 0; j < npend; ++j) {
      if (hn < s->H) {
        opho g = {l->cell, l->xi, pend[j].x, fabs(l->w), n + 1, pend[j].id};
        if (push_pho(s, g)) {
          s->n_pho_born++;
          log_event(s, 2, n, g.id, j, g.x, g.cell, g.xi, g.w);
        }
        l = &s->lep[i];                        /* (no realloc of lep here; kept for clarity) */
      }
    }
    deposit_one(s, l->cell, l->xi, l->w);
  }

  /* (2c) protons (Sect. 6.1: charge +1, m_p/m_e = 1836; no QED): kick
   * du/dt = E / 1836, drift dh/dt = u / gamma, boundaries, deposit */
  for (int64_t i = 0; i < s->npro; ++i) {
    olep* q = &s->pro[i];
    double Ep = (1.0 - q->xi) * s->Eb[q->cell] + q->xi * s->Eb[q->cell + 1];
    q->u += Ep * s->dt / ORC_MASS_P;
    double disp = q->u / sqrt(1.0 + q->u * q->u) * p->cfl;
    q->xi += disp;
    s->dcur += fabs(q->w) * disp;
    wrap_cell(s, &q->cell, &q->xi);
    if (!periodic && q->cell < 0) {
      s->dq += wt_fixed(q->w);
      s->n_pro_absorbed++;
      q->w = 0.0;
      continue;
    }
    if (!periodic && q->cell >= N) {
      s->n_pro_outflow++;
      q->w = 0.0;
      continue;
    }
    if (q->cell == 0) s->atm_prev[1]++;
    deposit_one(s, q->cell, q->xi, q->w);
  }

  /* (2b) frozen realisation: the recorded photon births of this step, with
   * their recorded states */
  if (replay) {
    for (const oevent* e = ev_kind_first(s, 2, n); e; e = ev_kind_next(s, e)) {
      opho g = {e->cell, e->xi, e->x, e->w, n + 1, e->id};
      if (push_pho(s, g)) s->n_pho_born++;
    }
  }

  /* (3) photons existing at the start of the step: free streaming at c,
   * one-photon pair creation (Sect. 3.2 eq. tau_bw; Sect. 6.1 accumulated
   * angle, QED off above H) */
  for (int64_t i = 0; i < npho0; ++i) {
    opho* g = &s->pho[i];
    double dir = g->x >= 0 ? 1.0 : -1.0;
    g->xi += dir * p->cfl;
    wrap_cell(s, &g->cell, &g->xi);
    double h = (g->cell + g->xi) * p->dx;
    if ((!periodic && (g->cell < 0 || g->cell >= N)) || h >= s->H) {
      s->n_pho_exit++;
      g->w = 0.0;
      continue;
    }
    if (!replay && (!qed || (p->flags & ORC_CONV_OFF))) continue;
    double path = (double)(n + 1 - g->n0) * s->dt;
    double sinpsi = fabs(sin(path / s->rc));
    double chi = fabs(g->x) * p->b * sinpsi;
    double dtau = ORC_ALPHA_EM * (p->b / s->lam) * sinpsi * orc_tbw(chi) * s->dt;
    double pc = -expm1(-dtau);
    if (pc > 0x1p-25) s->n_conv_eval++;
    int conv = 0;
    if (replay) {
      conv = ev_find(s, 1, n, g->id, 0) != NULL;
    } else {
      uint32_t r[4];
      draw(p->seed, g->id, n, TAG_CONV, 0, r);
      conv = u24(r[0]) < pc;
    }
    if (conv) {
      /* energy split: halves (R10), or the electron's fraction v from the
       * quantum pair spectrum at the photon's chi */
      double v = 0.5;
      if (p->flags & ORC_QUANTUM) {
        uint32_t r[4];
        draw(p->seed, g->id, n, TAG_CONV, 0, r);
        v = orc_qbw_inverse(chi, u24(r[1]));
      }
      double gm = v * fabs(g->x), gp = (1.0 - v) * fabs(g->x);
      olep em = {g->cell, g->xi, dir * sqrt(fmax(gm * gm - 1.0, 0.0)), -g->w, child_id(p->seed, g->id, n, 0)};
      olep ep = {g->cell, g->xi, dir * sqrt(fmax(gp * gp - 1.0, 0.0)), g->w, child_id(p->seed, g->id, n, 1)};
      log_event(s, 1, n, g->id, 0, fabs(g->x), 0, 0.0, 0.0);
      push_lep(s, em);
      push_lep(s, ep);
      s->n_conv++;
      g = &s->pho[i];
      g->w = 0.0;
    }
  }

  /* remove the dead (order is irrelevant to every result) */
  {
    int64_t j = 0;
    for (int64_t i = 0; i < s->nlep; ++i) if (s->lep[i].w != 0.0) s->lep[j++] = s->lep[i];
    s->nlep = j;
    j = 0;
    for (int64_t i = 0; i < s->npho; ++i) if (s->pho[i].w != 0.0) s->pho[j++] = s->pho[i];
    s->npho = j;
    j = 0;
    for (int64_t i = 0; i < s->npro; ++i) if (s->pro[i].w != 0.0) s->pro[j++] = s->pro[i];
    s->npro = j;
  }

  /* (4) field: Ampere drive and surface flux enter through E_s, then Gauss */
  if (!(p->flags & ORC_FIELD_FROZEN)) {
    if (!periodic) s->Es += (double)s->dq * s->w0 / ORC_FP_ONE + p->alpha * s->s_co * s->dt;
    else s->Es += -s->dcur * s->w0 * p->dx / (N * p->dx) + p->alpha * s->s_co * s->dt;
    field_from_rho(s);
    filter_field(s);
    node_field(s);
  }
  s->dq = 0;
  s->dcur = 0.0;
  s->step = n + 1;
}

int32_t orc_step(orc_sim* s, int64_t nsteps) {
  for (int64_t i = 0; i < nsteps; ++i) step_once(s);
  return s->err;
}

/* ------------------------------------------------------------------ */
/* Accessors for the tests.                                             */
/* ------------------------------------------------------------------ */
void orc_derived(const orc_sim* s, double out[8]) {
  out[0] = s->d_cm; out[1] = s->lam; out[2] = s->rc; out[3] = s->dt;
  out[4] = s->H; out[5] = s->w0; out[6] = s->s_co; out[7] = (double)s->N;
}

void orc_counts(const orc_sim* s, int64_t out[16]) {
  out[0] = s->nlep; out[1] = s->npho; out[2] = s->step; out[3] = s->n_emit;
  out[4] = s->n_pho_born; out[5] = s->n_conv; out[6] = s->n_absorbed; out[7] = s->n_outflow;
  out[8] = s->n_pho_exit; out[9] = s->n_dropped; out[10] = s->n_merged; out[11] = s->err;
  out[12] = s->nev; out[13] = (int64_t)s->inj_count; out[14] = s->n_emit_eval; out[15] = s->n_conv_eval;
}

double orc_es(const orc_sim* s) { return s->Es; }
/* the return flux since the last call, which clears it */
void orc_return(orc_sim* s, double out[ORC_RET_NB + 2]) {
  for (int i = 0; i < ORC_RET_NB + 2; ++i) { out[i] = s->ret[i]; s->ret[i] = 0.0; }
}
double orc_erad(const orc_sim* s) { return s->e_rad; }
void orc_field(const orc_sim* s, double* E) { memcpy(E, s->E, sizeof(double) * s->N); }
void orc_node_field(const orc_sim* s, double* Eb) { memcpy(Eb, s->Eb, sizeof(double) * (s->N + 1)); }
void orc_rho(const orc_sim* s, int64_t* rho) { memcpy(rho, s->rho, sizeof(int64_t) * (s->N + 1)); }

void orc_get_leptons(const orc_sim* s, int32_t* cell, double* xi, double* u, double* w, uint64_t* id) {
  for (int64_t i = 0; i < s->nlep; ++i) {
    cell[i] = s->lep[i].cell; xi[i] = s->lep[i].xi; u[i] = s->lep[i].u; w[i] = s->lep[i].w; id[i] = s->lep[i].id;
  }
}

void orc_get_photons(const orc_sim* s, int32_t* cell, double* xi, double* x, double* w, int64_t* n0, uint64_t* id) {
  for (int64_t i = 0; i < s->npho; ++i) {
    cell[i] = s->pho[i].cell; xi[i] = s->pho[i].xi; x[i] = s->pho[i].x; w[i] = s->pho[i].w;
    n0[i] = s->pho[i].n0; id[i] = s->pho[i].id;
  }
}

void orc_get_events(const orc_sim* s, int32_t* kind, int32_t* sub, int64_t* step, uint64_t* id, double* x,
                    int32_t* cell, double* xi, double* w) {
  for (int64_t i = 0; i < s->nev; ++i) {
    kind[i] = s->ev[i].kind; sub[i] = s->ev[i].sub; step[i] = s->ev[i].step; id[i] = s->ev[i].id; x[i] = s->ev[i].x;
    cell[i] = s->ev[i].cell; xi[i] = s->ev[i].xi; w[i] = s->ev[i].w;
  }
}

/* Replace the particle state (e.g. with a state exported from elsewhere);
 * the node charge and field are rebuilt from it with the given E_s. */
int32_t orc_set_state(orc_sim* s, int64_t nl, const int32_t* cell, const double* xi, const double* u,
                      const double* w, const uint64_t* id, int64_t np, const int32_t* pcell,
                      const double* pxi, const double* px, const double* pw, const int64_t* pn0,
                      const uint64_t* pid, double Es, int64_t step) {
  s->nlep = 0; s->npho = 0;
  s->atm_prev[0] = s->atm_prev[1] = s->p.atm_ppc;
  for (int64_t i = 0; i < nl; ++i) { olep l = {cell[i], xi[i], u[i], w[i], id[i]}; push_lep(s, l); }
  for (int64_t i = 0; i < np; ++i) { opho g = {pcell[i], pxi[i], px[i], pw[i], pn0[i], pid[i]}; push_pho(s, g); }
  s->Es = Es;
  s->step = step;
  s->dq = 0;
  deposit_all(s);
  field_from_rho(s);
  memcpy(s->E0, s->E, sizeof(double) * s->N);
  node_field(s);
  return s->err;
}

/* Protons: counts, state and replacement (the field is re-solved). */
void orc_proton_counts(const orc_sim* s, int64_t out[8]) {
  out[0] = s->npro; out[1] = s->n_pro_absorbed; out[2] = s->n_pro_outflow; out[3] = s->n_atm_e;
  out[4] = s->n_atm_p; out[5] = s->atm_prev[0]; out[6] = s->atm_prev[1]; out[7] = (int64_t)s->atm_count;
}
void orc_get_protons(const orc_sim* s, int32_t* cell, double* xi, double* u, double* w, uint64_t* id) {
  for (int64_t i = 0; i < s->npro; ++i) {
    cell[i] = s->pro[i].cell; xi[i] = s->pro[i].xi; u[i] = s->pro[i].u; w[i] = s->pro[i].w; id[i] = s->pro[i].id;
  }
}
int32_t orc_set_protons(orc_sim* s, int64_t n, const int32_t* cell, const double* xi, const double* u,
                        const double* w, const uint64_t* id) {
  s->npro = 0;
  for (int64_t i = 0; i < n; ++i) { olep l = {cell[i], xi[i], u[i], w[i], id[i]}; push_pro(s, l); }
  deposit_all(s);
  field_from_rho(s);
  memcpy(s->E0, s->E, sizeof(double) * s->N);
  node_field(s);
  return s->err;
}
void orc_set_atmosphere(orc_sim* s, int64_t prev_e, int64_t prev_p, uint64_t count) {
  s->atm_prev[0] = prev_e; s->atm_prev[1] = prev_p; s->atm_count = count;
}

/* Overwrite the cell field (FIELD_FROZEN tests). */
void orc_set_field(orc_sim* s, const double* E, double Es) {
  memcpy(s->E, E, sizeof(double) * s->N);
  memcpy(s->E0, E, sizeof(double) * s->N);
  s->Es = Es;
  node_field(s);
}

void orc_set_injection(orc_sim* s, double acc, uint64_t count) { s->inj_acc = acc; s->inj_count = count; }

/* Test hook: the merge of both species on the current state, as a step whose
 * merge check is due runs it first (draws keyed by the current step). */
void orc_merge_now(orc_sim* s) {
  merge_leptons(s);
  merge_photons(s);
}

/* Install a recorded event log for replay (sorted here by step/kind/id/sub). */
static int ev_sort_cmp(const void* a, const void* b) {
  const oevent* x = (const oevent*)a; const oevent* y = (const oevent*)b;
  return ev_cmp(x, y->kind, y->step, y->id, y->sub);
}
void orc_set_replay(orc_sim* s, int64_t n, const int32_t* kind, const int32_t* sub, const int64_t* step,
                    const uint64_t* id, const double* x, const int32_t* cell, const double* xi, const double* w) {
  oevent* e = (oevent*)malloc(sizeof(oevent) * (n ? n : 1));
  for (int64_t i = 0; i < n; ++i) {
    e[i].kind = kind[i]; e[i].sub = sub[i]; e[i].step = step[i]; e[i].id = id[i]; e[i].x = x[i];
    e[i].cell = cell[i]; e[i].xi = xi[i]; e[i].w = w[i];
  }
  qsort(e, n, sizeof(oevent), ev_sort_cmp);
  free((void*)s->rep);   /* a log installed before is replaced */
  s->rep = e; s->nrep = n;
}

/* Stand-alone access to the photon spectrum for the pins. */
double orc_sync_cdf(double xi) {
  orc_sim tmp; memset(&tmp, 0, sizeof(tmp));
  sync_nodes(&tmp);
  double t, d;
  sync_tail(&tmp, xi, &t, &d);
  free(tmp.q_cosh); free(tmp.q_g);
  return 1.0 - t;
}

void orc_sync_inverse_many(const double* r, double* xi, int64_t n) {
  orc_sim tmp; memset(&tmp, 0, sizeof(tmp));
  sync_nodes(&tmp);
  for (int64_t i = 0; i < n; ++i) xi[i] = sync_inverse(&tmp, r[i]);
  free(tmp.q_cosh); free(tmp.q_g);
}

double orc_u24(uint32_t r) { return u24(r); }
