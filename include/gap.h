/*
 * gap.h -- C ABI of libgap: the per-step particle loop of the 1D radiative
 * PIC of a pulsar polar-cap pair discharge (Nattila & Salmi), on one
 * MI355X (gfx950) GPU.
 *
 * One step of a flux tube (Sects. 2.2, 3, 4 and 6.1 of the paper):
 *   1. inject cold electrons at the stellar surface (atmosphere supply, Sect. 2.3);
 *   2. gather E_parallel and kick every lepton, du/dt = q E (Sect. 4, beads on a wire);
 *   3. curvature emission by Monte Carlo with recoil (Sect. 3.1 eqs. tau_syn,
 *      P_curv, x_curv; QED only below H_gap, Sect. 6.1);
 *   4. drift, absorption at h = 0, free outflow at h = L;
 *   5. charge-conserving fixed-point deposit (first-order shape, Sect. 6.1);
 *   6. photon free streaming and one-photon pair creation (Sect. 3.2 eq. tau_bw,
 *      accumulated angle sin(psi) = |sin(s/R_curv)|, Sect. 6.1);
 *   7. new pairs and photons compacted into the particle stores;
 *   8. field: Ampere drive alpha j_co and surface flux enter the surface field
 *      E_s, then Gauss's law dE/dh = rho - eta_co (Sect. 2.2) by an integer scan.
 *
 * Units: lengths in d = c/omega_p,co, times in 1/omega_p,co, c = 1,
 * u = gamma beta, E in m_e c omega_p,co / e, charge density in e n_co,
 * omega_p,co^2 = Omega omega_B with Omega = 2 pi / period (Sect. 2.2).
 *
 * Conventions for every entry point:
 *  - return 0 on success, a negative GAP_E* code otherwise; no exceptions
 *    cross the ABI;
 *  - device work is enqueued on the HIP stream given to gap_init and runs
 *    asynchronously (a step forks its photon pass onto an internal stream
 *    of default priority and joins it back before the step ends, so the
 *    order seen on the caller's stream is unchanged); errors raised on the
 *    device are sticky and reported by the next call that synchronises
 *    (gap_sync, gap_diag, gap_set_state); once reported, an error stops
 *    the run: gap_step, gap_step_graph and the window calls return it
 *    without enqueuing work;
 *  - one handle must not be used from two host threads at once.
 */
#ifndef GAP_H
#define GAP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* error codes */
#define GAP_OK        0
#define GAP_EINVAL   (-1)  /* invalid argument or parameter                          */
#define GAP_ENOMEM   (-2)  /* device or host allocation failed                       */
#define GAP_ECAP     (-3)  /* a particle store overflowed: particles were dropped    */
#define GAP_ETILE    (-4)  /* a particle left its tile window (rebucket too rare)    */
#define GAP_ENAN     (-5)  /* non-finite field                                       */
#define GAP_EDEVICE  (-6)  /* HIP runtime error                                      */
#define GAP_ESTATE   (-7)  /* call not valid in the current state                    */

/* flags (gap_params.flags) */
#define GAP_QED_OFF      1u     /* no emission, no conversion                          */
#define GAP_ETA_CO_OFF   2u     /* no co-rotation background charge in Gauss's law     */
#define GAP_FIELD_FROZEN 4u     /* E is not updated (set with gap_set_state)           */
#define GAP_RECOIL_OFF   8u     /* emission leaves the lepton momentum unchanged      */
#define GAP_PERIODIC     16u    /* periodic box; mean field advanced by Ampere's law   */
#define GAP_MERGE_ON     32u    /* weight-doubling merge above merge_frac * cap        */
#define GAP_TRACK_ALL    64u    /* store every emitted photon, also below x_thr        */
#define GAP_ANTI_ALIGNED 128u   /* eta_co = +e n_co instead of -e n_co                 */
#define GAP_CONV_OFF     1024u  /* photons never convert                               */
#define GAP_EMIT_OFF     2048u  /* leptons never emit                                  */
#define GAP_INJ_FIXED    4096u  /* injection count per step from inj_rate * ppc_ref
                                   alone: inj_weight scales the injected charge only
                                   (the injected density is inj_rate * inj_weight)    */
#define GAP_FILTER       8192u  /* the current is smoothed by the digital filter of
                                   Sect. 6.1: 8 passes per step of the binomial 3-point
                                   shape, ends repeating the end value (periodic: wrapped).
                                   Applied as E = E0 + F[E_u - E0], E_u the unfiltered
                                   Gauss field and E0 the field when the state was last
                                   set; E_s itself is not filtered.  Not with the
                                   differentiable window (GAP_EINVAL)                   */
#define GAP_QUANTUM      16384u /* quantum-corrected energies (Sect. 3.1, 3.2): an emitted
                                   photon takes the energy fraction x/gamma drawn from the
                                   first-order synchrotron spectrum at the lepton's chi
                                   (its mean carries the Gaunt factor g_Q into the recoil),
                                   and a pair's electron the fraction drawn from the
                                   one-photon pair spectrum at the photon's chi (the
                                   positron the rest).  The rates stay the fits T_syn and
                                   T_BW.  Without it: the classical spectrum and halves.
                                   Tables (~0.9 MB of device memory) are built on the host
                                   at the first handle that needs them                 */

/* initial states (gap_params.init_kind) */
#define GAP_INIT_GAP      0  /* vacuum below H, electrons at ppc_init per cell above H  */
#define GAP_INIT_UNIFORM  1  /* ppc_init electrons and ppc_init positrons in every cell */
#define GAP_INIT_EMPTY    2  /* no particles                                            */
#define GAP_INIT_ELECTRON 3  /* ppc_init electrons in every cell                        */
#define GAP_INIT_ATMOSPHERE 4 /* Sect. 6.1 initial state: ppc_init electrons in every cell
                                and ppc_init protons (weight 1, at rest) in every cell
                                below H, so that the charge is 0 below H and the
                                co-rotation charge above; not with GAP_PERIODIC     */

/* Physical inputs of one flux tube (the statement of the problem in Sects.
 * 2-3 and 6.1: grid, alpha, B/B_Q, curvature radius, injection, QED knobs). */
typedef struct gap_params {
  int32_t n_cells;        /* N >= 2                                                    */
  int32_t init_kind;      /* GAP_INIT_*                                                */
  int32_t ppc_init;       /* initial macro-particles per cell per species              */
  int32_t ppc_ref;        /* macro-particles per cell at n_co; w0 = dx / ppc_ref       */
  double dx;              /* cell size in skin depths                                  */
  double cfl;             /* c dt / dx, 0 < cfl < 1                                    */
  double alpha;           /* j_m / j_co                                                */
  double b;               /* B / B_Q                                                   */
  double r_curv_cm;       /* curvature radius of the field line [cm]                   */
  double period_s;        /* rotation period [s] (sets n_co)                           */
  double lambda_c_scale;  /* multiplies lambda_C / d (1 = physical)                    */
  double r_curv_scale;    /* multiplies R_curv / d (1 = physical)                      */
  double h_gap_frac;      /* H = h_gap_frac * N * dx; QED only below H                 */
  double inj_rate;        /* injected charge per step in units of n_co dx              */
  double inj_weight;      /* weight of one injected macro-electron (units of w0)       */
  double x_thr;           /* photons below this energy (m_e c^2) are not stored         */
  double xc_floor;        /* emission is evaluated only where x_c(gamma) >= xc_floor   */
  double u_init;          /* momentum of the initial particles                         */
  double merge_frac;      /* merge when a store holds more than merge_frac * cap       */
  uint64_t seed;          /* Philox key                                                */
  int64_t cap_leptons;    /* capacity of the lepton store (live particles)             */
  int64_t cap_photons;    /* capacity of the photon store                              */
  uint32_t flags;         /* GAP_* flags                                               */
  int32_t nsub_max;       /* cap on Monte Carlo sub-steps per step (>= 1)               */
  int32_t merge_every;    /* steps between merge checks                                */
  int32_t rebucket_every; /* steps between re-sorts of the stores (0 = the longest the
                             tile margin allows, (64 - 2)/cfl - 1 steps)                */
  double atm_temp;        /* thermal atmosphere: k_B T / (m_e c^2) of its particles (the
                             paper's 0.3); protons at the same temperature           */
  int32_t atm_ppc;        /* thermal atmosphere (Sect. 2.3, 6.1): 0 = none; else before
                             every push cell 0 is refilled to atm_ppc electrons and
                             atm_ppc protons (weight 1 each) from the count the previous
                             push left there, new particles uniform in the cell with
                             momenta from the 1D relativistic thermal distribution
                             exp(-gamma/Theta), Theta = atm_temp m_e/m, the charge they
                             bring taken from the star.  Protons (charge +1, m_p/m_e =
                             1836, no QED) are pushed by the field like the leptons,
                             absorbed at h = 0 and free to leave at h = L.  Not with
                             GAP_PERIODIC, nor with the differentiable window      */
  int32_t pad_atm;
} gap_params;

/* Optional device allocator (e.g. backed by torch's caching allocator). */
typedef struct gap_allocator {
  void* (*alloc)(size_t bytes, void* ctx);   /* returns device memory or NULL */
  void (*free)(void* ptr, void* ctx);
  void* ctx;
} gap_allocator;

typedef struct gap_t gap_t;

/* Create n_tubes >= 1 independent flux tubes described by p[0..n_tubes-1]
 * (host array, read during the call), place the initial particles and solve
 * the initial field.  stream: a hipStream_t (NULL = the null stream); all
 * device work of the handle is enqueued on it.  alloc: NULL = hipMalloc.
 * The handle owns all device buffers.  On success *out receives the handle. */
int gap_init(const gap_params* p, int32_t n_tubes, void* stream, const gap_allocator* alloc, gap_t** out);

/* Advance every tube by n_steps >= 0 steps (asynchronous, on the stream). */
int gap_step(gap_t* g, int64_t n_steps);

/* Capture the next n_steps of gap_step into a HIP graph and replay it; same
 * result as gap_step(g, n_steps).  Graph replays are reused while
 * n_steps stays the same. */
int gap_step_graph(gap_t* g, int64_t n_steps);

/* Wait for all queued work; return the sticky device error (or 0). */
int gap_sync(gap_t* g);

/* diagnostic kinds for gap_diag (layout of host_buf) */
#define GAP_DIAG_COUNTS   0  /* int64[32]: see GAP_C_* below                              */
#define GAP_DIAG_FIELD    1  /* float[N]: E at cell centres k+1/2                          */
#define GAP_DIAG_ES       2  /* double[1]: surface field (periodic: mean field)             */
#define GAP_DIAG_RHO      3  /* int64[N+1]: node charge of the last deposit (2^-24 w0 units) */
#define GAP_DIAG_LEPTONS  4  /* n x {int32 cell, uint32 frac24, float u, float w, uint64 id}  */
#define GAP_DIAG_PHOTONS  5  /* n x {int32 cell, uint32 frac24, float x, float w, int32 n0,
                                     int32 pad, uint64 id}                                 */
#define GAP_DIAG_NODE_E   6  /* float[N+1]: node field used by the gather                   */
#define GAP_DIAG_DERIVED  7  /* double[8]: d_cm, lambda~, R~, dt, H, w0, s_co, N            */
#define GAP_DIAG_TIMING   8  /* double[16]: (launches, summed ms) of the lepton pass, photon
                                pass, field, re-sort, prologue, tail passes of both
                                species (one launch), the merge check (and merge, when due) and
                                conversion draws since timing was enabled or last read
                                (tube ignored; resets the record)                           */
/* Discharge diagnostics (Sect. 5: Fig. 3 rows 5-7, Fig. 5, Fig. 7).  Bins are
 * GAP_STATE_PROFILE_BIN cells wide (default 64), nb = ceil(N / bin).  Groups,
 * in order: electrons moving up (u > 0), electrons moving down, positrons up,
 * positrons down, photons with |x| > 2 moving up (x > 0), and down. */
#define GAP_DIAG_PROFILE  9  /* double[nb][6][3]: per bin and group the multiplicity
                                n/n_co = sum |w| / (bin ppc_ref), the mean Lorentz factor
                                (photons: the mean |x|) and <gamma^-3> = sum |w| gamma^-3 /
                                sum |w| (0 for photons and for empty groups)              */
#define GAP_DIAG_PEAK    10  /* double[6]: over the bins whose centre lies below H, the
                                largest pair multiplicity (both species and directions; ties
                                to the lowest bin), the height of that bin's centre (skin
                                depths; -1 if none), <gamma^-3> of the pairs there, the
                                photon multiplicity (|x| > 2) there, then min E and max E
                                over the cells                                              */
#define GAP_DIAG_RETURN  11  /* double[66]: weight of the leptons absorbed at h = 0 since the
                                last read, per bin of 1/8 decade of gamma: bin b holds gamma
                                in [10^(b/8), 10^((b+1)/8)) (the last bin everything above),
                                decided on u^2 = gamma^2 - 1 of the absorbed lepton's FP32
                                momentum, taken exactly in FP64 against edges 10^(b/4) - 1;
                                then the total weight and the total weight x gamma (gamma in
                                FP32); reading resets it                                    */
#define GAP_DIAG_SPECTRA 14    /* double[3][90]: momentum spectra (Fig. 3, row 1), the weight of
                                  electrons and of positrons per 1/8 decade of |u| = gamma
                                  beta, and of photons per 1/8 decade of |x|: bin 0 below
                                  1e-2, bin b in [10^(-2+(b-1)/8), 10^(-2+b/8)) for b = 1 ..
                                  88, bin 89 from 1e9 on; decided on the FP32 value's
                                  square in FP64 against the squares of the edges        */
#define GAP_DIAG_PHASE   15    /* double[3][nb][180]: phase space (Fig. 3, rows 1-4), the weights
                                  of GAP_DIAG_SPECTRA per bin of GAP_STATE_PROFILE_BIN cells
                                  and signed momentum column: 90 + b for p > 0 and 89 - b
                                  for p <= 0 (p = u, photons x), b the spectrum bin of |p|;
                                  the first call for a bin width allocates device memory  */
#define GAP_DIAG_PROTONS 17    /* n x {int32 cell, uint32 frac24, float u, float w, uint64 id}:
                                  the tube's live protons (none without an atmosphere or the
                                  proton initial state)                                  */
#define GAP_DIAG_LAUNCH  16    /* int32[4]: the handle's launch shape, as GAP_STATE_LAUNCH sets it
                                  (workgroups of the sorted lepton pass, of the sorted photon
                                  pass and of the tail passes, re-sort interval; tube ignored) */
#define GAP_DIAG_ESPECTRUM 13  /* double[M/2 + 1], M the next power of two >= N: the power
                                  spectrum of E along the gap, P_k = |sum_j E_j
                                  exp(-2 pi i j k / M)|^2 / M with E zero-padded to M cells
                                  (FP64 FFT of the FP32 field; Parseval: the sum of P_k over
                                  all M wavenumbers is sum_j E_j^2)                       */
#define GAP_DIAG_WATERFALL 12  /* the space-time diagram of E^2 (Fig. 4), as recorded since the
                                  last read (GAP_STATE_WATERFALL): int64 n, int64 nb, then n
                                  step indices in ascending order, then n x nb doubles, the
                                  mean of E^2 over each bin of cells after the field update
                                  of that step (the last bin ragged).  Only the last
                                  `capacity` records are kept.  Reading empties the tube's
                                  record; GAP_ESTATE while recording is off               */

/* indices of GAP_DIAG_COUNTS */
#define GAP_C_LEPTONS     0   /* live leptons                      */
#define GAP_C_PHOTONS     1   /* live photons                      */
#define GAP_C_STEP        2   /* steps taken                       */
#define GAP_C_EMIT        3   /* emission events                   */
#define GAP_C_PHO_BORN    4   /* photons stored                    */
#define GAP_C_CONV        5   /* conversions                       */
#define GAP_C_ABSORBED    6   /* leptons absorbed at h = 0         */
#define GAP_C_OUTFLOW     7   /* leptons leaving at h = L          */
#define GAP_C_PHO_EXIT    8   /* photons leaving the QED zone      */
#define GAP_C_DROPPED     9   /* particles dropped (store full)    */
#define GAP_C_MERGED      10  /* merge events                      */
#define GAP_C_ERR         11  /* sticky error code                 */
#define GAP_C_INJECTED    12  /* injected electrons                */
#define GAP_C_EMIT_EVAL   13  /* lepton-steps that evaluated emission (read the id) */
#define GAP_C_CONV_EVAL   14  /* photon-steps that evaluated conversion (read id, w) */
#define GAP_C_LEP_STEPS   15  /* lepton-steps taken                */
#define GAP_C_PHO_STEPS   16  /* photon-steps taken                */
#define GAP_C_REBUCKETS   17  /* re-sorts of the stores            */
#define GAP_C_LEP_STEPS_TAIL 18  /* part of GAP_C_LEP_STEPS taken by the tail pass   */
#define GAP_C_EMIT_EVAL_TAIL 19  /* part of GAP_C_EMIT_EVAL taken by the tail pass   */
#define GAP_C_PHO_STEPS_TAIL 20  /* part of GAP_C_PHO_STEPS taken by the tail pass   */
#define GAP_C_CONV_EVAL_TAIL 21  /* part of GAP_C_CONV_EVAL taken by the tail pass   */
#define GAP_C_PROTONS     22  /* live protons                      */
#define GAP_C_PRO_ABSORBED 23 /* protons absorbed at h = 0         */
#define GAP_C_PRO_OUTFLOW 24  /* protons leaving at h = L          */
#define GAP_C_ATM_E       25  /* electrons the atmosphere supplied */
#define GAP_C_ATM_P       26  /* protons the atmosphere supplied   */

/* Copy a diagnostic of tube `tube` into host_buf (buf_bytes long); waits for
 * queued work.  *bytes_written receives the size used.  GAP_EINVAL if the
 * buffer is too small (then *bytes_written holds the size needed). */
int gap_diag(gap_t* g, int32_t kind, int32_t tube, void* host_buf, size_t buf_bytes, size_t* bytes_written);

/* state kinds for gap_set_state */
#define GAP_STATE_PARTICLES 0  /* host_buf: int64 nl, int64 np, then nl lepton records and np
                                  photon records in the GAP_DIAG_LEPTONS / PHOTONS layouts     */
#define GAP_STATE_ES_STEP   1  /* double E_s, then int64 step                                  */
#define GAP_STATE_FIELD     2  /* float E[N] then double E_s (for GAP_FIELD_FROZEN runs)       */
#define GAP_STATE_INJECTION 3  /* double accumulator, then uint64 injected count              */
#define GAP_STATE_TIMING    4  /* int32 on/off: HIP-event timing of each kernel group of
                                  eager gap_step calls (not of graph replays)                  */
#define GAP_STATE_DRIVE     5  /* double alpha, then double inj_weight: the imposed current
                                  j_m = alpha j_co (Sect. 2.2) and the weight of one injected
                                  electron from the next step on; ends a pending window        */
#define GAP_STATE_PROFILE_BIN 7  /* int32 cells per bin >= 1 of GAP_DIAG_PROFILE and
                                    GAP_DIAG_PEAK (all tubes)                                */
#define GAP_STATE_WATERFALL 8  /* int32[3]: every, bin cells >= 1, capacity in 1..65536: record
                                  GAP_DIAG_WATERFALL after every step whose index (counted
                                  by the field update) is a multiple of `every`, keeping the
                                  last `capacity` records per tube (all tubes); every = 0
                                  stops recording and frees the record.  Allocates device
                                  memory (GAP_ENOMEM if it cannot), drops a captured graph,
                                  waits for queued work and empties the record              */
#define GAP_STATE_PROTONS  10  /* int64 n, then n records as GAP_DIAG_PROTONS: the protons of
                                  the (single) tube, replacing all; the field is re-solved
                                  (FIELD_FROZEN: only the node charge).  GAP_ESTATE without
                                  proton storage (no atmosphere, no proton initial state) */
#define GAP_STATE_ATMOSPHERE 11 /* int32 electrons, int32 protons, uint64 count: what the last
                                  push left in cell 0 (the next refill tops up to atm_ppc)
                                  and the atmosphere particles made so far (their ids).
                                  Setting particles, protons or the step resets the counts
                                  to atm_ppc (no refill before the next push)           */
#define GAP_STATE_RAISE     9  /* int32 bits: OR them into the device error word, as a kernel
                                  that meets the condition does (1 store overflow -> GAP_ECAP,
                                  2 particle outside its tile window -> GAP_ETILE, 4 non-finite
                                  field -> GAP_ENAN, 8 field scan wait bound -> GAP_EDEVICE;
                                  any other bit GAP_EINVAL).  For tests of the error path:
                                  the next synchronising call reports the code              */
#define GAP_STATE_LAUNCH    6  /* int32[4]: workgroups of the sorted lepton pass, of the sorted
                                  photon pass and of the tail passes, and the re-sort interval
                                  (the values gap_autotune returns); grids must be multiples
                                  of 8 between 8 and four resident rounds, the interval
                                  between 1 and the longest the tile margin allows, else
                                  GAP_EINVAL.  Changes no result, only the speed.             */

/* Replace part of the state of tube `tube` (only valid when n_tubes == 1;
 * GAP_STATE_TIMING, GAP_STATE_DRIVE, GAP_STATE_LAUNCH, GAP_STATE_PROFILE_BIN and
 * GAP_STATE_WATERFALL are valid for any handle, the last three ignoring `tube`).
 * Loading particles rebuilds the node charge and, unless GAP_FIELD_FROZEN,
 * the field from the current E_s.  Waits for queued work. */
int gap_set_state(gap_t* g, int32_t kind, int32_t tube, const void* host_buf, size_t bytes);

/* Pick the launch shape of the particle passes and the re-sort interval for
 * this handle's workload: a coordinate search over the workgroup counts of
 * the sorted lepton pass, the sorted photon pass and the two tail passes (in
 * multiples of one resident round, kept multiples of 8 for the XCD-aware
 * range mapping) and over the re-sort interval (up to the longest the tile
 * margin allows), each candidate timed with HIP events over `trial_steps`
 * real steps of the simulation (at least two re-sorts for the interval).
 * The steps are part of the run: every result is independent of the launch
 * shape and of the re-sort interval.  chosen (host int32[4]) receives the
 * lepton, photon and tail workgroup counts and the interval, which the
 * handle keeps.  Discards a captured graph.  Blocks until done. */
int gap_autotune(gap_t* g, int32_t trial_steps, int32_t* chosen);

/* Differentiable window (frozen QED).
 *
 * gap_window_forward runs `window_steps` steps from the current state, as
 * gap_step would but with neither merge nor re-sort inside a segment of
 * `ckpt_every` steps, saving the state (device memory, owned by the handle)
 * at the start of every segment and at the end.  loss[t] (host array of
 * n_tubes doubles) receives the time-averaged field energy density
 *   L_t = 1/(W N_t) sum_{m=1..W} sum_k (E^{n0+m}_{k+1/2})^2
 * over the fields after each of the W steps (E in units of
 * m_e c omega_p,co / e).  Every tube must be non-periodic and not
 * GAP_FIELD_FROZEN; ckpt_every must keep particles inside their tile window,
 * i.e. ckpt_every <= (64 - 2) / cfl - 1 (136 steps at cfl = 0.45); GAP_EINVAL
 * otherwise.  Blocks until the window has run.
 *
 * gap_window_backward then returns, per tube, dL/dalpha and dL/dn_inj of that window
 * (host arrays of n_tubes doubles), where n_inj = inj_rate * inj_weight is the
 * injected charge per step in units of n_co dx (use GAP_INJ_FIXED so that the
 * number of injected macro-electrons does not depend on inj_weight).  The map
 * differentiated is the push (Sect. 4: kick by E, drift at u/gamma) and the
 * field (Sect. 2.2: Gauss integration from the surface field, which the drive
 * alpha j_co and the absorbed and injected charges advance) with the QED
 * events of the window frozen: an emission is a constant recoil offset, and
 * photons and pairs born inside the window are constants; the fixed-point
 * rounding of the charge split and drift counts as the identity.  Each
 * segment is recomputed from its saved state with a tape of the lepton
 * positions and momenta (device memory of (ckpt_every + 1) x slots x 8 bytes)
 * and run in reverse; afterwards the handle is back at the window's end
 * state.  GAP_ESTATE if no window was run, or if steps or state changes came
 * after it.  Blocks until done. */
int gap_window_forward(gap_t* g, int64_t window_steps, int32_t ckpt_every, double* loss);
int gap_window_backward(gap_t* g, double* dL_dalpha, double* dL_dninj);

/* Both halves in one call: gap_window_forward(g, window_steps, ckpt_every,
 * loss) then gap_window_backward(g, dL_dalpha, dL_dninj); loss, dL_dalpha
 * and dL_dninj are host arrays of n_tubes doubles.  Returns the first error
 * of the two.  The window's QED realisation is recorded implicitly: every
 * random decision is Philox keyed by (seed, particle id, step), so the
 * recomputation inside the reverse pass draws the same events and no event
 * log is kept. */
int gap_backward(gap_t* g, int64_t window_steps, int32_t ckpt_every, double* loss, double* dL_dalpha,
                 double* dL_dninj);

/* Release the handle and every buffer it owns (waits for queued work). */
void gap_free(gap_t* g);

/* Static description of an error code. */
const char* gap_strerror(int code);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the power
 * spectrum of GAP_DIAG_ESPECTRUM for tube `tube`, written to `power`, a
 * device buffer of power_len >= M/2 + 1 doubles (M the next power of two
 * >= N), owned by the caller.  Enqueued on the handle's stream, it neither
 * allocates nor waits: the FFT's two ping-pong buffers live in a static
 * workspace of the library on each device (2 x 2^18 complex doubles, 8 MiB,
 * held until the process ends), so M is at most 2^18 (N <= 262144 cells);
 * larger tubes, or a shorter buffer, give GAP_EINVAL.  Every call on one
 * device shares that workspace: calls that may overlap on one device (two
 * streams, two handles) race and must be ordered by the caller. */
int gap_e_spectrum_noalloc(gap_t* g, int32_t tube, double* power, int64_t power_len);

/* The quantum samplers the particle passes use (GAP_QUANTUM), evaluated on
 * the device at n given points: kind 0 gives the photon energy fraction
 * x/gamma for a lepton at chi[i], kind 1 the electron's energy fraction of a
 * pair created by a photon at chi[i]; words[i] is the Philox word whose top
 * 24 bits make the uniform r = (k + 1/2) 2^-24 (Sect. 3.1 spectrum S, Sect.
 * 3.2 pair creation).  Host pointers, out[i] as double; the call allocates
 * and waits.  GAP_EINVAL for another kind or a negative or non-finite chi. */
int gap_qed_sample(gap_t* g, int32_t kind, const double* chi, const uint32_t* words, int64_t n, double* out);

/* Host utility: invert the cumulative classical synchrotron photon-number
 * spectrum with the library's own table (the sampler the device uses):
 * xi[i] = C^-1(r[i]) for r in (0,1).  Host pointers; no device work. */
int gap_sync_inverse_host(const float* r, float* xi, int64_t n);

#ifdef __cplusplus
}
#endif
#endif /* GAP_H */
