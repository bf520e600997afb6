// gap_device.hpp -- device-side building blocks of libgap (gfx950, wave64):
// the state layout, Philox4x32-10, the QED rate fits and the photon-energy
// sampler.  Written for this library; shares nothing with the CPU oracle.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gap {

// ---------------------------------------------------------------- layout
// Particles live in per-species stores of fixed capacity, split into
//  * a sorted region: chunks of CHUNK slots, each chunk belonging to one tile
//    of TILE cells, padded with dead slots (a workgroup of TPB threads pushes
//    one chunk per iteration, VEC consecutive slots per thread);
//  * a tail: particles appended since the last re-sort (births, injection),
//    each carrying its tile index in `tt`.
// A position is a 32-bit fixed-point offset from the tile's window base
// (first cell - MARGIN): top 8 bits = cell offset, low 24 bits = fraction.
constexpr int TILE = 128;       // cells per tile
constexpr int MARGIN = 64;      // cells of slack on each side of a tile
constexpr int WIN = 256;        // cells addressable from a tile base
constexpr int TPB = 256;        // threads per workgroup
constexpr int VEC = 4;          // consecutive slots per thread in the sorted passes
constexpr int CHUNK = TPB * VEC; // slots per chunk
constexpr int PPC = CHUNK / TPB; // 256-slot pieces per chunk
constexpr int FRAC = 24;        // fractional bits of a position
constexpr int WAVE = 64;

constexpr int NTAB = 4096;      // photon-spectrum table segments
constexpr float TAB_YLO = 0.69314718055994531f;  // ln 2
constexpr float TAB_YHI = 17.5f;

// counters (mirrors the GAP_C_* indices of the ABI)
enum : int {
  C_LEPTONS = 0, C_PHOTONS = 1, C_STEP = 2, C_EMIT = 3, C_PHO_BORN = 4, C_CONV = 5, C_ABSORBED = 6,
  C_OUTFLOW = 7, C_PHO_EXIT = 8, C_DROPPED = 9, C_MERGED = 10, C_ERR = 11, C_INJECTED = 12,
  C_EMIT_EVAL = 13, C_CONV_EVAL = 14, C_LEP_STEPS = 15, C_PHO_STEPS = 16, C_REBUCKETS = 17,
  C_LEP_STEPS_TAIL = 18, C_EMIT_EVAL_TAIL = 19, C_PHO_STEPS_TAIL = 20, C_CONV_EVAL_TAIL = 21,
  C_PROTONS = 22, C_PRO_ABSORBED = 23, C_PRO_OUTFLOW = 24, C_ATM_E = 25, C_ATM_P = 26, C_N = 32
};

enum : uint32_t {
  F_QED_OFF = 1u, F_ETA_CO_OFF = 2u, F_FIELD_FROZEN = 4u, F_RECOIL_OFF = 8u, F_PERIODIC = 16u,
  F_MERGE_ON = 32u, F_TRACK_ALL = 64u, F_ANTI_ALIGNED = 128u, F_CONV_OFF = 1024u, F_EMIT_OFF = 2048u,
  F_INJ_FIXED = 4096u, F_FILTER = 8192u, F_QUANTUM = 16384u
};

// sticky device error bits
enum : int { E_CAP = 1, E_TILE = 2, E_NAN = 4, E_SCAN = 8 };

// Per-tube constants and mutable scalars (device memory).
struct Tube {
  // grid
  int32_t N, node_off, cell_off, tile_first;
  int32_t n_tiles, flags, nsub_max, pad0;
  // float constants of the push
  float dt, cfl24;          // dt; cfl * 2^24 (displacement of a beta = 1 particle, fixed point)
  float lr, inv_rc;         // lambda~/R~, 1/R~
  float b, b_over_lam;      // B/B_Q, b/lambda~
  float xc_floor, x_thr;
  float emit_k;             // alpha_em * dt / R~
  float conv_k;             // alpha_em * dt * b / lambda~
  float chi_skip;           // photons with chi below this cannot convert in one step
  float pad3;
  int32_t dpho;             // photon displacement per step: rint(cfl 2^24)
  int32_t pad1;
  // double constants of the field
  double dtd, scale;        // dt; w0 / 2^24
  double drive;             // alpha * s_co * dt
  double inj_per_step;      // macro-electrons injected per step
  double inv_len_scale;     // periodic: w0 dx / (2^24 2^24 L)
  int64_t bg_unit;          // -s_co ppc_ref 2^24 (0 with ETA_CO_OFF)
  int64_t hfix;             // ceil(H/dx 2^24): QED zone is cell*2^24 + frac < hfix
  int64_t inj_T;            // fixed-point charge of one injected electron
  float inj_w;              // weight of one injected electron (positive)
  float pad2;
  uint64_t seed;
  // mutable
  double Es, inj_acc;
  int64_t dq, dcur, step;   // step: steps completed (the field update of a step adds one)
  int64_t step_now;         // index of the step being taken (set by the prologue; read by the passes)
  uint64_t inj_count;
  int64_t cnt[C_N];
  // thermal atmosphere (atm_ppc > 0): Theta of its electrons and protons,
  // particles made so far (their ids), and the electrons (0, 1) and protons
  // (2, 3) in cell 0 after the push of a step of parity 0 or 1
  double atm_theta_e, atm_theta_p;
  int32_t atm_ppc, pad5;
  uint64_t atm_count;
  int32_t atm_cnt[4];
};

struct Tile {
  int32_t tube, first, base, ncell;   // base = first - MARGIN (tube-local cells)
};

struct Ctl {                  // control block of one store
  int64_t n_sorted_chunks;    // sorted region = slots [0, CHUNK * n_sorted_chunks)
  int64_t tail;               // tail length (slots after the sorted region)
  int64_t tail_snap;          // tail length at the start of the step's pass
  int64_t capacity;           // slots
  int64_t limit;              // appends stop at this slot (keeps room for re-sort padding)
  int64_t total_chunks_new;   // written by the re-sort scan
  int64_t cap_live;           // live-particle cap (merge threshold reference)
  int64_t tail_pre;           // tail length before this step's injection
  // photons: steps left in which no slot past a tile's hot prefix of the
  // sorted region can draw a conversion (set by the re-sort, counted down by
  // each step's prologue; < 0: no such guarantee)
  int64_t cold_steps;
};

struct LepBuf { uint32_t* pos; float* u; float* w; uint64_t* id; };
// protons: absolute cell and 24-bit fraction, momentum, weight, id, tube
struct ProBuf { int32_t* cell; uint32_t* frac; float* u; float* w; uint64_t* id; int32_t* tube; };
struct PhoBuf { uint32_t* pos; float* x; float* w; int32_t* n0; uint64_t* id; };

// ---------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon et al., SC'11): 10 rounds; each round multiplies
// words 0 and 2 by fixed 32-bit constants, swaps the high halves across and
// xors in the key, which is bumped by a Weyl increment between rounds.
struct u4 { uint32_t a, b, c, d; };

// Two equivalent forms of the same rounds: WIDE takes each product with one
// 32x32 -> 64 multiply, otherwise with separate low and high multiplies.
template <bool WIDE = false>
__device__ __forceinline__ u4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
    uint32_t hi0, lo0, hi1, lo1;
    if (WIDE) {
      const uint64_t p0 = (uint64_t)m0 * c0, p1 = (uint64_t)m1 * c2;
      hi0 = (uint32_t)(p0 >> 32); lo0 = (uint32_t)p0;
      hi1 = (uint32_t)(p1 >> 32); lo1 = (uint32_t)p1;
    } else {
      hi0 = __umulhi(m0, c0); lo0 = m0 * c0;
      hi1 = __umulhi(m1, c2); lo1 = m1 * c2;
    }
    uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
  }
  return {c0, c1, c2, c3};
}

// counter = (id lo, id hi, step, tag << 16 | sub), key = seed
template <bool WIDE = false>
__device__ __forceinline__ u4 draw(uint64_t seed, uint64_t id, int64_t step, uint32_t tag, uint32_t sub) {
  return philox<WIDE>((uint32_t)id, (uint32_t)(id >> 32), (uint32_t)step, (tag << 16) | (sub & 0xFFFFu),
                      (uint32_t)seed, (uint32_t)(seed >> 32));
}

enum : uint32_t { T_INIT = 1, T_EMIT = 2, T_CONV = 3, T_INJ = 4, T_MERGE = 5, T_CHILD = 6, T_ATM = 7 };

constexpr float MASS_P = 1836.0f;                 // proton to electron mass ratio (Sect. 6.1)
constexpr uint64_t ATM_ID_BASE = 3ull << 61;      // ids of atmosphere particles

// Bernoulli decision u < p with u = (k + 1/2) 2^-24, k = top 24 bits of r,
// taken exactly: 2k + 1 < p 2^25 (FP64 compare of exact values).
__device__ __forceinline__ bool bern(uint32_t r, float p) {
  return (double)(2u * (r >> 8) + 1u) < (double)p * 33554432.0;
}
// The same decision in integers: 2k + 1 < P (P = p 2^25, exact in FP32) holds
// iff 2k + 1 < ceil(P), and 2k + 1 = (r >> 7) | 1.
__device__ __forceinline__ uint32_t bern_thr(float p) { return (uint32_t)ceilf(p * 33554432.0f); }
__device__ __forceinline__ bool bern_t(uint32_t r, uint32_t thr) { return ((r >> 7) | 1u) < thr; }
__device__ __forceinline__ float unif(uint32_t r) { return ((float)(r >> 8) + 0.5f) * 5.9604645e-8f; }

__device__ __forceinline__ uint64_t child_id(uint64_t seed, uint64_t parent, int64_t step, uint32_t j) {
  u4 r = draw(seed, parent, step, T_CHILD, j);
  return (uint64_t)r.a | ((uint64_t)r.b << 32);
}

// ---------------------------------------------------------------- QED fits
// emission-rate function of Sect. 3.1 (fit quoted with eq. tau_syn):
// 5/(2 sqrt 3) (1 + 16 sqrt3/5 chi + 1.1 chi^2)^(-1/6), via the hardware
// base-2 logarithm and exponential
__device__ __forceinline__ float t_syn(float chi) {
  const float v = __fmaf_rn(__fmul_rn(1.1f, chi), chi, __fmaf_rn(5.5425625842204074f, chi, 1.0f));
  return __fmul_rn(1.4433756729740644f, __builtin_amdgcn_exp2f(__fmul_rn(__builtin_amdgcn_logf(v), -1.0f / 6.0f)));
}
// pair-creation function of Sect. 3.2 (fit quoted with eq. tau_bw):
// 0.23 exp(-8/(3 chi)) (1 + 0.22 chi)^(-1/3)
__device__ __forceinline__ float t_bw(float chi) {   // (chi = 0 gives 0 through 1/chi = inf)
  const float e = -3.8471206f * __builtin_amdgcn_rcpf(chi) -
                  __builtin_amdgcn_logf(1.0f + 0.22f * chi) * (1.0f / 3.0f);   // 8/3 log2(e)
  return 0.23f * __builtin_amdgcn_exp2f(e);
}

// Classical synchrotron number spectrum: xi = C^-1(r) from the table.
//  r <= 1/2: tab[i] = xi^(1/3) at r = i / (2 NTAB), linear in r near 0;
//  r > 1/2 : tab[NTAB+1+i] = xi at y = -ln(1-r) on [ln 2, TAB_YHI].
__device__ __forceinline__ float sync_sample(float r, const float* __restrict__ tab) {
  if (r <= 0.5f) {
    float t = r * (2.0f * NTAB);
    int i = min((int)t, NTAB - 1);
    float f = t - (float)i;
    float v = tab[i] + f * (tab[i + 1] - tab[i]);
    return v * v * v;
  }
  float y = -logf(1.0f - r);
  float t = (y - TAB_YLO) * ((float)NTAB / (TAB_YHI - TAB_YLO));
  t = fminf(fmaxf(t, 0.0f), (float)NTAB - 1e-3f);
  int i = (int)t;
  float f = t - (float)i;
  const float* h = tab + NTAB + 1;
  return h[i] + f * (h[i + 1] - h[i]);
}

// ---------------------------------------------------------------- quantum spectra
// Tables of the quantum-corrected photon spectrum and pair split (tubes with
// F_QUANTUM), built on the host at initialisation.
//
// Photon energy fraction d = x/gamma: column c holds ln z at the rows below,
// z = 2 d / (3 chi (1 - d)); column 0 is chi = 0 (the classical spectrum),
// column c >= 1 is chi = QS_CHI_LO 10^((c-1)/QS_PER_DEC).  Rows: r <= 1/2 at
// ln r uniform on [QS_ALO, ln 1/2] (QS_NR + 1 nodes), r > 1/2 at y = -ln(1-r)
// uniform on [ln 2, QS_YHI].  ln z is nearly linear in ln r for small r, in
// ln chi at both ends of the chi range (z -> its classical value as chi -> 0,
// z ~ 1/chi as chi -> inf), and columns are blended linearly in ln chi
// (linearly in chi between columns 0 and 1).
constexpr int QS_NR = 1024;
constexpr int QS_PER_DEC = 16;
constexpr int QS_COLS = 1 + 6 * QS_PER_DEC + 1;      // chi = 0 and 1e-3 .. 1e3
constexpr int QS_ROW = 2 * (QS_NR + 1);
constexpr float QS_CHI_LO = 1e-3f;
constexpr float QS_ALO = -17.328679513998633f;       // ln 2^-25, the smallest 24-bit midpoint uniform
constexpr float QS_AHI = -0.69314718055994531f;      // ln 1/2
constexpr float QS_YLO = 0.69314718055994531f;       // ln 2
constexpr float QS_YHI = 17.328679513998633f;        // -ln 2^-25
// Pair split, electron fraction v: by the symmetry v <-> 1 - v only r <= 1/2
// is tabulated, as s = w sqrt((1 + chi)/chi), w = 1/2 - v, at q = (2 r)^(1/4)
// uniform on [0, 1] (QB_NR + 1 nodes); column c is chi = QB_CHI_LO
// 10^(c/QB_PER_DEC), clamped to the table's range.
constexpr int QB_NR = 512;
constexpr int QB_PER_DEC = 16;
constexpr int QB_COLS = 5 * QB_PER_DEC + 1;           // chi = 1e-2 .. 1e3
constexpr float QB_CHI_LO = 1e-2f;

__device__ __forceinline__ float qtab_row(const float* __restrict__ col, int i, float f) {
  return col[i] + f * (col[i + 1] - col[i]);
}

// 1 - r for the 24-bit midpoint uniform r = unif(w), exact in FP32 (the
// difference 1 - r formed in FP32 is not: r rounds to 1 for the top word).
__device__ __forceinline__ float unif_hi(uint32_t w) { return ((float)(0xFFFFFFu - (w >> 8)) + 0.5f) * 5.9604645e-8f; }

// Photon energy fraction of the quantum spectrum at chi for the uniform of
// the Philox word rw.
__device__ __forceinline__ float qsyn_fraction(float chi, uint32_t rw, const float* __restrict__ qs) {
  int c;
  float fc;
  if (chi < QS_CHI_LO) {
    c = 0;
    fc = chi * (1.0f / QS_CHI_LO);
  } else {
    float pc = 1.0f + log2f(chi * (1.0f / QS_CHI_LO)) * (QS_PER_DEC / 3.3219280948873623f);
    pc = fminf(pc, (float)(QS_COLS - 1));
    c = min((int)pc, QS_COLS - 2);
    fc = pc - (float)c;
  }
  int half;
  float t;
  if ((rw >> 8) < 0x800000u) {          // r < 1/2
    half = 0;
    t = (logf(unif(rw)) - QS_ALO) * ((float)QS_NR / (QS_AHI - QS_ALO));
  } else {
    half = QS_NR + 1;
    t = (-logf(unif_hi(rw)) - QS_YLO) * ((float)QS_NR / (QS_YHI - QS_YLO));
  }
  t = fminf(fmaxf(t, 0.0f), (float)QS_NR - 1e-3f);
  const int i = (int)t;
  const float f = t - (float)i;
  const float a = qtab_row(qs + c * QS_ROW + half, i, f);
  const float b = qtab_row(qs + (c + 1) * QS_ROW + half, i, f);
  const float z = expf(a + fc * (b - a));
  const float q = 3.0f * chi * z;
  return q / (2.0f + q);
}

// Electron energy fraction of a pair created by a photon at chi, for the
// uniform of the Philox word rw.
__device__ __forceinline__ float qbw_fraction(float chi, uint32_t rw, const float* __restrict__ qb) {
  float pc = log2f(fmaxf(chi, QB_CHI_LO) * (1.0f / QB_CHI_LO)) * (QB_PER_DEC / 3.3219280948873623f);
  pc = fminf(pc, (float)(QB_COLS - 1));
  const int c = min((int)pc, QB_COLS - 2);
  const float fc = pc - (float)c;
  const bool upper = (rw >> 8) >= 0x800000u;
  const float rr = upper ? unif_hi(rw) : unif(rw);
  float t = sqrtf(sqrtf(2.0f * rr)) * (float)QB_NR;
  t = fminf(t, (float)QB_NR - 1e-3f);
  const int i = (int)t;
  const float f = t - (float)i;
  const float a = qtab_row(qb + c * (QB_NR + 1), i, f);
  const float b = qtab_row(qb + (c + 1) * (QB_NR + 1), i, f);
  // (below the first column s keeps its small-chi limit; w scales with chi)
  const float w = (a + fc * (b - a)) * sqrtf(chi / (1.0f + chi));
  return upper ? 0.5f + w : 0.5f - w;
}

// ---------------------------------------------------------------- wave utils
__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }
// number of set bits of `mask` below this lane
__device__ __forceinline__ int rank_in(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ void atomic_add_i64(int64_t* p, int64_t v) {
  atomicAdd(reinterpret_cast<unsigned long long*>(p), (unsigned long long)v);
}

// Wave-aggregated counter increment: one atomic per wave.
__device__ __forceinline__ void wave_count(int64_t* p, bool pred) {
  uint64_t m = __ballot(pred);
  if (m && lane_id() == __ffsll((long long)m) - 1) atomic_add_i64(p, (int64_t)__popcll(m));
}

}  // namespace gap
