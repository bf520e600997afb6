// gap_kernels.hpp -- the per-step kernels of libgap (gfx950, wave64).
#pragma once
#include "gap_device.hpp"

#include <type_traits>

namespace gap {

// Everything a step kernel needs; passed by value.
struct Ctx {
  Tube* tubes;
  const Tile* tiles;
  // lepton store (current buffers)
  LepBuf L;
  Ctl* lc;
  const int32_t* lchunk;  // chunk -> tile (sorted region)
  int32_t* ltt;           // slot -> tile (tail)
  // photon store
  PhoBuf P;
  Ctl* pc;
  const int32_t* pchunk;
  const uint16_t* pchot;  // hot slots at the start of each sorted chunk
  int32_t* ptt;
  // grid
  long long* rho;         // node charge accumulator, sum_t (N_t + 1)
  const float* ebar;      // node field, sum_t (N_t + 1)
  const float* tab;       // photon spectrum table
  const float* qs;        // quantum photon-spectrum table (tubes with F_QUANTUM), else null
  const float* qb;        // quantum pair-split table
  // protons (tubes with an atmosphere or the proton initial state): slots
  // [0, *pr_n) of R, dead ones with w = 0 until the next compaction
  ProBuf R;
  long long* pr_n;
  long long pr_cap;
  int* err;
  long long* shard;       // event counters [tube][NSHARD][C_N], summed by the host
  // conversion queue of the sorted photon pass: workgroup b of the photon
  // kernel writes its entries {slot, probability bits, tile, tube} from
  // entry c0(b) * CHUNK on, c0(b) being the first chunk of its range, and
  // their number to pq_count[b]
  uint4* pq;
  int* pq_count;
  // photon births of the sorted lepton pass, queued for the tail launch:
  // entries {slot, post-kick u bits, event mask low word, high word};
  // workgroup b of the pass (bq_groups of them) wrote bq_count[b] entries
  // from entry bq_start[b] on
  uint4* bq;
  int* bq_count;
  long long* bq_start;
  int bq_groups;
  // return spectrum per tube (RET_N doubles): absorbed weight per bin of
  // log10 gamma, then the total weight and the total weight x gamma; the
  // bins' lower edges in u^2 = gamma^2 - 1 (ret_thr[b] = 10^(b/4) - 1)
  double* ret;
  const double* ret_thr;
};

constexpr int RET_NB = 64;            // bins of 1/8 decade over gamma in [1, 1e8)
constexpr int RET_N = RET_NB + 2;

// A lepton of weight w and momentum u absorbed at the surface (Fig. 7's
// return flux): its bin is the last whose lower edge in u^2 it reaches, u^2
// taken exactly in FP64 from the FP32 u (a binary search over the edges, so
// that the lepton pass keeps its registers); gamma for the energy moment in
// FP32.
__device__ __forceinline__ void return_add(double* ret, const double* thr, int tube, float u, float w) {
  const double u2 = (double)u * (double)u;
  int b = 0;
#pragma unroll
  for (int st = RET_NB / 2; st >= 1; st >>= 1)
    if (thr[b + st] <= u2) b += st;
  double* r = ret + (size_t)tube * RET_N;
  const float aw = fabsf(w);
  atomicAdd(&r[b], (double)aw);
  atomicAdd(&r[RET_NB], (double)aw);
  atomicAdd(&r[RET_NB + 1], (double)(aw * __builtin_amdgcn_sqrtf(1.0f + u * u)));
}

constexpr int NSHARD = 64;

__device__ __forceinline__ long long* shard_at(long long* sh, int tube, int idx) {
  return sh + ((long long)tube * NSHARD + (blockIdx.x % NSHARD)) * C_N + idx;
}

__device__ __forceinline__ int wrap_cell(int c, int N) { return c < 0 ? c + N : (c >= N ? c - N : c); }

// Add `v` to counter `idx` of the tube `t` of each lane (t < 0: no-op), one
// atomic per distinct tube in the wave.
__device__ __forceinline__ void count_by_tube(long long* shard, int t, int idx, int64_t v) {
  while (true) {
    uint64_t m = __ballot(t >= 0);
    if (!m) break;
    int lead = __ffsll((long long)m) - 1;
    int k = __shfl(t, lead);
    long long s = (t == k) ? (long long)v : 0ll;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d);
    if (lane_id() == lead && s != 0) atomicAdd((unsigned long long*)shard_at(shard, k, idx), (unsigned long long)s);
    if (t == k) t = -1;
  }
}

// Per-thread event counts of one tube, reduced over the workgroup and added
// to the tube's shard once per flush (not once per wave).
struct LocalCounts {
  int v[8];
  __device__ void clear() {
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = 0;
  }
};

// counter slots of the lepton (KIND 0) and photon (KIND 1) passes; the tail
// passes (KIND 2, 3) count their particle-steps and evaluations separately
template <int KIND>
__device__ __forceinline__ int cnt_index(int i) {
  if (KIND == 2 && i == 0) return C_LEP_STEPS_TAIL;
  if (KIND == 2 && i == 1) return C_EMIT_EVAL_TAIL;
  if (KIND == 3 && i == 0) return C_PHO_STEPS_TAIL;
  if (KIND == 3 && i == 1) return C_CONV_EVAL_TAIL;
  if (KIND == 0 || KIND == 2) {
    switch (i) {
      case 0: return C_LEP_STEPS; case 1: return C_EMIT_EVAL; case 2: return C_EMIT; case 3: return C_PHO_BORN;
      case 4: return C_DROPPED; case 5: return C_ABSORBED; case 6: return C_OUTFLOW; default: return -1;
    }
  }
  switch (i) {
    case 0: return C_PHO_STEPS; case 1: return C_CONV_EVAL; case 2: return C_CONV; case 3: return C_DROPPED;
    case 4: return C_PHO_EXIT; default: return -1;
  }
}

template <int KIND>
__device__ void flush_counts(long long* shard, int tube, LocalCounts& lc, long long* s_cnt) {
  __syncthreads();
  if (threadIdx.x < 8) s_cnt[threadIdx.x] = 0;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    int x = lc.v[i];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d);
    if (lane_id() == 0 && x != 0) atomicAdd((unsigned long long*)&s_cnt[i], (unsigned long long)(long long)x);
  }
  __syncthreads();
  if (threadIdx.x < 8) {
    const int ci = cnt_index<KIND>(threadIdx.x);
    if (ci >= 0 && s_cnt[threadIdx.x] != 0)
      atomicAdd((unsigned long long*)shard_at(shard, tube, ci), (unsigned long long)s_cnt[threadIdx.x]);
  }
  lc.clear();
}

// Exclusive prefix sum of `v` over the wave; returns the exclusive value and
// writes the wave total to *total.
__device__ __forceinline__ int wave_excl_scan(int v, int* total) {
  int incl = v;
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    int o = __shfl_up(incl, d);
    if (lane_id() >= d) incl += o;
  }
  *total = __shfl(incl, WAVE - 1);
  return incl - v;
}

// Append room of a store during a pass: the sorted-region size and the append
// limit (neither changes while the particle passes run), read once per
// workgroup and held wave-uniform.
struct Room { long long S, L; };

__device__ __forceinline__ long long rfl64(long long v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v), hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (long long)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ Room load_room(const Ctl* c) {
  Room r;
  r.S = rfl64(c->n_sorted_chunks * CHUNK);
  r.L = rfl64(c->limit);
  return r;
}

// Reserve `n` tail slots of a store (one atomic per wave); returns the first
// slot index for this lane's records.  A wave whose reservation runs past the
// room left before the limit clamps the tail back to that room, so the tail
// never covers unwritten slots beyond the limit (every reservation made after
// a clamp starts at the room and is dropped whole).
__device__ __forceinline__ long long reserve_tail(Ctl* c, const Room& rm, int n, int* dropped) {
  int total;
  int ex = wave_excl_scan(n, &total);
  long long base = 0;
  if (lane_id() == WAVE - 1 && total > 0) {
    base = (long long)atomicAdd((unsigned long long*)&c->tail, (unsigned long long)total);
    const long long room = rm.L > rm.S ? rm.L - rm.S : 0;
    if (base + total > room) atomicMin((unsigned long long*)&c->tail, (unsigned long long)room);
  }
  base = __shfl(base, WAVE - 1);
  const long long first = rm.S + base + ex;
  // appends beyond the limit are dropped
  *dropped = 0;
  if (n > 0 && first + n > rm.L) {
    long long ok = rm.L - first;
    if (ok < 0) ok = 0;
    *dropped = n - (int)ok;
  }
  return first;
}

// ------------------------------------------------------------------ prologue
// Surface injection (cold electrons in cell 0 at a deterministic rate) and
// the snapshots of the tails that this step's passes will process.
__device__ __forceinline__ void clamp_tail(Ctl* c) {
  long long room = c->limit - c->n_sorted_chunks * CHUNK;
  if (room < 0) room = 0;
  if (c->tail > room) c->tail = room;
}

// ---- Thermal atmosphere (Sect. 2.3 atmospheric boundary; Sect. 6.1: k_B T
// = 0.3 m_e c^2, protons with m_p/m_e = 1836).  Reading: a reservoir in
// cell 0 holding atm_ppc electrons and atm_ppc protons (weight 1 each),
// refilled before each push from the count the previous push left there;
// new particles are uniform in the cell with momenta of the one-dimensional
// relativistic thermal distribution f(u) ~ exp(-gamma/Theta), and the charge
// they bring leaves the star.

__device__ __forceinline__ double u24d(uint32_t w) { return ((double)(w >> 8) + 0.5) * (1.0 / 16777216.0); }

// One momentum of f(u) ~ exp(-gamma/Theta) by rejection, in FP64: in the
// kinetic energy e = gamma - 1 the density is exp(-e/Theta) h(e), h = (1+e)
// / sqrt(e(2+e)) <= 1/sqrt(2e) + 1, and the envelope exp(-e/Theta)
// (1/sqrt(2e) + 1) is a mixture of e = Theta Z^2/2 (Z normal, Box-Muller),
// weight sqrt(pi Theta/2), and e = -Theta ln U, weight Theta.  Attempt j
// takes the words of draw(seed, id, step, T_ATM, j): a picks the component
// (and its bit 0 the sign of u), b and c make e, d accepts with probability
// h / (1/sqrt(2e) + 1).  After 64 rejections (probability below 1e-30) u = 0.
__device__ double atm_momentum(uint64_t seed, uint64_t id, int64_t step, double theta) {
  const double wa = sqrt(3.14159265358979323846 * theta / 2.0), wb = theta;
  for (uint32_t j = 0; j < 64; ++j) {
    const u4 r = draw(seed, id, step, T_ATM, j);
    double e;
    if (u24d(r.a) * (wa + wb) < wa) {
      const double c = cos(2.0 * 3.14159265358979323846 * u24d(r.c));
      e = -theta * log(u24d(r.b)) * c * c;
    } else {
      e = -theta * log(u24d(r.b));
    }
    if (!(e > 0.0)) continue;
    const double h = (1.0 + e) / sqrt(e * (2.0 + e));
    const double bnd = 1.0 / sqrt(2.0 * e) + 1.0;
    if (u24d(r.d) * bnd < h) {
      const double u = sqrt(e * (2.0 + e));
      return (r.a & 1u) ? u : -u;
    }
  }
  return 0.0;
}

// Refill of one tube's atmosphere (prologue thread of the tube): electrons
// into the lepton tail, protons after the proton slots in use.  The counts
// of the previous push are read from the slot of its step parity and
// cleared for the push after this one.
__device__ void atmosphere_refill(const Ctx& cx, Tube& T, int t, long long S, long long lim) {
  const int par = (int)((T.step - 1) & 1);
  const Tile& tl = cx.tiles[T.tile_first];
  int64_t dq = 0;
  for (int sp = 0; sp < 2; ++sp) {
    const int m = T.atm_ppc - T.atm_cnt[2 * sp + par];
    T.atm_cnt[2 * sp + par] = 0;
    if (m <= 0) continue;
    const double theta = sp == 0 ? T.atm_theta_e : T.atm_theta_p;
    const long long first = sp == 0 ? S + (long long)atomicAdd((unsigned long long*)&cx.lc->tail, (unsigned long long)m)
                                    : (long long)atomicAdd((unsigned long long*)cx.pr_n, (unsigned long long)m);
    for (int j = 0; j < m; ++j) {
      const uint64_t id = ATM_ID_BASE + T.atm_count++;
      const long long slot = first + j;
      if (slot >= (sp == 0 ? lim : cx.pr_cap)) { T.cnt[C_DROPPED]++; atomicOr(cx.err, E_CAP); continue; }
      const u4 r = draw(T.seed, id, T.step, T_ATM, 0xFFFFu);
      const float u = (float)atm_momentum(T.seed, id, T.step, theta);
      if (sp == 0) {
        cx.L.pos[slot] = ((uint32_t)(0 - tl.base) << FRAC) | (r.a >> 8);
        cx.L.u[slot] = u;
        cx.L.w[slot] = -1.0f;
        cx.L.id[slot] = id;
        cx.ltt[slot] = T.tile_first;
        dq += 16777216;                // E_s -= q w0 of the electron (q < 0)
        T.cnt[C_ATM_E]++;
      } else {
        cx.R.cell[slot] = 0;
        cx.R.frac[slot] = r.a >> 8;
        cx.R.u[slot] = u;
        cx.R.w[slot] = 1.0f;
        cx.R.id[slot] = id;
        cx.R.tube[slot] = t;
        dq -= 16777216;
        T.cnt[C_ATM_P]++;
        atomic_add_i64(&T.cnt[C_PROTONS], 1);
      }
    }
  }
  atomic_add_i64(&T.dq, dq);
}

constexpr int PRE_THREADS = 256;

// One workgroup of at most PRE_THREADS threads (a wave per 64 tubes);
// thread t handles tubes t, t + blockDim.x, ...  The launch bound asks for at
// most 96 registers a lane (5 waves a SIMD), so that the prologue's waves fit
// beside a SIMD's waves of the lepton pass as soon as one of them ends; with
// 1024 threads and 121 registers it needed a whole idle CU and waited for the
// lepton pass to drain before the photon side could start.  Each tube's
// injected electrons take tail slots through one atomic reservation (the
// order of tail slots changes no result).  The prologue belongs to the photon
// side of the step: it runs before the photon passes, while the lepton pass
// of the same step may already run, so it touches nothing that pass writes
// except through atomics (the surface charge dq); the photon tail's snapshot
// is taken by the field scan at the end of the previous step, after every
// photon birth of that step.
__global__ __launch_bounds__(PRE_THREADS, 5) void k_pre(Ctx cx, int n_tubes) {
  // (appends never leave the tails past the limit; the passes below stay
  // inside the stores whatever the tails hold)
  if (threadIdx.x == 0) {
    clamp_tail(cx.lc);
    cx.lc->tail_pre = cx.lc->tail;
    if (cx.pc->cold_steps >= 0) cx.pc->cold_steps -= 1;
  }
  __syncthreads();
  const long long S = cx.lc->n_sorted_chunks * CHUNK;
  const long long lim = cx.lc->limit;
  for (int t = threadIdx.x; t < n_tubes; t += blockDim.x) {
    Tube& T = cx.tubes[t];
    // the photon passes of this step read its index from step_now: the
    // field update (which counts the step) may run beside them
    T.step_now = T.step;
    if (T.atm_ppc > 0 && !(T.flags & F_PERIODIC)) atmosphere_refill(cx, T, t, S, lim);
    if (T.inj_per_step <= 0.0 || (T.flags & F_PERIODIC)) continue;
    T.inj_acc += T.inj_per_step;
    const double fl = floor(T.inj_acc);
    T.inj_acc -= fl;
    const int m = (int)fl;
    if (m <= 0) continue;
    const long long first = S + (long long)atomicAdd((unsigned long long*)&cx.lc->tail, (unsigned long long)m);
    const Tile& tl = cx.tiles[T.tile_first];
    int64_t dq = 0;
    for (int j = 0; j < m; ++j) {
      const long long slot = first + j;
      if (slot >= lim) { T.cnt[C_DROPPED]++; atomicOr(cx.err, E_CAP); continue; }
      const uint64_t id = (1ull << 62) + T.inj_count++;
      const u4 r = draw(T.seed, id, T.step, T_INJ, 0);
      cx.L.pos[slot] = ((uint32_t)(0 - tl.base) << FRAC) | (r.a >> 8);
      cx.L.u[slot] = 0.0f;
      cx.L.w[slot] = -T.inj_w;
      cx.L.id[slot] = id;
      cx.ltt[slot] = T.tile_first;
      dq += T.inj_T;                 // E_s -= q w0 of the injected electron (q < 0)
      T.cnt[C_INJECTED]++;
    }
    atomic_add_i64(&T.dq, dq);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    clamp_tail(cx.lc);               // (reservations past the limit were dropped)
    cx.lc->tail_snap = cx.lc->tail;
  }
}

// ------------------------------------------------------------------ leptons
// Flush the LDS node-charge window of tile `tile` into the global accumulator.
__device__ void flush_window(const Ctx& cx, int tile, long long* s_rho) {
  __syncthreads();
  const Tile tl = cx.tiles[tile];
  const Tube& T = cx.tubes[tl.tube];
  const bool per = (T.flags & F_PERIODIC) != 0;
  for (int j = threadIdx.x; j <= WIN; j += blockDim.x) {
    long long v = s_rho[j];
    if (v != 0) {
      int node = tl.base + j;
      if (per) node = wrap_cell(node, T.N);
      atomicAdd((unsigned long long*)&cx.rho[T.node_off + node], (unsigned long long)v);
      s_rho[j] = 0;
    }
  }
  __syncthreads();
}

// Constants of one tile and its tube, read once per tile switch and held in
// scalar registers (the tube records are also written by the kernels, so the
// compiler cannot turn per-lane reads of them into scalar loads).
struct KC {
  int tile, tube, base, N, node_off, flags, nsub_max, dpho;
  int64_t step, hfix;
  // a non-periodic tube's photon at tile-local position q (fixed point from
  // the window base) is outside [0, L) or above H when q < xlo or q >= xhi
  int64_t xlo, xhi;
  float dt, lr, inv_rc, b, xc_floor, x_thr, emit_k, conv_k, cfl24, chi_skip;
  uint64_t seed;
};

__device__ __forceinline__ int rfl(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float rfl(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }
__device__ __forceinline__ int64_t rfl(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v), hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// pho: the photon passes take the step index from step_now (set by the
// prologue), the lepton passes from step (they run on the stream of the field
// scan that advances it)
__device__ __forceinline__ KC load_kc(const Ctx& cx, int tile, bool pho) {
  KC k;
  tile = rfl(tile);
  const Tile tl = cx.tiles[tile];
  const Tube& T = cx.tubes[rfl(tl.tube)];
  k.tile = tile;
  k.tube = rfl(tl.tube);
  k.base = rfl(tl.base);
  k.N = rfl(T.N);
  k.node_off = rfl(T.node_off);
  k.flags = rfl(T.flags);
  k.nsub_max = rfl(T.nsub_max);
  k.dpho = rfl(T.dpho);
  k.step = rfl(pho ? (int64_t)T.step_now : (int64_t)T.step);
  k.hfix = rfl((int64_t)T.hfix);
  k.xlo = -((int64_t)k.base << FRAC);
  k.xhi = min(k.hfix - ((int64_t)k.base << FRAC), (int64_t)(k.N - k.base) << FRAC);
  k.dt = rfl(T.dt);
  k.lr = rfl(T.lr);
  k.inv_rc = rfl(T.inv_rc);
  k.b = rfl(T.b);
  k.xc_floor = rfl(T.xc_floor);
  k.x_thr = rfl(T.x_thr);
  k.emit_k = rfl(T.emit_k);
  k.conv_k = rfl(T.conv_k);
  k.cfl24 = rfl(T.cfl24);
  k.chi_skip = rfl(T.chi_skip);
  k.seed = (uint64_t)rfl((int64_t)T.seed);
  return k;
}

// The same constants for a lane's own tile (tail chunks: not uniform).
__device__ __forceinline__ KC lane_kc(const Ctx& cx, int tile, bool pho) {
  KC k;
  const Tile tl = cx.tiles[tile];
  const Tube& T = cx.tubes[tl.tube];
  k.tile = tile; k.tube = tl.tube; k.base = tl.base; k.N = T.N; k.node_off = T.node_off; k.flags = T.flags;
  k.nsub_max = T.nsub_max; k.dpho = T.dpho; k.step = pho ? T.step_now : T.step; k.hfix = T.hfix; k.dt = T.dt; k.lr = T.lr;
  k.xlo = -((int64_t)k.base << FRAC);
  k.xhi = min(k.hfix - ((int64_t)k.base << FRAC), (int64_t)(k.N - k.base) << FRAC);
  k.inv_rc = T.inv_rc; k.b = T.b; k.xc_floor = T.xc_floor; k.x_thr = T.x_thr; k.emit_k = T.emit_k;
  k.conv_k = T.conv_k; k.cfl24 = T.cfl24; k.chi_skip = T.chi_skip; k.seed = T.seed;
  return k;
}

// Small-argument forms used on the hot path (relative error < 1e-12 where
// they are selected, far below FP32 rounding).
// The rare branches are taken only by waves that have a lane needing them
// (a wave-uniform test), so the common path runs without exec-mask changes.
__device__ __forceinline__ float one_minus_exp_neg(float x) {   // 1 - exp(-x), x >= 0
  // Taylor series to x^7 up to 1/8 (truncation x^8/8! < 1.2e-11 relative)
  float r = x * (1.0f - 0.5f * x * (1.0f - (1.0f / 3.0f) * x * (1.0f - 0.25f * x * (1.0f - 0.2f * x *
            (1.0f - (1.0f / 6.0f) * x * (1.0f - (1.0f / 7.0f) * x))))));
  const bool big = x > 0.125f;
  if (__ballot(big)) {
    if (big) r = -expm1f(-x);
  }
  return r;
}

// Energy of an emitted photon from the Philox word rb: classical x = xi x_c
// (reading of the spectrum S), or with F_QUANTUM the quantum spectrum's
// energy fraction at the emitter's chi times its gamma (Sect. 3.1: the mean
// of this spectrum carries the Gaunt factor g_Q of P_syn into the recoil).
// gamma and chi are formed from the post-kick momentum with explicit
// roundings, so that the evaluation and the photon birth agree bit for bit.
// Q: the kernels are built for handles with quantum tubes (the branch is
// compiled out of the classical kernels, whose registers it would cost).
template <bool Q>
__device__ __forceinline__ float photon_energy(const Ctx& cx, uint32_t flags, uint32_t rb, float xc, float up,
                                               float lr) {
  if (Q && (flags & F_QUANTUM)) {
    const float g = __builtin_amdgcn_sqrtf(__fmaf_rn(up, up, 1.0f));
    return __fmul_rn(qsyn_fraction(__fmul_rn(__fmul_rn(g, g), lr), rb, cx.qs), g);
  }
  return sync_sample(unif(rb), cx.tab) * xc;
}

// Momenta of the pair a photon of energy |x| along dir creates: halves
// (reading of the split), or with F_QUANTUM the electron takes the fraction
// v of the quantum pair spectrum at the photon's chi (Sect. 3.2).
template <bool Q>
__device__ __forceinline__ void pair_momenta(const Ctx& cx, uint32_t flags, uint32_t rb, float chi, float x,
                                             float* ue, float* up) {
  const float dir = x >= 0.0f ? 1.0f : -1.0f;
  const float ax = fabsf(x);
  float ge = 0.5f * ax, gp = ge;
  if (Q && (flags & F_QUANTUM)) {
    const float v = qbw_fraction(chi, rb, cx.qb);
    ge = v * ax;
    gp = (1.0f - v) * ax;
  }
  *ue = dir * sqrtf(fmaxf(ge * ge - 1.0f, 0.0f));
  *up = dir * sqrtf(fmaxf(gp * gp - 1.0f, 0.0f));
}

// gamma, chi = gamma^2 lambda~/R~ and the characteristic photon energy
// x_c = 1.5 gamma chi of a lepton of momentum u, with explicit roundings: the
// emission evaluation and the photon births (which may run in another
// kernel) form them identically.
__device__ __forceinline__ float emit_xc(float u, float lr, float* g, float* chi) {
  *g = __builtin_amdgcn_sqrtf(__fmaf_rn(u, u, 1.0f));
  *chi = __fmul_rn(__fmul_rn(*g, *g), lr);
  return __fmul_rn(__fmul_rn(1.5f, *g), *chi);
}

// Birth queue of the sorted lepton pass.  Photon births take tail slots of
// the photon store, and the tail counter is one word that every reservation
// updates with a device-scope atomic; such atomics on one address are
// served one at a time, and in a cascade (hundreds of thousands of births
// per step) one reservation per wave and birth iteration made them the
// largest cost of the pass.  The birth code also held registers that the
// rest of the pass needs.  So the sorted pass only queues, per lepton with
// photons to store, its slot, its post-kick momentum and its event mask; the
// tail launch replays the events and writes the photons, one reservation per
// dense wave.  Workgroup b of the pass writes its entries from the first
// slot of its chunk range on (it has at most one entry per slot it pushes),
// counted in LDS, and their number and start to bq_count[b], bq_start[b].
__device__ __forceinline__ void queue_births(const Ctx& cx, int* s_bqn, long long seg0, bool has, uint32_t slot,
                                             float upk, uint64_t evmask) {
  const uint64_t m = __ballot(has);
  int base = 0;
  if (lane_id() == 0) base = atomicAdd(s_bqn, __popcll(m));
  base = __builtin_amdgcn_readfirstlane(base);
  if (has) cx.bq[seg0 + base + rank_in(m)] = make_uint4(slot, __float_as_uint(upk), (uint32_t)evmask,
                                                         (uint32_t)(evmask >> 32));
}

// One lepton: gather, kick, emission (Monte Carlo with recoil), drift,
// boundaries, deposit, photon births.  UNI: the lane's tile is the
// wave-uniform tile of a sorted chunk (tube constants come through scalar
// loads, gather and deposit go through the LDS window); otherwise the lane's
// own tile (tail) with global memory.  `tile` < 0: no particle in this lane.
template <bool UNI, bool Q, bool A>
__device__ void lepton_one(const Ctx& cx, uint32_t slot, int tile, const KC& ku, long long* s_rho, const float* s_eb,
                           LocalCounts& lcn, float w, uint32_t pos, float u, uint32_t* pos_out, float* u_out,
                           const Room& proom, int* s_bqn, long long seg0) {
  bool alive;
  KC k;
  if (UNI) {
    k = ku;
    alive = w != 0.0f;
  } else {
    alive = tile >= 0 && w != 0.0f;
    k = lane_kc(cx, alive ? tile : 0, false);   // tile 0 always exists; no branch on the struct
  }
  if (!alive) { pos = 0; u = 0.0f; }
  const int tube = alive ? k.tube : -1;
  const int N = k.N;
  const uint32_t flags = (uint32_t)k.flags;
  const bool per = (flags & F_PERIODIC) != 0;
  const int64_t step = k.step;
  struct { int base; } tl{k.base};

  // gather (node field, first-order shape) and kick
  const int off = (int)(pos >> FRAC);
  const int cell = tl.base + off;
  const uint32_t frac = pos & 0xFFFFFFu;
  const int cg = per ? wrap_cell(cell, N) : cell;
  const float xi = (float)frac * 5.9604645e-8f;
  float e0 = 0.0f, e1 = 0.0f;
  if (alive) {
    if (UNI) { e0 = s_eb[off]; e1 = s_eb[off + 1]; }
    else { e0 = cx.ebar[k.node_off + cg]; e1 = cx.ebar[k.node_off + cg + 1]; }
  }
  const float sg = w < 0.0f ? -1.0f : 1.0f;
  u += sg * ((1.0f - xi) * e0 + xi * e1) * k.dt;

  // curvature emission: rate alpha_em gamma/R~ T_syn(chi), chi = gamma^2 lambda~/R~,
  // photon energy xi_s x_c with x_c = 1.5 gamma chi, QED zone h < H
  const float upk = u;
  uint64_t evmask = 0;
  uint64_t id = 0;
  float xc = 0.0f;
  int ncand = 0, nev = 0;
  bool eval = false;
  if (alive && !(flags & (F_QED_OFF | F_EMIT_OFF)) && ((int64_t)cg << FRAC) + frac < k.hfix) {
    float g, chi;
    xc = emit_xc(u, k.lr, &g, &chi);
    if (xc >= k.xc_floor) {
      eval = true;
      id = cx.L.id[slot];
      const float dtau = k.emit_k * g * t_syn(chi);
      int nsub = (int)ceilf(dtau * 10.0f);
      nsub = max(1, min(nsub, k.nsub_max));
      const float p = one_minus_exp_neg(dtau / (float)nsub);
      float au = fabsf(u);
      for (int j = 0; j < nsub; ++j) {
        u4 r = draw(k.seed, id, step, T_EMIT, (uint32_t)j);
        if (bern(r.a, p)) {
          float x = fminf(photon_energy<Q>(cx, flags, r.b, xc, upk, k.lr), au);
          au -= x;
          evmask |= 1ull << j;
          ++nev;
          if (x >= k.x_thr || (flags & F_TRACK_ALL)) ++ncand;
        }
      }
      if (!(flags & F_RECOIL_OFF)) u = copysignf(au, upk);
    }
  }

  // drift: dh/dt = u / gamma, in fixed point
  const int dfix = __float2int_rn(u * __builtin_amdgcn_rsqf(1.0f + u * u) * k.cfl24);
  const long long npl = (long long)pos + dfix;
  const int noff = (int)(npl >> FRAC);
  const uint32_t nfrac = (uint32_t)npl & 0xFFFFFFu;
  bool dead = false;
  const int ncell = tl.base + noff;
  if (alive && (npl < 0 || noff >= WIN)) { atomicOr(cx.err, E_TILE); dead = true; }
  const int64_t Tw = alive ? __float2ll_rn(fabsf(w) * 16777216.0f) : 0;
  bool absorbed = false, outflow = false;
  if (alive && !dead && !per) {
    if (ncell < 0) { absorbed = true; dead = true; }
    else if (ncell >= N) { outflow = true; dead = true; }
  }
  if (alive && dead) cx.L.w[slot] = 0.0f;
  if (UNI) {           // the caller stores the chunk's records with vector stores
    *pos_out = (uint32_t)npl;
    *u_out = u;
  } else if (alive && !dead) {
    cx.L.pos[slot] = (uint32_t)npl;
    cx.L.u[slot] = u;
  }
  if (absorbed) {
    atomic_add_i64(&cx.tubes[tube].dq, sg > 0 ? Tw : -Tw);
    return_add(cx.ret, cx.ret_thr, tube, u, w);
  }
  if (per && alive && !dead) atomic_add_i64(&cx.tubes[tube].dcur, (sg > 0 ? Tw : -Tw) * (int64_t)dfix);

  // deposit at the new position: node k gets s (T - A), node k+1 gets s A,
  // A = round(T xi) (half up), exact integers
  const int ncg = per ? wrap_cell(ncell, N) : ncell;
  // electrons left in cell 0 by this push refill the atmosphere next step
  if (A && alive && !dead && sg < 0.0f && ncg == 0) atomicAdd(&cx.tubes[tube].atm_cnt[step & 1], 1);
  if (alive && !dead) {
    const unsigned long long Au = ((unsigned long long)Tw * nfrac + (1ull << 23)) >> FRAC;
    const long long a = sg > 0 ? (long long)Au : -(long long)Au;
    const long long ta = sg > 0 ? (long long)(Tw - (int64_t)Au) : -(long long)(Tw - (int64_t)Au);
    if (UNI) {
      atomicAdd((unsigned long long*)&s_rho[noff], (unsigned long long)ta);
      atomicAdd((unsigned long long*)&s_rho[noff + 1], (unsigned long long)a);
    } else {
      int n1 = ncg + 1;
      if (per && n1 == N) n1 = 0;
      atomicAdd((unsigned long long*)&cx.rho[k.node_off + ncg], (unsigned long long)ta);
      atomicAdd((unsigned long long*)&cx.rho[k.node_off + n1], (unsigned long long)a);
    }
  }

  // photon births at the post-drift position, inside the QED zone
  const bool keep = alive && !dead && (((int64_t)ncg << FRAC) + nfrac < k.hfix);
  const int nst = keep ? ncand : 0;
  if (UNI) {
    if (__ballot(nst > 0)) queue_births(cx, s_bqn, seg0, nst > 0, slot, upk, evmask);
  } else if (__ballot(nst > 0)) {
    int dropped = 0;
    const long long first = reserve_tail(cx.pc, proom, nst, &dropped);
    const long long lim = proom.L;
    if (nst > 0) {
      float au = fabsf(upk);
      const float dir = upk >= 0.0f ? 1.0f : -1.0f;
      const float aw = fabsf(w);
      long long q = first;
      uint64_t m = evmask;
      while (m) {
        const int j = __ffsll((long long)m) - 1;
        m &= m - 1;
        u4 r = draw(k.seed, id, step, T_EMIT, (uint32_t)j);
        float x = fminf(photon_energy<Q>(cx, flags, r.b, xc, upk, k.lr), au);
        au -= x;
        if (x >= k.x_thr || (flags & F_TRACK_ALL)) {
          if (q < lim) {
            const uint32_t kk = (uint32_t)q;
            cx.P.pos[kk] = (uint32_t)npl;
            cx.P.x[kk] = dir * x;
            cx.P.w[kk] = aw;
            cx.P.n0[kk] = (int32_t)(step + 1);
            cx.P.id[kk] = child_id(k.seed, id, step, 2u + (uint32_t)j);
            cx.ptt[kk] = tile;
          }
          ++q;
        }
      }
    }
    if (dropped) atomicOr(cx.err, E_CAP);
    lcn.v[3] += nst - dropped;
    lcn.v[4] += dropped;
  }

  // event counts: sorted chunks accumulate per thread (flushed per
  // workgroup); tail lanes may belong to different tubes
  lcn.v[0] += alive ? 1 : 0;
  lcn.v[1] += eval ? 1 : 0;
  lcn.v[2] += nev;
  lcn.v[5] += absorbed ? 1 : 0;
  lcn.v[6] += outflow ? 1 : 0;
  if (!UNI) {
#pragma unroll
    for (int i = 0; i < 7; ++i) {
      const int v = lcn.v[i];
      if (__ballot(v != 0)) count_by_tube(cx.shard, v != 0 ? tube : -1, cnt_index<2>(i), v);
    }
    lcn.clear();
  }
}

// Node field of a tile window into LDS (nodes base .. base + WIN).
__device__ void load_window(const Ctx& cx, int tile, float* s_eb) {
  const Tile tl = cx.tiles[tile];
  const Tube& T = cx.tubes[tl.tube];
  const bool per = (T.flags & F_PERIODIC) != 0;
  for (int j = threadIdx.x; j <= WIN; j += blockDim.x) {
    int node = tl.base + j;
    float v = 0.0f;
    if (per) v = cx.ebar[T.node_off + wrap_cell(node, T.N)];
    else if (node >= 0 && node <= T.N) v = cx.ebar[T.node_off + node];
    s_eb[j] = v;
  }
  __syncthreads();
}

// Records of VEC consecutive slots of a sorted chunk (one thread).
struct Lep4 { float4 w; uint4 pos; float4 u; int tile; uint32_t slot0; };

__device__ __forceinline__ Lep4 lep_load4(const Ctx& cx, long long c) {
  Lep4 r;
  r.slot0 = (uint32_t)c * CHUNK + VEC * threadIdx.x;
  r.tile = cx.lchunk[c];
  r.w = *reinterpret_cast<const float4*>(cx.L.w + r.slot0);
  r.pos = *reinterpret_cast<const uint4*>(cx.L.pos + r.slot0);
  r.u = *reinterpret_cast<const float4*>(cx.L.u + r.slot0);
  return r;
}

// Slot and tile of 256-slot piece q (sorted pieces first, then the tail).
__device__ __forceinline__ void piece_slot(long long q, long long nsq, long long S, long long tail, const int32_t* chunk,
                                           const int32_t* tt, uint32_t* slot, int* tile) {
  if (q < nsq) {
    *slot = (uint32_t)(q * TPB) + threadIdx.x;
    *tile = chunk[q / PPC];
  } else {
    *slot = (uint32_t)(S + (q - nsq) * TPB) + threadIdx.x;
    const int t = tt[*slot];            // in bounds: the store keeps a chunk of slack
    *tile = *slot < S + tail ? t : -1;
  }
}

// Lepton pass over the sorted region.  Each workgroup takes a contiguous
// range of chunks (XCD-aware: consecutive ranges go to the same XCD); each
// thread pushes VEC consecutive slots loaded and stored as 16-byte vectors,
// and the next chunk's records are prefetched while the current one is
// pushed.  The chunk's tile constants sit in scalar registers; gather and
// deposit go through an LDS window of the tile.
// (six waves per SIMD: the register cap spills one value, stored once on
// entry and reloaded once per chunk)
template <bool Q, bool A>
__global__ __launch_bounds__(TPB, 6) void k_leptons(Ctx cx) {
  const Room proom = load_room(cx.pc);
  __shared__ long long s_rho[WIN + 2];
  __shared__ float s_eb[WIN + 2];
  __shared__ long long s_cnt[8];
  LocalCounts lcn;
  lcn.clear();
  __shared__ int s_bqn;        // photon births queued by this workgroup
  int ctube = -1;
  for (int j = threadIdx.x; j < WIN + 2; j += blockDim.x) s_rho[j] = 0;
  if (threadIdx.x == 0) s_bqn = 0;
  __syncthreads();
  const long long nsc = cx.lc->n_sorted_chunks;
  const int G = gridDim.x, bx = blockIdx.x;
  const int r = (bx & 7) * (G >> 3) + (bx >> 3);
  const long long c0 = nsc * r / G, c1 = nsc * (r + 1) / G;
  int held = -1;
  KC kc;
  Lep4 cur;
  if (c0 < c1) cur = lep_load4(cx, c0);
  for (long long c = c0; c < c1; ++c) {
    Lep4 nxt;
    if (c + 1 < c1) nxt = lep_load4(cx, c + 1);
    const int tile = cur.tile;
    if (tile != held) {
      if (held >= 0) flush_window(cx, held, s_rho);
      held = tile;
      kc = load_kc(cx, tile, false);
      if (kc.tube != ctube) {
        if (ctube >= 0) flush_counts<0>(cx.shard, ctube, lcn, s_cnt);
        ctube = kc.tube;
      }
      load_window(cx, tile, s_eb);
    }
    float4 w = cur.w, u = cur.u;
    uint4 p = cur.pos;
    // one body, four records: process .x, write the result into .x, rotate
#pragma unroll 1
    for (int j = 0; j < VEC; ++j) {
      uint32_t po;
      float uo;
      lepton_one<true, Q, A>(cx, cur.slot0 + j, tile, kc, s_rho, s_eb, lcn, w.x, p.x, u.x, &po, &uo, proom, &s_bqn, c0 * CHUNK);
      w = make_float4(w.y, w.z, w.w, w.x);
      p = make_uint4(p.y, p.z, p.w, po);
      u = make_float4(u.y, u.z, u.w, uo);
    }
    *reinterpret_cast<uint4*>(cx.L.pos + cur.slot0) = p;
    *reinterpret_cast<float4*>(cx.L.u + cur.slot0) = u;
    cur = nxt;
  }
  if (held >= 0) flush_window(cx, held, s_rho);
  if (ctube >= 0) flush_counts<0>(cx.shard, ctube, lcn, s_cnt);
  // (flush_counts ends with a barrier: every wave has queued its births)
  if (threadIdx.x == 0) {
    cx.bq_count[blockIdx.x] = c0 < c1 ? s_bqn : 0;
    cx.bq_start[blockIdx.x] = c0 * CHUNK;
  }
}

// Lepton pass over the tail (particles appended since the last re-sort):
// one slot per thread, each lane with its own tile; global gather/deposit.
template <bool Q, bool A>
__device__ __forceinline__ void leptons_tail(const Ctx& cx, int bid, int nblk) {
  const Room proom = load_room(cx.pc);
  LocalCounts lcn;
  lcn.clear();
  const long long nsc = cx.lc->n_sorted_chunks;
  const long long S = nsc * CHUNK;
  const long long tail = cx.lc->tail_snap;
  const long long nq = (tail + TPB - 1) / TPB;
  const KC kc0 = load_kc(cx, 0, false);
  for (long long q = bid; q < nq; q += nblk) {
    uint32_t slot;
    int tile;
    piece_slot(S / TPB + q, S / TPB, S, tail, cx.lchunk, cx.ltt, &slot, &tile);
    const float w = cx.L.w[slot];
    const uint32_t pos = cx.L.pos[slot];
    const float u = cx.L.u[slot];
    lepton_one<false, Q, A>(cx, slot, tile, kc0, nullptr, nullptr, lcn, w, pos, u, nullptr, nullptr, proom, nullptr, 0);
  }
}

// ------------------------------------------------------------------ photons
// sin(a) for the accumulated angle; a power series where |a| < 0.05
// (truncation a^7/5040 < 2e-13 relative).
__device__ __forceinline__ float sin_small(float a) {
  const float a2 = a * a;
  float s = a * (1.0f - a2 * (1.0f / 6.0f) * (1.0f - a2 * (1.0f / 20.0f)));
  const bool big = !(fabsf(a) < 0.05f);
  if (__ballot(big)) {
    if (big) s = sinf(a);
  }
  return s;
}

// Conversion probability of a photon in this step: rate alpha_em (b/lambda~)
// sin(psi) T_BW(x b sin psi), sin(psi) = |sin(s/R~)| with s the path since
// birth.  Below chi_skip the fit gives p < 2^-27, under every 24-bit uniform:
// 0 is returned and no draw is made.  The age is taken in 32 bits, wrapping
// like the stored 32-bit birth step.
__device__ __forceinline__ float photon_chi(int64_t step, float dt, float inv_rc, float b, float x, int32_t n0,
                                            float* sp_out) {
  const int32_t age = (int32_t)((uint32_t)step + 1u - (uint32_t)n0);
  const float sp = fabsf(sin_small((float)age * dt * inv_rc));
  *sp_out = sp;
  return fabsf(x) * b * sp;
}
__device__ __forceinline__ float photon_prob(const KC& k, float x, int32_t n0) {
  float sp;
  const float chi = photon_chi(k.step, k.dt, k.inv_rc, k.b, x, n0, &sp);
  const float p = one_minus_exp_neg(k.conv_k * sp * t_bw(chi));
  return chi > k.chi_skip ? p : 0.0f;
}

// One photon: free streaming at c, exit above H, conversion with
// rate alpha_em (b/lambda~) sin(psi) T_BW(x b sin psi), sin(psi) = |sin(s/R~)|.
// Below chi_skip the fit gives p < 2^-27, under every 24-bit uniform: no
// draw is needed and none is made.
template <bool UNI, bool Q>
__device__ void photon_one(const Ctx& cx, uint32_t slot, int tile, const KC& ku, LocalCounts& lcn, float x, uint32_t pos,
                           int32_t n0, uint32_t* pos_out, float* x_out, const Room& lroom) {
  bool alive;
  KC k;
  if (UNI) {
    k = ku;
    alive = x != 0.0f;
  } else {
    alive = tile >= 0 && x != 0.0f;
    k = lane_kc(cx, alive ? tile : 0, true);
  }
  if (!alive) { x = 0.0f; pos = 0; n0 = 0; }
  const int tube = alive ? k.tube : -1;
  const int N = k.N;
  const uint32_t flags = (uint32_t)k.flags;
  const bool per = (flags & F_PERIODIC) != 0;
  const int64_t step = k.step;
  struct { int base; } tl{k.base};
  const float dir = x >= 0.0f ? 1.0f : -1.0f;
  const long long np = (long long)pos + (x >= 0.0f ? k.dpho : -k.dpho);
  const int noff = (int)(np >> FRAC);
  const uint32_t nfrac = (uint32_t)np & 0xFFFFFFu;
  const int ncell = tl.base + noff;
  bool dead = false;
  if (alive && (np < 0 || noff >= WIN)) { atomicOr(cx.err, E_TILE); dead = true; }
  const int ncg = per ? wrap_cell(ncell, N) : ncell;
  bool exited = false;
  if (alive && !dead) {
    if ((!per && (ncell < 0 || ncell >= N)) || (((int64_t)ncg << FRAC) + nfrac >= k.hfix)) { exited = true; dead = true; }
  }
  bool eval = false, conv = false;
  float w = 0.0f;
  uint64_t id = 0;
  uint32_t rsplit = 0;
  if (alive && !dead && !(flags & (F_QED_OFF | F_CONV_OFF))) {
    const float p = photon_prob(k, x, n0);
    if (p > 2.9802322e-8f) {   // below 2^-25 no 24-bit uniform can fall under p
      eval = true;
      id = cx.P.id[slot];
      u4 r = draw<true>(k.seed, id, step, T_CONV, 0);
      conv = bern(r.a, p);
      if (conv) w = cx.P.w[slot];
      rsplit = r.b;
    }
  }
  if (UNI) {           // the caller stores the chunk's records with vector stores
    *pos_out = (uint32_t)np;
    *x_out = (dead || conv) ? 0.0f : x;
  } else if (alive) {
    if (dead || conv) cx.P.x[slot] = 0.0f;
    else cx.P.pos[slot] = (uint32_t)np;
  }
  // pair births: e- and e+ at the photon position, gamma = x/2 each, along the photon
  if (__ballot(conv)) {
    int dropped = 0;
    const long long first = reserve_tail(cx.lc, lroom, conv ? 2 : 0, &dropped);
    const long long lim = lroom.L;
    if (conv) {
      float chi = 0.0f, sp;
      if (Q && (flags & F_QUANTUM)) chi = photon_chi(step, k.dt, k.inv_rc, k.b, x, n0, &sp);
      float ue, upo;
      pair_momenta<Q>(cx, flags, rsplit, chi, x, &ue, &upo);
      for (int e = 0; e < 2; ++e) {
        const long long sl = first + e;
        if (sl < lim) {
          const uint32_t s32 = (uint32_t)sl;
          cx.L.pos[s32] = (uint32_t)np;
          cx.L.u[s32] = e == 0 ? ue : upo;
          cx.L.w[s32] = e == 0 ? -w : w;
          cx.L.id[s32] = child_id(k.seed, id, step, (uint32_t)e);
          cx.ltt[s32] = tile;
        }
      }
    }
    if (dropped) atomicOr(cx.err, E_CAP);
    lcn.v[3] += dropped;
  }
  lcn.v[0] += alive ? 1 : 0;
  lcn.v[1] += eval ? 1 : 0;
  lcn.v[2] += conv ? 1 : 0;
  lcn.v[4] += exited ? 1 : 0;
  if (!UNI) {
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      const int v = lcn.v[i];
      if (__ballot(v != 0)) count_by_tube(cx.shard, v != 0 ? tube : -1, cnt_index<3>(i), v);
    }
    lcn.clear();
  }
}

struct Pho4 { float4 x; uint4 pos; int4 n0; int tile; int hot; uint32_t slot0; };

// One chunk's records for this thread.  hot: the chunk's leading slots that
// may draw (all of them without the re-sort's guarantee); a chunk with none
// does not need the birth steps.
__device__ __forceinline__ Pho4 pho_load4(const Ctx& cx, long long c, bool cold_ok) {
  Pho4 r;
  r.slot0 = (uint32_t)c * CHUNK + VEC * threadIdx.x;
  r.tile = cx.pchunk[c];
  r.hot = cold_ok ? (int)cx.pchot[c] : CHUNK;
  r.x = *reinterpret_cast<const float4*>(cx.P.x + r.slot0);
  r.pos = *reinterpret_cast<const uint4*>(cx.P.pos + r.slot0);
  r.n0 = r.hot > 0 ? *reinterpret_cast<const int4*>(cx.P.n0 + r.slot0) : make_int4(0, 0, 0, 0);
  return r;
}

// Sorted photon pass, first half for one photon: free streaming, exit, and
// the conversion probability.  Gives the new position, the energy (0 once
// the photon has left) and whether a conversion draw is due.
__device__ __forceinline__ void photon_move(const Ctx& cx, const KC& k, float x, uint32_t pos, int32_t n0, bool may_draw,
                                            LocalCounts& lcn, uint32_t* pos_out, float* x_out, float* p_out,
                                            bool* eval_out) {
  const bool alive = x != 0.0f;
  const uint32_t flags = (uint32_t)k.flags;
  const bool per = (flags & F_PERIODIC) != 0;
  // new tile-local position; leaving the 256-cell window (a tile error) is
  // the 32-bit add or subtract wrapping around
  const uint32_t d = (uint32_t)k.dpho;
  const uint32_t np = x >= 0.0f ? pos + d : pos - d;
  const bool fwd = x >= 0.0f;
  const bool oob = alive & ((fwd & (np < pos)) | (!fwd & (pos < d)));   // (no short-circuit: no branches)
  if (__ballot(oob)) {
    if (oob) atomicOr(cx.err, E_TILE);
  }
  bool out;
  if (per) {
    const int ncg = wrap_cell(k.base + (int)(np >> FRAC), k.N);
    out = ((int64_t)ncg << FRAC) + (np & 0xFFFFFFu) >= k.hfix;
  } else {
    out = ((int64_t)np < k.xlo) | ((int64_t)np >= k.xhi);
  }
  const bool exited = alive & !oob & out;
  const bool dead = oob | exited;
  // the probability is taken for every lane of a wave in which one may draw
  // (0 for an empty slot: chi = 0) and kept for the live ones; a slot that
  // cannot draw would get p <= 2^-25 and no draw
  const float pr = __ballot(may_draw) ? photon_prob(k, x, n0) : 0.0f;
  const float p = (alive & !dead & !(flags & (F_QED_OFF | F_CONV_OFF))) ? pr : 0.0f;
  const bool eval = p > 2.9802322e-8f;   // below 2^-25 no 24-bit uniform can fall under p
  *pos_out = np;
  *x_out = dead ? 0.0f : x;
  *p_out = p;
  *eval_out = eval;
  lcn.v[0] += alive ? 1 : 0;
  lcn.v[1] += eval ? 1 : 0;
  lcn.v[4] += exited ? 1 : 0;
}

// First chunk of the range of workgroup `bx` of a grid of G over nsc chunks
// (XCD-aware: consecutive ranges go to workgroups of the same XCD).
__device__ __forceinline__ void chunk_range(long long nsc, int G, int bx, long long* c0, long long* c1) {
  const int r = (bx & 7) * (G >> 3) + (bx >> 3);
  *c0 = nsc * r / G;
  *c1 = nsc * (r + 1) / G;
}

// Photon pass over the sorted region, first kernel: free streaming, exits
// and the conversion probability of every photon (a range of chunks per
// workgroup, VEC slots per thread, the next chunk prefetched).  Only a tenth
// or so of the photons must draw; they are queued, with their probability,
// in the workgroup's own segment of the conversion queue (at most one entry
// per slot of its range, so the segment cannot overflow), and the
// conversion kernel works through the queue.  No barrier stands between
// chunks.
__global__ __launch_bounds__(TPB) void k_photons(Ctx cx) {
  long long c0, c1;
  chunk_range(cx.pc->n_sorted_chunks, gridDim.x, blockIdx.x, &c0, &c1);
  __shared__ long long s_cnt[8];
  __shared__ int q_n;
  if (threadIdx.x == 0) q_n = 0;
  __syncthreads();
  uint4* const q = cx.pq + c0 * CHUNK;
  LocalCounts lcn;
  lcn.clear();
  int ctube = -1;
  KC kc;
  int held = -1;
  const bool cold_ok = cx.pc->cold_steps >= 0;
  Pho4 cur;
  if (c0 < c1) cur = pho_load4(cx, c0, cold_ok);
  for (long long c = c0; c < c1; ++c) {
    Pho4 nxt;
    if (c + 1 < c1) nxt = pho_load4(cx, c + 1, cold_ok);
    if (cur.tile != held) {
      held = cur.tile;
      kc = load_kc(cx, held, true);
      if (kc.tube != ctube) {
        if (ctube >= 0) flush_counts<1>(cx.shard, ctube, lcn, s_cnt);
        ctube = kc.tube;
      }
    }
    float4 x = cur.x;
    bool xchg = false;
    uint4 p = cur.pos;
    int4 n0 = cur.n0;
#pragma unroll 1
    for (int j = 0; j < VEC; ++j) {
      uint32_t po;
      float xo, pr;
      bool ev;
      photon_move(cx, kc, x.x, p.x, n0.x, (int)(VEC * threadIdx.x) + j < cur.hot, lcn, &po, &xo, &pr, &ev);
      xchg |= xo != x.x;
      const uint64_t m = __ballot(ev);
      if (m) {
        int base = 0;
        if (lane_id() == 0) base = atomicAdd(&q_n, (int)__popcll(m));
        base = __shfl(base, 0);
        if (ev) q[base + rank_in(m)] = make_uint4(cur.slot0 + j, __float_as_uint(pr), (uint32_t)held, (uint32_t)kc.tube);
      }
      x = make_float4(x.y, x.z, x.w, xo);
      p = make_uint4(p.y, p.z, p.w, po);
      n0 = make_int4(n0.y, n0.z, n0.w, n0.x);
    }
    *reinterpret_cast<uint4*>(cx.P.pos + cur.slot0) = p;
    if (xchg) *reinterpret_cast<float4*>(cx.P.x + cur.slot0) = x;   // only when a photon left
    cur = nxt;
  }
  if (ctube >= 0) flush_counts<1>(cx.shard, ctube, lcn, s_cnt);
  __syncthreads();
  if (threadIdx.x == 0) cx.pq_count[blockIdx.x] = q_n;
}

// Photon pass, second kernel: the conversion draws of the queued photons and
// the pairs they create: e- and e+ at the photon's new position, gamma = x/2
// each, moving along the photon; the converted photon is removed.
// The queue segment that workgroup k of the photon kernel (a grid of nseg)
// wrote is cut into `split` parts by rounds of TPB entries (part p takes
// rounds p, p + split, ...), so that the number of parts can fill the chip
// whatever the photon grid; workgroup b takes parts CONV_SEGS b .. CONV_SEGS
// b + CONV_SEGS - 1, one entry of each per thread and round, with all loads
// issued before the draws.  (With the segment as the unit, a photon grid of
// 768 left 384 workgroups to walk 4e7 entries, 1.7 ms per step.)
constexpr int CONV_SEGS = 2;
//
// The pairs take lepton tail slots from a block per wave (LDS state, one
// entry per wave): a new block is reserved with one atomic on the lepton
// tail counter only when the block cannot hold the iteration's pairs, which
// then fill the old block and continue in the new one.  The first block
// holds exactly the wave's first pairs; each later one is at least twice the
// last, up to PAIR_BLOCK_MAX.  The unused end of a wave's last block is
// written as dead leptons (weight 0, tile 0), which every pass skips and the
// re-sort drops.  (One atomic per wave and conversion iteration, on the one
// counter every reservation updates, cost a cascade of 1e5 conversions per
// step about a millisecond.)
constexpr int PAIR_BLOCK_MAX = 128;

template <bool Q>
__global__ __launch_bounds__(TPB) void k_conversions(Ctx cx, int nseg, int split) {
  const Room lroom = load_room(cx.lc);
  const long long nsc = cx.pc->n_sorted_chunks;
  __shared__ long long s_blk[TPB / WAVE][3];    // per wave: next slot, block end, next block size
  long long* blk = s_blk[threadIdx.x / WAVE];
  if (lane_id() == 0) { blk[0] = 0; blk[1] = 0; blk[2] = 2; }
  long long q0[CONV_SEGS];
  int n[CONV_SEGS];
  int nmax = 0;
#pragma unroll
  for (int j = 0; j < CONV_SEGS; ++j) {
    const int v = (int)blockIdx.x * CONV_SEGS + j;
    const int sg = v / split;
    long long c0 = 0, c1 = 0;
    n[j] = 0;
    if (sg < nseg) {
      chunk_range(nsc, nseg, sg, &c0, &c1);
      n[j] = __builtin_amdgcn_readfirstlane(cx.pq_count[sg]);
    }
    // rounds part, part + split, ... of the segment
    const int part = v - sg * split;
    q0[j] = c0 * CHUNK + (long long)part * TPB;
    n[j] -= part * TPB;
    nmax = max(nmax, n[j]);
  }
  const int stride = split * TPB;
  for (int i0 = 0; i0 < nmax; i0 += stride) {
    const int i = i0 + (int)threadIdx.x;
    uint4 e[CONV_SEGS];
    uint64_t id[CONV_SEGS], seed[CONV_SEGS];
    int64_t step[CONV_SEGS];
    bool act[CONV_SEGS];
#pragma unroll
    for (int j = 0; j < CONV_SEGS; ++j) {
      act[j] = i < n[j];
      e[j] = act[j] ? cx.pq[q0[j] + i] : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < CONV_SEGS; ++j) {
      id[j] = act[j] ? cx.P.id[e[j].x] : 0;
      seed[j] = act[j] ? cx.tubes[e[j].w].seed : 0;
      step[j] = act[j] ? cx.tubes[e[j].w].step_now : 0;
    }
#pragma unroll
    for (int j = 0; j < CONV_SEGS; ++j) {
      bool conv = false;
      uint32_t rsplit = 0;
      if (act[j]) {
        const u4 r = draw<true>(seed[j], id[j], step[j], T_CONV, 0);
        conv = bern(r.a, __uint_as_float(e[j].y));
        rsplit = r.b;
      }
      const uint64_t cm = __ballot(conv);
      if (cm) {
        const uint32_t slot = e[j].x;
        const int tube = conv ? (int)e[j].w : -1;
        // this lane's pair takes the wave's pair slots ex and ex + 1
        const long long total = 2 * __popcll(cm);
        const long long ex = 2 * rank_in(cm);
        const long long next = rfl64(blk[0]);
        const long long rem = rfl64(blk[1]) - next;
        long long nb = 0;
        if (total > rem) {
          const long long need = total - rem;
          const long long req = max(need, rfl64(blk[2]));
          long long base = 0;
          if (lane_id() == WAVE - 1) {
            base = (long long)atomicAdd((unsigned long long*)&cx.lc->tail, (unsigned long long)req);
            const long long room = lroom.L > lroom.S ? lroom.L - lroom.S : 0;
            if (base + req > room) atomicMin((unsigned long long*)&cx.lc->tail, (unsigned long long)room);
          }
          nb = lroom.S + rfl64(__shfl(base, WAVE - 1));
          if (lane_id() == 0) { blk[0] = nb + need; blk[1] = nb + req; blk[2] = min(2 * req, (long long)PAIR_BLOCK_MAX); }
        } else if (lane_id() == 0) {
          blk[0] = next + total;
        }
        int dropped = 0;
        if (conv) {
          const float x = cx.P.x[slot], w = cx.P.w[slot];
          const uint32_t np = cx.P.pos[slot];
          const Tube& T = cx.tubes[e[j].w];
          const uint32_t tflags = (uint32_t)T.flags;
          float chi = 0.0f, sp;
          if (Q && (tflags & F_QUANTUM)) chi = photon_chi(step[j], T.dt, T.inv_rc, T.b, x, cx.P.n0[slot], &sp);
          float ue, upo;
          pair_momenta<Q>(cx, tflags, rsplit, chi, x, &ue, &upo);
          for (int b = 0; b < 2; ++b) {
            const long long g = ex + b;
            const long long sl = g < rem ? next + g : nb + (g - rem);
            if (sl >= lroom.L) {
              ++dropped;
            } else {
              const uint32_t s32 = (uint32_t)sl;
              cx.L.pos[s32] = np;
              cx.L.u[s32] = b == 0 ? ue : upo;
              cx.L.w[s32] = b == 0 ? -w : w;
              cx.L.id[s32] = child_id(seed[j], id[j], step[j], (uint32_t)b);
              cx.ltt[s32] = (int32_t)e[j].z;
            }
          }
          cx.P.x[slot] = 0.0f;
        }
        if (dropped) atomicOr(cx.err, E_CAP);
        count_by_tube(cx.shard, tube, C_CONV, 1);
        if (__ballot(dropped != 0)) count_by_tube(cx.shard, dropped ? tube : -1, C_DROPPED, dropped);
      }
    }
  }
  // the unused end of the wave's last block: dead leptons
  const long long bend = min(rfl64(blk[1]), lroom.L);
  for (long long sl = rfl64(blk[0]) + lane_id(); sl < bend; sl += WAVE) {
    const uint32_t s32 = (uint32_t)sl;
    cx.L.pos[s32] = 0;
    cx.L.u[s32] = 0.0f;
    cx.L.w[s32] = 0.0f;
    cx.L.id[s32] = 0;
    cx.ltt[s32] = 0;
  }
}

template <bool Q>
__device__ __forceinline__ void photons_tail(const Ctx& cx, int bid, int nblk) {
  const Room lroom = load_room(cx.lc);
  LocalCounts lcn;
  lcn.clear();
  const long long nsc = cx.pc->n_sorted_chunks;
  const long long S = nsc * CHUNK;
  const long long tail = cx.pc->tail_snap;
  const long long nq = (tail + TPB - 1) / TPB;
  const KC kc0 = load_kc(cx, 0, true);
  for (long long q = bid; q < nq; q += nblk) {
    uint32_t slot;
    int tile;
    piece_slot(S / TPB + q, S / TPB, S, tail, cx.pchunk, cx.ptt, &slot, &tile);
    const float x = cx.P.x[slot];
    const uint32_t pos = cx.P.pos[slot];
    const int32_t n0 = cx.P.n0[slot];
    photon_one<false, Q>(cx, slot, tile, kc0, lcn, x, pos, n0, nullptr, nullptr, lroom);
  }
}

// The photon births queued by the sorted lepton pass (queue_births): a lane
// takes one entry and replays its lepton's emission events in order, with
// the draws, energies and recoil bookkeeping of the pass, once to count the
// photons to store and once to write them; the wave reserves tail slots
// once for all its lanes.  The lepton's position after its drift, weight and
// id are read from its slot (the pass has stored them); the step index is
// still the pass's, since the field update runs after this launch.
// Workgroup b0 takes the segments b0, b0 + nb, ..., TPB segments at a time:
// their counts are read together and scanned in LDS, and the entries of all
// of them are taken in dense pieces of TPB (a lane finds its segment by a
// binary search over the scan), so that a workgroup with few entries in many
// segments pays one chain of dependent loads, not one per segment.
template <bool Q>
__device__ __forceinline__ void births_queue(const Ctx& cx, int b0, int nb) {
  __shared__ int s_pre[TPB + 1];
  __shared__ long long s_st[TPB];
  __shared__ int s_wsum[TPB / WAVE];
  const Room proom = load_room(cx.pc);
  const long long lim = proom.L;
  const int ns = b0 < cx.bq_groups ? (cx.bq_groups - b0 + nb - 1) / nb : 0;
  for (int i0 = 0; i0 < ns; i0 += TPB) {
    const int i = i0 + (int)threadIdx.x;
    const int sg = b0 + i * nb;
    const int c = i < ns ? cx.bq_count[sg] : 0;
    s_st[threadIdx.x] = i < ns ? cx.bq_start[sg] : 0;
    int wt;
    const int ex = wave_excl_scan(c, &wt);
    if (lane_id() == 0) s_wsum[threadIdx.x / WAVE] = wt;
    __syncthreads();
    int before = 0, total = 0;
    for (int w = 0; w < TPB / WAVE; ++w) {
      if (w < (int)threadIdx.x / WAVE) before += s_wsum[w];
      total += s_wsum[w];
    }
    s_pre[threadIdx.x] = before + ex;
    if (threadIdx.x == 0) s_pre[TPB] = total;
    __syncthreads();
    for (int p = 0; p < total; p += TPB) {
      const int e = p + (int)threadIdx.x;
      const bool valid = e < total;
      // last segment whose first entry is at or before e (empty ones repeat
      // their successor's start, so the search lands on a segment that has e)
      int lo = 0, hi = TPB;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (s_pre[mid] <= e) lo = mid; else hi = mid;
      }
      const uint4 q = valid ? cx.bq[s_st[lo] + (e - s_pre[lo])] : make_uint4(0u, 0u, 0u, 0u);
      const uint32_t slot = q.x;
      const int tile = valid ? cx.lchunk[slot / CHUNK] : 0;
      const KC k = lane_kc(cx, tile, false);
      const uint32_t flags = (uint32_t)k.flags;
      const float upk = __uint_as_float(q.y);
      const uint64_t evmask = (uint64_t)q.z | ((uint64_t)q.w << 32);
      uint64_t id = 0;
      float aw = 0.0f;
      uint32_t npl = 0;
      if (valid) {
        id = cx.L.id[slot];
        aw = fabsf(cx.L.w[slot]);
        npl = cx.L.pos[slot];
      }
      float g, chi;
      const float xc = emit_xc(upk, k.lr, &g, &chi);
      int nst = 0;
      {
        float au = fabsf(upk);
        uint64_t m = evmask;
        while (m) {
          const int j = __ffsll((long long)m) - 1;
          m &= m - 1;
          const u4 r = draw(k.seed, id, k.step, T_EMIT, (uint32_t)j);
          const float x = fminf(photon_energy<Q>(cx, flags, r.b, xc, upk, k.lr), au);
          au -= x;
          if (x >= k.x_thr || (flags & F_TRACK_ALL)) ++nst;
        }
      }
      int dropped = 0;
      const long long first = reserve_tail(cx.pc, proom, nst, &dropped);
      if (nst > 0) {
        float au = fabsf(upk);
        const float dir = upk >= 0.0f ? 1.0f : -1.0f;
        long long qq = first;
        uint64_t m = evmask;
        while (m) {
          const int j = __ffsll((long long)m) - 1;
          m &= m - 1;
          const u4 r = draw(k.seed, id, k.step, T_EMIT, (uint32_t)j);
          const float x = fminf(photon_energy<Q>(cx, flags, r.b, xc, upk, k.lr), au);
          au -= x;
          if (x >= k.x_thr || (flags & F_TRACK_ALL)) {
            if (qq < lim) {
              const uint32_t kk = (uint32_t)qq;
              cx.P.pos[kk] = npl;
              cx.P.x[kk] = dir * x;
              cx.P.w[kk] = aw;
              cx.P.n0[kk] = (int32_t)(k.step + 1);
              cx.P.id[kk] = child_id(k.seed, id, k.step, 2u + (uint32_t)j);
              cx.ptt[kk] = tile;
            }
            ++qq;
          }
        }
      }
      if (__ballot(dropped != 0)) {
        if (dropped) atomicOr(cx.err, E_CAP);
        count_by_tube(cx.shard, dropped ? k.tube : -1, C_DROPPED, dropped);
      }
      if (__ballot(nst - dropped != 0)) count_by_tube(cx.shard, nst - dropped != 0 ? k.tube : -1, C_PHO_BORN, nst - dropped);
    }
    __syncthreads();                  // (s_pre and s_st are rewritten by the next batch)
  }
}

// Both tail passes in one launch.  They touch disjoint data: each reads its
// own store up to the snapshot taken before it, and its births (photons from
// the leptons, pairs from the photons) go past the other store's snapshot.
// Workgroups alternate roles in groups of eight, so both species spread over
// every XCD; the grid is a multiple of 16, so each role gets half of it with
// indexes 0 .. half - 1.  The first bq_wg workgroups, dispatched first,
// write the photon births that the sorted lepton pass queued instead (they
// go past the photon tail's snapshot, like every birth of the step): their
// chain of dependent loads then runs beside the tail passes.
template <bool Q, bool A>
__global__ __launch_bounds__(TPB) void k_tails(Ctx cx, int bq_wg) {
  if ((int)blockIdx.x < bq_wg) {
    births_queue<Q>(cx, (int)blockIdx.x, bq_wg);
    return;
  }
  const int bx = (int)blockIdx.x - bq_wg;
  const int bid = ((bx >> 4) << 3) | (bx & 7);
  const int nblk = ((int)gridDim.x - bq_wg) >> 1;
  if ((bx >> 3) & 1) photons_tail<Q>(cx, bid, nblk);
  else leptons_tail<Q, A>(cx, bid, nblk);
}

// ------------------------------------------------------------------ field
// Blocks of FB_NODES cells of one tube.  Pass A: block sums of the node
// charge (and, periodic, sum rho_i (N - i)), and the surface-field update
//   E_s += dq w0 2^-24 + alpha s_co dt     (Ampere at the surface)
// Pass B: inclusive scan (Gauss) and conversion to E and the node field.
constexpr int FB_THREADS = 256;
constexpr int FB_PER = 4;
constexpr int FB_NODES = FB_THREADS * FB_PER;

struct FBlk { int32_t tube, k0, first_blk, nblk; };

struct FieldCtx {
  Tube* tubes;
  const FBlk* fb;
  long long* rho;
  long long* rho_last;
  float* E;
  float* ebar;
  long long* part;    // per block: sum rho
  long long* part2;   // per block: sum rho_i (N - i)
  int* err;
  unsigned long long* fs;   // single-pass form: a four-word record per block, then the epoch and a done count
  double* E0;         // filtered tubes: the reference field (set in mode 1)
  double* Du;         // filtered tubes, mode 0: E_u - E0, which k_filter smooths
  Ctl* pc;            // photon store: its tail snapshot for the next step is taken here
  int mode;           // 0: step (surface update, step += 1); 1: rebuild E only
};

__device__ __forceinline__ long long block_sum_ll(long long v, long long* sh) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
  const int w = threadIdx.x / WAVE;
  if (lane_id() == 0) sh[w] = v;
  __syncthreads();
  long long t = 0;
  if (threadIdx.x < WAVE) {
    t = threadIdx.x < (int)(blockDim.x / WAVE) ? sh[threadIdx.x] : 0;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) t += __shfl_xor(t, d);
  }
  if (threadIdx.x == 0) sh[0] = t;
  __syncthreads();
  t = sh[0];
  __syncthreads();
  return t;
}

// Sum of v[first, last) taken by every wave of the workgroup, 64 entries per
// load round.
__device__ __forceinline__ long long wave_range_sum(const long long* v, int first, int last) {
  long long acc = 0;
  for (int j0 = first; j0 < last; j0 += WAVE) {
    const int j = j0 + lane_id();
    long long x = j < last ? v[j] : 0;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d);
    acc += x;
  }
  return acc;
}

__global__ __launch_bounds__(FB_THREADS) void k_field_a(FieldCtx f) {
  __shared__ long long sh[FB_THREADS / WAVE];
  const FBlk b = f.fb[blockIdx.x];
  Tube& T = f.tubes[b.tube];
  const int N = T.N;
  long long s1 = 0, s2 = 0;
  const int k = b.k0 + threadIdx.x * FB_PER;
#pragma unroll
  for (int i = 0; i < FB_PER; ++i) {
    if (k + i < N) {
      long long r = f.rho[T.node_off + k + i];
      s1 += r;
      s2 += r * (long long)(N - (k + i));
    }
  }
  s1 = block_sum_ll(s1, sh);
  s2 = block_sum_ll(s2, sh);
  if (threadIdx.x == 0) {
    f.part[blockIdx.x] = s1;
    f.part2[blockIdx.x] = s2;
    if (b.k0 == 0 && f.mode == 0) {
      if (!(T.flags & F_FIELD_FROZEN)) {
        if (T.flags & F_PERIODIC) T.Es += -(double)T.dcur * T.inv_len_scale + T.drive;
        else T.Es += (double)T.dq * T.scale + T.drive;
      }
      T.dq = 0;
      T.dcur = 0;
    }
  }
}

__global__ __launch_bounds__(FB_THREADS) void k_field_b(FieldCtx f) {
  __shared__ long long sh[FB_THREADS / WAVE];
  const FBlk b = f.fb[blockIdx.x];
  Tube& T = f.tubes[b.tube];
  const int N = T.N;
  const bool per = (T.flags & F_PERIODIC) != 0;
  const bool frozen = (T.flags & F_FIELD_FROZEN) != 0;
  const bool filt = (T.flags & F_FILTER) != 0;
  // carry from the tube's earlier blocks
  const long long carry = wave_range_sum(f.part, b.first_blk, (int)blockIdx.x);
  double mean = 0.0;
  if (per) {
    const long long s2 = wave_range_sum(f.part2, b.first_blk, b.first_blk + b.nblk);
    mean = ((double)s2 + (double)T.bg_unit * 0.5 * (double)N * (double)N) / (double)N;
  }
  const int k = b.k0 + threadIdx.x * FB_PER;
  long long r[FB_PER];
  long long loc = 0;
#pragma unroll
  for (int i = 0; i < FB_PER; ++i) {
    r[i] = (k + i < N) ? f.rho[T.node_off + k + i] : 0;
    loc += r[i];
  }
  // block exclusive scan of loc
  long long incl = loc;
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    long long o = __shfl_up(incl, d);
    if (lane_id() >= d) incl += o;
  }
  const int wv = threadIdx.x / WAVE;
  if (lane_id() == WAVE - 1) sh[wv] = incl;
  __syncthreads();
  if (threadIdx.x < WAVE) {
    long long v = threadIdx.x < FB_THREADS / WAVE ? sh[threadIdx.x] : 0;
    long long iv = v;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
      long long o = __shfl_up(iv, d);
      if (lane_id() >= d) iv += o;
    }
    if (threadIdx.x < FB_THREADS / WAVE) sh[threadIdx.x] = iv - v;
  }
  __syncthreads();
  long long run = carry + sh[wv] + (incl - loc);   // sum of rho over cells < k
  const double Es = T.Es;
  const long long bgu = T.bg_unit;
  // E_{k-1/2} for the node field
  double eprev;
  if (k == 0) eprev = per ? 0.0 : Es;
  else {
    long long eint = run + bgu * (long long)(k - 1) + bgu / 2;
    eprev = per ? ((double)eint - mean) * T.scale + Es : (double)eint * T.scale + Es;
  }
#pragma unroll
  for (int i = 0; i < FB_PER; ++i) {
    const int kk = k + i;
    if (kk >= N) break;
    run += r[i];
    const long long eint = run + bgu * (long long)kk + bgu / 2;
    const double e = per ? ((double)eint - mean) * T.scale + Es : (double)eint * T.scale + Es;
    if (!frozen) {
      if (filt && f.mode == 0) {
        f.Du[T.cell_off + kk] = e - f.E0[T.cell_off + kk];
      } else {
        f.E[T.cell_off + kk] = (float)e;
        if (kk > 0 || !per) f.ebar[T.node_off + kk] = (float)(0.5 * (eprev + e));
        if (filt) f.E0[T.cell_off + kk] = e;
      }
      if (!isfinite(e)) atomicOr(f.err, E_NAN);
    }
    f.rho_last[T.node_off + kk] = r[i];
    f.rho[T.node_off + kk] = 0;
    eprev = e;
    if (kk == N - 1) {
      // last node: non-periodic ghost E_{N+1/2} = E_{N-1/2}; periodic node 0 = node N
      if (!frozen && !per && !(filt && f.mode == 0)) f.ebar[T.node_off + N] = (float)e;
      f.rho_last[T.node_off + N] = f.rho[T.node_off + N];
      f.rho[T.node_off + N] = 0;
    }
  }
  if (threadIdx.x == 0 && f.mode == 0 && b.k0 == 0) T.step += 1;
  // the photon tail the next step's photon tail pass takes: every photon
  // born in this step (the lepton passes, earlier on this stream) is in it
  if (threadIdx.x == 0 && blockIdx.x == 0 && f.mode == 0) {
    clamp_tail(f.pc);
    f.pc->tail_snap = f.pc->tail;
  }
}

// Single-pass form of the two passes above, for grids without periodic tubes.
// Each block publishes its charge sum, finds the sum over its tube's earlier
// blocks by looking back over their records (a block's own sum, or its
// inclusive prefix once known, the nearest such ending the search), publishes
// its inclusive prefix, then scans.  A block waits only on blocks of lower
// index, which every XCD dispatches before it, so each wait ends; a bounded
// spin turns a record that never appears into an error rather than a hang.
// The tube's first block updates E_s and every inclusive record carries it on.
//
// A record is four 64-bit words: the high half of each holds the record's
// 32-bit tag (launch epoch and status), the low halves hold the sum and E_s
// 32 bits at a time.  Each word is one single-copy-atomic, device-coherent
// access, so a reader that finds one tag in all four words holds a whole
// record, with no fence between the writer's stores.  The last block out
// advances the epoch, so no record is cleared between launches.
constexpr uint32_t FS_AGG = 1, FS_INCL = 2;
constexpr int FS_SPIN = 1 << 18;

__device__ __forceinline__ void fs_word_put(unsigned long long* p, uint32_t tag, uint32_t v) {
  __hip_atomic_store(p, ((unsigned long long)tag << 32) | v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void fs_put(unsigned long long* r, uint32_t tag, long long v, double es) {
  const unsigned long long e = __builtin_bit_cast(unsigned long long, es);
  fs_word_put(r + 0, tag, (uint32_t)(unsigned long long)v);
  fs_word_put(r + 1, tag, (uint32_t)((unsigned long long)v >> 32));
  fs_word_put(r + 2, tag, (uint32_t)e);
  fs_word_put(r + 3, tag, (uint32_t)(e >> 32));
}
// The record's tag if all four words agree, else 0 (no tag is 0).
__device__ __forceinline__ uint32_t fs_get(const unsigned long long* r, long long* v, double* es) {
  unsigned long long w[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) w[i] = __hip_atomic_load(r + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint32_t t = (uint32_t)(w[0] >> 32);
  if ((uint32_t)(w[1] >> 32) != t || (uint32_t)(w[2] >> 32) != t || (uint32_t)(w[3] >> 32) != t) return 0;
  *v = (long long)((w[1] << 32) | (uint32_t)w[0]);
  *es = __builtin_bit_cast(double, (w[3] << 32) | (uint32_t)w[2]);
  return t;
}

__global__ __launch_bounds__(FB_THREADS) void k_field_1p(FieldCtx f) {
  constexpr int NW = FB_THREADS / WAVE;
  __shared__ long long sh[NW];
  __shared__ long long s_carry;
  __shared__ double s_es;
  __shared__ unsigned long long s_ep;
  const FBlk b = f.fb[blockIdx.x];
  Tube& T = f.tubes[b.tube];
  const int N = T.N;
  const bool frozen = (T.flags & F_FIELD_FROZEN) != 0;
  const bool filt = (T.flags & F_FILTER) != 0;
  unsigned long long* rec = f.fs;                       // 4 words per block
  unsigned long long* epoch = f.fs + 4 * gridDim.x;     // then the done count
  const int k = b.k0 + threadIdx.x * FB_PER;
  long long r[FB_PER];
  long long loc = 0;
#pragma unroll
  for (int i = 0; i < FB_PER; ++i) {
    r[i] = (k + i < N) ? f.rho[T.node_off + k + i] : 0;
    loc += r[i];
  }
  long long incl = loc;
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    long long o = __shfl_up(incl, d);
    if (lane_id() >= d) incl += o;
  }
  const int wv = threadIdx.x / WAVE;
  if (lane_id() == WAVE - 1) sh[wv] = incl;
  if (threadIdx.x == 0) s_ep = __hip_atomic_load(epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  if (threadIdx.x < WAVE) {
    const long long v = threadIdx.x < NW ? sh[threadIdx.x] : 0;
    long long iv = v;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
      long long o = __shfl_up(iv, d);
      if (lane_id() >= d) iv += o;
    }
    if (threadIdx.x < NW) sh[threadIdx.x] = iv - v;
    const long long tot = __shfl(iv, NW - 1);
    const uint32_t cur = (uint32_t)(s_ep + 1) << 2;   // the status bits are 1 or 2, so no tag is 0
    const int bx = (int)blockIdx.x;
    long long carry = 0;
    double es = 0.0;
    if (bx == b.first_blk) {
      es = T.Es;
      if (f.mode == 0 && !frozen) es += (double)T.dq * T.scale + T.drive;
      if (lane_id() == 0) {
        if (f.mode == 0) {
          T.Es = es;
          T.dq = 0;
          T.dcur = 0;
        }
        fs_put(rec + 4 * bx, cur | FS_INCL, tot, es);
      }
    } else {
      if (lane_id() == 0) fs_put(rec + 4 * bx, cur | FS_AGG, tot, 0.0);
      for (int top = bx - 1; top >= b.first_blk; top -= WAVE) {
        const int p = top - lane_id();
        const bool in = p >= b.first_blk;
        uint32_t t = 0;
        long long pv = 0;
        double pe = 0.0;
        if (in) {
          int spin = 0;
          t = fs_get(rec + 4 * p, &pv, &pe);
          while ((t & ~3u) != cur && ++spin < FS_SPIN) {
            __builtin_amdgcn_s_sleep(2);
            t = fs_get(rec + 4 * p, &pv, &pe);
          }
          if ((t & ~3u) != cur) atomicOr(f.err, E_SCAN);
        }
        const unsigned long long im = __ballot(in && t == (cur | FS_INCL));
        const int stop = im ? __ffsll((long long)im) - 1 : WAVE;
        long long x = (in && lane_id() <= stop && (t & ~3u) == cur) ? pv : 0;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d);
        carry += x;
        if (im) {
          es = __shfl(pe, stop);
          break;
        }
      }
      if (lane_id() == 0) fs_put(rec + 4 * bx, cur | FS_INCL, carry + tot, es);
    }
    if (lane_id() == 0) {
      s_carry = carry;
      s_es = es;
    }
  }
  __syncthreads();
  long long run = s_carry + sh[wv] + (incl - loc);   // sum of rho over cells < k
  const double Es = s_es;
  const long long bgu = T.bg_unit;
  double eprev = k == 0 ? Es : (double)(run + bgu * (long long)(k - 1) + bgu / 2) * T.scale + Es;
#pragma unroll
  for (int i = 0; i < FB_PER; ++i) {
    const int kk = k + i;
    if (kk >= N) break;
    run += r[i];
    const double e = (double)(run + bgu * (long long)kk + bgu / 2) * T.scale + Es;
    if (!frozen) {
      if (filt && f.mode == 0) {
        f.Du[T.cell_off + kk] = e - f.E0[T.cell_off + kk];
      } else {
        f.E[T.cell_off + kk] = (float)e;
        f.ebar[T.node_off + kk] = (float)(0.5 * (eprev + e));
        if (filt) f.E0[T.cell_off + kk] = e;
      }
      if (!isfinite(e)) atomicOr(f.err, E_NAN);
    }
    f.rho_last[T.node_off + kk] = r[i];
    f.rho[T.node_off + kk] = 0;
    eprev = e;
    if (kk == N - 1) {
      if (!frozen && !(filt && f.mode == 0)) f.ebar[T.node_off + N] = (float)e;   // ghost E_{N+1/2} = E_{N-1/2}
      f.rho_last[T.node_off + N] = f.rho[T.node_off + N];
      f.rho[T.node_off + N] = 0;
    }
  }
  if (threadIdx.x == 0 && f.mode == 0 && b.k0 == 0) T.step += 1;
  if (threadIdx.x == 0 && blockIdx.x == 0 && f.mode == 0) {
    clamp_tail(f.pc);
    f.pc->tail_snap = f.pc->tail;
  }
  // the last block out advances the epoch (every block read it before this)
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    const unsigned long long d = __hip_atomic_fetch_add(epoch + 1, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (d == gridDim.x - 1) {
      __hip_atomic_store(epoch + 1, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(epoch, s_ep + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// Periodic node 0 (= node N): average of E_{N-1/2} and E_{1/2}; runs after k_field_b.
__global__ void k_field_periodic_ends(FieldCtx f, int n_tubes) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tubes) return;
  Tube& T = f.tubes[t];
  if (!(T.flags & F_PERIODIC) || (T.flags & F_FIELD_FROZEN)) return;
  const float v = 0.5f * (f.E[T.cell_off + T.N - 1] + f.E[T.cell_off]);
  f.ebar[T.node_off] = v;
  f.ebar[T.node_off + T.N] = v;
}

// The digital filter of the current (Sect. 6.1), for tubes with F_FILTER,
// after the field update of a step: E = E0 + F[E_u - E0] with F eight
// passes of (x_{i-1} + 2 x_i + x_{i+1}) / 4 (E_u - E0 is in Du).  Repeating
// the end value at every pass is the same as extending the array once by its
// mirror image about the end face, so each block loads its cells with a halo
// of FLT_PASSES + 1 cells on the left (the node field needs the cell before
// the block) and FLT_PASSES on the right, mirrored (or wrapped, periodic)
// at the ends, smooths in LDS, and writes E and the node field.
// Grid (ceil(max N / FLT_CELLS), tubes); filtered tubes have N >= 2 FLT_PASSES.
constexpr int FLT_PASSES = 8;
constexpr int FLT_CELLS = 256;
constexpr int FLT_W = FLT_CELLS + 2 * FLT_PASSES + 1;

__global__ __launch_bounds__(FLT_CELLS) void k_filter(FieldCtx f) {
  __shared__ double a[FLT_W], b[FLT_W];
  const Tube& T = f.tubes[blockIdx.y];
  if (!(T.flags & F_FILTER) || (T.flags & F_FIELD_FROZEN)) return;
  const int N = T.N;
  const int c0 = blockIdx.x * FLT_CELLS;
  if (c0 >= N) return;
  const bool per = (T.flags & F_PERIODIC) != 0;
  // (window cells past N + FLT_PASSES feed no output: clamped into the tube)
  auto src = [&](int j) {
    if (per) return ((j % N) + N) % N;
    const int m = j < 0 ? -1 - j : (j >= N ? 2 * N - 1 - j : j);
    return min(max(m, 0), N - 1);
  };
  for (int i = threadIdx.x; i < FLT_W; i += blockDim.x) a[i] = f.Du[T.cell_off + src(c0 - FLT_PASSES - 1 + i)];
  __syncthreads();
  double* x = a;
  double* y = b;
  for (int p = 0; p < FLT_PASSES; ++p) {
    for (int i = threadIdx.x; i < FLT_W; i += blockDim.x)
      y[i] = (i > 0 && i < FLT_W - 1) ? (x[i - 1] + 2.0 * x[i] + x[i + 1]) / 4.0 : x[i];
    __syncthreads();
    double* t = x;
    x = y;
    y = t;
  }
  // x[FLT_PASSES + 1 + c - c0] is the smoothed value of cell c (exact for
  // cells c0 - 1 .. c0 + FLT_CELLS - 1)
  const int c = c0 + (int)threadIdx.x;
  if (c < N) {
    const double e = f.E0[T.cell_off + c] + x[FLT_PASSES + 1 + threadIdx.x];
    double ep;
    if (c > 0 || per) {
      const int cp = c > 0 ? c - 1 : N - 1;
      ep = f.E0[T.cell_off + cp] + x[FLT_PASSES + threadIdx.x];
    } else {
      ep = T.Es;   // ghost E_{-1/2} = E_s
    }
    f.E[T.cell_off + c] = (float)e;
    f.ebar[T.node_off + c] = (float)(0.5 * (ep + e));
    if (per && c == 0) f.ebar[T.node_off + N] = (float)(0.5 * (ep + e));   // node N is node 0
    if (!per && c == N - 1) f.ebar[T.node_off + N] = (float)e;             // ghost E_{N+1/2} = E_{N-1/2}
  }
}

// ------------------------------------------------------------------ re-sort
template <class B> __device__ __forceinline__ bool rec_alive(const B& b, long long i);
template <> __device__ __forceinline__ bool rec_alive<LepBuf>(const LepBuf& b, long long i) { return b.w[i] != 0.0f; }
template <> __device__ __forceinline__ bool rec_alive<PhoBuf>(const PhoBuf& b, long long i) { return b.x[i] != 0.0f; }

__device__ __forceinline__ void rec_copy(const LepBuf& s, long long i, const LepBuf& d, long long j, uint32_t pos) {
  d.pos[j] = pos; d.u[j] = s.u[i]; d.w[j] = s.w[i]; d.id[j] = s.id[i];
}
__device__ __forceinline__ void rec_copy(const PhoBuf& s, long long i, const PhoBuf& d, long long j, uint32_t pos) {
  d.pos[j] = pos; d.x[j] = s.x[i]; d.w[j] = s.w[i]; d.n0[j] = s.n0[i]; d.id[j] = s.id[i];
}
__device__ __forceinline__ void rec_kill(const LepBuf& d, long long j) { d.w[j] = 0.0f; }
__device__ __forceinline__ void rec_kill(const PhoBuf& d, long long j) { d.x[j] = 0.0f; }

template <class B>
struct RbCtx {
  const Tube* tubes;
  const Tile* tiles;
  B src, dst;
  Ctl* ctl;
  const int32_t* chunk_old;
  int32_t* chunk_new;
  const int32_t* tt;
  int32_t* tcount;       // live particles per tile
  // Within a tile the particles are placed by class (RbClasses<B>::N of
  // them, class 0 first): photons that can draw a conversion before the next
  // re-sort ahead of those that cannot, leptons by how close they are to
  // the emission threshold.  Waves of the particle passes then meet the
  // rare branches only where their particles need them.
  int32_t* ccount;       // [N - 1][n_tiles]: particles of classes 0 .. N - 2 per tile
  int32_t* ccur;         // [N][n_tiles]: placement cursor per class and tile
  uint8_t* cls;          // per source slot: the class the count kernel decided
  uint16_t* chot;        // photons, per chunk of the new layout: class-0 slots at its start
  int window;            // steps until the next re-sort
  long long* tchunk;     // first chunk of each tile in the new layout (n_tiles + 1)
  int32_t* wh;           // [grid][RB_HW][N]: each count workgroup's window counts by tile and class
  int n_tiles;
};

// A photon is cold when no step of the coming re-sort window can draw its
// conversion.  Over the window its age runs from a1 to a2; |sin psi| is at
// most the larger of its values at the two ends while both angles stay
// within 1.5 rad, and at most 1 otherwise.  The step's exponent
// alpha_em (b/lambda~) sin psi T_BW(x b sin psi) grows with |sin psi| (the
// fit's log-derivative in chi stays above -1/3), so its value at that bound
// caps every step's.  Cold needs the cap at or below 2^-27: a factor 4 under
// the 2^-25 that a draw needs, far beyond the rounding differences between
// this FP32 bound and the pass's FP32 probability.  The photon pass skips
// the probability of cold slots only while the window lasts, so the
// classification changes no result.
template <class B> struct RbClasses;
template <> struct RbClasses<PhoBuf> { static constexpr int N = 2; };
template <> struct RbClasses<LepBuf> { static constexpr int N = 4; };

// The loads of one slot of a re-sort row, issued before any use, so that a
// group of rows keeps its loads in flight together.  a: the field that marks
// a live record (photon x, lepton w); b: lepton u; n0: photon birth step;
// cls: the class the count kernel decided (scatter).
struct RbIn { long long slot; int tile; uint32_t pos; float a, b; uint32_t n0; int cls; };

__device__ __forceinline__ bool rb_hot(const RbCtx<PhoBuf>& cx, const Tube& T, float x, uint32_t n0) {
  const int32_t a1 = (int32_t)((uint32_t)T.step + 1u - n0);
  const int32_t a2 = (int32_t)((uint32_t)T.step + (uint32_t)cx.window - n0);
  if (a2 < a1) return true;                 // the 32-bit age wraps inside the window
  const float s1 = (float)a1 * T.dt * T.inv_rc, s2 = (float)a2 * T.dt * T.inv_rc;
  const float sp = fmaxf(fabsf(s1), fabsf(s2)) < 1.5f ? fmaxf(fabsf(sinf(s1)), fabsf(sinf(s2))) : 1.0f;
  const float chi = fabsf(x) * T.b * sp;
  return T.conv_k * sp * t_bw(chi) > 7.4505806e-9f;   // 2^-27
}
__device__ __forceinline__ int rb_class(const RbCtx<PhoBuf>& cx, const Tube& T, const RbIn& r, int, uint32_t) {
  return rb_hot(cx, T, r.a, r.n0) ? 0 : 1;
}
// Leptons: class 0 evaluates emission now (x_c >= x_c,floor inside the QED
// zone, the pass's test on the stored momentum), classes 1 and 2 are within
// factors 4 and 64 of the threshold in x_c (gamma within 1.6 and 4), class 3
// is the rest and everything outside the zone.  Those that cross the
// threshold during the window sit next to the evaluating ones.
__device__ __forceinline__ int rb_class(const RbCtx<LepBuf>&, const Tube& T, const RbIn& r, int cell, uint32_t frac) {
  if ((T.flags & (F_QED_OFF | F_EMIT_OFF)) || ((int64_t)cell << FRAC) + frac >= T.hfix) return 3;
  const float u = r.b;
  const float g = __builtin_amdgcn_sqrtf(1.0f + u * u);
  const float xc = 1.5f * g * (g * g * T.lr);
  return xc >= T.xc_floor ? 0 : xc >= 0.25f * T.xc_floor ? 1 : xc >= (1.0f / 64.0f) * T.xc_floor ? 2 : 3;
}

// Tile (new) of the particle in `slot`, or -1 if the slot is dead/empty.
// cls: computed (decide) or read back from the count kernel's decision; the
// scatter must place exactly the particles the count kernel counted in each
// class (a recomputed class could differ in its last rounding between
// kernels).
template <class B>
__device__ __forceinline__ int rb_locate(const RbCtx<B>& cx, const RbIn& r, int* cell_out, uint32_t* frac_out, int* cls,
                                         bool decide) {
  *cls = 0;
  if (r.tile < 0 || r.a == 0.0f) return -1;
  const Tile tl = cx.tiles[r.tile];
  const Tube& T = cx.tubes[tl.tube];
  int cell = tl.base + (int)(r.pos >> FRAC);
  if (T.flags & F_PERIODIC) cell = wrap_cell(cell, T.N);
  *cell_out = cell;
  *frac_out = r.pos & 0xFFFFFFu;
  if (decide) {
    *cls = rb_class(cx, T, r, cell, r.pos & 0xFFFFFFu);
    cx.cls[r.slot] = (uint8_t)*cls;
  } else {
    *cls = r.cls;
  }
  return T.tile_first + cell / TILE;
}

// Row q of a re-sort pass: the slot of this thread and its loads (a row past
// the workgroup's last gives a dead slot).  Slots past the tail are inside
// the store (it keeps a chunk of slack), so every load is in bounds.
template <class B>
__device__ __forceinline__ void rb_load(const RbCtx<B>& cx, bool have, long long q, long long nsq, long long S,
                                        long long tail, bool decide, RbIn& r) {
  r.slot = 0;
  r.tile = -1;
  r.pos = 0;
  r.a = 0.0f;
  r.b = 0.0f;
  r.n0 = 0;
  r.cls = 0;
  if (!have) return;
  uint32_t s32;
  piece_slot(q, nsq, S, tail, cx.chunk_old, cx.tt, &s32, &r.tile);
  r.slot = s32;
  r.pos = cx.src.pos[s32];
  if constexpr (std::is_same<B, PhoBuf>::value) {
    r.a = cx.src.x[s32];
    if (decide) r.n0 = (uint32_t)cx.src.n0[s32];
  } else {
    r.a = cx.src.w[s32];
    if (decide) r.b = cx.src.u[s32];
  }
  if (!decide) r.cls = cx.cls[s32];
}
constexpr int RB_U = 4;   // rows whose loads a thread keeps in flight together

// Destination tiles of one workgroup's contiguous chunk range are counted in
// an LDS histogram over a window of RB_HW tiles (a range of sorted chunks
// only reaches its own tiles +- 1); tiles outside the window go straight to
// global atomics, aggregated per wave.  A store of at most RB_HW tiles puts
// the window at tile 0, so that every tile is in it and the tail rows, whose
// tiles are in no order, need no global atomics either (the production
// gap's re-sort 0.83 -> 0.65 ms).
constexpr int RB_HW = 1024;

__device__ __forceinline__ void rb_range(long long nch, long long* c0, long long* c1) {
  const int G = gridDim.x, bx = blockIdx.x;
  const int r = (bx & 7) * (G >> 3) + (bx >> 3);
  *c0 = nch * r / G;
  *c1 = nch * (r + 1) / G;
}

// Rows (256-slot pieces) of this workgroup in a re-sort pass: a contiguous
// range [c0, c1) of the sorted rows (so that the LDS window of destination
// tiles applies), then every G-th row of the tail.  Tail particles are in no
// tile order and cost more per row; striding them over all workgroups keeps
// the pass balanced.
__device__ __forceinline__ long long rb_nrows(long long c0, long long c1, long long nsq, long long nq) {
  const long long nt = nq - nsq - (long long)blockIdx.x;
  return (c1 - c0) + (nt > 0 ? (nt + gridDim.x - 1) / gridDim.x : 0);
}
__device__ __forceinline__ long long rb_row(long long i, long long c0, long long c1, long long nsq) {
  return i < c1 - c0 ? c0 + i : nsq + (long long)blockIdx.x + (i - (c1 - c0)) * (long long)gridDim.x;
}

// Wave-aggregated add of 1 per lane to bin `k` (k < 0: no-op).  `lds`: bins
// are LDS entries relative to dlo, else global tile counters.  Returns this
// lane's rank-based position (old value + rank) when `ret` is set.
__device__ __forceinline__ int rb_wave_add(int k, int* lds_bins, int dlo, int* gbins, bool lds, bool ret) {
  int out = -1;
  while (true) {
    uint64_t m = __ballot(k >= 0);
    if (!m) break;
    const int lead = __ffsll((long long)m) - 1;
    const int kk = __shfl(k, lead);
    const uint64_t mk = __ballot(k == kk);
    int base = 0;
    if (lane_id() == lead) {
      if (lds) base = atomicAdd(&lds_bins[kk - dlo], (int)__popcll(mk));
      else base = atomicAdd(&gbins[kk], (int)__popcll(mk));
    }
    if (ret) base = __shfl(base, lead);
    if (k == kk) { out = base + rank_in(mk); k = -1; }
  }
  return out;
}

template <class B>
__global__ __launch_bounds__(TPB) void k_rb_count(RbCtx<B> cx) {
  constexpr int NC = RbClasses<B>::N;
  __shared__ int s_h[RB_HW];
  __shared__ int s_c[RB_HW * (NC - 1)];     // (tile - dlo) (NC - 1) + class, classes 0 .. NC - 2
  const long long nsc = cx.ctl->n_sorted_chunks, S = nsc * CHUNK, tail = cx.ctl->tail;
  const long long nsq = S / TPB, nq = nsq + (tail + TPB - 1) / TPB;
  long long c0, c1;
  rb_range(nsq, &c0, &c1);
  const long long nrow = rb_nrows(c0, c1, nsq, nq);
  for (int j = threadIdx.x; j < RB_HW; j += blockDim.x) s_h[j] = 0;
  for (int j = threadIdx.x; j < RB_HW * (NC - 1); j += blockDim.x) s_c[j] = 0;
  __syncthreads();
  const int dlo = cx.n_tiles <= RB_HW ? 0 : (c0 < nsq ? cx.chunk_old[c0 / PPC] - 1 : -(1 << 30));
  for (long long i0 = 0; i0 < nrow; i0 += RB_U) {
    RbIn in[RB_U];
#pragma unroll
    for (int u = 0; u < RB_U; ++u)
      rb_load(cx, i0 + u < nrow, rb_row(i0 + u, c0, c1, nsq), nsq, S, tail, true, in[u]);
#pragma unroll
    for (int u = 0; u < RB_U; ++u) {
      int cell; uint32_t frac; int k;
      const int nt = rb_locate(cx, in[u], &cell, &frac, &k, true);
      const bool inw = nt >= 0 && nt - dlo >= 0 && nt - dlo < RB_HW;
      rb_wave_add(inw ? nt : -1, s_h, dlo, cx.tcount, true, false);
      rb_wave_add((nt >= 0 && !inw) ? nt : -1, s_h, dlo, cx.tcount, false, false);
      const bool ck = nt >= 0 && k < NC - 1;
      rb_wave_add((ck && inw) ? (nt - dlo) * (NC - 1) + k : -1, s_c, 0, nullptr, true, false);
      rb_wave_add((ck && !inw) ? k * cx.n_tiles + nt : -1, nullptr, 0, cx.ccount, false, false);
    }
  }
  __syncthreads();
  // the window counts by (tile, class) for the scatter, whose workgroup b
  // takes the same rows as this one
  int32_t* wh = cx.wh + (long long)blockIdx.x * (RB_HW * NC);
  for (int j = threadIdx.x; j < RB_HW; j += blockDim.x) {
    int rest = s_h[j];
    for (int k = 0; k < NC - 1; ++k) {
      const int c = s_c[j * (NC - 1) + k];
      wh[j * NC + k] = c;
      rest -= c;
    }
    wh[j * NC + NC - 1] = rest;
  }
  for (int j = threadIdx.x; j < RB_HW; j += blockDim.x)
    if (s_h[j] > 0) atomicAdd(&cx.tcount[dlo + j], s_h[j]);
  for (int j = threadIdx.x; j < RB_HW * (NC - 1); j += blockDim.x)
    if (s_c[j] > 0) atomicAdd(&cx.ccount[(j % (NC - 1)) * cx.n_tiles + dlo + j / (NC - 1)], s_c[j]);
}

// Exclusive scan of the chunk counts of the tiles (one workgroup of
// RB_SCAN_T threads, RB_SCAN_V consecutive tiles per thread and round).  A
// small workgroup starts beside the other store's re-sort kernels, which run
// at the same time on the second stream; one of 1024 threads waited for a
// whole idle CU.
constexpr int RB_SCAN_T = 256;
constexpr int RB_SCAN_V = 4;
template <class B>
__global__ __launch_bounds__(RB_SCAN_T) void k_rb_scan(RbCtx<B> cx) {
  __shared__ long long sh[RB_SCAN_T / WAVE];
  long long carry = 0;
  for (int base = 0; base < cx.n_tiles; base += RB_SCAN_T * RB_SCAN_V) {
    const int t0 = base + (int)threadIdx.x * RB_SCAN_V;
    long long v[RB_SCAN_V];
    long long sum = 0;
#pragma unroll
    for (int j = 0; j < RB_SCAN_V; ++j) {
      const int t = t0 + j;
      v[j] = 0;
      if (t < cx.n_tiles) {
        v[j] = (cx.tcount[t] + CHUNK - 1) / CHUNK;
        for (int k = 0; k < RbClasses<B>::N; ++k) cx.ccur[k * cx.n_tiles + t] = 0;
      }
      sum += v[j];
    }
    long long incl = sum;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
      long long o = __shfl_up(incl, d);
      if (lane_id() >= d) incl += o;
    }
    const int wv = threadIdx.x / WAVE;
    if (lane_id() == WAVE - 1) sh[wv] = incl;
    __syncthreads();
    long long before = carry, tot = carry;
    for (int w = 0; w < RB_SCAN_T / WAVE; ++w) {
      if (w < wv) before += sh[w];
      tot += sh[w];
    }
    long long ex = before + incl - sum;
#pragma unroll
    for (int j = 0; j < RB_SCAN_V; ++j) {
      if (t0 + j < cx.n_tiles) cx.tchunk[t0 + j] = ex;
      ex += v[j];
    }
    carry = tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    cx.tchunk[cx.n_tiles] = carry;
    cx.ctl->total_chunks_new = carry;
  }
}

template <class B>
__global__ void k_rb_chunks(RbCtx<B> cx) {
  const long long tot = cx.ctl->total_chunks_new;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < tot; c += (long long)gridDim.x * blockDim.x) {
    int lo = 0, hi = cx.n_tiles;      // find last t with tchunk[t] <= c
    while (hi - lo > 1) {
      int mid = (lo + hi) >> 1;
      if (cx.tchunk[mid] <= c) lo = mid; else hi = mid;
    }
    cx.chunk_new[c] = lo;
    if (cx.chot) {
      const long long h = (long long)cx.ccount[lo] - (c - cx.tchunk[lo]) * CHUNK;
      cx.chot[c] = (uint16_t)(h < 0 ? 0 : (h > CHUNK ? CHUNK : h));
    }
  }
}

// First slot of class k in tile t of the new layout.
template <class B>
__device__ __forceinline__ long long rb_class_start(const RbCtx<B>& cx, int t, int k) {
  long long o = cx.tchunk[t] * CHUNK;
  for (int j = 0; j < k; ++j) o += cx.ccount[j * cx.n_tiles + t];
  return o;
}

template <class B>
__global__ __launch_bounds__(TPB) void k_rb_scatter(RbCtx<B> cx) {
  constexpr int NC = RbClasses<B>::N;
  __shared__ int s_h[RB_HW * NC];            // (tile - dlo) NC + class
  __shared__ uint32_t s_base[RB_HW * NC];
  const long long nsc = cx.ctl->n_sorted_chunks, S = nsc * CHUNK, tail = cx.ctl->tail;
  const long long nsq = S / TPB, nq = nsq + (tail + TPB - 1) / TPB;
  long long c0, c1;
  rb_range(nsq, &c0, &c1);
  const long long nrow = rb_nrows(c0, c1, nsq, nq);
  const int dlo = cx.n_tiles <= RB_HW ? 0 : (c0 < nsq ? cx.chunk_old[c0 / PPC] - 1 : -(1 << 30));
  // how many of this range go to each window tile and class: counted by the
  // count kernel's workgroup of the same index, which took the same rows
  // with the same window
  {
    const int32_t* wh = cx.wh + (long long)blockIdx.x * (RB_HW * NC);
    for (int j = threadIdx.x; j < RB_HW * NC; j += blockDim.x) s_h[j] = wh[j];
  }
  __syncthreads();
  // one reservation per (workgroup, tile, class)
  for (int j = threadIdx.x; j < RB_HW * NC; j += blockDim.x) {
    const int n = s_h[j];
    if (n > 0) {
      const int t = dlo + j / NC, k = j % NC;
      s_base[j] = (uint32_t)(rb_class_start(cx, t, k) + atomicAdd(&cx.ccur[k * cx.n_tiles + t], n));
      s_h[j] = 0;
    }
  }
  __syncthreads();
  // pass B: place the records
  for (long long i0 = 0; i0 < nrow; i0 += RB_U) {
    RbIn in[RB_U];
#pragma unroll
    for (int u = 0; u < RB_U; ++u)
      rb_load(cx, i0 + u < nrow, rb_row(i0 + u, c0, c1, nsq), nsq, S, tail, false, in[u]);
#pragma unroll
    for (int u = 0; u < RB_U; ++u) {
      int cell = 0, k; uint32_t frac = 0;
      const int nt = rb_locate(cx, in[u], &cell, &frac, &k, false);
      const bool inw = nt >= 0 && nt - dlo >= 0 && nt - dlo < RB_HW;
      const int ri = rb_wave_add(inw ? (nt - dlo) * NC + k : -1, s_h, 0, nullptr, true, true);
      const int ro = rb_wave_add((nt >= 0 && !inw) ? k * cx.n_tiles + nt : -1, nullptr, 0, cx.ccur, false, true);
      if (nt >= 0) {
        const long long dst = inw ? (long long)s_base[(nt - dlo) * NC + k] + ri : rb_class_start(cx, nt, k) + ro;
        const Tile tl = cx.tiles[nt];
        rec_copy(cx.src, in[u].slot, cx.dst, dst, ((uint32_t)(cell - tl.base) << FRAC) | frac);
      }
    }
  }
}

// The slots of the new layout past each tile's last particle, up to the end
// of its last chunk, hold dead records (the scatter writes every other slot).
// Workgroup b takes tiles b, b + G, ...: the work is the padding alone.
template <class B>
__global__ __launch_bounds__(TPB) void k_rb_pad(RbCtx<B> cx) {
  for (int t = blockIdx.x; t < cx.n_tiles; t += gridDim.x) {
    const long long hi = cx.tchunk[t + 1] * CHUNK;
    for (long long slot = cx.tchunk[t] * CHUNK + cx.tcount[t] + threadIdx.x; slot < hi; slot += blockDim.x)
      rec_kill(cx.dst, slot);
  }
}

template <class B>
__global__ void k_rb_finish(RbCtx<B> cx) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    cx.ctl->n_sorted_chunks = cx.ctl->total_chunks_new;
    cx.ctl->tail = 0;
    cx.ctl->tail_snap = 0;
    cx.ctl->cold_steps = cx.chot ? cx.window : -1;
  }
}

// ------------------------------------------------------------------ init
struct InitCtx {
  const Tube* tubes;
  const Tile* tiles;
  LepBuf L;
  int32_t* ltt;
  long long base_slot;
  const long long* tube_off;   // first init index of each tube (n_tubes + 1)
  const int32_t* kind;         // init kind per tube
  const int32_t* ppc;          // ppc_init per tube
  const int32_t* k_lo;         // first initialised cell per tube
  const float* u0;             // initial momentum per tube
  int n_tubes;
};

__global__ void k_init_particles(InitCtx cx) {
  const long long tot = cx.tube_off[cx.n_tubes];
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += (long long)gridDim.x * blockDim.x) {
    int lo = 0, hi = cx.n_tubes;
    while (hi - lo > 1) { int mid = (lo + hi) >> 1; if (cx.tube_off[mid] <= i) lo = mid; else hi = mid; }
    const int t = lo;
    const Tube& T = cx.tubes[t];
    const long long li = i - cx.tube_off[t];
    const int ppc = cx.ppc[t];
    const long long ncell = T.N - cx.k_lo[t];
    const long long per_sp = ncell * ppc;
    const int sp = (int)(li / per_sp);
    const long long rem = li - (long long)sp * per_sp;
    const int cell = cx.k_lo[t] + (int)(rem / ppc);
    const uint64_t id = (uint64_t)li + 1;
    u4 r = draw(T.seed, id, 0, T_INIT, 0);
    const int tile = T.tile_first + cell / TILE;
    const Tile tl = cx.tiles[tile];
    const long long slot = cx.base_slot + i;
    cx.L.pos[slot] = ((uint32_t)(cell - tl.base) << FRAC) | (r.a >> 8);
    cx.L.u[slot] = cx.u0[t];
    cx.L.w[slot] = (cx.kind[t] == 1 && sp == 1) ? 1.0f : -1.0f;
    cx.L.id[slot] = id;
    cx.ltt[slot] = tile;
  }
}

// Deposit every live lepton (initial field, loaded states): global atomics.
__global__ __launch_bounds__(TPB) void k_deposit_all(Ctx cx) {
  const long long nsc = cx.lc->n_sorted_chunks, S = nsc * CHUNK, tail = cx.lc->tail;
  const long long nsq = S / TPB, nq = nsq + (tail + TPB - 1) / TPB;
  for (long long c = blockIdx.x; c < nq; c += gridDim.x) {
    uint32_t slot; int tile;
    piece_slot(c, nsq, S, tail, cx.lchunk, cx.ltt, &slot, &tile);
    if (tile < 0) continue;
    const float w = cx.L.w[slot];
    if (w == 0.0f) continue;
    const Tile tl = cx.tiles[tile];
    const Tube& T = cx.tubes[tl.tube];
    const bool per = (T.flags & F_PERIODIC) != 0;
    const uint32_t pos = cx.L.pos[slot];
    int cell = tl.base + (int)(pos >> FRAC);
    if (per) cell = wrap_cell(cell, T.N);
    const uint32_t frac = pos & 0xFFFFFFu;
    const int64_t Tw = __float2ll_rn(fabsf(w) * 16777216.0f);
    const unsigned long long A = ((unsigned long long)Tw * frac + (1ull << 23)) >> FRAC;
    const long long a = w > 0 ? (long long)A : -(long long)A;
    const long long ta = w > 0 ? (long long)(Tw - (int64_t)A) : -(long long)(Tw - (int64_t)A);
    int n1 = cell + 1;
    if (per && n1 == T.N) n1 = 0;
    atomicAdd((unsigned long long*)&cx.rho[T.node_off + cell], (unsigned long long)ta);
    atomicAdd((unsigned long long*)&cx.rho[T.node_off + n1], (unsigned long long)a);
  }
}

// Live particles per tube: per-workgroup LDS counts (tubes < 1024), one
// global add per workgroup and tube.
template <class B>
__global__ __launch_bounds__(TPB) void k_count_live(B buf, const Ctl* ctl, const int32_t* chunk, const int32_t* tt,
                                                     const Tile* tiles, long long* out, int n_tubes,
                                                     const uint32_t* gate = nullptr) {
  if (gate != nullptr && *gate == 0) return;   // (a merge check that cannot merge)
  __shared__ int s_n[1024];
  for (int j = threadIdx.x; j < 1024; j += blockDim.x) s_n[j] = 0;
  __syncthreads();
  const long long nsc = ctl->n_sorted_chunks, S = nsc * CHUNK, tail = ctl->tail;
  const long long nsq = S / TPB, nq = nsq + (tail + TPB - 1) / TPB;
  for (long long c = blockIdx.x; c < nq; c += gridDim.x) {
    uint32_t slot; int tile;
    piece_slot(c, nsq, S, tail, chunk, tt, &slot, &tile);
    int t = (tile >= 0 && rec_alive<B>(buf, slot)) ? tiles[tile].tube : -1;
    while (true) {
      uint64_t m = __ballot(t >= 0);
      if (!m) break;
      int lead = __ffsll((long long)m) - 1;
      int k = __shfl(t, lead);
      uint64_t mk = __ballot(t == k);
      if (lane_id() == lead) {
        if (k < 1024) atomicAdd(&s_n[k], (int)__popcll(mk));
        else atomicAdd((unsigned long long*)&out[k], (unsigned long long)__popcll(mk));
      }
      if (t == k) t = -1;
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < 1024 && j < n_tubes; j += blockDim.x)
    if (s_n[j]) atomicAdd((unsigned long long*)&out[j], (unsigned long long)s_n[j]);
}

}  // namespace gap
