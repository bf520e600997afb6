// gap_diag.hpp -- discharge diagnostics of libgap (gfx950, wave64): the
// quantities the paper reads off its simulations (Sect. 5, Figs. 3, 5, 7).
//
//  * Profile (Fig. 3, rows 5-7): per bin of B cells and per group -- e- and
//    e+ moving up (u > 0) and down, photons with |x| > 2 moving up (x > 0)
//    and down -- the multiplicity m = n / n_co = sum |w| / (B ppc_ref) (a
//    weight-w macro-particle stands for w dx / ppc_ref particles per unit
//    area), the mean Lorentz factor <gamma> (photons: <|x|>) and the
//    plasma-inertia measure <gamma^-3> = n^-1 sum w gamma^-3 (its definition
//    with eq. omega_osc, Sect. 3).
//  * Peak (Fig. 5): the largest pair multiplicity m_+- (e- plus e+, both
//    directions) over the bins inside the gap zone h < H, the height of that
//    bin, <gamma^-3> of the pairs there, the photon multiplicity there, and
//    the extremes of E over the cells.
//  * Return spectrum (Fig. 7): the weight of the leptons absorbed at the
//    surface, binned in log10 gamma, filled by the lepton passes (gap_kernels).
//  * Waterfall (Fig. 4): the space-time diagram of E^2, the mean of E^2 over
//    bins of cells recorded after the field update of every k-th step.
//  * Power spectrum of E along the gap: the field zero-padded to M, the next
//    power of two >= N, transformed by a radix-2 Stockham FFT in FP64,
//    P_k = |X_k|^2 / M for k = 0 .. M/2.
#pragma once
#include "gap_kernels.hpp"

namespace gap {

constexpr int PROF_G = 6;   // groups: e- up, e- down, e+ up, e+ down, photons (|x| > 2) up, down
constexpr int PROF_M = 3;   // moments per group: sum |w|, sum |w| gamma (photons |x|), sum |w| gamma^-3

// Adds (v0, v1, v2) to acc[key * 3 + m] for every lane with key >= 0, one
// atomic per distinct key of the wave.
__device__ __forceinline__ void prof_wave_add(int key, double v0, double v1, double v2, double* acc) {
  while (true) {
    const uint64_t m = __ballot(key >= 0);
    if (!m) break;
    const int lead = __ffsll((long long)m) - 1;
    const int kk = __shfl(key, lead);
    double a = key == kk ? v0 : 0.0, b = key == kk ? v1 : 0.0, c = key == kk ? v2 : 0.0;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      a += __shfl_xor(a, d);
      b += __shfl_xor(b, d);
      c += __shfl_xor(c, d);
    }
    if (lane_id() == lead) {
      atomicAdd(&acc[(size_t)kk * PROF_M + 0], a);
      atomicAdd(&acc[(size_t)kk * PROF_M + 1], b);
      if (c != 0.0) atomicAdd(&acc[(size_t)kk * PROF_M + 2], c);
    }
    if (key == kk) key = -1;
  }
}

// Profile moments of one slot: key = bin * PROF_G + group (-1: none).
__device__ __forceinline__ int prof_moments(const Ctx& cx, bool lep, uint32_t slot, int tile, int tube, int B,
                                            double* v0, double* v1, double* v2) {
  *v0 = *v1 = *v2 = 0.0;
  if (tile < 0) return -1;
  const Tile tl = cx.tiles[tile];
  const float a = lep ? cx.L.w[slot] : cx.P.x[slot];
  if (tl.tube != tube || a == 0.0f) return -1;
  const Tube& T = cx.tubes[tube];
  const uint32_t pos = lep ? cx.L.pos[slot] : cx.P.pos[slot];
  int cell = tl.base + (int)(pos >> FRAC);
  if (T.flags & F_PERIODIC) cell = wrap_cell(cell, T.N);
  const int bin = min(max(cell, 0), T.N - 1) / B;
  if (lep) {
    const double u = (double)cx.L.u[slot];
    const double w = fabs((double)a);
    const double g = sqrt(1.0 + u * u);
    *v0 = w;
    *v1 = w * g;
    *v2 = w / (g * g * g);
    return bin * PROF_G + (a < 0.0f ? 0 : 2) + (u > 0.0 ? 0 : 1);
  }
  if (!(fabsf(a) > 2.0f)) return -1;
  const double w = (double)cx.P.w[slot];
  *v0 = w;
  *v1 = w * fabs((double)a);
  return bin * PROF_G + 4 + (a > 0.0f ? 0 : 1);
}

constexpr int PROF_LW = 80;   // LDS window of bins per workgroup (bins of >= 4 cells cover a tile's 256-cell window)

// Moments of tube `tube`'s particles into acc[nb][PROF_G][PROF_M], which the
// caller has zeroed.  Each workgroup takes a contiguous range of the sorted
// rows of each store (one slot per thread and 256-slot row): their particles
// lie within a tile's window, so with bins of at least 4 cells they are summed
// into an LDS window of bins (FP64 LDS atomics), flushed to acc when the tile
// changes and at the end; tail rows (and narrower bins) add to acc directly,
// one atomic per distinct key of a wave.
__global__ __launch_bounds__(TPB) void k_profile(Ctx cx, int tube, int B, int nb, double* acc) {
  __shared__ double s_w[PROF_LW * PROF_G * PROF_M];
  const bool win = B >= 4;
  for (int j = threadIdx.x; j < PROF_LW * PROF_G * PROF_M; j += blockDim.x) s_w[j] = 0.0;
  int lo = -1;                              // first bin of the LDS window (block-uniform)
  __syncthreads();
  for (int sp = 0; sp < 2; ++sp) {
    const bool lep = sp == 0;
    const Ctl* ctl = lep ? cx.lc : cx.pc;
    const long long S = ctl->n_sorted_chunks * CHUNK, tail = ctl->tail;
    const long long nsq = S / TPB, nq = nsq + (tail + TPB - 1) / TPB;
    const int32_t* chunk = lep ? cx.lchunk : cx.pchunk;
    const int32_t* tt = lep ? cx.ltt : cx.ptt;
    // sorted rows: a contiguous range per workgroup
    const long long r0 = nsq * blockIdx.x / gridDim.x, r1 = nsq * (blockIdx.x + 1) / gridDim.x;
    for (long long q = r0; q < r1; ++q) {
      uint32_t slot;
      int tile;
      piece_slot(q, nsq, S, tail, chunk, tt, &slot, &tile);
      double v0, v1, v2;
      const int key = prof_moments(cx, lep, slot, tile, tube, B, &v0, &v1, &v2);
      if (win) {
        // the row's tile (uniform: a sorted row lies in one chunk) sets the window
        const int wl = __builtin_amdgcn_readfirstlane(max(cx.tiles[tile].base, 0) / B);
        if (wl != lo) {
          __syncthreads();
          if (lo >= 0)
            for (int j = threadIdx.x; j < PROF_LW * PROF_G * PROF_M; j += blockDim.x) {
              const double v = s_w[j];
              if (v != 0.0) {
                const int bb = lo + j / (PROF_G * PROF_M);
                if (bb < nb) atomicAdd(&acc[(size_t)lo * PROF_G * PROF_M + j], v);
                s_w[j] = 0.0;
              }
            }
          lo = wl;
          __syncthreads();
        }
        const int kb = key >= 0 ? key / PROF_G - lo : -1;
        const bool in = kb >= 0 && kb < PROF_LW;
        if (in) {
          double* e = &s_w[((size_t)kb * PROF_G + key % PROF_G) * PROF_M];
          atomicAdd(&e[0], v0);
          atomicAdd(&e[1], v1);
          if (v2 != 0.0) atomicAdd(&e[2], v2);
        }
        prof_wave_add(in ? -1 : key, v0, v1, v2, acc);   // (every lane takes part)
      } else {
        prof_wave_add(key, v0, v1, v2, acc);
      }
    }
    // tail rows: strided over all workgroups
    for (long long q = nsq + blockIdx.x; q < nq; q += gridDim.x) {
      uint32_t slot;
      int tile;
      piece_slot(q, nsq, S, tail, chunk, tt, &slot, &tile);
      double v0, v1, v2;
      const int key = prof_moments(cx, lep, slot, tile, tube, B, &v0, &v1, &v2);
      prof_wave_add(key, v0, v1, v2, acc);
    }
  }
  __syncthreads();
  if (lo >= 0)
    for (int j = threadIdx.x; j < PROF_LW * PROF_G * PROF_M; j += blockDim.x) {
      const double v = s_w[j];
      if (v != 0.0 && lo + j / (PROF_G * PROF_M) < nb) atomicAdd(&acc[(size_t)lo * PROF_G * PROF_M + j], v);
    }
}

// Sums to the profile: out[nb][PROF_G][3] = multiplicity, <gamma> (photons
// <|x|>), <gamma^-3> (0 for photons and for empty groups).
__global__ void k_profile_finish(const double* acc, int nb, double bppc, double* out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nb * PROF_G; i += gridDim.x * blockDim.x) {
    const double w = acc[(size_t)i * PROF_M], wg = acc[(size_t)i * PROF_M + 1], wg3 = acc[(size_t)i * PROF_M + 2];
    out[(size_t)i * 3 + 0] = w / bppc;
    out[(size_t)i * 3 + 1] = w > 0.0 ? wg / w : 0.0;
    out[(size_t)i * 3 + 2] = w > 0.0 ? wg3 / w : 0.0;
  }
}

// Peak of the pair multiplicity over the bins whose centre lies in the gap
// zone (h < H), with ties to the lowest bin, and the field's extremes; one
// workgroup.  out: m_+- at the peak, the peak bin's centre height, <gamma^-3>
// of the pairs there, the photon multiplicity (|x| > 2) there, min E, max E.
constexpr int PEAK_T = 1024;   // one workgroup of 1024 threads

__global__ __launch_bounds__(PEAK_T) void k_profile_peak(const double* acc, int nb, int B, double dx, double H,
                                                         double bppc, const float* E, int N, double* out) {
  __shared__ double s_v[PEAK_T];
  __shared__ int s_i[PEAK_T];
  __shared__ double s_lo[PEAK_T], s_hi[PEAK_T];
  double best = -1.0;
  int arg = -1;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    if (!(((double)b + 0.5) * B * dx < H)) continue;
    double m = 0.0;
    for (int g = 0; g < 4; ++g) m += acc[((size_t)b * PROF_G + g) * PROF_M];
    if (m > best) { best = m; arg = b; }   // (b grows within a thread: the first of equal values stays)
  }
  // four independent loads per round
  double lo = 1e300, hi = -1e300;
  const int bd = blockDim.x;
  for (int k = threadIdx.x; k < N; k += 4 * bd) {
    float v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = k + u * bd < N ? E[k + u * bd] : E[k];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      lo = fmin(lo, (double)v[u]);
      hi = fmax(hi, (double)v[u]);
    }
  }
  s_v[threadIdx.x] = best;
  s_i[threadIdx.x] = arg;
  s_lo[threadIdx.x] = lo;
  s_hi[threadIdx.x] = hi;
  __syncthreads();
  for (int d = blockDim.x / 2; d >= 1; d >>= 1) {
    if ((int)threadIdx.x < d) {
      const double v = s_v[threadIdx.x + d];
      const int i = s_i[threadIdx.x + d];
      if (v > s_v[threadIdx.x] || (v == s_v[threadIdx.x] && i >= 0 && (s_i[threadIdx.x] < 0 || i < s_i[threadIdx.x]))) {
        s_v[threadIdx.x] = v;
        s_i[threadIdx.x] = i;
      }
      s_lo[threadIdx.x] = fmin(s_lo[threadIdx.x], s_lo[threadIdx.x + d]);
      s_hi[threadIdx.x] = fmax(s_hi[threadIdx.x], s_hi[threadIdx.x + d]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int b = s_i[0];
    double m = 0.0, g3 = 0.0, mx = 0.0;
    if (b >= 0) {
      double w = 0.0;
      for (int g = 0; g < 4; ++g) {
        w += acc[((size_t)b * PROF_G + g) * PROF_M];
        g3 += acc[((size_t)b * PROF_G + g) * PROF_M + 2];
      }
      m = w / bppc;
      g3 = w > 0.0 ? g3 / w : 0.0;
      mx = (acc[((size_t)b * PROF_G + 4) * PROF_M] + acc[((size_t)b * PROF_G + 5) * PROF_M]) / bppc;
    }
    out[0] = m;
    out[1] = b >= 0 ? ((double)b + 0.5) * B * dx : -1.0;
    out[2] = g3;
    out[3] = mx;
    out[4] = N > 0 ? s_lo[0] : 0.0;
    out[5] = N > 0 ? s_hi[0] : 0.0;
  }
}

// Waterfall record of the step that the field update just counted, when
// its index is a multiple of `every`: the mean of E^2 over each bin of B
// cells (the last bin ragged) goes to ring slot (step / every) mod cap of
// the tube, and the step index beside it.  One wave per bin, FP64 sums of
// squares of the FP32 field; grid (ceil(nbmax / waves per block), tubes).
struct WfCtx {
  const Tube* tubes;
  const float* E;
  double* ring;        // [tube][cap][nbmax]
  long long* steps;    // [tube][cap], -1 for an empty slot
  int every, B, cap, nbmax;
};

__global__ __launch_bounds__(TPB) void k_waterfall(WfCtx w) {
  const int t = blockIdx.y;
  const Tube& T = w.tubes[t];
  const long long step = T.step;
  if (step < 0 || step % w.every != 0) return;
  const int N = T.N;
  const int nb = (N + w.B - 1) / w.B;
  const long long slot = (step / w.every) % w.cap;
  const int bin = blockIdx.x * (TPB / WAVE) + (int)(threadIdx.x / WAVE);
  if (bin < nb) {
    const int c0 = bin * w.B, c1 = min(N, c0 + w.B);
    double s = 0.0;
    for (int c = c0 + lane_id(); c < c1; c += WAVE) {
      const double e = (double)w.E[T.cell_off + c];
      s += e * e;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d);
    if (lane_id() == 0) w.ring[((size_t)t * w.cap + slot) * w.nbmax + bin] = s / (double)(c1 - c0);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) w.steps[(size_t)t * w.cap + slot] = step;
}

// Power spectrum of E: load (zero-padded), log2 M Stockham stages (each
// output in natural order after the last), |X|^2 / M.  One thread per pair
// of the stage; every index is below M (M a power of two).
__global__ void k_fft_load(const float* E, int N, int M, double2* x) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < M; j += gridDim.x * blockDim.x)
    x[j] = make_double2(j < N ? (double)E[j] : 0.0, 0.0);
}

// Stage with sub-transforms of length Ns (1, 2, 4, ..., M/2): pair j takes
// in[j] and in[j + M/2], turns the second by exp(-i pi k / Ns) with
// k = j mod Ns, and writes the sum and difference Ns apart at 2 (j - k) + k.
__global__ void k_fft_stage(const double2* in, double2* out, int M, int Ns) {
  const int h = M / 2;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < h; j += gridDim.x * blockDim.x) {
    const int k = j & (Ns - 1);
    double s, c;
    sincospi(-(double)k / (double)Ns, &s, &c);
    const double2 a = in[j], b = in[j + h];
    const double2 t = make_double2(b.x * c - b.y * s, b.x * s + b.y * c);
    const int o = 2 * (j - k) + k;
    out[o] = make_double2(a.x + t.x, a.y + t.y);
    out[o + Ns] = make_double2(a.x - t.x, a.y - t.y);
  }
}

__global__ void k_fft_power(const double2* X, int M, double* P) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k <= M / 2; k += gridDim.x * blockDim.x)
    P[k] = (X[k].x * X[k].x + X[k].y * X[k].y) / (double)M;
}

// Momentum spectra (Fig. 3, row 1): the weight of electrons and positrons
// per 1/8 decade of |u| and of photons per 1/8 decade of |x|, from 1e-2 to
// 1e9, with an underflow and an overflow bin.  A value's bin is the number of
// edges 10^(-2 + b/8) (b = 0 .. 88) whose square its square reaches, taken
// in FP64 against a host-computed table of the squares (binary search).  Each
// workgroup sums into an LDS histogram over a strided set of 256-slot pieces
// of both stores and adds it to acc[3][SPEC_NB] once.
constexpr int SPEC_EDGES = 89;
constexpr int SPEC_NB = SPEC_EDGES + 1;

__device__ __forceinline__ int spec_bin(const double* thr, double p2) {
  int lo = 0, hi = SPEC_EDGES;              // count of edges <= p2, in [0, SPEC_EDGES]
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (thr[mid] <= p2) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(TPB) void k_spectra(Ctx cx, int tube, const double* thr, double* acc) {
  __shared__ double s_h[3 * SPEC_NB];
  __shared__ double s_thr[SPEC_EDGES];
  for (int j = threadIdx.x; j < 3 * SPEC_NB; j += blockDim.x) s_h[j] = 0.0;
  for (int j = threadIdx.x; j < SPEC_EDGES; j += blockDim.x) s_thr[j] = thr[j];
  __syncthreads();
  for (int sp = 0; sp < 2; ++sp) {
    const bool lep = sp == 0;
    const Ctl* ctl = lep ? cx.lc : cx.pc;
    const long long S = ctl->n_sorted_chunks * CHUNK, tail = ctl->tail;
    const long long nsq = S / TPB, nq = nsq + (tail + TPB - 1) / TPB;
    const int32_t* chunk = lep ? cx.lchunk : cx.pchunk;
    const int32_t* tt = lep ? cx.ltt : cx.ptt;
    for (long long q = blockIdx.x; q < nq; q += gridDim.x) {
      uint32_t slot;
      int tile;
      piece_slot(q, nsq, S, tail, chunk, tt, &slot, &tile);
      if (tile < 0 || cx.tiles[tile].tube != tube) continue;
      if (lep) {
        const float w = cx.L.w[slot];
        if (w == 0.0f) continue;
        const double u = (double)cx.L.u[slot];
        atomicAdd(&s_h[(w < 0.0f ? 0 : 1) * SPEC_NB + spec_bin(s_thr, u * u)], (double)fabsf(w));
      } else {
        const float x = cx.P.x[slot];
        if (x == 0.0f) continue;
        const double xd = (double)x;
        atomicAdd(&s_h[2 * SPEC_NB + spec_bin(s_thr, xd * xd)], (double)cx.P.w[slot]);
      }
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < 3 * SPEC_NB; j += blockDim.x)
    if (s_h[j] != 0.0) atomicAdd(&acc[j], s_h[j]);
}

// Phase space (Fig. 3, rows 1-4): the weights of the momentum spectra, per
// bin of B cells and signed momentum column (column SPEC_NB + b for p > 0,
// SPEC_NB - 1 - b for p <= 0, b the spectrum bin of |p|), added to
// acc[3][nb][2 SPEC_NB] with one atomic per distinct key of a wave.
constexpr int PHASE_NP = 2 * SPEC_NB;

__device__ __forceinline__ void phase_wave_add(long long key, double v, double* acc) {
  while (true) {
    const uint64_t m = __ballot(key >= 0);
    if (!m) break;
    const int lead = __ffsll((long long)m) - 1;
    const long long kk = __shfl(key, lead);
    double a = key == kk ? v : 0.0;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) a += __shfl_xor(a, d);
    if (lane_id() == lead) atomicAdd(&acc[kk], a);
    if (key == kk) key = -1;
  }
}

__global__ __launch_bounds__(TPB) void k_phase(Ctx cx, int tube, int B, int nb, const double* thr, double* acc) {
  __shared__ double s_thr[SPEC_EDGES];
  for (int j = threadIdx.x; j < SPEC_EDGES; j += blockDim.x) s_thr[j] = thr[j];
  __syncthreads();
  const Tube& T = cx.tubes[tube];
  for (int sp = 0; sp < 2; ++sp) {
    const bool lep = sp == 0;
    const Ctl* ctl = lep ? cx.lc : cx.pc;
    const long long S = ctl->n_sorted_chunks * CHUNK, tail = ctl->tail;
    const long long nsq = S / TPB, nq = nsq + (tail + TPB - 1) / TPB;
    const int32_t* chunk = lep ? cx.lchunk : cx.pchunk;
    const int32_t* tt = lep ? cx.ltt : cx.ptt;
    for (long long q = blockIdx.x; q < nq; q += gridDim.x) {
      uint32_t slot;
      int tile;
      piece_slot(q, nsq, S, tail, chunk, tt, &slot, &tile);
      long long key = -1;
      double v = 0.0;
      if (tile >= 0 && cx.tiles[tile].tube == tube) {
        const float a = lep ? cx.L.w[slot] : cx.P.x[slot];
        if (a != 0.0f) {
          const Tile tl = cx.tiles[tile];
          const uint32_t pos = lep ? cx.L.pos[slot] : cx.P.pos[slot];
          int cell = tl.base + (int)(pos >> FRAC);
          if (T.flags & F_PERIODIC) cell = wrap_cell(cell, T.N);
          cell = min(max(cell, 0), T.N - 1);
          const double p = lep ? (double)cx.L.u[slot] : (double)a;
          const int b = spec_bin(s_thr, p * p);
          const int col = p > 0.0 ? SPEC_NB + b : SPEC_NB - 1 - b;
          const int s3 = lep ? (a < 0.0f ? 0 : 1) : 2;
          key = ((long long)s3 * nb + cell / B) * PHASE_NP + col;
          v = lep ? (double)fabsf(a) : (double)cx.P.w[slot];
        }
      }
      phase_wave_add(key, v, acc);
    }
  }
}

}  // namespace gap
