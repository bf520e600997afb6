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

// Moments of tube `tube`'s particles (sorted regions and tails of both
// stores, one slot per thread and 256-slot row) into acc[nb][PROF_G][PROF_M],
// which the caller has zeroed.
__global__ __launch_bounds__(TPB) void k_profile(Ctx cx, int tube, int B, int nb, double* acc) {
  const long long Sl = cx.lc->n_sorted_chunks * CHUNK, tl_ = cx.lc->tail;
  const long long Sp = cx.pc->n_sorted_chunks * CHUNK, tp_ = cx.pc->tail;
  const long long nql = (Sl + tl_ + TPB - 1) / TPB, nqp = (Sp + tp_ + TPB - 1) / TPB;
  for (long long q = blockIdx.x; q < nql + nqp; q += gridDim.x) {
    const bool lep = q < nql;
    const long long qq = lep ? q : q - nql;
    const long long S = lep ? Sl : Sp, tail = lep ? tl_ : tp_;
    uint32_t slot;
    int tile;
    piece_slot(qq, S / TPB, S, tail, lep ? cx.lchunk : cx.pchunk, lep ? cx.ltt : cx.ptt, &slot, &tile);
    int key = -1;
    double v0 = 0.0, v1 = 0.0, v2 = 0.0;
    if (tile >= 0) {
      const Tile tl = cx.tiles[tile];
      const float a = lep ? cx.L.w[slot] : cx.P.x[slot];
      if (tl.tube == tube && a != 0.0f) {
        const Tube& T = cx.tubes[tube];
        const uint32_t pos = lep ? cx.L.pos[slot] : cx.P.pos[slot];
        int cell = tl.base + (int)(pos >> FRAC);
        if (T.flags & F_PERIODIC) cell = wrap_cell(cell, T.N);
        const int bin = min(max(cell, 0), T.N - 1) / B;
        if (lep) {
          const double u = (double)cx.L.u[slot];
          const double w = fabs((double)a);
          const double g = sqrt(1.0 + u * u);
          const int grp = (a < 0.0f ? 0 : 2) + (u > 0.0 ? 0 : 1);
          key = bin * PROF_G + grp;
          v0 = w;
          v1 = w * g;
          v2 = w / (g * g * g);
        } else if (fabsf(a) > 2.0f) {
          const double w = (double)cx.P.w[slot];
          key = bin * PROF_G + 4 + (a > 0.0f ? 0 : 1);
          v0 = w;
          v1 = w * fabs((double)a);
        }
      }
    }
    prof_wave_add(key, v0, v1, v2, acc);
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
__global__ void k_profile_peak(const double* acc, int nb, int B, double dx, double H, double bppc,
                               const float* E, int N, double* out) {
  __shared__ double s_v[TPB];
  __shared__ int s_i[TPB];
  __shared__ double s_lo[TPB], s_hi[TPB];
  double best = -1.0;
  int arg = -1;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    if (!(((double)b + 0.5) * B * dx < H)) continue;
    double m = 0.0;
    for (int g = 0; g < 4; ++g) m += acc[((size_t)b * PROF_G + g) * PROF_M];
    if (m > best) { best = m; arg = b; }   // (b grows within a thread: the first of equal values stays)
  }
  double lo = 1e300, hi = -1e300;
  for (int k = threadIdx.x; k < N; k += blockDim.x) {
    const double e = (double)E[k];
    lo = fmin(lo, e);
    hi = fmax(hi, e);
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

}  // namespace gap
