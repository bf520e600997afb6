// gap_protons.hpp -- the proton species (Sect. 6.1: electrons, positrons and
// protons with m_p/m_e = 1836; protons take no part in the QED processes).
// Protons exist only in tubes with a thermal atmosphere or the proton initial
// state, and are few next to the leptons, so they live in one flat array per
// handle, each lane pushing one proton with global gather and deposit; dead
// slots are squeezed out at every re-sort.
#pragma once
#include "gap_kernels.hpp"

namespace gap {

// Kick du/dt = E / 1836 (charge +1), drift dh/dt = u / gamma in the same
// 2^-24 fixed point as the leptons, absorption at h = 0 (the charge returns
// to the star), free outflow at h = L, deposit of the first-order split.
// Protons left in cell 0 are counted for the atmosphere refill.
__global__ __launch_bounds__(TPB) void k_protons(Ctx cx) {
  const long long n = min(*cx.pr_n, cx.pr_cap);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float w = cx.R.w[i];
    if (w == 0.0f) continue;
    const int t = cx.R.tube[i];
    Tube& T = cx.tubes[t];
    const int N = T.N;
    const bool per = (T.flags & F_PERIODIC) != 0;
    const int cell = cx.R.cell[i];
    const uint32_t frac = cx.R.frac[i];
    float u = cx.R.u[i];
    const float xi = (float)frac * 5.9604645e-8f;
    const float e0 = cx.ebar[T.node_off + cell], e1 = cx.ebar[T.node_off + cell + 1];
    u += ((1.0f - xi) * e0 + xi * e1) * T.dt * (1.0f / MASS_P);
    const int dfix = __float2int_rn(u * __builtin_amdgcn_rsqf(1.0f + u * u) * T.cfl24);
    const long long np = ((long long)cell << FRAC) + (long long)frac + dfix;
    int ncell = (int)(np >> FRAC);
    const uint32_t nfrac = (uint32_t)np & 0xFFFFFFu;
    const int64_t Tw = __float2ll_rn(fabsf(w) * 16777216.0f);
    if (per) {
      ncell = wrap_cell(ncell, N);
      atomic_add_i64(&T.dcur, Tw * (int64_t)dfix);
    } else if (ncell < 0 || ncell >= N) {
      cx.R.w[i] = 0.0f;
      if (ncell < 0) {
        atomic_add_i64(&T.dq, Tw);
        atomic_add_i64(&T.cnt[C_PRO_ABSORBED], 1);
      } else {
        atomic_add_i64(&T.cnt[C_PRO_OUTFLOW], 1);
      }
      atomic_add_i64(&T.cnt[C_PROTONS], -1);
      continue;
    }
    const long long A = (long long)(((unsigned long long)Tw * nfrac + (1ull << 23)) >> FRAC);
    int n1 = ncell + 1;
    if (per && n1 == N) n1 = 0;
    atomicAdd((unsigned long long*)&cx.rho[T.node_off + ncell], (unsigned long long)(Tw - A));
    atomicAdd((unsigned long long*)&cx.rho[T.node_off + n1], (unsigned long long)A);
    if (ncell == 0) atomicAdd(&T.atm_cnt[2 + (int)(T.step & 1)], 1);
    cx.R.cell[i] = ncell;
    cx.R.frac[i] = nfrac;
    cx.R.u[i] = u;
  }
}

// Charge of every live proton into rho (initial field, loaded states).
__global__ __launch_bounds__(TPB) void k_deposit_protons(Ctx cx) {
  const long long n = min(*cx.pr_n, cx.pr_cap);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float w = cx.R.w[i];
    if (w == 0.0f) continue;
    const Tube& T = cx.tubes[cx.R.tube[i]];
    const int cell = cx.R.cell[i];
    const int64_t Tw = __float2ll_rn(fabsf(w) * 16777216.0f);
    const long long A = (long long)(((unsigned long long)Tw * cx.R.frac[i] + (1ull << 23)) >> FRAC);
    int n1 = cell + 1;
    if ((T.flags & F_PERIODIC) && n1 == T.N) n1 = 0;
    atomicAdd((unsigned long long*)&cx.rho[T.node_off + cell], (unsigned long long)(Tw - A));
    atomicAdd((unsigned long long*)&cx.rho[T.node_off + n1], (unsigned long long)A);
  }
}

// Initial protons (proton initial state): ppc per cell in cells [0, k_h) of
// each such tube, ids continuing after the tube's initial electrons, positions
// from draw(seed, id, 0, T_INIT, 0) like those.
struct ProInit {
  const Tube* tubes;
  ProBuf R;
  const long long* off;      // first slot of each tube's protons (n_tubes + 1)
  const int32_t* ppc;
  const int64_t* id0;        // id of the tube's first proton
  int n_tubes;
};

__global__ void k_init_protons(ProInit ic) {
  const long long tot = ic.off[ic.n_tubes];
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += (long long)gridDim.x * blockDim.x) {
    int lo = 0, hi = ic.n_tubes;
    while (hi - lo > 1) { const int mid = (lo + hi) >> 1; if (ic.off[mid] <= i) lo = mid; else hi = mid; }
    const int t = lo;
    const long long li = i - ic.off[t];
    const uint64_t id = (uint64_t)ic.id0[t] + (uint64_t)li;
    const u4 r = draw(ic.tubes[t].seed, id, 0, T_INIT, 0);
    ic.R.cell[i] = (int32_t)(li / ic.ppc[t]);
    ic.R.frac[i] = r.a >> 8;
    ic.R.u[i] = 0.0f;
    ic.R.w[i] = 1.0f;
    ic.R.id[i] = id;
    ic.R.tube[i] = t;
  }
}

// Squeeze the dead slots out (one workgroup, order kept): src -> dst, *n the
// new count.
constexpr int PRO_COMPACT_THREADS = 1024;
__global__ __launch_bounds__(PRO_COMPACT_THREADS) void k_pro_compact(ProBuf src, ProBuf dst, long long* n_io,
                                                                      long long cap) {
  __shared__ int s_wave[PRO_COMPACT_THREADS / WAVE];
  const long long n = min(*n_io, cap);
  long long base = 0;
  for (long long c0 = 0; c0 < n; c0 += PRO_COMPACT_THREADS) {
    const long long i = c0 + threadIdx.x;
    const bool alive = i < n && src.w[i] != 0.0f;
    const uint64_t m = __ballot(alive);
    const int wv = threadIdx.x / WAVE;
    if (lane_id() == 0) s_wave[wv] = __popcll(m);
    __syncthreads();
    int before = 0, total = 0;
    for (int k = 0; k < PRO_COMPACT_THREADS / WAVE; ++k) {
      if (k < wv) before += s_wave[k];
      total += s_wave[k];
    }
    if (alive) {
      const long long j = base + before + rank_in(m);
      dst.cell[j] = src.cell[i];
      dst.frac[j] = src.frac[i];
      dst.u[j] = src.u[i];
      dst.w[j] = src.w[i];
      dst.id[j] = src.id[i];
      dst.tube[j] = src.tube[i];
    }
    base += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) *n_io = base;
}

}  // namespace gap
