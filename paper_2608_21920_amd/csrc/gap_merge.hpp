// gap_merge.hpp -- weight-doubling merge of over-full stores: a stable LSD
// radix sort of (group key, id) written for this library, and the pairing
// kernel.  Groups are (cell, charge sign, direction, floor(log2 gamma)) for
// leptons and (cell, direction, floor(log2 x)) for photons; within a group
// consecutive particles in id order fuse pairwise, the survivor (one random
// bit of Philox(seed; id of the first, step, MERGE)) taking both weights.
#pragma once
#include "gap_kernels.hpp"

namespace gap {

constexpr int RS_TPB = 256;
constexpr int RS_TILES = 64;                    // 256-item tiles per block
constexpr int RS_ITEMS = RS_TPB * RS_TILES;     // items per block

struct SortBuf {
  uint32_t* major[2];   // group key
  uint64_t* id[2];      // minor key
  uint32_t* val[2];     // slot of the record
  uint32_t* bhist;      // [256][nblocks] digit counts per block
  uint32_t* dtot;       // [256] items per digit
  long long* live;      // per tube: live particles of the store
  uint32_t* start;      // per item: first index of its group
  uint32_t* bmax;       // per block of the max-scan: its maximum, then its carry
  uint32_t* flags;      // per tube: merge this step
  uint32_t* gate;       // [0]: 0 when no tube of the store can be over its threshold; [1]: some tube is flagged
  long long* n;         // number of items
  int max_blocks;
};

// floor(log2 v) + 64 clamped to [0, 127] from the FP64 exponent (v >= 1 here)
__device__ __forceinline__ uint32_t lg2bin_d(double v) {
  const int e = (int)((__double_as_longlong(v) >> 52) & 0x7FF) - 1023;
  const int b = e + 64;
  return (uint32_t)(b < 0 ? 0 : (b > 127 ? 127 : b));
}
__device__ __forceinline__ uint32_t rec_group(const LepBuf& b, uint32_t slot, uint32_t gcell) {
  const double u = (double)b.u[slot];
  const double g = sqrt(1.0 + u * u);
  return (gcell << 9) | ((b.w[slot] > 0.0f ? 1u : 0u) << 8) | ((u >= 0.0 ? 1u : 0u) << 7) | lg2bin_d(g);
}
__device__ __forceinline__ uint32_t rec_group(const PhoBuf& b, uint32_t slot, uint32_t gcell) {
  const float x = b.x[slot];
  return (gcell << 9) | ((x >= 0.0f ? 1u : 0u) << 7) | lg2bin_d(fabs((double)x));
}

// Gate of a merge check: the occupied slots of a store (sorted region plus
// tail) bound the live particles of all its tubes together, so a store whose
// occupancy stays at or below the smallest tube threshold holds no tube over
// its threshold.  The check's counting and gathering kernels then return at
// once (and the sort passes find nothing to sort).
__global__ void k_merge_gate(const Ctl* ctl, double thresh_min, uint32_t* gate) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    gate[0] = (double)(ctl->n_sorted_chunks * CHUNK + ctl->tail) > thresh_min ? 1u : 0u;
    gate[1] = 0u;
  }
}

// Per-tube decision: merge when the live count exceeds merge_frac * cap.
__global__ void k_merge_flags(const long long* live, const double* thresh, uint32_t* flags, int n_tubes,
                              uint32_t* gate) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n_tubes) {
    const bool f = gate[0] != 0 && (double)live[t] > thresh[t];
    flags[t] = f ? 1u : 0u;
    if (f) atomicOr(&gate[1], 1u);
  }
}

// Gather the merge candidates (live particles of flagged tubes) with their
// keys.  The order of the gathered list does not matter: the sort's full key
// (group, id) is unique.  With no tube flagged it returns at once (the store
// may be over the smallest threshold without any tube over its own; reading
// every particle for nothing took a millisecond in the QED-active
// ensemble).  A workgroup takes MK_PIECES pieces of TPB slots at
// a time and reserves their entries with one atomic on the list counter.
// (One atomic per wave and piece, on the one counter, cost the photon store
// of the QED-active ensemble 10 ms per merge.)
constexpr int MK_PIECES = 8;
template <class B>
__global__ __launch_bounds__(TPB) void k_merge_keys(B buf, const Ctl* ctl, const int32_t* chunk, const int32_t* tt,
                                                    const Tile* tiles, const Tube* tubes, SortBuf sb) {
  if (sb.gate[1] == 0) return;
  __shared__ int s_w[TPB / WAVE];
  __shared__ long long s_base;
  const long long nsc = ctl->n_sorted_chunks, S = nsc * CHUNK, tail = ctl->tail;
  const long long nsq = S / TPB, nq = nsq + (tail + TPB - 1) / TPB;
  const int wv = (int)threadIdx.x / WAVE;
  for (long long q0 = (long long)blockIdx.x * MK_PIECES; q0 < nq; q0 += (long long)gridDim.x * MK_PIECES) {
    bool take[MK_PIECES];
    uint32_t key[MK_PIECES], slot[MK_PIECES];
    int before[MK_PIECES];
    int wtot = 0;
#pragma unroll
    for (int u = 0; u < MK_PIECES; ++u) {
      take[u] = false;
      key[u] = 0;
      slot[u] = 0;
      if (q0 + u < nq) {
        int tile;
        piece_slot(q0 + u, nsq, S, tail, chunk, tt, &slot[u], &tile);
        if (tile >= 0 && rec_alive<B>(buf, slot[u])) {
          const Tile tl = tiles[tile];
          const Tube& T = tubes[tl.tube];
          if (sb.flags[tl.tube]) {
            int cell = tl.base + (int)(buf.pos[slot[u]] >> FRAC);
            if (T.flags & F_PERIODIC) cell = wrap_cell(cell, T.N);
            const uint32_t gcell = (uint32_t)(T.cell_off + cell);
            key[u] = rec_group(buf, slot[u], gcell);
            take[u] = true;
          }
        }
      }
      const uint64_t m = __ballot(take[u]);
      before[u] = wtot + (int)rank_in(m);
      wtot += (int)__popcll(m);
    }
    if (lane_id() == 0) s_w[wv] = wtot;
    __syncthreads();
    int off = 0, total = 0;
#pragma unroll
    for (int w = 0; w < TPB / WAVE; ++w) {
      off += w < wv ? s_w[w] : 0;
      total += s_w[w];
    }
    if (threadIdx.x == 0)
      s_base = total ? (long long)atomicAdd((unsigned long long*)sb.n, (unsigned long long)total) : 0;
    __syncthreads();
    const long long base = s_base + off;
#pragma unroll
    for (int u = 0; u < MK_PIECES; ++u) {
      if (take[u]) {
        const long long i = base + before[u];
        sb.major[0][i] = key[u];
        sb.id[0][i] = buf.id[slot[u]];
        sb.val[0][i] = slot[u];
      }
    }
    __syncthreads();   // (s_w and s_base are rewritten by the next round)
  }
}

// digit d of the composite key (passes 0..7: id bytes, 8..11: group bytes)
__device__ __forceinline__ uint32_t rs_digit(uint32_t major, uint64_t id, int pass) {
  return pass < 8 ? (uint32_t)(id >> (8 * pass)) & 0xFFu : (major >> (8 * (pass - 8))) & 0xFFu;
}

__global__ __launch_bounds__(RS_TPB) void k_rs_hist(SortBuf sb, int src, int pass) {
  __shared__ uint32_t h[256];
  const long long n = *sb.n;
  const int nb = (int)((n + RS_ITEMS - 1) / RS_ITEMS);
  h[threadIdx.x] = 0;
  __syncthreads();
  for (int b = blockIdx.x; b < nb; b += gridDim.x) {
    const long long i0 = (long long)b * RS_ITEMS;
    for (int k = threadIdx.x; k < RS_ITEMS; k += RS_TPB) {
      const long long i = i0 + k;
      if (i < n) atomicAdd(&h[rs_digit(sb.major[src][i], sb.id[src][i], pass)], 1u);
    }
    __syncthreads();
    sb.bhist[(long long)threadIdx.x * sb.max_blocks + b] = h[threadIdx.x];
    h[threadIdx.x] = 0;
    __syncthreads();
  }
}

// Exclusive scan of each digit's row of bhist, RS_SCAN_WG workgroups taking
// every RS_SCAN_WG-th digit: bhist[d][b] becomes the number of items with
// digit d in the blocks before b, and dtot[d] the number of items with digit
// d.  A thread takes a run of consecutive blocks, so a row is read twice and
// written once.  (One workgroup over all 256 rows took a quarter of a
// millisecond per pass at 3e8 items; a workgroup per digit cost a gated
// merge check, which finds nothing to sort, 3 us per launch.)  Workgroups
// of RS_SCAN_T threads start beside the other store's sort kernels, which
// run at the same time on the second stream; 1024-thread ones waited up to
// 0.8 ms for an idle CU in the QED-active ensemble.
constexpr int RS_SCAN_WG = 64;
constexpr int RS_SCAN_T = 256;
__global__ __launch_bounds__(RS_SCAN_T) void k_rs_scan(SortBuf sb) {
  __shared__ uint32_t sh[RS_SCAN_T / WAVE];
  const long long n = *sb.n;
  const int nb = (int)((n + RS_ITEMS - 1) / RS_ITEMS);
  if (nb == 0) {
    for (int d = (int)blockIdx.x; d < 256; d += gridDim.x)
      if (threadIdx.x == 0) sb.dtot[d] = 0;
    return;
  }
  const int per = (nb + RS_SCAN_T - 1) / RS_SCAN_T;
  const int b0 = min(nb, (int)threadIdx.x * per), b1 = min(nb, b0 + per);
  const int wv = (int)threadIdx.x / WAVE;
  for (int d = (int)blockIdx.x; d < 256; d += gridDim.x) {
    uint32_t* row = sb.bhist + (long long)d * sb.max_blocks;
    uint32_t s = 0;
    for (int b = b0; b < b1; ++b) s += row[b];
    uint32_t incl = s;
#pragma unroll
    for (int k = 1; k < WAVE; k <<= 1) {
      const uint32_t o = __shfl_up(incl, k);
      if (lane_id() >= k) incl += o;
    }
    if (lane_id() == WAVE - 1) sh[wv] = incl;
    __syncthreads();
    uint32_t before = 0;
    for (int w = 0; w < wv; ++w) before += sh[w];
    uint32_t run = before + incl - s;
    for (int b = b0; b < b1; ++b) {
      const uint32_t v = row[b];
      row[b] = run;
      run += v;
    }
    if (threadIdx.x == RS_SCAN_T - 1) sb.dtot[d] = run;
    __syncthreads();
  }
}

// Stable scatter: items keep their order among equal digits.  Each block
// walks its items in 256-item tiles; a lane's rank is the number of earlier
// items of its block with the same digit.
__global__ __launch_bounds__(RS_TPB) void k_rs_scatter(SortBuf sb, int src, int pass) {
  static_assert(RS_TPB == 256, "one thread per digit");
  __shared__ uint32_t run[256];          // per digit: next output position of this block
  __shared__ uint32_t wcnt[RS_TPB / WAVE][256];
  __shared__ uint32_t dbase[256];        // per digit: items with smaller digits
  const long long n = *sb.n;
  const int nb = (int)((n + RS_ITEMS - 1) / RS_ITEMS);
  if (nb <= (int)blockIdx.x) return;
  const int dst = src ^ 1;
  const int w = threadIdx.x / WAVE;
  const uint64_t lt = (1ull << lane_id()) - 1ull;
  {
    const uint32_t v = sb.dtot[threadIdx.x];
    uint32_t incl = v;
#pragma unroll
    for (int k = 1; k < WAVE; k <<= 1) {
      const uint32_t o = __shfl_up(incl, k);
      if (lane_id() >= k) incl += o;
    }
    if (lane_id() == WAVE - 1) wcnt[0][w] = incl;
    __syncthreads();
    uint32_t before = 0;
    for (int ww = 0; ww < w; ++ww) before += wcnt[0][ww];
    dbase[threadIdx.x] = before + incl - v;
    __syncthreads();
  }
  for (int b = blockIdx.x; b < nb; b += gridDim.x) {
    run[threadIdx.x] = dbase[threadIdx.x] + sb.bhist[(long long)threadIdx.x * sb.max_blocks + b];
    __syncthreads();
    const long long i0 = (long long)b * RS_ITEMS;
    for (int tile = 0; tile < RS_TILES; ++tile) {
      const long long i = i0 + (long long)tile * RS_TPB + threadIdx.x;
      const bool ok = i < n;
      uint32_t mj = 0, v = 0;
      uint64_t id = 0;
      uint32_t d = 256;
      if (ok) { mj = sb.major[src][i]; id = sb.id[src][i]; v = sb.val[src][i]; d = rs_digit(mj, id, pass); }
      // lanes of this wave with the same digit
      uint64_t same = __ballot(ok);
#pragma unroll
      for (int bit = 0; bit < 8; ++bit) {
        const uint64_t bb = __ballot(ok && ((d >> bit) & 1u));
        same &= ((d >> bit) & 1u) ? bb : ~bb;
      }
      if (!ok) same = 0;
      for (int k = threadIdx.x; k < (RS_TPB / WAVE) * 256; k += RS_TPB) (&wcnt[0][0])[k] = 0;
      __syncthreads();
      // the highest lane of each digit group records the group size
      if (ok && (same >> lane_id()) == 1ull) wcnt[w][d] = (uint32_t)__popcll(same);
      __syncthreads();
      if (ok) {
        uint32_t before = run[d] + (uint32_t)__popcll(same & lt);
        for (int ww = 0; ww < w; ++ww) before += wcnt[ww][d];
        const long long o = (long long)before;
        sb.major[dst][o] = mj;
        sb.id[dst][o] = id;
        sb.val[dst][o] = v;
      }
      __syncthreads();
      {
        uint32_t add = 0;
        for (int ww = 0; ww < RS_TPB / WAVE; ++ww) add += wcnt[ww][threadIdx.x];
        run[threadIdx.x] += add;
      }
      __syncthreads();
    }
  }
}

// Pairing: the k-th particle of a group (in id order) pairs with the (k+1)-th
// when k is even; k = i - (first index of the group), the first index coming
// from a max-scan of the group starts.
__global__ void k_merge_bounds(SortBuf sb, int src, uint32_t* start) {
  const long long n = *sb.n;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    start[i] = (i == 0 || sb.major[src][i] != sb.major[src][i - 1]) ? (uint32_t)i : 0u;
}

// Inclusive max-scan of start[] in place, in three launches over blocks of
// MX_ITEMS entries: each block's maximum, an exclusive max-scan of those (one
// workgroup, over n / MX_ITEMS values), and each block's own scan from that
// carry.  (One workgroup over all n entries took milliseconds per merge of
// 1e8 candidates.)
constexpr int MX_TILES = 16;
constexpr int MX_ITEMS = RS_TPB * MX_TILES;

__global__ __launch_bounds__(RS_TPB) void k_mx_reduce(SortBuf sb, const uint32_t* start, uint32_t* bmax) {
  __shared__ uint32_t sh[RS_TPB / WAVE];
  const long long n = *sb.n;
  const int nb = (int)((n + MX_ITEMS - 1) / MX_ITEMS);
  for (int b = blockIdx.x; b < nb; b += gridDim.x) {
    uint32_t m = 0;
    for (int k = threadIdx.x; k < MX_ITEMS; k += RS_TPB) {
      const long long i = (long long)b * MX_ITEMS + k;
      if (i < n) m = max(m, start[i]);
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, d));
    if (lane_id() == 0) sh[threadIdx.x / WAVE] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t t = 0;
      for (int w = 0; w < RS_TPB / WAVE; ++w) t = max(t, sh[w]);
      bmax[b] = t;
    }
    __syncthreads();
  }
}

// Exclusive max-scan of bmax[0, nb) in place (one workgroup).
__global__ __launch_bounds__(1024) void k_mx_carry(SortBuf sb, uint32_t* bmax) {
  __shared__ uint32_t sh[1024 / WAVE];
  const long long n = *sb.n;
  const int nb = (int)((n + MX_ITEMS - 1) / MX_ITEMS);
  uint32_t carry = 0;
  for (int base = 0; base < nb; base += 1024) {
    const int i = base + (int)threadIdx.x;
    const uint32_t v = i < nb ? bmax[i] : 0u;
    uint32_t incl = v;
#pragma unroll
    for (int k = 1; k < WAVE; k <<= 1) {
      const uint32_t o = (uint32_t)__shfl_up((int)incl, k);
      if (lane_id() >= k) incl = max(incl, o);
    }
    const int wv = threadIdx.x / WAVE;
    if (lane_id() == WAVE - 1) sh[wv] = incl;
    __syncthreads();
    uint32_t pre = carry;
    for (int ww = 0; ww < wv; ++ww) pre = max(pre, sh[ww]);
    // exclusive: the maximum of everything before entry i
    const uint32_t up = (uint32_t)__shfl_up((int)incl, 1);
    const uint32_t ex = lane_id() == 0 ? pre : max(pre, up);
    uint32_t tot = carry;
    for (int ww = 0; ww < 1024 / WAVE; ++ww) tot = max(tot, sh[ww]);
    __syncthreads();
    if (i < nb) bmax[i] = ex;
    carry = tot;
  }
}

__global__ __launch_bounds__(RS_TPB) void k_mx_apply(SortBuf sb, uint32_t* start, const uint32_t* bcarry) {
  __shared__ uint32_t sh[RS_TPB / WAVE];
  const long long n = *sb.n;
  const int nb = (int)((n + MX_ITEMS - 1) / MX_ITEMS);
  for (int b = blockIdx.x; b < nb; b += gridDim.x) {
    uint32_t carry = bcarry[b];
    for (int tile = 0; tile < MX_TILES; ++tile) {
      const long long i = (long long)b * MX_ITEMS + (long long)tile * RS_TPB + threadIdx.x;
      const uint32_t v = i < n ? start[i] : 0u;
      uint32_t incl = v;
#pragma unroll
      for (int k = 1; k < WAVE; k <<= 1) {
        const uint32_t o = (uint32_t)__shfl_up((int)incl, k);
        if (lane_id() >= k) incl = max(incl, o);
      }
      const int wv = threadIdx.x / WAVE;
      if (lane_id() == WAVE - 1) sh[wv] = incl;
      __syncthreads();
      uint32_t pre = carry, tot = carry;
      for (int ww = 0; ww < RS_TPB / WAVE; ++ww) {
        if (ww < wv) pre = max(pre, sh[ww]);
        tot = max(tot, sh[ww]);
      }
      if (i < n) start[i] = max(pre, incl);
      __syncthreads();
      carry = tot;
    }
  }
}

template <class B>
__global__ void k_merge_pairs(B buf, SortBuf sb, int src, const uint32_t* start, const Tube* tubes, const Tile* tiles,
                              const int32_t* chunk, const int32_t* tt, const Ctl* ctl, long long* shard) {
  const long long n = *sb.n;
  const long long nsorted_slots = ctl->n_sorted_chunks * CHUNK;
  // (the loop bound is uniform over the workgroup, so that the per-tube
  // count below is taken with every lane of the wave active)
  for (long long i0 = (long long)blockIdx.x * blockDim.x; i0 + 1 < n; i0 += (long long)gridDim.x * blockDim.x) {
    const long long i = i0 + threadIdx.x;
    int t = -1;
    if (i + 1 < n && sb.major[src][i + 1] == sb.major[src][i] && ((i - (long long)start[i]) & 1) == 0) {
      const uint32_t sa = sb.val[src][i], sbb = sb.val[src][i + 1];
      const int tile = sa < nsorted_slots ? chunk[sa / CHUNK] : tt[sa];
      t = tiles[tile].tube;
      const Tube& T = tubes[t];
      const u4 r = draw(T.seed, sb.id[src][i], T.step, T_MERGE, 0);
      const uint32_t keep = (r.a & 1u) ? sbb : sa, drop = (r.a & 1u) ? sa : sbb;
      buf.w[keep] += buf.w[drop];
      rec_kill(buf, drop);
    }
    count_by_tube(shard, t, C_MERGED, 1);
  }
}

}  // namespace gap
