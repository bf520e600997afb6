// gap_adjoint.hpp -- reverse pass of the particle loop over a window with the
// QED realisation frozen: every emission is a constant recoil offset on its
// lepton, and photons and pairs born inside the window are constants.  The
// differentiated map is the push and the field of one step (Sect. 4 kick and
// drift, Sect. 2.2 Gauss integration from the surface field E_s, which the
// Ampere drive alpha j_co advances):
//   E_{j+1/2} = E_s + w0 sum_{i<=j} rho_i - background,  rho from the
//   first-order split (w (1 - xi) on node k, w xi on node k + 1);
//   u' = u + sign(w) E_p dt, E_p = (1 - xi) Eb_k + xi Eb_{k+1};
//   u'' = u' - x (recorded recoil);  xi' = xi + cfl u'' / sqrt(1 + u''^2);
//   E_s' = E_s + w0 (absorbed w + injected |w|) + alpha s_co dt.
// The fixed-point rounding of the deposit and drift is taken as the identity.
//
// Within a checkpoint segment no re-sort runs, so a lepton keeps its slot;
// the tape holds each slot's position and momentum at the start of every
// step (TAPE_DEAD for empty or dead slots) and the node field each step used.
#pragma once
#include "gap_kernels.hpp"

namespace gap {

constexpr uint32_t TAPE_DEAD = 0xFFFFFFFFu;

struct AdjTube {            // per tube (device)
  double lamEs;             // adjoint of the surface field
  double dalpha;            // dL/dalpha
  double dinjw;             // dL/d(weight of one injected electron)
  // w0 sum_k lamE_k summed over the reverse steps taken so far: the part of
  // every live lepton's weight adjoint that does not depend on its cell.
  // The slots hold their weight adjoints less this sum (FP32 then keeps the
  // small cell-dependent rest, and an injected electron's -lam_w + lamEs w0,
  // a near cancellation of two large sums, is formed in FP64).
  double cw;
  double w0, s_co, dt, cfl, lossw;   // lossw = 2 / (window steps * N)
  int32_t N, cell_off, node_off, pad;
};

struct TapeMeta {           // lepton store at one tape point
  int64_t S;                // sorted-region slots
  int64_t tail_pre;         // tail before this step's injection
  int64_t tail_post;        // tail after it
  int64_t used;             // slots taped: S + tail_post
};

struct AdjCtx {
  const Tile* tiles;
  const int32_t* chunk;     // lepton chunk -> tile (layout of the segment)
  const int32_t* tt;        // lepton tail slot -> tile
  const float* wlast;       // weight of each slot while alive
  const uint32_t* pos0;     // tape at the start of step j
  const float* u0;
  const uint32_t* pos1;     // tape at the start of step j + 1
  const float* u1;
  const TapeMeta* meta0;
  const float* eb0;         // node field used by step j
  float* lxi;
  float* lu;
  float* lw;
  const double* lamE;       // adjoint of the cell field after step j
  const double* suf;        // suffix sums of lamE per tube node: suf_k = sum_{m>=k} lamE_m
  double* lamEb;            // adjoint of the node field of step j (accumulated)
  AdjTube* at;
};

// ------------------------------------------------------------------ tape
// Copy the lepton positions and momenta of slots [0, S + tail) into one tape
// point; `final` marks the point after a segment's last step (no injection).
__global__ __launch_bounds__(TPB) void k_tape(LepBuf L, const Ctl* lc, uint32_t* tpos, float* tu, float* wlast,
                                              TapeMeta* meta, long long M, int final_point, int* err) {
  const long long S = lc->n_sorted_chunks * CHUNK;
  long long used = S + lc->tail;
  if (used > M) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(err, E_CAP);
    used = M;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    TapeMeta m;
    m.S = S;
    m.tail_post = lc->tail;
    m.tail_pre = final_point ? lc->tail : lc->tail_pre;
    m.used = used;
    *meta = m;
  }
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < used; i += (long long)gridDim.x * blockDim.x) {
    const float w = L.w[i];
    const bool alive = w != 0.0f;
    tpos[i] = alive ? L.pos[i] : TAPE_DEAD;
    tu[i] = L.u[i];
    if (alive) wlast[i] = w;
  }
}

// Sum of E^2 over each tube's cells, added to acc[tube] (one workgroup per
// tube, fixed reduction order).
__device__ __forceinline__ double block_sum_d(double v, double* sh) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
  const int w = threadIdx.x / WAVE;
  if (lane_id() == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x < WAVE) {
    t = threadIdx.x < (int)(blockDim.x / WAVE) ? sh[threadIdx.x] : 0.0;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) t += __shfl_xor(t, d);
  }
  if (threadIdx.x == 0) sh[0] = t;
  __syncthreads();
  t = sh[0];
  __syncthreads();
  return t;
}

constexpr int ADJ_THREADS = 1024;

__global__ __launch_bounds__(ADJ_THREADS) void k_loss(const float* E, const Tube* tubes, double* acc) {
  __shared__ double sh[ADJ_THREADS / WAVE];
  const Tube& T = tubes[blockIdx.x];
  double s = 0.0;
  for (int k = threadIdx.x; k < T.N; k += blockDim.x) {
    const double e = (double)E[T.cell_off + k];
    s += e * e;
  }
  s = block_sum_d(s, sh);
  if (threadIdx.x == 0) acc[blockIdx.x] += s;
}

// lamE = lossw * E (adjoint of the loss at the window's last field)
__global__ __launch_bounds__(ADJ_THREADS) void k_adj_init(double* lamE, const float* E, const AdjTube* at) {
  const AdjTube& a = at[blockIdx.x];
  for (int k = threadIdx.x; k < a.N; k += blockDim.x) lamE[a.cell_off + k] = a.lossw * (double)E[a.cell_off + k];
}

// ------------------------------------------------------------------ reverse
// Field after step j: E_s receives sum_k lamE_k; suffix sums for the weights;
// alpha enters E_s as alpha s_co dt.  One workgroup per tube: thread t sums
// a run of consecutive cells, one block scan gives each run the sum of the
// runs above it, and each thread then writes its run's suffix sums from the
// top down (one round of barriers instead of one per ADJ_THREADS cells).
__global__ __launch_bounds__(ADJ_THREADS) void k_adj_field(const double* lamE, double* suf, AdjTube* at) {
  __shared__ double sh[ADJ_THREADS / WAVE];
  AdjTube& a = at[blockIdx.x];
  const int N = a.N;
  const double* lm = lamE + a.cell_off;
  const int per = (N + ADJ_THREADS - 1) / ADJ_THREADS;
  const int k0 = min(N, (int)threadIdx.x * per), k1 = min(N, k0 + per);
  double t = 0.0;
  for (int k = k0; k < k1; ++k) t += lm[k];
  // inclusive suffix of the run sums over the wave's lanes, then over waves
  double incl = t;
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    const double o = __shfl_down(incl, d);
    if (lane_id() + d < WAVE) incl += o;
  }
  const int wv = threadIdx.x / WAVE;
  if (lane_id() == 0) sh[wv] = incl;
  __syncthreads();
  double after = 0.0;
  for (int q = ADJ_THREADS / WAVE - 1; q > wv; --q) after += sh[q];
  // the sum of the runs above this one, then this run's suffix sums
  const double above = __shfl_down(incl, 1);
  double s = (lane_id() + 1 < WAVE ? above : 0.0) + after;
  for (int k = k1 - 1; k >= k0; --k) {
    s += lm[k];
    suf[a.node_off + k] = s;
  }
  if (threadIdx.x == 0) {
    const double total = s;          // thread 0's run starts at cell 0
    suf[a.node_off + N] = 0.0;
    a.lamEs += total;
    a.cw += a.w0 * total;
    a.dalpha += a.lamEs * a.s_co * a.dt;
  }
}

// One lepton slot, step j in reverse: field term at the post-step position,
// drift, recoil (identity), kick; node-field adjoint into LDS (s_eb, sorted
// chunks) or global memory (tail).
__device__ __forceinline__ void adj_one(const AdjCtx& c, long long slot, int tile, double* s_eb, long long inj0,
                                        long long inj1) {
  const uint32_t p0 = c.pos0[slot];
  if (p0 == TAPE_DEAD) return;
  const Tile tl = c.tiles[tile];
  AdjTube& a = c.at[tl.tube];
  const double w0 = a.w0;
  const float dt = (float)a.dt, cfl = (float)a.cfl;
  const float w = c.wlast[slot];
  const float sg = w < 0.0f ? -1.0f : 1.0f;
  const int off0 = (int)(p0 >> FRAC);
  const int cell0 = tl.base + off0;
  const float xi0 = (float)(p0 & 0xFFFFFFu) * 5.9604645e-8f;
  float lxi = c.lxi[slot], lu = c.lu[slot], lw = c.lw[slot];
  const uint32_t p1 = c.pos1[slot];
  if (p1 != TAPE_DEAD) {
    const int cell1 = tl.base + (int)(p1 >> FRAC);
    const double xi1 = (double)(p1 & 0xFFFFFFu) * 5.9604644775390625e-8;
    const double e = c.lamE[a.cell_off + cell1];
    lxi += (float)(-w0 * (double)w * e);
    // w0 ((1 - xi) lamE_k + sum_{m>k} lamE_m), less the common w0 sum_m lamE_m
    lw += (float)(w0 * ((1.0 - xi1) * e + (c.suf[a.node_off + cell1 + 1] - c.suf[a.node_off])));
    const float u1 = c.u1[slot];
    const float g = sqrtf(1.0f + u1 * u1);
    lu += lxi * cfl / (g * g * g);
  } else {
    // gone during step j: absorbed below the surface (its charge enters E_s)
    // or out of the top of the box
    lxi = 0.0f;
    lu = 0.0f;
    lw = (float)((cell0 < a.N / 2 ? a.lamEs * w0 : 0.0) - a.cw);
  }
  const float e0 = c.eb0[a.node_off + cell0], e1 = c.eb0[a.node_off + cell0 + 1];
  const float lEp = sg * dt * lu;
  lxi += lEp * (e1 - e0);
  const double d0 = (double)((1.0f - xi0) * lEp), d1 = (double)(xi0 * lEp);
  if (s_eb) {
    atomicAdd(&s_eb[off0], d0);
    atomicAdd(&s_eb[off0 + 1], d1);
  } else {
    atomicAdd(&c.lamEb[a.node_off + cell0], d0);
    atomicAdd(&c.lamEb[a.node_off + cell0 + 1], d1);
  }
  if (slot >= inj0 && slot < inj1) {
    // injected at the start of step j with weight -inj_w; its injection also
    // raised E_s by inj_w w0
    atomicAdd(&a.dinjw, -(double)lw + (a.lamEs * w0 - a.cw));
    lxi = 0.0f;
    lu = 0.0f;
    lw = 0.0f;
  }
  c.lxi[slot] = lxi;
  c.lu[slot] = lu;
  c.lw[slot] = lw;
}

__global__ __launch_bounds__(TPB) void k_adj_leptons(AdjCtx c) {
  __shared__ double s_eb[WIN + 2];
  const TapeMeta m = *c.meta0;
  const long long S = m.S, used = m.used;
  const long long inj0 = S + m.tail_pre, inj1 = S + m.tail_post;
  const long long nsc = S / CHUNK, ntp = (used - S + TPB - 1) / TPB;
  for (long long q = blockIdx.x; q < nsc + ntp; q += gridDim.x) {
    if (q < nsc) {
      const int tile = c.chunk[q];
      for (int j = threadIdx.x; j < WIN + 2; j += blockDim.x) s_eb[j] = 0.0;
      __syncthreads();
#pragma unroll
      for (int v = 0; v < VEC; ++v) adj_one(c, q * CHUNK + v * TPB + threadIdx.x, tile, s_eb, inj0, inj1);
      __syncthreads();
      const Tile tl = c.tiles[tile];
      const AdjTube& a = c.at[tl.tube];
      for (int j = threadIdx.x; j <= WIN; j += blockDim.x) {
        const double v = s_eb[j];
        if (v != 0.0) atomicAdd(&c.lamEb[a.node_off + tl.base + j], v);
      }
      __syncthreads();
    } else {
      const long long slot = S + (q - nsc) * TPB + threadIdx.x;
      if (slot < used) adj_one(c, slot, c.tt[slot], nullptr, inj0, inj1);
    }
  }
}

// Node field -> cell field and surface field of the start of step j; the
// loss term of that field (when it lies inside the window); clears lamEb.
__global__ __launch_bounds__(ADJ_THREADS) void k_adj_nodes(double* lamE, double* lamEb, const float* Eprev, AdjTube* at) {
  AdjTube& a = at[blockIdx.x];
  const int N = a.N;
  const double* nb = lamEb + a.node_off;
  for (int k = threadIdx.x; k < N; k += blockDim.x) {
    double v = (k < N - 1) ? 0.5 * (nb[k] + nb[k + 1]) : 0.5 * nb[N - 1] + nb[N];
    if (Eprev) v += a.lossw * (double)Eprev[a.cell_off + k];
    lamE[a.cell_off + k] = v;
  }
  if (threadIdx.x == 0) a.lamEs += 0.5 * nb[0];
  __syncthreads();
  for (int k = threadIdx.x; k <= N; k += blockDim.x) lamEb[a.node_off + k] = 0.0;
}

// ------------------------------------------------------------------ id map
__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  // splitmix64 finaliser (Steele, Lea & Flood, OOPSLA 2014)
  x ^= x >> 30;
  x *= 0xBF58476D1CE4E5B9ull;
  x ^= x >> 27;
  x *= 0x94D049BB133111EBull;
  x ^= x >> 31;
  return x;
}

// The table holds slots of a saved layout (HASH_EMPTY32 = free); a particle
// is found by (tube, id), read back through the saved arrays.
constexpr uint32_t HASH_EMPTY32 = 0xFFFFFFFFu;

__device__ __forceinline__ uint64_t hkey(uint64_t id, int tube) {
  return mix64(id ^ mix64((uint64_t)tube + 0x632BE59BD9B4E019ull));
}

__global__ void k_hash_clear(uint32_t* vals, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    vals[i] = HASH_EMPTY32;
}

// Insert the live slots [0, n) of a saved lepton store (sorted region only).
__global__ void k_hash_insert(const uint64_t* ids, const float* w, const int32_t* chunk, const Tile* tiles, long long n,
                              uint32_t* vals, uint64_t mask) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    if (w[i] == 0.0f) continue;
    const int tube = tiles[chunk[i / CHUNK]].tube;
    uint64_t h = hkey(ids[i], tube) & mask;
    for (uint64_t probe = 0; probe <= mask; ++probe) {
      if (atomicCAS(&vals[h], HASH_EMPTY32, (uint32_t)i) == HASH_EMPTY32) break;
      h = (h + 1) & mask;
    }
  }
}

// The adjoint of every live slot of the current lepton store, taken from the
// slot of the same particle (same tube and id) in the saved layout (zero for
// dead slots).
__global__ void k_lam_map(LepBuf L, const Ctl* lc, const int32_t* chunk, const int32_t* tt, const Tile* tiles,
                          const uint64_t* sid, const int32_t* schunk, const uint32_t* vals, uint64_t mask,
                          const float* sxi, const float* su, const float* sw, float* dxi, float* du, float* dw,
                          long long M, int* err) {
  const long long S = lc->n_sorted_chunks * CHUNK;
  long long used = S + lc->tail;
  if (used > M) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(err, E_CAP);
    used = M;
  }
  for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < used; r += (long long)gridDim.x * blockDim.x) {
    float a = 0.0f, b = 0.0f, c = 0.0f;
    if (L.w[r] != 0.0f) {
      const uint64_t id = L.id[r];
      const int tube = tiles[r < S ? chunk[r / CHUNK] : tt[r]].tube;
      uint64_t h = hkey(id, tube) & mask;
      bool found = false;
      for (uint64_t probe = 0; probe <= mask; ++probe) {
        const uint32_t q = vals[h];
        if (q == HASH_EMPTY32) break;
        if (sid[q] == id && tiles[schunk[q / CHUNK]].tube == tube) {
          a = sxi[q]; b = su[q]; c = sw[q];
          found = true;
          break;
        }
        h = (h + 1) & mask;
      }
      if (!found) atomicOr(err, E_TILE);
    }
    dxi[r] = a;
    du[r] = b;
    dw[r] = c;
  }
}

}  // namespace gap
