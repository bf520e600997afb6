// replay.cpp -- drives libgap's C ABI through the call sequences of the
// batched launch-shape sweep (launch shape set, graph dropped and captured
// again, replays, eager steps, reads) and of every other host-side path, on
// the strict HIP stand-in of hip_stub.cpp, under ASan/UBSan.  Test
// infrastructure: nothing here runs on a GPU.
#include "gap.h"

#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

extern "C" void hipstub_report(long long* out);

namespace {

int g_fail = 0;

void expect(int code, const char* what, int ok2 = 0) {
  if (code != 0 && code != ok2) {
    fprintf(stderr, "REPLAY: %s returned %d (%s)\n", what, code, gap_strerror(code));
    g_fail = 1;
  }
}

gap_params base_params() {
  gap_params p;
  std::memset(&p, 0, sizeof p);
  p.n_cells = 1024; p.init_kind = GAP_INIT_UNIFORM; p.ppc_init = 4; p.ppc_ref = 16;
  p.dx = 0.25; p.cfl = 0.45; p.alpha = 1.5; p.b = 0.1; p.r_curv_cm = 1e7; p.period_s = 1.0;
  p.lambda_c_scale = 1.0; p.r_curv_scale = 1.0; p.h_gap_frac = 0.8; p.inj_rate = 0.0; p.inj_weight = 1.0;
  p.x_thr = 2.0; p.xc_floor = 1e-2; p.u_init = 0.0; p.merge_frac = 0.9; p.seed = 1;
  p.cap_leptons = 1 << 16; p.cap_photons = 1 << 15; p.flags = 0; p.nsub_max = 64; p.merge_every = 64;
  p.rebucket_every = 0;
  return p;
}

// caching allocator in the manner of a framework's pool: freed blocks are
// kept and handed out again
struct Pool {
  std::vector<std::pair<void*, size_t>> free_blocks;
  std::vector<std::pair<void*, size_t>> all;
  long long live = 0;
};
void* pool_alloc(size_t n, void* ctx) {
  Pool* P = (Pool*)ctx;
  for (size_t i = 0; i < P->free_blocks.size(); ++i)
    if (P->free_blocks[i].second >= n && P->free_blocks[i].second <= 2 * n + 4096) {
      void* p = P->free_blocks[i].first;
      P->free_blocks.erase(P->free_blocks.begin() + (long)i);
      ++P->live;
      return p;
    }
  void* p = nullptr;
  if (hipMalloc(&p, n) != hipSuccess) return nullptr;
  P->all.push_back({p, n});
  ++P->live;
  return p;
}
void pool_free(void* p, void* ctx) {
  Pool* P = (Pool*)ctx;
  for (auto& b : P->free_blocks)
    if (b.first == p) { fprintf(stderr, "REPLAY: double free of %p through the allocator\n", p); abort(); }
  for (auto& b : P->all)
    if (b.first == p) { P->free_blocks.push_back(b); --P->live; return; }
  fprintf(stderr, "REPLAY: allocator asked to free %p, never handed out\n", p);
  abort();
}

void read_all(gap_t* g, int n_tubes, bool waterfall) {
  std::vector<char> buf(1 << 22);
  size_t wr = 0;
  int kinds[] = {GAP_DIAG_COUNTS, GAP_DIAG_FIELD, GAP_DIAG_ES, GAP_DIAG_RHO, GAP_DIAG_NODE_E, GAP_DIAG_DERIVED,
                 GAP_DIAG_PROFILE, GAP_DIAG_PEAK, GAP_DIAG_RETURN, GAP_DIAG_SPECTRA, GAP_DIAG_ESPECTRUM,
                 GAP_DIAG_PHASE, GAP_DIAG_LEPTONS, GAP_DIAG_PHOTONS, GAP_DIAG_WATERFALL};
  for (int t = 0; t < n_tubes; t += 3)
    for (int k : kinds) {
      if (k == GAP_DIAG_WATERFALL && !waterfall) continue;
      int e = gap_diag(g, k, t, buf.data(), buf.size(), &wr);
      if (e == GAP_EINVAL && wr > buf.size()) continue;   // buffer too small: reported, not written
      expect(e, "gap_diag");
      if (wr > buf.size()) { fprintf(stderr, "REPLAY: diag %d wrote %zu > %zu\n", k, wr, buf.size()); g_fail = 1; }
    }
  // too small a buffer must be refused without writing past it
  std::vector<char> small(8);
  int e = gap_diag(g, GAP_DIAG_FIELD, 0, small.data(), small.size(), &wr);
  if (e != GAP_EINVAL) { fprintf(stderr, "REPLAY: short buffer accepted\n"); g_fail = 1; }
}

void sweep(bool pool) {
  // an uneven ensemble in the manner of the batched recipe, at small sizes
  const int nt = 12;
  std::vector<gap_params> P(nt);
  uint64_t s = 12345;
  auto rnd = [&]() { s = s * 6364136223846793005ull + 1442695040888963407ull; return (double)(s >> 11) / 9007199254740992.0; };
  for (int t = 0; t < nt; ++t) {
    P[t] = base_params();
    P[t].n_cells = 256 + (int)(rnd() * 1793);
    P[t].alpha = -1.0 + 3.0 * rnd();
    P[t].b = 0.01 * std::pow(30.0, rnd());
    P[t].ppc_init = 1 + (int)(rnd() * 8);
    P[t].seed = 100003 + t;
    P[t].cap_leptons = 4 * 2 * P[t].ppc_init * P[t].n_cells + 1024;
    P[t].cap_photons = 2 * P[t].ppc_init * P[t].n_cells + 1024;
    if (t % 4 == 1) P[t].flags |= GAP_MERGE_ON;
    if (t % 5 == 2) P[t].flags |= GAP_FILTER;
  }
  hipStream_t st;
  hipStreamCreateWithFlags(&st, 0);
  Pool pl;
  gap_allocator al{pool_alloc, pool_free, &pl};
  gap_t* g = nullptr;
  expect(gap_init(P.data(), nt, st, pool ? &al : nullptr, &g), "gap_init");
  if (!g) return;
  int32_t chosen[4];
  expect(gap_autotune(g, 16, chosen), "gap_autotune");
  // the launch-shape sweep: every call changes the shape, which drops the
  // graph; replays whose length flips the store parity capture again
  const int shapes[8][4] = {{512, 512, 512, 68}, {1024, 2048, 1024, 34}, {256, 1024, 2048, 136},
                            {2048, 4096, 512, 17},  {512, 512, 4096, 68}, {1024, 512, 512, 136},
                            {256, 256, 256, 5},     {1536, 1536, 1536, 68}};
  for (int cyc = 0; cyc < 24; ++cyc) {
    int32_t v[4];
    std::memcpy(v, shapes[cyc % 8], sizeof v);
    expect(gap_set_state(g, GAP_STATE_LAUNCH, 0, v, sizeof v), "set launch");
    const int n = v[3] + (cyc & 1);
    expect(gap_step_graph(g, n), "step_graph");
    expect(gap_step_graph(g, n), "step_graph again");
    expect(gap_step(g, 3), "step");
    if (cyc % 3 == 0) expect(gap_step_graph(g, 2 * v[3]), "step_graph two intervals");
    size_t wr;
    int64_t c[32];
    for (int t = 0; t < nt; ++t) expect(gap_diag(g, GAP_DIAG_COUNTS, t, c, sizeof c, &wr), "counts");
    if (cyc % 4 == 3) expect(gap_sync(g), "sync");
  }
  // timing of eager steps, with graph replays between (which are not timed)
  int32_t on = 1, off = 0;
  expect(gap_set_state(g, GAP_STATE_TIMING, 0, &on, 4), "timing on");
  expect(gap_step(g, 5), "timed steps");
  expect(gap_step_graph(g, 7), "graph while timing");
  expect(gap_step(g, 2), "timed steps");
  double tim[16];
  size_t wr;
  expect(gap_diag(g, GAP_DIAG_TIMING, 0, tim, sizeof tim, &wr), "timing read");
  expect(gap_set_state(g, GAP_STATE_TIMING, 0, &off, 4), "timing off");
  // waterfall on, graph, read, off; profile bin; drive
  int32_t wf[3] = {2, 16, 8};
  expect(gap_set_state(g, GAP_STATE_WATERFALL, 0, wf, sizeof wf), "waterfall on");
  expect(gap_step_graph(g, 9), "graph with waterfall");
  expect(gap_step(g, 4), "steps with waterfall");
  int32_t pb = 7;
  expect(gap_set_state(g, GAP_STATE_PROFILE_BIN, 0, &pb, 4), "profile bin");
  read_all(g, nt, true);
  int32_t wf0[3] = {0, 1, 1};
  expect(gap_set_state(g, GAP_STATE_WATERFALL, 0, wf0, sizeof wf0), "waterfall off");
  double drive[2] = {0.5, 1.0};
  for (int t = 0; t < nt; t += 5) expect(gap_set_state(g, GAP_STATE_DRIVE, t, drive, sizeof drive), "drive");
  expect(gap_autotune(g, 8, chosen), "autotune again");
  expect(gap_step_graph(g, 3), "graph after autotune");
  gap_free(g);
  hipStreamDestroy(st);
  if (pool) {
    if (pl.live != 0) { fprintf(stderr, "REPLAY: %lld allocations not returned\n", pl.live); g_fail = 1; }
    for (auto& b : pl.all) hipFree(b.first);
  }
}

void single_tube() {
  gap_params p = base_params();
  p.n_cells = 300;
  p.flags = GAP_MERGE_ON;
  p.inj_rate = 0.1;
  p.init_kind = GAP_INIT_GAP;
  hipStream_t st;
  hipStreamCreateWithFlags(&st, 0);
  gap_t* g = nullptr;
  expect(gap_init(&p, 1, st, nullptr, &g), "gap_init single");
  if (!g) return;
  // particles: header + 3 leptons + 2 photons in the ABI's record layouts
  std::vector<char> buf(16 + 3 * 24 + 2 * 32, 0);
  int64_t hdr[2] = {3, 2};
  std::memcpy(buf.data(), hdr, 16);
  for (int i = 0; i < 3; ++i) {
    char* r = buf.data() + 16 + 24 * i;
    int32_t cell = 10 * i; uint32_t frac = 1u << 20; float u = 1.0f + i, w = (i & 1) ? -1.0f : 1.0f;
    uint64_t id = 100 + i;
    std::memcpy(r, &cell, 4); std::memcpy(r + 4, &frac, 4); std::memcpy(r + 8, &u, 4);
    std::memcpy(r + 12, &w, 4); std::memcpy(r + 16, &id, 8);
  }
  for (int i = 0; i < 2; ++i) {
    char* r = buf.data() + 16 + 3 * 24 + 32 * i;
    int32_t cell = 20 + i; uint32_t frac = 5; float x = 50.0f, w = 1.0f; int32_t n0 = 0; uint64_t id = 900 + i;
    std::memcpy(r, &cell, 4); std::memcpy(r + 4, &frac, 4); std::memcpy(r + 8, &x, 4);
    std::memcpy(r + 12, &w, 4); std::memcpy(r + 16, &n0, 4); std::memcpy(r + 24, &id, 8);
  }
  expect(gap_set_state(g, GAP_STATE_PARTICLES, 0, buf.data(), buf.size()), "set particles");
  // a short buffer (header promises more records than it holds) is refused
  if (gap_set_state(g, GAP_STATE_PARTICLES, 0, buf.data(), buf.size() - 1) != GAP_EINVAL) {
    fprintf(stderr, "REPLAY: short particle buffer accepted\n");
    g_fail = 1;
  }
  char es[16];
  double E_s = 0.25;
  int64_t step = 40;
  std::memcpy(es, &E_s, 8);
  std::memcpy(es + 8, &step, 8);
  expect(gap_set_state(g, GAP_STATE_ES_STEP, 0, es, sizeof es), "set es");
  std::vector<char> fld(sizeof(float) * 300 + 8, 0);
  expect(gap_set_state(g, GAP_STATE_FIELD, 0, fld.data(), fld.size()), "set field");
  char inj[16] = {0};
  expect(gap_set_state(g, GAP_STATE_INJECTION, 0, inj, sizeof inj), "set injection");
  expect(gap_step(g, 70), "steps");
  expect(gap_step_graph(g, 70), "graph");
  read_all(g, 1, false);
  double loss[1], da[1], dn[1];
  // the window needs the device to re-sort (kernels do not run here): either
  // result is a clean return
  int e = gap_window_forward(g, 12, 5, loss);
  if (e == 0) expect(gap_window_backward(g, da, dn), "backward");
  e = gap_backward(g, 12, 5, loss, da, dn);
  if (e != 0 && e != GAP_ESTATE) expect(e, "backward in one call");
  // the allocation-free spectrum: into a caller's buffer, twice (then a
  // smaller request), and its refusals
  {
    void* pw = nullptr;
    hipMalloc(&pw, sizeof(double) * 257);
    expect(gap_e_spectrum_noalloc(g, 0, (double*)pw, 257), "noalloc spectrum");
    expect(gap_e_spectrum_noalloc(g, 0, (double*)pw, 200), "noalloc spectrum (short)", GAP_EINVAL);
    if (gap_e_spectrum_noalloc(g, 0, (double*)pw, 256) != GAP_EINVAL || gap_e_spectrum_noalloc(g, 0, nullptr, 257) != GAP_EINVAL) {
      fprintf(stderr, "REPLAY: bad spectrum buffer accepted\n");
      g_fail = 1;
    }
    gap_sync(g);
    hipFree(pw);
  }
  // the error hook (no kernel runs here, so the word itself stays clear)
  int32_t bits = 2;
  expect(gap_set_state(g, GAP_STATE_RAISE, 0, &bits, 4), "raise");
  bits = 64;
  if (gap_set_state(g, GAP_STATE_RAISE, 0, &bits, 4) != GAP_EINVAL) {
    fprintf(stderr, "REPLAY: unknown error bit accepted\n");
    g_fail = 1;
  }
  gap_free(g);
  hipStreamDestroy(st);
}

}  // namespace

int main() {
  sweep(false);
  sweep(true);
  single_tube();
  // refusals
  gap_params bad = base_params();
  bad.n_cells = 1;
  gap_t* g = nullptr;
  if (gap_init(&bad, 1, nullptr, nullptr, &g) != GAP_EINVAL || g) { fprintf(stderr, "REPLAY: bad params\n"); g_fail = 1; }
  long long r[6];
  hipstub_report(r);
  printf("replay: %lld HIP calls; left: %lld allocations, %lld streams, %lld events, %lld graphs, %lld execs\n",
         r[5], r[0], r[1], r[2], r[3], r[4]);
  if (r[0] || r[1] || r[2] || r[3] || r[4]) { fprintf(stderr, "REPLAY: handles leaked\n"); g_fail = 1; }
  if (!g_fail) printf("REPLAY OK\n");
  return g_fail;
}
