// hip_stub.cpp -- a strict stand-in for the HIP runtime, for host-only runs of
// libgap's host code under AddressSanitizer and UndefinedBehaviorSanitizer.
//
// Test infrastructure: no GPU work happens.  Device memory is host memory
// (zeroed), kernels are not run, and every handle (stream, event, graph, graph
// exec, allocation) is tracked so that its misuse is reported at the call that
// misuses it, with the call sequence that led there:
//   * copies and fills must stay inside one live allocation;
//   * hipFree / destroy of an unknown or already released handle;
//   * a graph exec destroyed while one of its launches may still run (no
//     synchronisation of the launching stream since the launch);
//   * synchronous calls (hipMemcpy, hipStreamSynchronize, hipMalloc, ...)
//     while a stream of this thread is being captured;
//   * a capture that ends with a forked stream not joined back;
//   * an event recorded inside one capture and waited on outside it or in
//     another capture, or timed with hipEventElapsedTime.
// Any finding prints "HIPSTUB ERROR: ..." and aborts.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <set>
#include <string>

namespace {

struct Stream {
  unsigned flags = 0;
  int capture = 0;         // id of the capture this stream takes part in (0: none)
  bool origin = false;     // began the capture
  long long seq = 0;       // work items enqueued so far
  long long joined_seq = -1;   // seq of this stream's work that another capture member waited for
  std::set<struct Exec*> inflight;   // graph launches not yet synchronised
};
struct Event {
  unsigned flags = 0;
  int recorded_in_capture = 0;   // capture id of the last record (0: recorded on a live stream)
  bool recorded = false;
  Stream* rec_stream = nullptr;
  long long rec_seq = 0;         // the recording stream's seq at the record
};
struct Graph { long long nodes = 0; };
struct Exec { long long nodes = 0; std::set<Stream*> launched_on; };

std::map<uintptr_t, size_t> g_mem;            // live device allocations
std::set<Stream*> g_streams;
std::set<Event*> g_events;
std::set<Graph*> g_graphs;
std::set<Exec*> g_execs;
Stream g_null;                                 // the null stream
int g_next_capture = 1;
std::map<int, std::set<Stream*>> g_capture_members;
std::deque<std::string> g_trail;              // last API calls, printed on an error
long long g_calls = 0;

void trail(const char* fmt, ...) {
  char buf[256];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_trail.push_back(buf);
  if (g_trail.size() > 40) g_trail.pop_front();
  ++g_calls;
}

[[noreturn]] void fail(const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  fprintf(stderr, "HIPSTUB ERROR: %s\n  after %lld calls; last calls:\n", buf, g_calls);
  for (const std::string& s : g_trail) fprintf(stderr, "    %s\n", s.c_str());
  fflush(stderr);
  abort();
}

Stream* S(hipStream_t s) {
  if (!s) return &g_null;
  Stream* p = (Stream*)s;
  if (!g_streams.count(p)) fail("use of an unknown or destroyed stream %p", (void*)s);
  return p;
}

Event* E(hipEvent_t e) {
  Event* p = (Event*)e;
  if (!p || !g_events.count(p)) fail("use of an unknown or destroyed event %p", (void*)e);
  return p;
}

bool any_capture() {
  if (g_null.capture) return true;
  for (Stream* s : g_streams)
    if (s->capture) return true;
  return false;
}

void no_capture(const char* what) {
  if (any_capture()) fail("%s while a stream is being captured", what);
}

void check_dev(const void* p, size_t bytes, const char* what) {
  const uintptr_t a = (uintptr_t)p;
  auto it = g_mem.upper_bound(a);
  if (it == g_mem.begin()) fail("%s: %p is not device memory", what, p);
  --it;
  if (a < it->first || a + bytes > it->first + it->second)
    fail("%s: [%p, +%zu) is outside the allocation [%p, +%zu)", what, p, bytes, (void*)it->first, it->second);
}

// synchronisation of a stream: its graph launches are complete
void sync_stream(Stream* s) {
  for (Exec* x : s->inflight) x->launched_on.erase(s);
  s->inflight.clear();
}

void sync_all() {
  sync_stream(&g_null);
  for (Stream* s : g_streams) sync_stream(s);
}

void enqueue(Stream* s) { s->seq++; }

struct LaunchCfg { dim3 g, b; size_t sh; hipStream_t s; };
LaunchCfg g_cfg[8];
int g_cfg_n = 0;

}  // namespace

extern "C" {

void** __hipRegisterFatBinary(const void*) {
  static void* dummy = nullptr;
  return &dummy;
}
void __hipRegisterFunction(void**, const void*, char*, const char*, unsigned int, void*, void*, void*, void*,
                           int*) {}
void __hipUnregisterFatBinary(void**) {}

// device variables: each registered host shadow gets a stand-in allocation of
// its size, which hipGetSymbolAddress returns
// (constructed on first use: the library's module constructor registers its
// variables before this file's globals are initialised)
std::map<const void*, std::pair<void*, size_t>>& vars() {
  static std::map<const void*, std::pair<void*, size_t>> m;
  return m;
}
void __hipRegisterVar(void**, void* var, char*, char*, int, size_t size, int, int) {
  void* q = aligned_alloc(256, (size + 255) / 256 * 256);
  memset(q, 0, size);
  vars()[var] = {q, size};
}
hipError_t hipGetSymbolAddress(void** p, const void* sym) {
  trail("hipGetSymbolAddress(%p)", sym);
  auto it = vars().find(sym);
  if (it == vars().end()) fail("hipGetSymbolAddress of an unregistered symbol %p", sym);
  g_mem[(uintptr_t)it->second.first] = it->second.second;   // device memory from now on, never freed
  *p = it->second.first;
  return hipSuccess;
}

hipError_t __hipPushCallConfiguration(dim3 g, dim3 b, size_t sh, hipStream_t s) {
  if (g_cfg_n == 8) fail("launch configuration stack overflow");
  g_cfg[g_cfg_n++] = LaunchCfg{g, b, sh, s};
  return hipSuccess;
}
hipError_t __hipPopCallConfiguration(dim3* g, dim3* b, size_t* sh, hipStream_t* s) {
  if (g_cfg_n == 0) fail("launch configuration stack underflow");
  const LaunchCfg& c = g_cfg[--g_cfg_n];
  *g = c.g; *b = c.b; *sh = c.sh; *s = c.s;
  return hipSuccess;
}

hipError_t hipLaunchKernel(const void* f, dim3 g, dim3 b, void**, size_t, hipStream_t s) {
  trail("hipLaunchKernel(%p, %u x %u, stream %p)", f, g.x * g.y * g.z, b.x, (void*)s);
  if (g.x == 0 || g.y == 0 || g.z == 0 || b.x == 0 || b.x * b.y * b.z > 1024)
    fail("kernel launch with grid %u,%u,%u block %u,%u,%u", g.x, g.y, g.z, b.x, b.y, b.z);
  enqueue(S(s));
  return hipSuccess;
}

hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);

hipError_t hipExtLaunchKernel(const void* f, dim3 g, dim3 b, void** a, size_t sh, hipStream_t s, hipEvent_t start,
                              hipEvent_t stop, int) {
  if (start) hipEventRecord(start, s);
  hipLaunchKernel(f, g, b, a, sh, s);
  if (stop) hipEventRecord(stop, s);
  return hipSuccess;
}

hipError_t hipGetDeviceCount(int* n) { *n = 1; return hipSuccess; }
hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t a, int) {
  *v = a == hipDeviceAttributeMultiprocessorCount ? 256 : 1;
  return hipSuccess;
}
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, const void*, int, size_t) {
  *n = 6;
  return hipSuccess;
}
hipError_t hipGetLastError(void) { return hipSuccess; }

hipError_t hipMalloc(void** p, size_t bytes) {
  trail("hipMalloc(%zu)", bytes);
  no_capture("hipMalloc");
  void* q = aligned_alloc(256, (bytes + 255) / 256 * 256);
  if (!q) return hipErrorOutOfMemory;
  memset(q, 0xA5, bytes);   // device memory starts undefined
  g_mem[(uintptr_t)q] = bytes;
  *p = q;
  return hipSuccess;
}
hipError_t hipFree(void* p) {
  trail("hipFree(%p)", p);
  no_capture("hipFree");
  if (!p) return hipSuccess;
  auto it = g_mem.find((uintptr_t)p);
  if (it == g_mem.end()) fail("hipFree of %p, not a live allocation", p);
  sync_all();   // hipFree synchronises the device
  g_mem.erase(it);
  free(p);
  return hipSuccess;
}

hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind k) {
  trail("hipMemcpy(%p, %p, %zu, %d)", d, s, n, (int)k);
  no_capture("hipMemcpy");
  if (k == hipMemcpyHostToDevice || k == hipMemcpyDeviceToDevice) check_dev(d, n, "hipMemcpy dst");
  if (k == hipMemcpyDeviceToHost || k == hipMemcpyDeviceToDevice) check_dev(s, n, "hipMemcpy src");
  if (k != hipMemcpyHostToDevice && k != hipMemcpyDeviceToHost && k != hipMemcpyDeviceToDevice)
    fail("hipMemcpy kind %d", (int)k);
  sync_stream(&g_null);
  memmove(d, s, n);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind k, hipStream_t st) {
  trail("hipMemcpyAsync(%p, %p, %zu, %d, %p)", d, s, n, (int)k, (void*)st);
  Stream* q = S(st);
  if (q->capture && k != hipMemcpyDeviceToDevice) fail("host copy captured into a graph");
  if (k == hipMemcpyHostToDevice || k == hipMemcpyDeviceToDevice) check_dev(d, n, "hipMemcpyAsync dst");
  if (k == hipMemcpyDeviceToHost || k == hipMemcpyDeviceToDevice) check_dev(s, n, "hipMemcpyAsync src");
  enqueue(q);
  if (!q->capture) memmove(d, s, n);
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t st) {
  trail("hipMemsetAsync(%p, %d, %zu, %p)", d, v, n, (void*)st);
  Stream* q = S(st);
  if (q->capture) fail("hipMemsetAsync captured into a graph");
  check_dev(d, n, "hipMemsetAsync");
  memset(d, v, n);
  return hipSuccess;
}

hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned flags) {
  trail("hipStreamCreateWithFlags");
  Stream* p = new Stream();
  p->flags = flags;
  g_streams.insert(p);
  *s = (hipStream_t)p;
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  trail("hipStreamDestroy(%p)", (void*)s);
  Stream* p = S(s);
  if (p == &g_null) fail("hipStreamDestroy of the null stream");
  if (p->capture) fail("hipStreamDestroy of a stream under capture");
  sync_stream(p);
  g_streams.erase(p);
  delete p;
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
  trail("hipStreamSynchronize(%p)", (void*)s);
  Stream* p = S(s);
  if (p->capture) fail("hipStreamSynchronize of a stream under capture");
  no_capture("hipStreamSynchronize");
  sync_stream(p);
  return hipSuccess;
}

hipError_t hipEventCreate(hipEvent_t* e) {
  trail("hipEventCreate");
  no_capture("hipEventCreate");
  Event* p = new Event();
  g_events.insert(p);
  *e = (hipEvent_t)p;
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned flags) {
  hipEventCreate(e);
  ((Event*)*e)->flags = flags;
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
  trail("hipEventDestroy(%p)", (void*)e);
  Event* p = E(e);
  g_events.erase(p);
  delete p;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  trail("hipEventRecord(%p, %p)", (void*)e, (void*)s);
  Event* p = E(e);
  Stream* q = S(s);
  p->recorded = true;
  p->recorded_in_capture = q->capture;
  p->rec_stream = q;
  p->rec_seq = q->seq;
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) {
  trail("hipStreamWaitEvent(%p, %p)", (void*)s, (void*)e);
  Stream* q = S(s);
  Event* p = E(e);
  if (p->recorded_in_capture) {
    if (!g_capture_members.count(p->recorded_in_capture))
      fail("wait on an event recorded inside a capture that has ended");
    if (q->capture && q->capture != p->recorded_in_capture) fail("wait across two captures");
    if (!q->capture) {
      // a stream joins the capture through the event (a fork)
      q->capture = p->recorded_in_capture;
      q->origin = false;
      q->joined_seq = -1;
      g_capture_members[q->capture].insert(q);
    } else if (p->rec_stream && p->rec_stream != q) {
      p->rec_stream->joined_seq = std::max(p->rec_stream->joined_seq, p->rec_seq);   // joined back up to there
    }
  } else if (q->capture && p->recorded) {
    fail("a captured stream waits on an event recorded outside the capture");
  }
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
  trail("hipEventSynchronize(%p)", (void*)e);
  Event* p = E(e);
  no_capture("hipEventSynchronize");
  if (p->recorded_in_capture) fail("hipEventSynchronize on an event recorded only inside a capture");
  if (p->rec_stream) sync_stream(p->rec_stream);
  return hipSuccess;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  trail("hipEventElapsedTime(%p, %p)", (void*)a, (void*)b);
  Event* x = E(a);
  Event* y = E(b);
  if ((x->flags | y->flags) & hipEventDisableTiming) fail("hipEventElapsedTime on an event without timing");
  if (!x->recorded || !y->recorded) fail("hipEventElapsedTime on an event never recorded");
  if (x->recorded_in_capture || y->recorded_in_capture) fail("hipEventElapsedTime on an event recorded in a capture");
  *ms = 0.001f;
  return hipSuccess;
}

hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  trail("hipStreamBeginCapture(%p)", (void*)s);
  Stream* q = S(s);
  if (q == &g_null) fail("capture of the null stream");
  if (q->capture) fail("hipStreamBeginCapture of a stream already under capture");
  q->capture = g_next_capture++;
  q->origin = true;
  g_capture_members[q->capture] = {q};
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
  trail("hipStreamEndCapture(%p)", (void*)s);
  Stream* q = S(s);
  if (!q->capture || !q->origin) fail("hipStreamEndCapture on a stream that did not begin a capture");
  const int id = q->capture;
  for (Stream* m : g_capture_members[id]) {
    if (m != q && m->joined_seq != m->seq)
      fail("capture ends with a forked stream not joined back (work after the last join)");
    m->capture = 0;
    m->origin = false;
  }
  g_capture_members.erase(id);
  Graph* gr = new Graph();
  g_graphs.insert(gr);
  *g = (hipGraph_t)gr;
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
  trail("hipGraphInstantiate(%p)", (void*)g);
  if (!g_graphs.count((Graph*)g)) fail("hipGraphInstantiate of an unknown graph");
  Exec* e = new Exec();
  g_execs.insert(e);
  *x = (hipGraphExec_t)e;
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
  trail("hipGraphDestroy(%p)", (void*)g);
  if (!g_graphs.erase((Graph*)g)) fail("hipGraphDestroy of an unknown or destroyed graph");
  delete (Graph*)g;
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s) {
  trail("hipGraphLaunch(%p, %p)", (void*)x, (void*)s);
  Exec* e = (Exec*)x;
  if (!g_execs.count(e)) fail("hipGraphLaunch of an unknown or destroyed graph exec");
  Stream* q = S(s);
  if (q->capture) fail("graph launch inside a capture");
  e->launched_on.insert(q);
  q->inflight.insert(e);
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t x) {
  trail("hipGraphExecDestroy(%p)", (void*)x);
  Exec* e = (Exec*)x;
  if (!g_execs.count(e)) fail("hipGraphExecDestroy of an unknown or destroyed graph exec");
  if (!e->launched_on.empty()) fail("graph exec destroyed while a launch of it may still run");
  g_execs.erase(e);
  delete e;
  return hipSuccess;
}

// summary for the driver
void hipstub_report(long long* out) {
  long long statics = 0;
  for (auto& v : vars()) statics += g_mem.count((uintptr_t)v.second.first);
  out[0] = (long long)g_mem.size() - statics;
  out[1] = (long long)g_streams.size();
  out[2] = (long long)g_events.size();
  out[3] = (long long)g_graphs.size();
  out[4] = (long long)g_execs.size();
  out[5] = g_calls;
}

}  // extern "C"
