// A host-only stand-in for the HIP runtime, for running the library's host code on a machine
// without a GPU under AddressSanitizer (test infrastructure; never linked into libpic.so).
//
// Device memory is host memory here: hipMemcpyAsync is a plain memcpy, so every table the
// host code writes into a "device" workspace is bounds-checked by ASan.  Kernel launches are
// accepted and do nothing.  Streams, events, graphs and executable graphs are heap objects
// with a live flag: using or destroying one that was already destroyed, destroying a graph
// executable that may still run, synchronising a stream that is being captured or leaving a
// stream that was pulled into a capture unjoined aborts the process with a message naming the
// call, so the lifetime rules of the HIP runtime are checked, not assumed.
#include <hip/hip_runtime_api.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <set>
#include <vector>

struct ihipStream_t {
  int capture = 0;       // capture id this stream records into (0: not capturing)
  bool origin = false;   // the stream the capture was begun on
  long ops = 0;          // operations recorded on it in the current capture
  long joined = 0;       // its `ops` when the origin last waited on an event recorded on it
  long submitted = 0;    // graph launches enqueued on it
  long completed = 0;    // graph launches known complete (a stream or event synchronisation)
};
struct ihipEvent_t {
  int capture = 0;       // recorded during capture `capture` (0: outside any capture)
  ihipStream_t* src = nullptr;  // the stream it was last recorded on, and its ops then
  long src_ops = 0;
  long src_submitted = 0;       // the graph launches enqueued on src before the record
};
struct ihipGraph {
  int id;
};
struct hipGraphExec {
  int id;
  int launches = 0;
  ihipStream_t* last_stream = nullptr;  // the stream of its last launch and that launch's number
  long last_submit = 0;
};

namespace {

std::set<const void*> g_live;
std::set<ihipStream_t*> g_streams;
int g_next_capture = 0;
int g_next_graph = 0;
dim3 g_grid, g_block;
size_t g_shmem = 0;
hipStream_t g_cfg_stream = nullptr;
long long g_launches = 0;

[[noreturn]] void die(const char* what, const void* h) {
  std::fprintf(stderr, "hip_stub: %s (handle %p)\n", what, h);
  std::fflush(stderr);
  std::abort();
}

void need_live(const void* h, const char* what) {
  if (h && !g_live.count(h)) die(what, h);
}

}  // namespace

extern "C" {

long long hip_stub_launch_count() { return g_launches; }
int hip_stub_live_handles() { return (int)g_live.size(); }

hipError_t hipGetDeviceCount(int* n) {
  *n = 1;
  return hipSuccess;
}

hipError_t hipGetLastError(void) { return hipSuccess; }

const char* hipGetErrorString(hipError_t) { return "hip_stub"; }

hipError_t hipFuncSetAttribute(const void*, hipFuncAttribute, int) { return hipSuccess; }

hipError_t __hipPushCallConfiguration(dim3 grid, dim3 block, size_t shmem, hipStream_t s) {
  g_grid = grid;
  g_block = block;
  g_shmem = shmem;
  g_cfg_stream = s;
  return hipSuccess;
}

hipError_t __hipPopCallConfiguration(dim3* grid, dim3* block, size_t* shmem, hipStream_t* s) {
  *grid = g_grid;
  *block = g_block;
  *shmem = g_shmem;
  *s = g_cfg_stream;
  return hipSuccess;
}

void** __hipRegisterFatBinary(const void*) {
  static void* module = nullptr;
  return &module;
}

void __hipUnregisterFatBinary(void**) {}

void __hipRegisterFunction(void**, const void*, char*, const char*, unsigned int, uint3*, uint3*,
                           dim3*, dim3*, int*) {}

hipError_t hipLaunchKernel(const void*, dim3 grid, dim3 block, void**, size_t shmem,
                           hipStream_t s) {
  need_live(s, "kernel launch on a destroyed stream");
  if (grid.x == 0 || grid.y == 0 || grid.z == 0 || block.x * block.y * block.z == 0 ||
      block.x * block.y * block.z > 1024 || grid.y > 65535 || grid.z > 65535)
    die("kernel launch with an invalid grid or block", s);
  if (shmem > 160 * 1024) die("kernel launch with more than 160 KB of LDS", s);
  if (s && s->capture) ++s->ops;
  ++g_launches;
  return hipSuccess;
}

hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind, hipStream_t s) {
  need_live(s, "copy on a destroyed stream");
  if (s && s->capture) die("copy recorded into a capture (a graph memcpy node)", s);
  if (bytes) std::memmove(dst, src, bytes);
  return hipSuccess;
}

hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) {
  *s = new ihipStream_t;
  g_live.insert(*s);
  g_streams.insert(*s);
  return hipSuccess;
}

hipError_t hipStreamDestroy(hipStream_t s) {
  need_live(s, "hipStreamDestroy of a destroyed stream");
  if (!s) die("hipStreamDestroy of the null stream", s);
  if (s->capture) die("hipStreamDestroy of a stream in a capture", s);
  g_live.erase(s);
  g_streams.erase(s);
  delete s;
  return hipSuccess;
}

hipError_t hipStreamSynchronize(hipStream_t s) {
  need_live(s, "hipStreamSynchronize of a destroyed stream");
  if (s && s->capture) die("hipStreamSynchronize of a capturing stream", s);
  if (s) s->completed = s->submitted;
  return hipSuccess;
}

hipError_t hipEventCreate(hipEvent_t* e) {
  *e = new ihipEvent_t;
  g_live.insert(*e);
  return hipSuccess;
}

hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }

hipError_t hipEventDestroy(hipEvent_t e) {
  need_live(e, "hipEventDestroy of a destroyed event");
  if (!e) die("hipEventDestroy(NULL)", e);
  g_live.erase(e);
  delete e;
  return hipSuccess;
}

hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  need_live(e, "hipEventRecord of a destroyed event");
  need_live(s, "hipEventRecord on a destroyed stream");
  e->capture = s ? s->capture : 0;
  e->src = s;
  e->src_ops = s ? s->ops : 0;
  e->src_submitted = s ? s->submitted : 0;
  return hipSuccess;
}

hipError_t hipEventSynchronize(hipEvent_t e) {
  need_live(e, "hipEventSynchronize of a destroyed event");
  if (e->capture) die("hipEventSynchronize of an event recorded in a capture", e);
  if (e->src && g_streams.count(e->src) && e->src->completed < e->src_submitted)
    e->src->completed = e->src_submitted;
  return hipSuccess;
}

hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  need_live(a, "hipEventElapsedTime of a destroyed event");
  need_live(b, "hipEventElapsedTime of a destroyed event");
  *ms = 0.0f;
  return hipSuccess;
}

hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned int) {
  need_live(s, "hipStreamWaitEvent on a destroyed stream");
  need_live(e, "hipStreamWaitEvent on a destroyed event");
  if (e->capture) {
    // waiting on an event of a capture pulls the stream into that capture
    if (s && s->capture && s->capture != e->capture) die("stream joins two captures", s);
    if (s) {
      s->capture = e->capture;
      ++s->ops;
      if (s->origin && e->src) e->src->joined = e->src_ops;  // the origin joins e's stream
    }
  } else if (s && s->capture && !s->origin) {
    die("captured stream waits on an event outside its capture", s);
  }
  return hipSuccess;
}

hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  need_live(s, "capture on a destroyed stream");
  if (!s) die("capture on the null stream", s);
  if (s->capture) die("capture begun twice", s);
  s->capture = ++g_next_capture;
  s->origin = true;
  s->ops = s->joined = 0;
  return hipSuccess;
}

hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
  need_live(s, "end of capture on a destroyed stream");
  if (!s->origin) die("capture ended on a stream that did not begin it", s);
  const int id = s->capture;
  // every other stream pulled into the capture must have been joined back into the origin
  // after its last captured operation
  for (ihipStream_t* t : g_streams)
    if (t != s && t->capture == id) {
      if (t->ops != t->joined) die("capture ended with unjoined work on a forked stream", t);
      t->capture = 0;
      t->ops = t->joined = 0;
    }
  s->capture = 0;
  s->origin = false;
  s->ops = s->joined = 0;
  *g = new ihipGraph{++g_next_graph};
  g_live.insert(*g);
  return hipSuccess;
}

hipError_t hipGraphInstantiate(hipGraphExec_t* ex, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
  need_live(g, "instantiation of a destroyed graph");
  *ex = new hipGraphExec{g->id};
  g_live.insert(*ex);
  return hipSuccess;
}

hipError_t hipGraphDestroy(hipGraph_t g) {
  need_live(g, "hipGraphDestroy of a destroyed graph");
  g_live.erase(g);
  delete g;
  return hipSuccess;
}

hipError_t hipGraphLaunch(hipGraphExec_t ex, hipStream_t s) {
  need_live(ex, "launch of a destroyed graph executable");
  need_live(s, "graph launch on a destroyed stream");
  if (!s) die("graph launch on the null stream", s);
  ++ex->launches;
  ex->last_stream = s;
  ex->last_submit = ++s->submitted;
  return hipSuccess;
}

hipError_t hipGraphExecDestroy(hipGraphExec_t ex) {
  need_live(ex, "hipGraphExecDestroy of a destroyed graph executable");
  if (ex->last_stream && (!g_streams.count(ex->last_stream) ||
                          ex->last_stream->completed < ex->last_submit))
    die("graph executable destroyed while its last launch may still run", ex);
  g_live.erase(ex);
  delete ex;
  return hipSuccess;
}

}  // extern "C"
