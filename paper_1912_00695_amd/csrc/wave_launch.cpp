// wave_launch.cpp -- recorded launch lists and their graph cache.
//
// On MI355X a kernel launched back to back on one stream costs about 2.4 us of
// host time; replayed from an instantiated graph the host cost is a few us per
// graph and the GPU-side gap between dependent kernels stays (about 1.7 us for
// tiny kernels). Solves whose steps take less than the host launch time (small
// grids) are host-bound without graphs. A graph is captured from the same launch
// calls a direct run makes, so replaying it runs the same kernels with the same
// arguments: results are bitwise those of the direct run.
#include "wave_launch.h"

#include <cstring>
#include <mutex>

#include "../../include/wave.h"

namespace wave {

LaunchRec& LaunchList::add(int kind) {
  recs_.emplace_back();
  LaunchRec& r = recs_.back();
  std::memset(static_cast<void*>(&r), 0, sizeof(LaunchRec));  // padding too: lists compare by bytes
  r.kind = kind;
  return r;
}

void LaunchList::step(const StepArgs& a, int r, bool grad, int st, bool diff, bool nt) {
  LaunchRec& q = add(LaunchRec::STEP);
  std::memcpy(static_cast<void*>(&q.a), &a, sizeof(StepArgs));
  q.r = r; q.grad = grad; q.st = st; q.diff = diff; q.nt = nt;
}

void LaunchList::step_basic(const StepArgs& a, int r) {
  LaunchRec& q = add(LaunchRec::STEP_BASIC);
  std::memcpy(static_cast<void*>(&q.a), &a, sizeof(StepArgs));
  q.r = r;
}

void LaunchList::fused2(const Fused2Args& f, int r, bool nt) {
  LaunchRec& q = add(LaunchRec::FUSED2);
  std::memcpy(static_cast<void*>(&q.f), &f, sizeof(Fused2Args));
  q.r = r; q.nt = nt;
}

void LaunchList::sample(const void* field, int st, LevelMeta meta, int m, const int* idx,
                        const float* w, int n, float* out) {
  if (n <= 0) return;
  LaunchRec& q = add(LaunchRec::SAMPLE);
  q.st = st;
  q.smp.field = field; q.smp.meta = meta; q.smp.m = m; q.smp.n = n;
  q.smp.idx = idx; q.smp.w = w; q.smp.out = out;
}

void LaunchList::pack(const float* src, float* dst, Geom g) {
  LaunchRec& q = add(LaunchRec::PACK);
  q.el.src = src; q.el.dst = dst; q.el.g = g;
}

void LaunchList::unpack(const float* src, float* dst, Geom g) {
  LaunchRec& q = add(LaunchRec::UNPACK);
  q.el.src = src; q.el.dst = dst; q.el.g = g;
}

void LaunchList::copy(const float* src, float* dst, int64_t n) {
  if (n <= 0) return;
  LaunchRec& q = add(LaunchRec::COPY);
  q.el.src = src; q.el.dst = dst; q.el.count = n;
}

void LaunchList::zero_words(unsigned* p, int64_t n) {
  if (n <= 0) return;
  LaunchRec& q = add(LaunchRec::ZERO);
  q.el.dst = reinterpret_cast<float*>(p); q.el.count = n;
}

hipError_t LaunchList::play(hipStream_t s) const {
  for (const LaunchRec& q : recs_) {
    hipError_t e = hipSuccess;
    switch (q.kind) {
      case LaunchRec::STEP: e = launch_step(q.a, q.r, q.grad, q.st, q.diff, q.nt, s); break;
      case LaunchRec::STEP_BASIC: e = launch_step_basic(q.a, q.r, s); break;
      case LaunchRec::FUSED2: e = launch_fused2(q.f, q.r, q.nt, s); break;
      case LaunchRec::SAMPLE:
        e = launch_sample(q.smp.field, q.st, q.smp.meta, q.smp.m, q.smp.idx, q.smp.w, q.smp.n,
                          q.smp.out, s);
        break;
      case LaunchRec::PACK: e = launch_pack(q.el.src, q.el.dst, q.el.g, s); break;
      case LaunchRec::UNPACK: e = launch_unpack(q.el.src, q.el.dst, q.el.g, s); break;
      case LaunchRec::COPY: e = launch_copy(q.el.src, q.el.dst, q.el.count, s); break;
      case LaunchRec::ZERO:
        e = launch_zero_words(reinterpret_cast<unsigned*>(q.el.dst), q.el.count, s);
        break;
      default: e = hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

namespace {

constexpr size_t kMinGraphLaunches = 8;  // shorter lists always run directly
constexpr size_t kMaxGraphs = 16;        // instantiated graphs kept (least recently used out)
constexpr size_t kMaxSeen = 256;         // lists seen once (hash and device)
constexpr int kMaxDevices = 64;

uint64_t fnv1a(const void* p, size_t n) {
  const unsigned char* b = static_cast<const unsigned char*>(p);
  uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
  return h;
}

struct Graph {
  uint64_t hash;
  int dev;
  std::vector<LaunchRec> recs;
  hipGraphExec_t exec;
  hipEvent_t done;  // recorded after each replay: an evicted graph is idle once it completed
  uint64_t used;
};

struct GraphCache {
  std::mutex mu;
  std::vector<Graph> graphs;
  std::vector<std::pair<uint64_t, int>> seen;
  uint64_t tick = 0;
  hipStream_t capture[kMaxDevices] = {};
};

GraphCache& cache() {
  static GraphCache* c = new GraphCache;  // never destroyed: graphs may be in flight at exit
  return *c;
}

bool same(const std::vector<LaunchRec>& a, const std::vector<LaunchRec>& b) {
  return a.size() == b.size() &&
         std::memcmp(a.data(), b.data(), a.size() * sizeof(LaunchRec)) == 0;
}

}  // namespace

hipError_t LaunchList::run(hipStream_t s, int path) {
  if (recs_.empty()) return hipSuccess;
  if ((path & WAVE_PATH_DIRECT) || recs_.size() < kMinGraphLaunches) return play(s);
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return play(s);
  const uint64_t h = fnv1a(recs_.data(), recs_.size() * sizeof(LaunchRec));
  GraphCache& C = cache();
  std::lock_guard<std::mutex> lk(C.mu);
  Graph* g = nullptr;
  for (Graph& q : C.graphs)
    if (q.hash == h && q.dev == dev && same(q.recs, recs_)) g = &q;
  if (g == nullptr) {
    const std::pair<uint64_t, int> key{h, dev};
    bool seen = false;
    for (const auto& k : C.seen) seen = seen || k == key;
    if (!seen && !(path & WAVE_PATH_GRAPH)) {
      if (C.seen.size() >= kMaxSeen) C.seen.erase(C.seen.begin());
      C.seen.push_back(key);
      return play(s);
    }
    if (C.capture[dev] == nullptr) {
      e = hipStreamCreateWithFlags(&C.capture[dev], hipStreamNonBlocking);
      if (e != hipSuccess) return e;
    }
    hipStream_t cs = C.capture[dev];
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    const hipError_t ep = play(cs);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    if (ep != hipSuccess || e != hipSuccess) {
      if (graph != nullptr) (void)hipGraphDestroy(graph);
      return ep != hipSuccess ? ep : e;
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return e;
    hipEvent_t done = nullptr;
    e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
    if (e != hipSuccess) {
      (void)hipGraphExecDestroy(exec);
      return e;
    }
    if (C.graphs.size() >= kMaxGraphs) {
      size_t old = 0;
      for (size_t i = 1; i < C.graphs.size(); ++i)
        if (C.graphs[i].used < C.graphs[old].used) old = i;
      Graph& v = C.graphs[old];
      (void)hipEventSynchronize(v.done);
      (void)hipGraphExecDestroy(v.exec);
      (void)hipEventDestroy(v.done);
      C.graphs.erase(C.graphs.begin() + old);
    }
    C.graphs.push_back(Graph{h, dev, recs_, exec, done, 0});
    g = &C.graphs.back();
  }
  g->used = ++C.tick;
  e = hipGraphLaunch(g->exec, s);
  if (e != hipSuccess) return e;
  return hipEventRecord(g->done, s);
}

}  // namespace wave
