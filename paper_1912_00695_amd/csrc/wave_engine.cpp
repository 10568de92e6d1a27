// wave_engine.cpp -- continuous-batching shot server behind include/wave.h.
//
// One engine owns one HBM pool (allocated once, at create), a descriptor array of
// resident shots, and a worker thread that drives the GPU:
//   * submit() copies a request's inputs to the host side of the engine and queues
//     it (a request that can never fit the budget is rejected with WAVE_EBUSY);
//   * the worker admits queued requests first-come first-served, skipping ahead to
//     later ones that fit when the head does not, whenever a slot and pool space
//     are free; an uploader thread then copies the inputs and builds the shot's
//     tables on an upload stream while resident shots keep running (host-pageable
//     copies block the calling thread, so they stay off the thread that feeds
//     the GPU);
//   * resident shots advance in groups (one space order, per-step arrays that fit
//     the Infinity Cache together): a captured graph of kReplaySteps launches of
//     the batched step kernel per group, group after group, is replayed; each
//     group's launch table lists (shot, xy tile, planes) per workgroup, with the
//     group's own z-chunk length; per-shot step counters live in device memory, so
//     one graph serves any mix of shots at any step, and is re-captured only when
//     the set of resident shots changes;
//   * the graph is launched several times back to back (up to the first shot's
//     finish, bounded by kSyncWork of estimated GPU time while requests wait)
//     before the worker reads the counters back, completes finished shots (traces
//     copied to the caller's host buffer, latency recorded; their pool space is
//     freed at the next rebuild) and admits more.
// Every shot's arithmetic is the single-shot kernel's (shared tile function), so
// a result does not depend on the batch it ran in.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/wave.h"
#include "wave_host.h"
#include "wave_internal.h"
#include "wave_sched.h"

namespace wave {
namespace {

constexpr int kReplaySteps = 16;    // launches per group in one captured graph (even)
constexpr double kSyncWork = 2e-3;  // GPU seconds of work between host syncs while shots wait
constexpr double kSyncWorkIdle = 10e-3;  // ... and while none waits
constexpr double kUpdateRate = 250e9;  // grid-point updates per second, for that estimate
// z-chunk length of a cache group's shots, chosen when the group's table is built
// (the injection tables do not depend on it): the longest of 32, 24, ..., 1 planes
// that gives the group at least 512 stencil workgroups (a grid that fixes its
// zchunk keeps it). A group of one mid-sized shot gets short chunks that fill the
// GPU (192^3 SO8 alone: 32-plane chunks, 217 workgroups, ran 29 us per step against
// 20.6 with 14-plane chunks); a group of several shots keeps long chunks, which
// re-read fewer planes to prime their queues.
constexpr int kChunkLens[] = {32, 24, 16, 12, 8, 6, 4, 3, 2, 1};
// Cache groups whose 64 x 32 workgroups fill the CUs evenly are stepped on them.
#ifndef WAVE_ENGINE_TALL
#define WAVE_ENGINE_TALL 1
#endif
constexpr bool kEngineTall = WAVE_ENGINE_TALL != 0;
constexpr int kEngineZChunk = 32;  // tiling of a shot's context (tables are chunk-free)
// Shots stepped together in one run of kReplaySteps launches: their per-step arrays
// (two levels and v^2 dt^2) fit the 256 MB Infinity Cache together, so they stay
// cache-resident across the run's steps. wave_engine_set_group_bytes overrides.
constexpr size_t kCacheGroupBytes = (size_t)224 << 20;

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

using sched::PoolAlloc;

enum ShotState { QUEUED = 0, ADMITTED = 5, UPLOADING = 1, ACTIVE = 2, DONE = 3, FAILED = 4 };

struct Shot {
  uint64_t id = 0;
  wave_grid g{};
  std::vector<float> vel, wavelet;
  std::vector<double> src, rec;
  int nsrc = 0, nrec = 0;
  float* rec_out_h = nullptr;
  // device placement
  size_t off = 0, bytes = 0;
  int slot = -1;
  Ctx C{};
  size_t off_wav = 0, off_tr = 0;
  std::unique_ptr<Blob> blob;
  ShotDesc desc{};
  hipEvent_t ready = nullptr;
  std::atomic<int> state{QUEUED};
  int counter = 0;
  int status = WAVE_EAGAIN;
  int cnt0[2] = {0, 0};  // initial step counters (upload source)
  size_t entries = 0;    // its workgroups in the current graph's table
  double t_submit = 0, t_admit = 0, t_done = 0;
};

size_t shot_bytes(const wave_grid* g, int nsrc, int nrec) {
  const Layout L = make_layout(g, nsrc, nrec, WAVE_MODE_FORWARD, 0, false);
  return L.total + align_up((size_t)g->nt * nsrc * sizeof(float)) +
         align_up((size_t)g->nt * nrec * sizeof(float));
}

class Engine {
 public:
  Engine(size_t budget, int max_slots) : budget_(budget), max_slots_(max_slots), alloc_(budget) {}

  void set_group_bytes(size_t b) { group_bytes_.store(b); }

  int init() {
    HIP_TRY(hipGetDevice(&device_));
    HIP_TRY(hipMalloc(&pool_, budget_));
    HIP_TRY(hipMalloc(&d_desc_, sizeof(ShotDesc) * max_slots_));
    HIP_TRY(hipMalloc(&d_cnt_, sizeof(int) * 2 * max_slots_));
    table_cap_ = 1 << 20;
    for (int k = 0; k < 2; ++k) HIP_TRY(hipMalloc(&d_table_[k], sizeof(BatchEntry) * table_cap_));
    HIP_TRY(hipMalloc(&d_slots_, sizeof(int) * max_slots_));
    HIP_TRY(hipMalloc(&d_counts_, sizeof(int) * max_slots_));
    HIP_TRY(hipHostMalloc(&h_counts_, sizeof(int) * max_slots_, hipHostMallocDefault));
    HIP_TRY(hipStreamCreateWithFlags(&s_exec_, hipStreamNonBlocking));
    HIP_TRY(hipStreamCreateWithFlags(&s_up_, hipStreamNonBlocking));
    slot_used_.assign(max_slots_, 0);
    worker_ = std::thread([this] { loop(); });
    uploader_ = std::thread([this] { upload_loop(); });
    return WAVE_OK;
  }

  ~Engine() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    {
      std::lock_guard<std::mutex> lk(up_mu_);
      stop_up_ = true;
    }
    cv_.notify_all();
    up_cv_.notify_all();
    if (worker_.joinable()) worker_.join();
    if (uploader_.joinable()) uploader_.join();
    (void)hipSetDevice(device_);
    if (s_exec_) (void)hipStreamSynchronize(s_exec_);
    if (s_up_) (void)hipStreamSynchronize(s_up_);
    if (gexec_) (void)hipGraphExecDestroy(gexec_);
    for (auto& kv : shots_)
      if (kv.second->ready) (void)hipEventDestroy(kv.second->ready);
    if (s_exec_) (void)hipStreamDestroy(s_exec_);
    if (s_up_) (void)hipStreamDestroy(s_up_);
    if (h_counts_) (void)hipHostFree(h_counts_);
    if (d_counts_) (void)hipFree(d_counts_);
    if (d_slots_) (void)hipFree(d_slots_);
    for (int k = 0; k < 2; ++k)
      if (d_table_[k]) (void)hipFree(d_table_[k]);
    if (d_desc_) (void)hipFree(d_desc_);
    if (d_cnt_) (void)hipFree(d_cnt_);
    if (pool_) (void)hipFree(pool_);
  }

  int submit(const wave_request* r, uint64_t* id) {
    if (r == nullptr || id == nullptr) return WAVE_EINVAL;
    const wave_grid* g = &r->grid;
    int st = validate(g);
    if (st) return st;
    if (g->storage != WAVE_STORE_F32) return WAVE_EINVAL;
    if (r->vel_h == nullptr || r->nsrc < 0 || r->nrec < 0) return WAVE_EINVAL;
    if (r->nsrc > 0 && r->wavelet_h == nullptr) return WAVE_EINVAL;
    if (r->nrec > 0 && r->rec_out_h == nullptr) return WAVE_EINVAL;
    if (!points_ok(g, r->src_xyz_h, r->nsrc) || !points_ok(g, r->rec_xyz_h, r->nrec))
      return WAVE_EINVAL;
    auto sh = std::make_unique<Shot>();
    sh->g = *g;
    sh->nsrc = r->nsrc;
    sh->nrec = r->nrec;
    sh->bytes = shot_bytes(g, r->nsrc, r->nrec);
    {
      std::lock_guard<std::mutex> lk(mu_);
      ++submitted_;
      if (sh->bytes > budget_) {
        ++rejected_;
        return WAVE_EBUSY;
      }
    }
    const size_t n = (size_t)g->nx * g->ny * g->nz;
    sh->vel.assign(r->vel_h, r->vel_h + n);
    if (r->nsrc > 0)
      sh->wavelet.assign(r->wavelet_h, r->wavelet_h + (size_t)g->nt * r->nsrc);
    if (r->nsrc > 0) sh->src.assign(r->src_xyz_h, r->src_xyz_h + 3 * (size_t)r->nsrc);
    if (r->nrec > 0) sh->rec.assign(r->rec_xyz_h, r->rec_xyz_h + 3 * (size_t)r->nrec);
    sh->rec_out_h = r->rec_out_h;
    sh->t_submit = now_s();
    {
      std::lock_guard<std::mutex> lk(mu_);
      sh->id = ++next_id_;
      *id = sh->id;
      if (first_submit_ == 0) first_submit_ = sh->t_submit;
      queue_.push_back(sh.get());
      shots_[sh->id] = std::move(sh);
    }
    cv_.notify_all();
    return WAVE_OK;
  }

  int poll(uint64_t id, wave_result* res) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = shots_.find(id);
    if (it == shots_.end()) return WAVE_EINVAL;
    const Shot* s = it->second.get();
    if (res != nullptr) {
      res->status = s->status;
      res->t_submit = s->t_submit;
      res->t_admit = s->t_admit;
      res->t_done = s->t_done;
    }
    return s->status;
  }

  int stats(wave_stats* st) {
    if (st == nullptr) return WAVE_EINVAL;
    std::lock_guard<std::mutex> lk(mu_);
    std::memset(st, 0, sizeof(*st));
    st->submitted = submitted_;
    st->admitted = admitted_;
    st->completed = lat_.size();
    st->rejected = rejected_;
    st->queued = queue_.size();
    st->resident = resident_;
    if (!lat_.empty()) {
      st->p50_latency_s = sched::percentile(lat_, 0.50);
      st->p99_latency_s = sched::percentile(lat_, 0.99);
      double sum = 0, mx = 0;
      for (double x : lat_) {
        sum += x;
        mx = std::max(mx, x);
      }
      st->mean_latency_s = sum / lat_.size();
      st->max_latency_s = mx;
    }
    st->total_gpt = total_updates_ / 1e9;
    st->busy_s = busy_s_;
    st->span_s = last_done_ > first_submit_ ? last_done_ - first_submit_ : 0.0;
    st->graph_builds = graph_builds_;
    st->replays = replays_;
    st->max_resident = max_resident_;
    st->max_pool_bytes = max_pool_bytes_;
    return WAVE_OK;
  }

  int drain(double timeout_s) {
    const double t_end = now_s() + timeout_s;
    std::unique_lock<std::mutex> lk(mu_);
    while (!(queue_.empty() && resident_ == 0)) {
      if (now_s() > t_end) return WAVE_EAGAIN;
      done_cv_.wait_for(lk, std::chrono::milliseconds(5));
    }
    return WAVE_OK;
  }

 private:
  // ---- worker ----
  void loop() {
    (void)hipSetDevice(device_);
    std::vector<Shot*> resident;  // UPLOADING or ACTIVE, worker-owned view
    std::vector<Shot*> finished;  // done, slot and pool space not yet released
    bool dirty = true;
    double busy_t0 = 0;
    while (true) {
      std::vector<Shot*> incoming;
      {
        std::unique_lock<std::mutex> lk(mu_);
        if (stop_) break;
        if (resident.empty() && queue_.empty()) {
          if (!finished.empty()) {
            lk.unlock();
            for (Shot* s : finished) release(s);
            finished.clear();
            dirty = true;
            continue;
          }
          cv_.wait_for(lk, std::chrono::milliseconds(2));
          continue;
        }
        // admission: FIFO with skip-ahead over requests that fit
        int nfree = 0;
        for (int i = 0; i < max_slots_; ++i) nfree += slot_used_[i] ? 0 : 1;
        std::vector<size_t> qb;
        for (Shot* s : queue_) qb.push_back(s->bytes);
        const std::vector<sched::Admission> adm = sched::admit(qb, alloc_, nfree);
        for (const sched::Admission& ad : adm) {
          Shot* s = queue_[ad.pos];
          const int slot = free_slot();
          s->off = ad.off;
          s->slot = slot;
          slot_used_[slot] = 1;
          pool_used_ += align_up(s->bytes);
          max_pool_bytes_ = std::max(max_pool_bytes_, pool_used_);
          ++admitted_;
          ++resident_;
          max_resident_ = std::max<uint64_t>(max_resident_, resident_);
          s->t_admit = now_s();
          incoming.push_back(s);
        }
        for (size_t k = adm.size(); k-- > 0;) queue_.erase(queue_.begin() + adm[k].pos);
      }
      if (!incoming.empty()) {
        for (Shot* s : incoming) {
          s->state = ADMITTED;
          resident.push_back(s);
        }
        {
          std::lock_guard<std::mutex> lk(up_mu_);
          for (Shot* s : incoming) upload_q_.push_back(s);
        }
        up_cv_.notify_all();
      }
      // drop shots whose upload failed
      {
        std::vector<Shot*> keep;
        for (Shot* s : resident)
          if (s->state != FAILED) keep.push_back(s);
        resident.swap(keep);
      }
      // promote finished uploads (the graph is rebuilt: finished shots leave it)
      for (Shot* s : resident)
        if (s->state.load(std::memory_order_acquire) == UPLOADING &&
            hipEventQuery(s->ready) == hipSuccess) {
          s->state = ACTIVE;
          s->blob.reset();
          std::vector<float>().swap(s->vel);
          dirty = true;
        }
      if (dirty && !finished.empty()) {
        for (Shot* s : finished) release(s);
        finished.clear();
      }
      std::vector<Shot*> active;
      for (Shot* s : resident)
        if (s->state == ACTIVE) active.push_back(s);
      if (active.empty()) {
        if (!resident.empty()) std::this_thread::sleep_for(std::chrono::microseconds(50));
        continue;
      }
      if (busy_t0 == 0) busy_t0 = now_s();
      if (dirty) {
        if (rebuild_graph(active) != WAVE_OK) {
          for (Shot* s : active) fail(s);
          resident.clear();
          continue;
        }
        dirty = false;
      }
      // Replays back to back until the first resident shot can have finished (its
      // remaining steps are known), within a time budget: short while shots are
      // waiting to be admitted or promoted (they join at the next sync), longer
      // otherwise; then read back the counters.
      double pts = 0;
      int to_finish = INT_MAX;
      for (Shot* s : active) {
        pts += (double)s->g.nx * s->g.ny * s->g.nz;
        const int left = std::max(1, s->g.nt + 1 - s->counter);
        to_finish = std::min(to_finish, (left + kReplaySteps - 1) / kReplaySteps);
      }
      bool pending = resident.size() > active.size();
      {
        std::lock_guard<std::mutex> lk(mu_);
        pending = pending || !queue_.empty();
      }
      const double step_s = std::max(2e-6, pts / kUpdateRate);
      const double budget = pending ? kSyncWork : kSyncWorkIdle;
      const int reps = std::max(
          1, std::min({to_finish, 256, (int)(budget / (kReplaySteps * step_s))}));
      bool launched = true;
      for (int k = 0; k < reps && launched; ++k) launched = hipGraphLaunch(gexec_, s_exec_) == hipSuccess;
      // counters of the shots in the graph, in the slot order the last rebuild uploaded
      // (the active set can shrink between rebuilds: finished shots stay in the graph)
      const int ng = (int)graph_shots_.size();
      if (!launched ||
          launch_gather_counters(d_cnt_, d_slots_, ng, d_counts_, s_exec_) != hipSuccess ||
          hipMemcpyAsync(h_counts_, d_counts_, sizeof(int) * ng, hipMemcpyDeviceToHost,
                         s_exec_) != hipSuccess ||
          hipStreamSynchronize(s_exec_) != hipSuccess) {
        for (Shot* s : resident) fail(s);
        resident.clear();
        continue;
      }
      ++replays_;
      // Finished shots complete at once (traces copied back, latency recorded); their
      // slots and pool space stay reserved, and their table entries in the graph
      // (which do nothing past nt), until the graph is rebuilt anyway (new shots
      // active), a queued request or an idle engine needs them back, or their idle
      // workgroups reach a quarter of a launch.
      std::vector<Shot*> keep;
      for (int i = 0; i < ng; ++i) graph_shots_[i]->counter = h_counts_[i];
      for (Shot* s : resident) {
        if (s->state == ACTIVE && s->counter > s->g.nt) {
          finish(s);
          finished.push_back(s);
        } else {
          keep.push_back(s);
        }
      }
      resident.swap(keep);
      bool any_active = false, waiting = false;
      for (Shot* s : resident) any_active = any_active || s->state == ACTIVE;
      {
        std::lock_guard<std::mutex> lk(mu_);
        waiting = !queue_.empty();
      }
      // idle workgroups of finished shots: rebuild once they are a quarter of a launch
      size_t idle_entries = 0;
      for (Shot* s : finished) idle_entries += s->entries;
      if (!finished.empty() && (waiting || !any_active || 4 * idle_entries > graph_entries_)) {
        for (Shot* s : finished) release(s);
        finished.clear();
        dirty = true;
      }
      if (resident.empty() && busy_t0 > 0) {
        std::lock_guard<std::mutex> lk(mu_);
        busy_s_ += now_s() - busy_t0;
        busy_t0 = 0;
      }
    }
  }

  // Uploader thread: runs start_upload for admitted shots in admission order.
  void upload_loop() {
    (void)hipSetDevice(device_);
    while (true) {
      Shot* s = nullptr;
      {
        std::unique_lock<std::mutex> lk(up_mu_);
        up_cv_.wait_for(lk, std::chrono::milliseconds(5),
                        [this] { return stop_up_ || !upload_q_.empty(); });
        if (stop_up_) return;
        if (upload_q_.empty()) {
          std::lock_guard<std::mutex> lk2(mu_);
          if (stop_) return;
          continue;
        }
        s = upload_q_.front();
        upload_q_.pop_front();
      }
      if (start_upload(s) != WAVE_OK) fail(s);
    }
  }

  int free_slot() const {
    for (int i = 0; i < max_slots_; ++i)
      if (!slot_used_[i]) return i;
    return -1;
  }

  // Device layout of a shot inside its pool region: the forward-mode workspace,
  // then the wavelet, then the traces.
  int start_upload(Shot* s) {
    char* base = static_cast<char*>(pool_) + s->off;
    const wave_grid* g = &s->g;
    // the launch's chunking is chosen per cache group (rebuild_graph); the tables
    // and the values do not depend on it
    int st = init_ctx(s->C, g, s->nsrc, s->nrec, WAVE_MODE_FORWARD, 0, base, s->bytes, s_up_,
                      kEngineZChunk, false);
    if (st) return st;
    s->C.g = &s->g;
    s->off_wav = s->C.L.total;
    s->off_tr = s->off_wav + align_up((size_t)g->nt * s->nsrc * sizeof(float));
    s->blob.reset(build_blob(s->C, s->src.data(), s->nsrc, s->rec.data(), s->nrec));
    float* U0 = s->C.at<float>(s->C.L.u[0]);
    float* U1 = s->C.at<float>(s->C.L.u[1]);
    // the velocity is staged in u[1] (dense fits in pitched), turned into c2, then
    // both u levels are cleared
    HIP_TRY(upload_blob(*s->blob, base + s->C.L.tables_beg, s_up_));
    HIP_TRY(hipMemcpyAsync(U1, s->vel.data(), s->vel.size() * sizeof(float),
                           hipMemcpyHostToDevice, s_up_));
    HIP_TRY(launch_prep_c2(U1, s->C.at<float>(s->C.L.c2), s->C.G, g->dt, s_up_));
    HIP_TRY(launch_pack(nullptr, U0, s->C.G, s_up_));
    HIP_TRY(launch_pack(nullptr, U1, s->C.G, s_up_));
    float* wav = reinterpret_cast<float*>(base + s->off_wav);
    if (s->nsrc > 0)
      HIP_TRY(hipMemcpyAsync(wav, s->wavelet.data(), s->wavelet.size() * sizeof(float),
                             hipMemcpyHostToDevice, s_up_));
    ShotDesc& d = s->desc;
    d.a = base_args(s->C);
    set_inj(d.a, s->C, 0, s->nsrc, s->nsrc > 0 ? wav : nullptr);
    set_samp(d.a, s->C, 1, s->nrec, reinterpret_cast<float*>(base + s->off_tr));
    d.buf[0] = U0;
    d.buf[1] = U1;
    d.wavelet = wav;
    d.traces = reinterpret_cast<float*>(base + s->off_tr);
    d.nsrc = s->nsrc;
    d.nrec = s->nrec;
    d.nt = g->nt;
    HIP_TRY(hipMemcpyAsync(d_desc_ + s->slot, &s->desc, sizeof(ShotDesc), hipMemcpyHostToDevice,
                           s_up_));
    HIP_TRY(hipMemcpyAsync(d_cnt_ + 2 * s->slot, s->cnt0, sizeof(s->cnt0), hipMemcpyHostToDevice,
                           s_up_));
    HIP_TRY(hipEventCreateWithFlags(&s->ready, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(s->ready, s_up_));
    s->state.store(UPLOADING, std::memory_order_release);
    return WAVE_OK;
  }

  // Tables of (shot, tile) per group, and the captured replay graph. A group holds
  // shots of one space order whose per-step arrays fit the Infinity Cache together
  // (first fit in admission order); the graph runs kReplaySteps launches of each
  // group back to back, so a group's fields are re-read from the cache on every
  // step of its run rather than streamed from HBM with every other resident shot's.
  int rebuild_graph(const std::vector<Shot*>& active) {
    struct Group {
      int r;
      size_t bytes;
      std::vector<Shot*> shots;
      std::vector<BatchEntry> e;  // stencil blocks of every shot, then sampling blocks
      int nstencil = 0;
      int ky = 1;  // workgroup height of the group's launches, in one-step tiles
    };
    const size_t gb = group_bytes_.load();
    const size_t cap = gb > 0 ? gb : kCacheGroupBytes;
    std::vector<Group> groups;
    std::vector<int> slots;
    graph_shots_.clear();
    for (Shot* s : active) {
      slots.push_back(s->slot);
      graph_shots_.push_back(s);
      const int r = s->g.so / 2;
      const size_t b = (size_t)s->C.G.nfield * 12;  // two FP32 levels and v^2 dt^2
      size_t gi = 0;
      while (gi < groups.size() && (groups[gi].r != r || groups[gi].bytes + b > cap)) ++gi;
      if (gi == groups.size()) groups.push_back(Group{r, 0, {}});
      Group& G = groups[gi];
      G.bytes += b;
      G.shots.push_back(s);
    }
    for (Group& G : groups) {
      int zc = 1;
      for (const int len : kChunkLens) {
        int64_t wg = 0;
        for (const Shot* s : G.shots) {
          const int z = s->g.zchunk > 0 ? s->g.zchunk : len;
          wg += (int64_t)s->C.T.ntile_x * s->C.T.ntile_y * ((s->g.nz + z - 1) / z);
        }
        if (wg >= 512) {
          zc = len;
          break;
        }
      }
      // Workgroups of two one-step tiles along y (the single-solve rule): where the
      // radius has them and the group's taller workgroups fill the CUs evenly, e.g. a
      // 256^3 shot alone in its group, in 32-plane chunks (256 workgroups).
      if (kEngineTall && tall_tiles_ok(G.r)) {
        int64_t tall = 0;
        for (const Shot* s : G.shots) {
          const int z = s->g.zchunk > 0 ? s->g.zchunk : zc;
          tall += (int64_t)s->C.T.ntile_x * ((s->C.T.ntile_y + 1) / 2) * ((s->g.nz + z - 1) / z);
        }
        if (tall >= kCUs && tall % kCUs == 0) G.ky = 2;
      }
      // every shot's stencil blocks chunk-major (the single-solve tile order), then
      // every shot's sampling blocks
      const int nth = G.ky * NTHREADS;
      for (Shot* s : G.shots) {
        const int z = s->g.zchunk > 0 ? s->g.zchunk : zc;
        const int bxy = s->C.T.ntile_x * ((s->C.T.ntile_y + G.ky - 1) / G.ky);
        const size_t e0 = G.e.size();
        for (int z0 = 0; z0 < s->g.nz; z0 += z)
          for (int xy = 0; xy < bxy; ++xy)
            G.e.push_back(BatchEntry{s->slot, xy, z0, std::min(z0 + z, s->g.nz)});
        s->entries = G.e.size() - e0;
      }
      G.nstencil = (int)G.e.size();
      for (Shot* s : G.shots) {
        const int nsb = s->nrec > 0 ? (s->nrec + nth - 1) / nth : 0;
        for (int k = 0; k < nsb; ++k) G.e.push_back(BatchEntry{s->slot, -1 - k, 0, 0});
        s->entries += nsb;
      }
    }
    struct Seg {
      int r, ky, off, count, nstencil;
    };
    std::vector<BatchEntry> all;
    std::vector<Seg> segs;
    graph_entries_ = 0;
    for (auto& G : groups) {
      segs.push_back(Seg{G.r, G.ky, (int)all.size(), (int)G.e.size(), G.nstencil});
      all.insert(all.end(), G.e.begin(), G.e.end());
    }
    if ((int)all.size() > table_cap_) return WAVE_ENOMEM;
    graph_entries_ = all.size();
    cur_table_ ^= 1;
    BatchEntry* tab = d_table_[cur_table_];
    HIP_TRY(hipMemcpyAsync(tab, all.data(), all.size() * sizeof(BatchEntry),
                           hipMemcpyHostToDevice, s_exec_));
    HIP_TRY(hipMemcpyAsync(d_slots_, slots.data(), slots.size() * sizeof(int),
                           hipMemcpyHostToDevice, s_exec_));
    HIP_TRY(hipStreamSynchronize(s_exec_));
    hipGraph_t graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(s_exec_, hipStreamCaptureModeThreadLocal));
    hipError_t err = hipSuccess;
    for (const Seg& sg : segs)
      for (int k = 0; k < kReplaySteps && err == hipSuccess; ++k)
        err = launch_batched(d_desc_, d_cnt_, tab + sg.off, sg.count, sg.nstencil, sg.r, sg.ky, k & 1,
                             s_exec_);
    hipError_t e2 = hipStreamEndCapture(s_exec_, &graph);
    if (err != hipSuccess || e2 != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return WAVE_EDEVICE;
    }
    if (gexec_) (void)hipGraphExecDestroy(gexec_);
    gexec_ = nullptr;
    err = hipGraphInstantiate(&gexec_, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (err != hipSuccess) return WAVE_EDEVICE;
    ++graph_builds_;
    return WAVE_OK;
  }

  // The shot's traces go back to the caller's buffer and its request completes.
  void finish(Shot* s) {
    bool ok = true;
    if (s->nrec > 0 && s->rec_out_h != nullptr)
      ok = hipMemcpyAsync(s->rec_out_h, s->desc.traces, sizeof(float) * (size_t)s->g.nt * s->nrec,
                          hipMemcpyDeviceToHost, s_exec_) == hipSuccess &&
           hipStreamSynchronize(s_exec_) == hipSuccess;
    if (s->ready) {
      (void)hipEventDestroy(s->ready);
      s->ready = nullptr;
    }
    std::lock_guard<std::mutex> lk(mu_);
    s->t_done = now_s();
    s->status = ok ? WAVE_OK : WAVE_EDEVICE;
    s->state = ok ? DONE : FAILED;
    if (ok) {
      lat_.push_back(s->t_done - s->t_submit);
      total_updates_ += (double)s->g.nx * s->g.ny * s->g.nz * s->g.nt;
      last_done_ = s->t_done;
    }
    std::vector<float>().swap(s->wavelet);
    done_cv_.notify_all();
  }

  // Slot and pool space of a finished shot become free (the caller rebuilds the
  // graph before the next replay, so no launch refers to them any more).
  void release(Shot* s) {
    std::lock_guard<std::mutex> lk(mu_);
    if (s->slot < 0) return;
    alloc_.release(s->off, s->bytes);
    pool_used_ -= align_up(s->bytes);
    slot_used_[s->slot] = 0;
    s->slot = -1;
    --resident_;
    done_cv_.notify_all();
  }

  void fail(Shot* s) {
    std::lock_guard<std::mutex> lk(mu_);
    s->status = WAVE_EDEVICE;
    s->state = FAILED;
    s->t_done = now_s();
    if (s->slot >= 0) {
      alloc_.release(s->off, s->bytes);
      pool_used_ -= align_up(s->bytes);
      slot_used_[s->slot] = 0;
      s->slot = -1;
      --resident_;
    }
    done_cv_.notify_all();
  }

  size_t budget_;
  int max_slots_;
  std::atomic<size_t> group_bytes_{0};
  int device_ = 0;
  void* pool_ = nullptr;
  PoolAlloc alloc_;
  size_t pool_used_ = 0, max_pool_bytes_ = 0;
  ShotDesc* d_desc_ = nullptr;
  int* d_cnt_ = nullptr;  // step counters, two per slot (cnts[2 * slot + parity])
  BatchEntry* d_table_[2] = {nullptr, nullptr};
  int table_cap_ = 0, cur_table_ = 0;
  int* d_slots_ = nullptr;
  int* d_counts_ = nullptr;
  int* h_counts_ = nullptr;
  hipStream_t s_exec_ = nullptr, s_up_ = nullptr;
  hipGraphExec_t gexec_ = nullptr;
  std::vector<Shot*> graph_shots_;  // shots of the current graph, in d_slots_ order
  size_t graph_entries_ = 0;        // table entries (workgroups) of one launch of each group
  std::vector<char> slot_used_;
  std::thread worker_, uploader_;
  std::mutex mu_, up_mu_;
  std::condition_variable up_cv_;
  std::deque<Shot*> upload_q_;
  bool stop_up_ = false;
  std::condition_variable cv_, done_cv_;
  bool stop_ = false;
  std::deque<Shot*> queue_;
  std::unordered_map<uint64_t, std::unique_ptr<Shot>> shots_;
  uint64_t next_id_ = 0, submitted_ = 0, admitted_ = 0, rejected_ = 0, resident_ = 0;
  uint64_t max_resident_ = 0, graph_builds_ = 0, replays_ = 0;
  std::vector<double> lat_;
  double total_updates_ = 0, busy_s_ = 0, first_submit_ = 0, last_done_ = 0;
};

}  // namespace
}  // namespace wave

using wave::Engine;

extern "C" {

int wave_engine_create(size_t hbm_budget_bytes, int max_slots, void** engine) {
  if (engine == nullptr || max_slots < 1 || max_slots > 4096 || hbm_budget_bytes < 4096)
    return WAVE_EINVAL;
  *engine = nullptr;
  Engine* e = new Engine(hbm_budget_bytes, max_slots);
  const int st = e->init();
  if (st != WAVE_OK) {
    delete e;
    return st;
  }
  *engine = e;
  return WAVE_OK;
}

int wave_engine_submit(void* engine, const wave_request* req, uint64_t* id) {
  if (engine == nullptr) return WAVE_EINVAL;
  return static_cast<Engine*>(engine)->submit(req, id);
}

int wave_engine_poll(void* engine, uint64_t id, wave_result* res) {
  if (engine == nullptr) return WAVE_EINVAL;
  return static_cast<Engine*>(engine)->poll(id, res);
}

int wave_engine_stats(void* engine, wave_stats* st) {
  if (engine == nullptr) return WAVE_EINVAL;
  return static_cast<Engine*>(engine)->stats(st);
}

int wave_engine_drain(void* engine, double timeout_s) {
  if (engine == nullptr) return WAVE_EINVAL;
  return static_cast<Engine*>(engine)->drain(timeout_s);
}

void wave_engine_destroy(void* engine) { delete static_cast<Engine*>(engine); }

int wave_engine_set_group_bytes(void* engine, size_t bytes) {
  if (engine == nullptr) return WAVE_EINVAL;
  static_cast<Engine*>(engine)->set_group_bytes(bytes);
  return WAVE_OK;
}

size_t wave_engine_request_bytes(const wave_grid* g, int nsrc, int nrec) {
  if (!wave::grid_ok(g) || nsrc < 0 || nrec < 0) return 0;
  return wave::align_up(wave::shot_bytes(g, nsrc, nrec));
}

}  // extern "C"
