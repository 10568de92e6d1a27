// wave_launch.h -- the kernel launches of one solve, recorded on the host and then
// either issued directly on the caller's stream or replayed from a cached HIP graph
// (internal; not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "wave_internal.h"

namespace wave {

struct LaunchRec {
  enum Kind : int { STEP = 1, STEP_BASIC, FUSED2, SAMPLE, PACK, UNPACK, COPY, ZERO };
  int kind, r, st;
  int grad, diff, nt;
  union {
    StepArgs a;  // STEP, STEP_BASIC
    Fused2Args f;  // FUSED2
    struct {
      const void* field;
      LevelMeta meta;
      int m, n;
      const int* idx;
      const float* w;
      float* out;
    } smp;  // SAMPLE
    struct {
      const float* src;
      float* dst;
      Geom g;
      int64_t count;
    } el;  // PACK, UNPACK, COPY, ZERO (dst as words)
  };
};

// Launches of one solve in order. Every recorded launch carries all of its
// arguments, so two lists with equal bytes launch the same kernels on the same
// data.
class LaunchList {
 public:
  void step(const StepArgs& a, int r, bool grad, int st, bool diff, bool nt);
  void step_basic(const StepArgs& a, int r);
  void fused2(const Fused2Args& f, int r, bool nt);
  void sample(const void* field, int st, LevelMeta meta, int m, const int* idx, const float* w,
              int n, float* out);
  void pack(const float* src, float* dst, Geom g);
  void unpack(const float* src, float* dst, Geom g);
  void copy(const float* src, float* dst, int64_t n);
  void zero_words(unsigned* p, int64_t n);
  size_t size() const { return recs_.size(); }
  // Issue the launches on s: directly, or from a cached graph of the same list.
  // path: the grid's WAVE_PATH_* flags. By default a list is captured into a graph
  // the second time the same list is run (equal bytes, same device) and replayed
  // from then on; WAVE_PATH_GRAPH captures at the first run, WAVE_PATH_DIRECT never.
  hipError_t run(hipStream_t s, int path);
  // Issue the launches directly on s.
  hipError_t play(hipStream_t s) const;

 private:
  LaunchRec& add(int kind);
  std::vector<LaunchRec> recs_;
};

}  // namespace wave
