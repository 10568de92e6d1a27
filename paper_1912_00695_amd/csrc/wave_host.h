// wave_host.h -- host-side helpers shared by the solver entry points
// (wave_api.cpp) and the serving engine (wave_engine.cpp); internal.
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <utility>
#include <vector>

#include "../../include/wave.h"
#include "wave_internal.h"

namespace wave {

constexpr size_t kAlign = 256;
constexpr int kDefaultCkpt = 50;

constexpr int kCUs = 256;  // compute units of an MI355X

struct Tiling {
  int ntile_x, ntile_y, nchunk, zchunk, nblocks;  // in one-step (TX x TY) tiles
  int tiles_y;  // one-step tiles per workgroup of the one-step kernel along y
};

struct PointTables {  // offsets into the workspace
  size_t tile_beg, ent, csr_idx, csr_w, samp_idx, samp_w;
};

// Workspace layout of one call (offsets from the workspace base).
struct Layout {
  size_t c2, bx, by, bz, u[2], d, meta;
  PointTables pts[2];  // 0: sources, 1: receivers
  bool fused;          // FP32 forward with radius <= 4: two more levels and the
  size_t ux[2];        //   extended-tile source tables of the two-step kernel
  PointTables epts;
  size_t tables_beg, tables_end;
  size_t graw, lam[2], seg, ick;  // gradient mode
  int ckpt_every, nseg;
  size_t total;
};

// Host image of the table region, in page-locked memory from a process-wide pool of
// staging buffers (plain heap memory if that allocation fails), so that its upload
// is an asynchronous copy; the buffer returns to the pool when the Blob is deleted
// (after the upload, from the stream's host callback). Uninitialised (the point
// tables are sized for 8 corners per point, most of it unused for on-grid points):
// the builders record the ranges they write, and only those are uploaded.
struct Blob {
  char* bytes = nullptr;
  bool pinned = false;
  size_t base = 0;
  std::vector<std::pair<size_t, size_t>> used;  // (offset from base, bytes)
  Blob() = default;
  Blob(const Blob&) = delete;
  Blob& operator=(const Blob&) = delete;
  ~Blob();
  // take n bytes of storage: page-locked from the staging pool when pinned is set
  // (and the pool can provide it), else ordinary heap memory
  void alloc(size_t n, bool pinned = true);
  template <class T>
  T* at(size_t off) { return reinterpret_cast<T*>(bytes + (off - base)); }
  void mark(size_t off, size_t n) {
    if (n > 0) used.push_back({off - base, n});
  }
};
// Enqueue the upload of b's written ranges into the table region at dst (the
// device address of the region's start).
hipError_t upload_blob(const Blob& b, char* dst, hipStream_t s);

// Per-call state.
struct Ctx {
  const wave_grid* g;
  Geom G;
  Tiling T;
  Layout L;
  char* ws;
  hipStream_t s;
  bool nt;  // streamed arrays bypass the caches (working set above the Infinity Cache)
  int path;  // the grid's WAVE_PATH_* flags
  double wx[MAXR + 1], wy[MAXR + 1], wz[MAXR + 1], wc;
  template <class T>
  T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
};

#define HIP_TRY(x)                              \
  do {                                          \
    if ((x) != hipSuccess) return WAVE_EDEVICE; \
  } while (0)

// Static workspace of wave_forward_noalloc (wave_scratch.cpp): its size, and its
// device address on the current device (WAVE_OK, or WAVE_EDEVICE).
constexpr size_t kScratchBytes = (size_t)64 << 20;
int scratch_address(void** out);

size_t align_up(size_t v);
bool grid_ok(const wave_grid* g);
int validate(const wave_grid* g);  // grid_ok + stability limit
bool points_ok(const wave_grid* g, const double* xyz, int np);
Geom make_geom(const wave_grid* g);
// zchunk > 0 fixes the z-chunk length; 0 applies the single-solve policy (which
// depends on the storage, WAVE_STORE_* flags). r, path (WAVE_PATH_* flags) and the
// storage choose the one-step kernel's workgroup height.
Tiling make_tiling(const Geom& G, int r, int path, int zchunk, int storage);
// fused_levels: an FP32 forward layout at radius <= 4 also holds the two-step
// kernel's two extra levels and extended-tile tables (false: one-step only)
Layout make_layout(const wave_grid* g, int nsrc, int nrec, int mode, int ckpt_every,
                   bool fused_levels = true);
// geometry, tiling, layout and weights of a call on workspace ws (no device work)
int init_ctx(Ctx& C, const wave_grid* g, int nsrc, int nrec, int mode, int ckpt_every, void* ws,
             size_t ws_bytes, void* stream, int zchunk = 0, bool fused_levels = true);
Blob* build_blob(const Ctx& C, const double* src, int nsrc, const double* rec, int nrec,
                 bool pinned = true);
StepArgs base_args(const Ctx& C);
void set_inj(StepArgs& a, const Ctx& C, int set, int np, const float* row);
void set_samp(StepArgs& a, const Ctx& C, int set, int np, float* row);

}  // namespace wave
