// wave_internal.h -- data structures shared by the host runtime and the gfx950
// kernels of the acoustic solver (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wave {

// Stencil tile: TX x TY columns in the xy-plane, streamed along z. Each of the
// 256 threads owns VX consecutive x points of one row and keeps a register
// queue of 2r+1 z-planes; x/y neighbours come from an LDS copy of the plane.
constexpr int TX = 64;
constexpr int TY = 16;
constexpr int VX = 4;
constexpr int NTX = TX / VX;     // threads along x
constexpr int NTHREADS = NTX * TY;
constexpr int MAXR = 12;         // SO <= 24
constexpr int MAXZCHUNK = 256;   // planes per z-chunk at most (<= NTHREADS)
// One-step tiles stacked along y in one workgroup's tile of the one-step kernel:
// 1 (TX x TY points, NTHREADS threads) or 2 (TX x 2TY points, twice the threads:
// half the y-halo per point). The taller tile exists for the radii whose bit is set
// in WAVE_TALL_MASK; the host picks it per call (StepArgs::tiles_y) where the grid
// fills the CUs evenly with it. The injection tables stay in TY-row tiles; a taller
// tile reads them per sub-tile. Measured at 256^3 (one 512-thread workgroup per CU
// instead of two of 256): SO2 +1.5 %, SO4 +2.9 %, SO6 +2.9 %, SO8 +6.7 %, SO16
// +2.2 %, SO20 +1.8 %; SO14 level; SO10 -2.7 %, SO12 -2.9 %, SO18 -6.4 %, SO22
// -4.7 %, SO24 -3.6 %.
#ifndef WAVE_TALL_MASK
#define WAVE_TALL_MASK 0x51E  // radius 1-4, 8 and 10
#endif
constexpr bool tall_tiles_ok(int r) { return (((WAVE_TALL_MASK) >> r) & 1) != 0; }
constexpr int SAMPLE_THREADS = 256;

// Pitched field geometry: rows padded to a multiple of 32 floats (128 bytes);
// padding columns hold zeros, also in the v^2 dt^2 array, so they stay zero.
struct Geom {
  int nx, ny, nz, pitch;
  int64_t plane;    // pitch * ny
  int64_t nfield;   // pitch * ny * nz (elements)
};

// One injection entry: a grid point inside a tile at plane z, with its local
// index in the tile and a range of (trace index, weight) terms.
struct InjEntry {
  int z;        // plane
  int local;    // (j - tile_y) * TX + (i - tile_x)
  int csr_beg;  // terms [csr_beg, csr_end)
  int csr_end;
  int grp_end;  // end of the run of entries on this entry's plane (in its tile)
  int tidx;     // an entry with a single term: its trace index (else -1)
  float w;      //   and its weight
  int pad;
};
static_assert(sizeof(InjEntry) == 32, "entries are loaded as two 16-byte vectors");

// Storage formats of the wavefield levels (arithmetic is FP32 in all of them).
enum StoreKind { ST_F32 = 0, ST_F16 = 1, ST_BF16 = 2 };

// Reduced-precision levels are stored as value * 2^e (e an integer chosen per level
// so that the level's bound maps below 2^kScaleTarget). Per-level bookkeeping in
// device memory, L = nt + 3 entries each, level m at index m + 1:
//   mu[(m+1)*kMaxSlots + s], md[...]  bits of max|u^m| and max|u^m - u^{m-1}|
//                     (atomicMax of the non-negative float bits written while
//                     encoding level m); workgroup b updates slot b % kMaxSlots, so
//                     the atomics of one launch spread over kMaxSlots addresses, and
//                     the level's maximum is the maximum over its slots
//   injb[n]           bound on the injected increment of step n
//   eu[m+1], ed[m+1]  scale exponents of level m's u and difference arrays
constexpr int kScaleTarget = 12;
constexpr int kMaxSlots = 32;
struct LevelMeta {
  unsigned* mu;
  unsigned* md;
  float* injb;
  int* eu;
  int* ed;
};

struct StepArgs {
  // fields (pitched); element type given by the storage kind
  const void* cur;    // level read with neighbours (u^n or lambda^{n+1})
  const void* prev;   // read at the point only: u^{n-1} (or the difference u^n - u^{n-1})
  void* out;          // result written in place of prev (u^{n+1}, or the new difference)
  void* out_u;        // difference form only: u^{n+1} (the other u buffer)
  const float* c2;    // v^2 dt^2 (FP32)
  const float* bx;    // dt gamma_x / 2 per x (pitch entries, zero padded)
  const float* by;    // per y
  const float* bz;    // per z
  Geom g;
  // tiling
  int ntile_x, ntile_y, nchunk, zchunk;
  int nstencil_blocks;
  int tiles_y;        // one-step tiles per workgroup along y (1, or 2 where tall_tiles_ok)
  int xcd_remap;      // 1: contiguous tile ranges per XCD
  // weights pre-scaled by h_a^-2; wc = -2 sum_{q>=2} (wx+wy+wz) (the q = 1 pairs are
  // taken about the centre)
  float wx[MAXR + 1], wy[MAXR + 1], wz[MAXR + 1];
  float wc;
  float dt;           // time step (the unfactorised ablation kernel only)
  // fused injection into `out`: entry lists per column (xy tile, plane), numbered
  // (ty * ntile_x + tx) * nz + z; tile_beg[c] is column c's first entry, so a
  // workgroup's planes [z0, z1) of xy tile xy are entries tile_beg[xy nz + z0] ..
  // tile_beg[xy nz + z1] whatever the chunking
  const int* tile_beg;         // [ntile_x * ntile_y * nz + 1]
  const InjEntry* ent;
  const int* csr_idx;          // trace index
  const float* csr_w;          // weight
  const float* trace_row;      // samples of this step (indexed by csr_idx) or null
  // fused sampling of `cur` (extra blocks after the stencil blocks)
  const int* samp_idx;         // [nsamp][8] pitched element index
  const float* samp_w;         // [nsamp][8]
  int nsamp;
  float* samp_out;             // row of nsamp outputs, or null for none
  // fused accumulation (gradient kernels): grad += ufwd * c2 * (L_h cur + injection),
  // or with acc_image set grad += ufwd * cur (zero-lag cross-correlation image)
  const float* ufwd;
  float* grad;
  int acc_image;
  // reduced-precision storage: level index n of `cur`, and the bookkeeping
  int level;
  LevelMeta meta;
};

// Two fused leapfrog steps per pass (FP32 forward, radius <= 4): u^n, u^{n-1} ->
// u^{n+1}, u^{n+2}. In `a`: cur = u^n, prev = u^{n-1}, out = u^{n+1}; the tile
// injection tables with trace_row = step n+1's samples (added to u^{n+2});
// sampling of cur into samp_out. The extended-tile tables inject step n's samples
// into u^{n+1} over each tile's extended region.
// A two-step tile is K one-step tiles stacked along y (TX x K*TY points): K = 1
// (512 threads) up to radius 3, K = 2 (768 threads) at radius 4, where the taller
// tile halves the extended region's overhead per point and a workgroup has 12
// waves. The launch's tile counts (a.ntile_y, a.nstencil_blocks) are in two-step
// tiles; the tile injection tables are the one-step tiling's (ntile_y1 tiles along
// y), read per sub-tile.
constexpr int f2_tiles_y(int r) { return r == 4 ? 2 : 1; }
constexpr int f2_threads(int r) { return r == 4 ? 768 : 512; }
constexpr int F2_THREADS_MAX = 768;
struct Fused2Args {
  StepArgs a;
  int ntile_y1;              // one-step tiles along y (the tile tables' tiling)
  float* out2;               // u^{n+2}
  const int* etile_beg;      // [ntiles + 1] entries over the extended tiles
  const InjEntry* eent;      // local = row * (TX + 8) + column within the extended tile
  const int* ecsr_idx;
  const float* ecsr_w;
  const float* etrace_row;   // step n's samples, or null
  float* samp_out2;          // samples of prev (u^{n-1}), or null
};

// Serving: a resident shot and one entry of a batched launch's tile table.
struct ShotDesc {
  StepArgs a;              // static per-shot arguments (tables, geometry, weights)
  float* buf[2];           // the two pitched u buffers: level n lives in buf[n & 1]
  const float* wavelet;    // [nt][nsrc]
  float* traces;           // [nt][nrec]
  int nsrc, nrec, nt;
};
// The engine's step counters live beside the descriptors, two per slot
// (cnts[2 * slot + parity], see batched_step_kernel): the descriptors stay
// read-only in the kernel, so its arguments can be held like kernel arguments.
struct BatchEntry {
  int shot;   // slot in the descriptor array
  int xy;     // xy tile ty * ntile_x + tx of a stencil block (ty in rows of the launch's
              // workgroup tiles), or -1-k for sampling block k
  int z0, z1; // the stencil block's planes [z0, z1) (at most MAXZCHUNK)
};

// Launchers (wave_kernels.hip). All return hipGetLastError() after the launch.
// st: StoreKind; diff: difference-form storage (reduced precision only); nt:
// non-temporal loads/stores of the streamed arrays (prev, c2, out).
hipError_t launch_step(const StepArgs& a, int r, bool grad, int st, bool diff, bool nt,
                       hipStream_t s);
// ablation: one FP32 forward step in the unfactorised form of the paper's SO2
// listing (every term divided by r0 separately), radius r in {4, 6, 8, 12}
hipError_t launch_step_basic(const StepArgs& a, int r, hipStream_t s);
// two fused steps (radius r <= 4); nt: non-temporal stores of the two outputs
hipError_t launch_fused2(const Fused2Args& f, int r, bool nt, hipStream_t s);
// one batched step of every shot in table: nentries entries, the first nstencil of them
// stencil blocks, then sampling blocks (space-order radius r, workgroups of tiles_y
// one-step tiles along y: 1, or 2 where tall_tiles_ok(r); launch parity)
hipError_t launch_batched(const ShotDesc* shots, int* cnts, const BatchEntry* table, int nentries,
                          int nstencil, int r, int tiles_y, int parity, hipStream_t s);
// out[i] = shots[slots[i]].cnt[0]
hipError_t launch_gather_counters(const int* cnts, const int* slots, int n, int* out,
                                  hipStream_t s);
// out[i] = sum_c w[8i+c] field[idx[8i+c]], the field decoded with level m's scale
hipError_t launch_sample(const void* field, int st, LevelMeta meta, int m, const int* idx,
                         const float* w, int n, float* out, hipStream_t s);
// dst (pitched, zero padded) = src (dense) or zero when src is null
hipError_t launch_pack(const float* src, float* dst, Geom g, hipStream_t s);
// dst (dense) = src (pitched)
hipError_t launch_unpack(const float* src, float* dst, Geom g, hipStream_t s);
// c2 (pitched) = (float)(v^2 dt^2) computed in double
hipError_t launch_prep_c2(const float* vel, float* c2, Geom g, double dt, hipStream_t s);
// grad_vel (dense) = scale * graw / v^3
hipError_t launch_grad_finalize(const float* graw, const float* vel, float* grad_vel, Geom g,
                                double scale, hipStream_t s);
// dst = src for n floats
hipError_t launch_copy(const float* src, float* dst, int64_t n, hipStream_t s);
// reduced precision: zero n words
hipError_t launch_zero_words(unsigned* p, int64_t n, hipStream_t s);
// injb[k] = c2max * 8 * max_j |trace[k][j]| for k < nt (bound of one step's injection)
hipError_t launch_inj_bound(const float* trace, int nt, int ntr, float c2max, float* injb,
                            hipStream_t s);
// initial levels (dense FP32, null = zero): record max|a| (and max|a - b| when
// diff) for level m, choose its scales, then encode a (and a - b, or b as level
// m - 1 in the naive form) into the pitched stores
hipError_t launch_encode_initial(const float* a, const float* b, void* ua, void* ub, int st,
                                 bool diff, LevelMeta meta, int m, Geom g, hipStream_t s);
// dst (dense FP32) = decoded level m of src (pitched, storage st)
hipError_t launch_decode(const void* src, int st, LevelMeta meta, int m, float* dst, Geom g,
                         hipStream_t s);

}  // namespace wave
