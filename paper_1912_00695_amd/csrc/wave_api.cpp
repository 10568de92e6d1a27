// wave_api.cpp -- host runtime behind include/wave.h: argument validation,
// workspace layout, injection/sampling tables, and the time-loop drivers of
// the forward, adjoint and gradient solves.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/wave.h"
#include "wave_host.h"
#include "wave_internal.h"
#include "wave_launch.h"

namespace wave {

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Centred second-derivative weights of order 2r, closed form:
// w_q = 2 (-1)^{q+1} (r!)^2 / (q^2 (r-q)! (r+q)!), w_0 = -2 sum_q 1/q^2.
void fd_weights(int so, double* w) {
  const int r = so / 2;
  double s = 0.0;
  for (int q = 1; q <= r; ++q) {
    // (r!)^2 / ((r-q)! (r+q)!) = prod_{i=1..q} (r-q+i) / (r+i)
    double ratio = 1.0;
    for (int i = 1; i <= q; ++i) ratio *= (double)(r - q + i) / (double)(r + i);
    w[q] = 2.0 * ((q % 2) ? 1.0 : -1.0) * ratio / ((double)q * q);
    s += 1.0 / ((double)q * q);
  }
  w[0] = -2.0 * s;
}

bool grid_ok(const wave_grid* g) {
  if (g == nullptr) return false;
  if (g->nx < 1 || g->ny < 1 || g->nz < 1) return false;
  if (g->so < 2 || g->so > 2 * MAXR || g->so % 2) return false;
  if (!(g->hx > 0 && g->hy > 0 && g->hz > 0 && g->dt > 0 && g->vmax > 0)) return false;
  if (!std::isfinite(g->hx) || !std::isfinite(g->hy) || !std::isfinite(g->hz) ||
      !std::isfinite(g->dt) || !std::isfinite(g->vmax))
    return false;
  if (g->nt < 0) return false;
  const int n[3] = {g->nx, g->ny, g->nz};
  for (int a = 0; a < 3; ++a) {
    if (g->nbl[2 * a] < 0 || g->nbl[2 * a + 1] < 0) return false;
    if (g->nbl[2 * a] + g->nbl[2 * a + 1] > n[a]) return false;
  }
  const int st = g->storage & ~WAVE_STORE_DIFF;
  if (st != WAVE_STORE_F32 && st != WAVE_STORE_F16 && st != WAVE_STORE_BF16) return false;
  if (st == WAVE_STORE_F32 && (g->storage & WAVE_STORE_DIFF)) return false;
  if (g->path & ~(WAVE_PATH_ONE_STEP | WAVE_PATH_TWO_STEP | WAVE_PATH_STREAM |
                  WAVE_PATH_CACHED | WAVE_PATH_LINEAR | WAVE_PATH_GRAPH | WAVE_PATH_DIRECT |
                  WAVE_PATH_TILE16 | WAVE_PATH_TILE32))
    return false;
  if ((g->path & WAVE_PATH_TILE16) && (g->path & WAVE_PATH_TILE32)) return false;
  if ((g->path & WAVE_PATH_GRAPH) && (g->path & WAVE_PATH_DIRECT)) return false;
  if ((g->path & WAVE_PATH_ONE_STEP) && (g->path & WAVE_PATH_TWO_STEP)) return false;
  if ((g->path & WAVE_PATH_STREAM) && (g->path & WAVE_PATH_CACHED)) return false;
  if (g->zchunk < 0 || g->zchunk > MAXZCHUNK) return false;
  const int64_t pitch = (g->nx + 31) / 32 * 32;
  if (pitch * g->ny * (int64_t)g->nz >= ((int64_t)1 << 31)) return false;
  // one FP32 plane must stay below 2 GiB (the kernels' buffer loads use 32-bit offsets)
  if (pitch * g->ny * (int64_t)sizeof(float) >= ((int64_t)1 << 31)) return false;
  return true;
}

Geom make_geom(const wave_grid* g) {
  Geom G;
  G.nx = g->nx; G.ny = g->ny; G.nz = g->nz;
  G.pitch = (g->nx + 31) / 32 * 32;
  G.plane = (int64_t)G.pitch * G.ny;
  G.nfield = G.plane * G.nz;
  return G;
}

// z-chunking: floor(512 / tiles per plane) chunks (at least one): about 512
// workgroups, two per CU, all resident at once, each sweeping one long chunk.
// Measured on MI355X at SO8, among the chunk lengths tried: 256^3 best at 32 planes
// (512 workgroups), 384^3 at 128 (432), 448^3 at 224 (392), 512^3 at 256 (512). More
// workgroups at once (576-1024) lost 5-15 %, several rounds of short chunks (the
// previous policy for large grids: 20 planes) lost 3-6 % at SO8, fewer than ~400
// workgroups leave CUs idle. Long chunks also amortise the 2r planes each chunk
// re-reads to prime its z queue, so the gain grows with the order (512^3 over
// 20-plane chunks: +5 % SO8, +11 % SO16, +23 % SO24; FP32 and the 16-bit difference
// form). Small grids get short chunks from the same rule (64^3: 1 plane, 256
// workgroups; 128^3: 4 planes): there a step takes a few microseconds and the
// workgroup count sets it (64^3 SO4 with graph replay: 4.5 us per step at 1-plane
// chunks against 8.5 at 8-plane chunks; 128^3 SO4: 7.5 against 9.0). The naive
// 16-bit form (short_chunks) keeps chunks of 8..32 planes for about 512 workgroups,
// and balanced chunks of about 20 planes, swept in several rounds, for grids that
// would need more than 1024 workgroups at 32 planes: 546 Gpt/s at 512^3 SO8 against
// 498 with one long chunk per workgroup. A positive zchunk fixes the chunk length
// (the grid's zchunk, or the caller's policy).
Tiling make_tiling(const Geom& G, int r, int path, int zchunk, int storage) {
  const int kind = storage & ~WAVE_STORE_DIFF;
  const bool short_chunks = kind != WAVE_STORE_F32 && !(storage & WAVE_STORE_DIFF);
  Tiling T;
  T.ntile_x = (G.nx + TX - 1) / TX;
  T.ntile_y = (G.ny + TY - 1) / TY;
  const int bxy = T.ntile_x * T.ntile_y;
  int zc = zchunk;
  if (zc <= 0 && short_chunks) {
    const int want = std::max(1, (512 + bxy - 1) / bxy);
    zc = std::min(std::max((G.nz + want - 1) / want, 8), 32);
    if ((int64_t)bxy * ((G.nz + 31) / 32) > 1024) {
      const int nch = (G.nz + 19) / 20;
      zc = (G.nz + nch - 1) / nch;
    }
  } else if (zc <= 0) {
    const int nch = std::max(1, 512 / bxy);
    zc = (G.nz + nch - 1) / nch;
  }
  zc = std::max(1, std::min({zc, G.nz, MAXZCHUNK}));
  T.zchunk = zc;
  T.nchunk = (G.nz + zc - 1) / zc;
  T.nblocks = bxy * T.nchunk;
  // Workgroup height of the one-step kernel: two one-step tiles along y where the
  // radius has that form and the taller workgroups fill the 256 CUs evenly (a
  // multiple of 256). Measured at SO8 with the chunks above: 256^3 +6.7 % and 512^3
  // +2.2 % (256 workgroups each); 320^3 -6 %, 384^3 -6 %, 448^3 -4 % (250, 216 and 196
  // workgroups: idle CUs). Uneven counts are worse still: a CU given two of them runs
  // out of VALU issue (the kernel keeps about 45 % of it busy at SO8): 288 workgroups
  // at 384^3 (96-plane chunks) -23 %. With 16-bit storage (2-byte halos) the taller
  // tiles do not pay: 512^3 SO8 -0.5 % in the difference form, -2.3 % naive (FP32
  // +3 %), so those keep 64 x 16 unless WAVE_PATH_TILE32 asks.
  T.tiles_y = 1;
  if (tall_tiles_ok(r) && !(path & WAVE_PATH_TILE16)) {
    const int64_t tall = (int64_t)T.ntile_x * ((T.ntile_y + 1) / 2) * T.nchunk;
    if ((path & WAVE_PATH_TILE32) ||
        (kind == WAVE_STORE_F32 && tall >= kCUs && tall % kCUs == 0))
      T.tiles_y = 2;
  }
  return T;
}

int64_t max_tiles(const Geom& G) {
  return (int64_t)((G.nx + TX - 1) / TX) * ((G.ny + TY - 1) / TY) * G.nz;
}

// ---------------------------------------------------------------------------
// Workspace layout.
int store_kind(const wave_grid* g) { return g->storage & ~WAVE_STORE_DIFF; }
bool store_diff(const wave_grid* g) { return (g->storage & WAVE_STORE_DIFF) != 0; }

Layout make_layout(const wave_grid* g, int nsrc, int nrec, int mode, int ckpt_every,
                   bool fused_levels) {
  const Geom G = make_geom(g);
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
  const size_t fbytes = (size_t)G.nfield * sizeof(float);
  const size_t ubytes = (size_t)G.nfield * (store_kind(g) == WAVE_STORE_F32 ? 4 : 2);
  L.c2 = take(fbytes);
  L.u[0] = take(ubytes);
  L.u[1] = take(ubytes);
  L.d = store_diff(g) ? take(ubytes) : 0;
  L.meta = store_kind(g) != WAVE_STORE_F32
               ? take((size_t)(2 * kMaxSlots + 3) * (g->nt + 3) * sizeof(unsigned))
               : 0;
  L.tables_beg = off;
  L.bx = take((size_t)G.pitch * sizeof(float));
  L.by = take((size_t)G.ny * sizeof(float));
  L.bz = take((size_t)G.nz * sizeof(float));
  const int64_t nt = max_tiles(G);
  const int np[2] = {nsrc, nrec};
  for (int s = 0; s < 2; ++s) {
    const size_t n8 = (size_t)8 * std::max(np[s], 0);
    L.pts[s].tile_beg = take((size_t)(nt + 1) * sizeof(int));
    L.pts[s].ent = take(n8 * sizeof(InjEntry));
    L.pts[s].csr_idx = take(n8 * sizeof(int));
    L.pts[s].csr_w = take(n8 * sizeof(float));
    L.pts[s].samp_idx = take(n8 * sizeof(int));
    L.pts[s].samp_w = take(n8 * sizeof(float));
  }
  L.fused = fused_levels && mode == WAVE_MODE_FORWARD && store_kind(g) == WAVE_STORE_F32 &&
            g->so / 2 <= 4;
  if (L.fused) {
    // each corner of a source lies in the extended region of at most 2 tiles per
    // axis (x extension 4 < TX, y extension r <= 4 < TY, z extension r <= 4 <= half
    // the shortest chunk)
    const size_t n64 = (size_t)64 * std::max(nsrc, 0);
    L.epts.tile_beg = take((size_t)(max_tiles(G) + 1) * sizeof(int));
    L.epts.ent = take(n64 * sizeof(InjEntry));
    L.epts.csr_idx = take(n64 * sizeof(int));
    L.epts.csr_w = take(n64 * sizeof(float));
  }
  L.tables_end = off;
  if (L.fused) {
    L.ux[0] = take(fbytes);
    L.ux[1] = take(fbytes);
  }
  if (mode == WAVE_MODE_GRADIENT) {
    const int C = ckpt_every > 0 ? ckpt_every : kDefaultCkpt;
    L.ckpt_every = C;
    L.nseg = g->nt > 0 ? (g->nt + C - 1) / C : 0;
    const int seglen = std::min(C, std::max(g->nt, 1));
    L.graw = take(fbytes);
    L.lam[0] = take(fbytes);
    L.lam[1] = take(fbytes);
    L.seg = take(fbytes * (size_t)(seglen + 2));
    L.ick = take(fbytes * (size_t)(2 * L.nseg));
  }
  L.total = off;
  return L;
}

// ---------------------------------------------------------------------------
// Trilinear corners of a point (metres); corners of weight exactly 0 dropped.
// Returns false when the point lies outside [0, (n-1) h] on some axis.
bool corners(const wave_grid* g, const double* xyz, int* ijk, double* w, int* cnt) {
  const double f[3] = {xyz[0] / g->hx, xyz[1] / g->hy, xyz[2] / g->hz};
  const int n[3] = {g->nx, g->ny, g->nz};
  int i0[3];
  double t[3];
  for (int a = 0; a < 3; ++a) {
    if (!(f[a] >= 0.0) || f[a] > (double)(n[a] - 1)) return false;
    i0[a] = (int)std::floor(f[a]);
    t[a] = f[a] - (double)i0[a];
  }
  int c = 0;
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        const double wt = (dx ? t[0] : 1.0 - t[0]) * (dy ? t[1] : 1.0 - t[1]) *
                          (dz ? t[2] : 1.0 - t[2]);
        if (wt == 0.0) continue;
        ijk[3 * c + 0] = i0[0] + dx;
        ijk[3 * c + 1] = i0[1] + dy;
        ijk[3 * c + 2] = i0[2] + dz;
        w[c] = wt;
        ++c;
      }
  *cnt = c;
  return true;
}

bool points_ok(const wave_grid* g, const double* xyz, int np) {
  if (np < 0) return false;
  if (np > 0 && xyz == nullptr) return false;
  int ijk[24], c;
  double w[8];
  for (int p = 0; p < np; ++p)
    if (!corners(g, xyz + 3 * p, ijk, w, &c)) return false;
  return true;
}


// Injection tables in "column" order, independent of the z-chunking: a column is
// one xy tile (TX x TY points) on one plane, numbered (xy tile) * nz + z with xy
// tile = ty * ntile_x + tx; tile_beg[c] is the first entry of column c, so the
// entries of xy tile xy on planes [z0, z1) are tile_beg[xy nz + z0] ..
// tile_beg[xy nz + z1], for any chunk a kernel is given.
void build_point_tables(const wave_grid* g, const Geom& G, const Tiling& T, const double* xyz,
                        int np, const PointTables& P, Blob& B) {
  int* tile_beg = B.at<int>(P.tile_beg);
  const int ntiles = T.ntile_x * T.ntile_y * G.nz;  // columns
  std::fill(tile_beg, tile_beg + ntiles + 1, 0);
  // One term per (point, trilinear corner) in point order: the corner's column and
  // local index in the tile, the point and the weight. A stable counting sort by
  // column, then a stable sort of each column's terms by local index (skipped where
  // they are in that order already, as for points given in raster order on a grid
  // plane), puts the terms of one grid point together in point order, the order in
  // which the kernels sum them.
  struct Term {
    int tile, z, local, p;
    float w;
  };
  std::vector<Term> terms;
  terms.reserve((size_t)np * 8);
  std::vector<int> cnt((size_t)ntiles + 1, 0);
  int* sidx = B.at<int>(P.samp_idx);
  float* sw = B.at<float>(P.samp_w);
  for (int p = 0; p < np; ++p) {
    int ijk[24], c = 0;
    double w[8];
    corners(g, xyz + 3 * p, ijk, w, &c);
    for (int k = 0; k < 8; ++k) {
      sidx[8 * p + k] = 0;
      sw[8 * p + k] = 0.f;
    }
    for (int k = 0; k < c; ++k) {
      const int i = ijk[3 * k], j = ijk[3 * k + 1], z = ijk[3 * k + 2];
      sidx[8 * p + k] = (int)((int64_t)z * G.plane + (int64_t)j * G.pitch + i);
      sw[8 * p + k] = (float)w[k];
      const int tile = ((j / TY) * T.ntile_x + i / TX) * G.nz + z;
      terms.push_back(Term{tile, z, (j % TY) * TX + (i % TX), p, (float)w[k]});
      ++cnt[(size_t)tile + 1];
    }
  }
  for (int t = 0; t < ntiles; ++t) cnt[(size_t)t + 1] += cnt[t];
  std::vector<Term> sorted(terms.size());
  {
    std::vector<int> pos(cnt.begin(), cnt.end() - 1);
    for (const Term& q : terms) sorted[pos[q.tile]++] = q;
  }
  std::vector<Term>().swap(terms);
  // All terms of a column lie on one plane; each column is ordered by a stable
  // counting sort on the index in the tile (in cache).
  const auto by_local = [](const Term& a, const Term& b) { return a.local < b.local; };
  std::vector<Term> tmp;
  std::vector<int> pos;
  for (int t = 0; t < ntiles; ++t) {
    const auto b0 = sorted.begin() + cnt[t], b1 = sorted.begin() + cnt[(size_t)t + 1];
    if (b1 - b0 <= 1 || std::is_sorted(b0, b1, by_local)) continue;
    pos.assign((size_t)TX * TY + 1, 0);
    for (auto it = b0; it != b1; ++it) ++pos[(size_t)it->local + 1];
    for (int k = 0; k < TX * TY; ++k) pos[(size_t)k + 1] += pos[k];
    tmp.resize(b1 - b0);
    for (auto it = b0; it != b1; ++it) tmp[pos[(size_t)it->local]++] = *it;
    std::copy(tmp.begin(), tmp.end(), b0);
  }
  // one entry per distinct (column, local index), its terms in CSR order
  InjEntry* ent = B.at<InjEntry>(P.ent);
  int* cidx = B.at<int>(P.csr_idx);
  float* cw = B.at<float>(P.csr_w);
  int e = 0;
  const size_t nterm = sorted.size();
  for (size_t a = 0; a < nterm;) {
    const Term& h = sorted[a];
    size_t b = a;
    for (; b < nterm && sorted[b].tile == h.tile && sorted[b].z == h.z && sorted[b].local == h.local;
         ++b) {
      cidx[b] = sorted[b].p;
      cw[b] = sorted[b].w;
    }
    InjEntry en{};
    en.z = h.z;
    en.local = h.local;
    en.csr_beg = (int)a;
    en.csr_end = (int)b;
    en.tidx = b - a == 1 ? h.p : -1;
    en.w = b - a == 1 ? h.w : 0.f;
    ent[e++] = en;
    tile_beg[h.tile + 1]++;
    a = b;
  }
  for (int t = 0; t < ntiles; ++t) tile_beg[t + 1] += tile_beg[t];
  // group ends: a plane's group is its column
  for (int t = 0; t < ntiles; ++t)
    for (int k = tile_beg[t]; k < tile_beg[t + 1]; ++k) ent[k].grp_end = tile_beg[t + 1];
  B.mark(P.tile_beg, ((size_t)ntiles + 1) * sizeof(int));
  B.mark(P.ent, (size_t)e * sizeof(InjEntry));
  B.mark(P.csr_idx, nterm * sizeof(int));
  B.mark(P.csr_w, nterm * sizeof(float));
  B.mark(P.samp_idx, (size_t)8 * np * sizeof(int));
  B.mark(P.samp_w, (size_t)8 * np * sizeof(float));
}

// The two-step kernel needs chunks of at least 2r planes (a source corner then
// lies in the extended region of at most two chunks, which sizes its tables).
bool fused_tiling_ok(const Ctx& C) { return C.L.fused && C.T.zchunk >= C.g->so; }

// Whether an FP32 forward solve without checkpoints takes the two-step kernel, and
// its z-chunk length. Measured on MI355X (100-step solves, cubic grids, two-step vs
// the one-step kernel with its default tiling, halo ring and hints): SO2 +5 % at
// 320^3, -2.4 % at 352^3, +2 % at 384^3, +19 % at 512^3; SO4 -5 % at 320^3, -8 % at
// 384^3, +12 % at 416^3, 448^3 and 512^3; SO6 -15 % at 384^3, +1.7 % at 416^3, +1.5 %
// at 448^3, +2.5 % at 512^3; SO8 (tiles twice as tall, one 768-thread workgroup per CU)
// -8 % at 448^3, -3.5 % at 512^3, so at SO8 the one-step kernel is the default at
// every size. Below these sizes the one-step kernel's working set is largely served
// by the 256 MiB Infinity Cache; longer two-step chunks (128, 256 planes) lost at
// SO2/SO4/SO6. Chosen by the library: at least kFusedMinPoints[r] grid points.
// WAVE_PATH_TWO_STEP asks for it at radius <= 4, WAVE_PATH_ONE_STEP never takes it;
// its z-chunks are the grid's zchunk, else fused_zchunk's (at SO8 128-plane chunks
// where they give 512 workgroups: +5 % over 64-plane chunks at 512^3).
constexpr int64_t kFusedMinPoints[5] = {0, 30000000, 60000000, 80000000, INT64_MAX};
constexpr int kFusedZChunk = 64;
int fused_zchunk(const wave_grid* g) {
  const int r = g->so / 2;
  if (r == 4) {  // one 768-thread workgroup per CU: 128-plane chunks where they still
                 // give 512 workgroups, else 64 or 32 planes for at least 256
    const int64_t cols = (int64_t)((g->nx + TX - 1) / TX) *
                         ((g->ny + f2_tiles_y(r) * TY - 1) / (f2_tiles_y(r) * TY));
    if (cols * ((g->nz + 127) / 128) >= 512) return 128;
    if (cols * ((g->nz + 63) / 64) >= 256) return 64;
    return 32;
  }
  return kFusedZChunk;
}
bool want_fused(const wave_grid* g, int* zchunk) {
  *zchunk = g->zchunk > 0 ? g->zchunk : fused_zchunk(g);
  if (store_kind(g) != WAVE_STORE_F32 || g->so / 2 > 4) return false;
  if (g->path & WAVE_PATH_ONE_STEP) return false;
  if (g->path & WAVE_PATH_TWO_STEP) return true;
  const int64_t npts = (int64_t)g->nx * g->ny * g->nz;
  return npts >= kFusedMinPoints[g->so / 2];
}

// Source tables of the two-step kernel: for every two-step tile (f2_tiles_y(r)
// one-step tiles of T stacked along y, TY2 = f2_tiles_y(r) * TY rows), the grid
// points of its extended region (x in [xt - 4, xt + TX + 4), y in [yt - r, yt +
// TY2 + r), z in [z0 - r, z1 + r)), with local index row * (TX + 8) + column in
// that region. A point near a tile edge appears in the tables of every tile whose
// region holds it; each copy carries its own (point, weight) terms in the same order.
void build_ext_tables(const wave_grid* g, const Geom& G, const Tiling& T, int r, const double* xyz,
                      int np, const PointTables& P, Blob& B) {
  constexpr int XE = 4;
  const int TY2 = f2_tiles_y(r) * TY;
  const int nty = (T.ntile_y + f2_tiles_y(r) - 1) / f2_tiles_y(r);
  int* tile_beg = B.at<int>(P.tile_beg);
  const int ntiles = T.ntile_x * nty * T.nchunk;
  std::fill(tile_beg, tile_beg + ntiles + 1, 0);
  struct Key {
    int tile, z, local;
    bool operator<(const Key& o) const {
      return tile != o.tile ? tile < o.tile : z != o.z ? z < o.z : local < o.local;
    }
  };
  std::map<Key, std::vector<std::pair<int, float>>> uniq;
  for (int p = 0; p < np; ++p) {
    int ijk[24], c = 0;
    double w[8];
    corners(g, xyz + 3 * p, ijk, w, &c);
    for (int k = 0; k < c; ++k) {
      const int i = ijk[3 * k], j = ijk[3 * k + 1], z = ijk[3 * k + 2];
      for (int tx = std::max(0, i / TX - 1); tx <= std::min(T.ntile_x - 1, i / TX + 1); ++tx) {
        const int xt = tx * TX;
        if (i < xt - XE || i >= xt + TX + XE) continue;
        for (int ty = std::max(0, j / TY2 - 1); ty <= std::min(nty - 1, j / TY2 + 1); ++ty) {
          const int yt = ty * TY2;
          if (j < yt - r || j >= yt + TY2 + r) continue;
          for (int zc = std::max(0, z / T.zchunk - 1);
               zc <= std::min(T.nchunk - 1, z / T.zchunk + 1); ++zc) {
            const int z0 = zc * T.zchunk, z1 = std::min(z0 + T.zchunk, G.nz);
            if (z < z0 - r || z >= z1 + r) continue;
            const int tile = (zc * nty + ty) * T.ntile_x + tx;
            const int local = (j - (yt - r)) * (TX + 2 * XE) + (i - (xt - XE));
            uniq[Key{tile, z, local}].push_back({p, (float)w[k]});
          }
        }
      }
    }
  }
  InjEntry* ent = B.at<InjEntry>(P.ent);
  int* cidx = B.at<int>(P.csr_idx);
  float* cw = B.at<float>(P.csr_w);
  int e = 0, c = 0;
  for (auto& kv : uniq) {
    InjEntry en{};
    en.z = kv.first.z;
    en.local = kv.first.local;
    en.csr_beg = c;
    for (auto& pw : kv.second) {
      cidx[c] = pw.first;
      cw[c] = pw.second;
      ++c;
    }
    en.csr_end = c;
    en.tidx = c - en.csr_beg == 1 ? cidx[en.csr_beg] : -1;
    en.w = c - en.csr_beg == 1 ? cw[en.csr_beg] : 0.f;
    ent[e] = en;
    tile_beg[kv.first.tile + 1]++;
    ++e;
  }
  for (int t = 0; t < ntiles; ++t) tile_beg[t + 1] += tile_beg[t];
  for (int t = 0; t < ntiles; ++t) {
    int b = tile_beg[t], end = tile_beg[t + 1];
    while (b < end) {
      int q = b;
      while (q < end && ent[q].z == ent[b].z) ++q;
      for (int k = b; k < q; ++k) ent[k].grp_end = q;
      b = q;
    }
  }
  B.mark(P.tile_beg, ((size_t)ntiles + 1) * sizeof(int));
  B.mark(P.ent, (size_t)e * sizeof(InjEntry));
  B.mark(P.csr_idx, (size_t)c * sizeof(int));
  B.mark(P.csr_w, (size_t)c * sizeof(float));
}

void sponge_1d(int n, int lo, int hi, double h, double vmax, double dt, float* b) {
  const double pi = 3.14159265358979323846;
  std::vector<double> gam(n, 0.0);
  const int nbl[2] = {lo, hi};
  for (int f = 0; f < 2; ++f) {
    if (nbl[f] <= 0) continue;
    const double gmax = 3.0 * vmax * std::log(1000.0) / (2.0 * nbl[f] * h);
    for (int d = 0; d < nbl[f] && d < n; ++d) {
      const double p = (double)(nbl[f] - d) / nbl[f];
      gam[f == 0 ? d : n - 1 - d] += gmax * (p - std::sin(2.0 * pi * p) / (2.0 * pi));
    }
  }
  for (int i = 0; i < n; ++i) b[i] = (float)(0.5 * dt * gam[i]);
}

// Page-locked staging buffers for the table uploads, reused across calls: a buffer
// is taken for one call's tables and returned when that call's Blob is deleted,
// which for a solve happens in the stream's host callback after the upload has run
// (no HIP call is made there). The pool only grows, to at most the number of
// calls in flight at once, and lives until the process ends.
class StagingPool {
 public:
  char* take(size_t n) {
    std::lock_guard<std::mutex> lk(mu_);
    Buf* best = nullptr;
    for (Buf& b : bufs_)
      if (!b.busy && b.n >= n && (best == nullptr || b.n < best->n)) best = &b;
    if (best != nullptr) {
      best->busy = true;
      return best->p;
    }
    size_t sz = (size_t)1 << 20;
    while (sz < n) sz <<= 1;
    void* p = nullptr;
    if (hipHostMalloc(&p, sz, hipHostMallocDefault) != hipSuccess || p == nullptr) return nullptr;
    bufs_.push_back(Buf{static_cast<char*>(p), sz, true});
    return static_cast<char*>(p);
  }
  void give(char* p) {
    std::lock_guard<std::mutex> lk(mu_);
    for (Buf& b : bufs_)
      if (b.p == p) b.busy = false;
  }

 private:
  struct Buf {
    char* p;
    size_t n;
    bool busy;
  };
  std::mutex mu_;
  std::vector<Buf> bufs_;
};

StagingPool& staging() {
  static StagingPool* pool = new StagingPool;  // never destroyed: callbacks may run late
  return *pool;
}

void Blob::alloc(size_t n, bool want_pinned) {
  bytes = want_pinned ? staging().take(n) : nullptr;
  pinned = bytes != nullptr;
  if (!pinned) bytes = new char[n];
}

Blob::~Blob() {
  if (bytes == nullptr) return;
  if (pinned)
    staging().give(bytes);
  else
    delete[] bytes;
}

void delete_blob(void* p) { delete static_cast<Blob*>(p); }

hipError_t upload_blob(const Blob& b, char* dst, hipStream_t s) {
  for (const auto& r : b.used) {
    const hipError_t e =
        hipMemcpyAsync(dst + r.first, b.bytes + r.first, r.second, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

int init_ctx(Ctx& C, const wave_grid* g, int nsrc, int nrec, int mode, int ckpt_every, void* ws,
             size_t ws_bytes, void* stream, int zchunk, bool fused_levels) {
  C.g = g;
  C.G = make_geom(g);
  C.T = make_tiling(C.G, g->so / 2, g->path, zchunk > 0 ? zchunk : g->zchunk, g->storage);
  C.L = make_layout(g, nsrc, nrec, mode, ckpt_every, fused_levels);
  if (ws == nullptr || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0) return WAVE_EINVAL;
  if (ws_bytes < C.L.total) return WAVE_ENOMEM;
  C.ws = static_cast<char*>(ws);
  C.s = static_cast<hipStream_t>(stream);
  C.path = g->path;
  // Non-temporal hints on the streamed arrays when one step's fields (v^2 dt^2 and
  // the stored levels) exceed the 256 MiB Infinity Cache: measured on MI355X at
  // 512^3 they gain ~10 %; below it the cache serves the next step's reads and the
  // hints lose ~20 %. WAVE_PATH_STREAM / WAVE_PATH_CACHED decide instead.
  {
    const size_t es = store_kind(g) == WAVE_STORE_F32 ? 4 : 2;
    const size_t ws_bytes_step = (size_t)C.G.nfield * (4 + es * (store_diff(g) ? 3 : 2));
    C.nt = (g->path & WAVE_PATH_STREAM)   ? true
           : (g->path & WAVE_PATH_CACHED) ? false
                                          : ws_bytes_step > ((size_t)256 << 20);
  }
  double w[MAXR + 1];
  fd_weights(g->so, w);
  const double ix = 1.0 / (g->hx * g->hx), iy = 1.0 / (g->hy * g->hy), iz = 1.0 / (g->hz * g->hz);
  for (int q = 0; q <= MAXR; ++q) {
    const double v = q <= g->so / 2 ? w[q] : 0.0;
    C.wx[q] = v * ix; C.wy[q] = v * iy; C.wz[q] = v * iz;
  }
  // Centre weight of the terms q >= 2 (the q = 1 pairs are taken about the centre
  // in the kernel): minus twice the sum of the FP32-rounded weights, so that the
  // weights the kernel uses sum to zero up to one rounding of this value.
  double wc = 0.0;
  for (int q = 2; q <= g->so / 2; ++q)
    wc -= 2.0 * ((double)(float)C.wx[q] + (double)(float)C.wy[q] + (double)(float)C.wz[q]);
  C.wc = wc;
  return WAVE_OK;
}

// Host image of the tables (sponge profiles, injection and sampling tables).
Blob* build_blob(const Ctx& C, const double* src, int nsrc, const double* rec, int nrec,
                 bool pinned) {
  const wave_grid* g = C.g;
  Blob* B = new Blob;
  B->base = C.L.tables_beg;
  B->alloc(C.L.tables_end - C.L.tables_beg, pinned);
  float* bx = B->at<float>(C.L.bx);
  sponge_1d(g->nx, g->nbl[0], g->nbl[1], g->hx, g->vmax, g->dt, bx);
  std::fill(bx + g->nx, bx + C.G.pitch, 0.f);  // padding columns
  sponge_1d(g->ny, g->nbl[2], g->nbl[3], g->hy, g->vmax, g->dt, B->at<float>(C.L.by));
  sponge_1d(g->nz, g->nbl[4], g->nbl[5], g->hz, g->vmax, g->dt, B->at<float>(C.L.bz));
  B->mark(C.L.bx, (size_t)C.G.pitch * sizeof(float));
  B->mark(C.L.by, (size_t)g->ny * sizeof(float));
  B->mark(C.L.bz, (size_t)g->nz * sizeof(float));
  build_point_tables(g, C.G, C.T, src, nsrc, C.L.pts[0], *B);
  build_point_tables(g, C.G, C.T, rec, nrec, C.L.pts[1], *B);
  if (fused_tiling_ok(C)) build_ext_tables(g, C.G, C.T, g->so / 2, src, nsrc, C.L.epts, *B);
  return B;
}

// noalloc: one-step layout and tables staged in ordinary heap memory (no HIP
// allocation anywhere in the call)
int setup(Ctx& C, const wave_grid* g, const float* vel, const double* src, int nsrc,
          const double* rec, int nrec, int mode, int ckpt_every, void* ws, size_t ws_bytes,
          void* stream, int zchunk = 0, bool noalloc = false) {
  int st = init_ctx(C, g, nsrc, nrec, mode, ckpt_every, ws, ws_bytes, stream, zchunk, !noalloc);
  if (st) return st;
  Blob* B = build_blob(C, src, nsrc, rec, nrec, !noalloc);
  if (upload_blob(*B, C.ws + C.L.tables_beg, C.s) != hipSuccess) {
    delete B;
    return WAVE_EDEVICE;
  }
  if (hipLaunchHostFunc(C.s, delete_blob, B) != hipSuccess) {
    (void)hipStreamSynchronize(C.s);
    delete B;
    return WAVE_EDEVICE;
  }
  HIP_TRY(launch_prep_c2(vel, C.at<float>(C.L.c2), C.G, g->dt, C.s));
  return WAVE_OK;
}

LevelMeta level_meta(const Ctx& C) {
  LevelMeta m{};
  if (C.L.meta == 0) return m;
  const int64_t L = C.g->nt + 3;
  unsigned* base = C.at<unsigned>(C.L.meta);
  m.mu = base;
  m.md = base + kMaxSlots * L;
  m.injb = reinterpret_cast<float*>(base + 2 * kMaxSlots * L);
  m.eu = reinterpret_cast<int*>(base + (2 * kMaxSlots + 1) * L);
  m.ed = reinterpret_cast<int*>(base + (2 * kMaxSlots + 2) * L);
  return m;
}

StepArgs base_args(const Ctx& C) {
  StepArgs a{};
  a.meta = level_meta(C);
  a.c2 = C.at<float>(C.L.c2);
  a.bx = C.at<float>(C.L.bx);
  a.by = C.at<float>(C.L.by);
  a.bz = C.at<float>(C.L.bz);
  a.g = C.G;
  a.ntile_x = C.T.ntile_x;
  a.ntile_y = C.T.ntile_y;
  a.nchunk = C.T.nchunk;
  a.zchunk = C.T.zchunk;
  // the one-step kernel's workgroups tile T.tiles_y one-step tiles along y
  a.tiles_y = C.T.tiles_y;
  a.nstencil_blocks = C.T.ntile_x * ((C.T.ntile_y + a.tiles_y - 1) / a.tiles_y) * C.T.nchunk;
  a.xcd_remap = (C.g->path & WAVE_PATH_LINEAR) == 0;
  for (int q = 0; q <= MAXR; ++q) {
    a.wx[q] = (float)C.wx[q];
    a.wy[q] = (float)C.wy[q];
    a.wz[q] = (float)C.wz[q];
  }
  a.wc = (float)C.wc;
  a.dt = (float)C.g->dt;
  return a;
}

void set_inj(StepArgs& a, const Ctx& C, int set, int np, const float* row) {
  if (np > 0 && row != nullptr) {
    const PointTables& P = C.L.pts[set];
    a.tile_beg = C.at<int>(P.tile_beg);
    a.ent = C.at<InjEntry>(P.ent);
    a.csr_idx = C.at<int>(P.csr_idx);
    a.csr_w = C.at<float>(P.csr_w);
    a.trace_row = row;
  } else {
    a.tile_beg = nullptr; a.ent = nullptr; a.csr_idx = nullptr; a.csr_w = nullptr;
    a.trace_row = nullptr;
  }
}

void set_samp(StepArgs& a, const Ctx& C, int set, int np, float* row) {
  if (np > 0 && row != nullptr) {
    const PointTables& P = C.L.pts[set];
    a.samp_idx = C.at<int>(P.samp_idx);
    a.samp_w = C.at<float>(P.samp_w);
    a.nsamp = np;
    a.samp_out = row;
  } else {
    a.samp_idx = nullptr; a.samp_w = nullptr; a.nsamp = 0; a.samp_out = nullptr;
  }
}

// Forward solve with 16-bit wavefield storage (FP32 arithmetic). Naive form:
// levels u^n, u^{n-1}; difference form: u^n and d^n = u^n - u^{n-1}.
int forward_reduced(Ctx& C, const float* wavelet, int nsrc, int nrec, float* rec_out,
                    const float* u0, const float* um1, float* u_final) {
  const wave_grid* g = C.g;
  const int stk = store_kind(g) == WAVE_STORE_F16 ? ST_F16 : ST_BF16;
  const bool diff = store_diff(g);
  const LevelMeta meta = level_meta(C);
  void* U[2] = {C.ws + C.L.u[0], C.ws + C.L.u[1]};
  void* D = diff ? C.ws + C.L.d : nullptr;
  HIP_TRY(launch_zero_words(meta.mu, (int64_t)(2 * kMaxSlots + 3) * (g->nt + 3), C.s));
  const float c2max = (float)(g->vmax * g->vmax * g->dt * g->dt);
  if (nsrc > 0) HIP_TRY(launch_inj_bound(wavelet, g->nt, nsrc, c2max, meta.injb, C.s));
  HIP_TRY(launch_encode_initial(u0, um1, U[0], diff ? D : U[1], stk, diff, meta, 0, C.G, C.s));
  StepArgs a = base_args(C);
  const int r = g->so / 2;
  LaunchList LL;
  for (int n = 0; n < g->nt; ++n) {
    a.level = n;
    a.cur = U[n & 1];
    if (diff) {
      a.prev = D;
      a.out = D;
      a.out_u = U[(n + 1) & 1];
    } else {
      a.prev = U[(n + 1) & 1];
      a.out = U[(n + 1) & 1];
      a.out_u = nullptr;
    }
    set_inj(a, C, 0, nsrc, nsrc > 0 ? wavelet + (int64_t)n * nsrc : nullptr);
    set_samp(a, C, 1, nrec, n >= 1 && nrec > 0 ? rec_out + (int64_t)(n - 1) * nrec : nullptr);
    LL.step(a, r, false, stk, diff, C.nt);
  }
  if (nrec > 0 && g->nt > 0) {
    const PointTables& P = C.L.pts[1];
    LL.sample(U[g->nt & 1], stk, meta, g->nt, C.at<int>(P.samp_idx), C.at<float>(P.samp_w), nrec,
              rec_out + (int64_t)(g->nt - 1) * nrec);
  }
  HIP_TRY(LL.run(C.s, C.path));
  if (u_final != nullptr) HIP_TRY(launch_decode(U[g->nt & 1], stk, meta, g->nt, u_final, C.G, C.s));
  return WAVE_OK;
}

// FP32 forward solve with two fused steps per launch (radius <= 4). Four level
// buffers: a pass reads u^n and u^{n-1} (with halos, also from neighbouring
// workgroups) and writes u^{n+1} and u^{n+2} into the other two. A pass at n >= 2
// also samples its two input levels: d^{n-1} = R u^n and d^{n-2} = R u^{n-1}. An
// odd step count ends with one single step.
int forward_fused(Ctx& C, const float* wavelet, int nsrc, int nrec, float* rec_out,
                  const float* u0, const float* um1, float* u_final) {
  const wave_grid* g = C.g;
  float* X[4] = {C.at<float>(C.L.u[0]), C.at<float>(C.L.u[1]), C.at<float>(C.L.ux[0]),
                 C.at<float>(C.L.ux[1])};
  LaunchList LL;
  LL.pack(u0, X[0], C.G);
  LL.pack(um1, X[1], C.G);
  LL.pack(nullptr, X[2], C.G);  // padding columns are never written
  LL.pack(nullptr, X[3], C.G);
  const int r = g->so / 2;
  const PointTables& PR = C.L.pts[1];
  Fused2Args f{};
  f.a = base_args(C);
  // launch in two-step tiles; the tile tables stay in the one-step tiling
  f.ntile_y1 = C.T.ntile_y;
  f.a.ntile_y = (C.T.ntile_y + f2_tiles_y(r) - 1) / f2_tiles_y(r);
  f.a.nstencil_blocks = C.T.ntile_x * f.a.ntile_y * C.T.nchunk;
  int cur = 0, prv = 1, o1 = 2, o2 = 3;
  int n = 0;
  for (; n + 2 <= g->nt; n += 2) {
    f.a.cur = X[cur];
    f.a.prev = X[prv];
    f.a.out = X[o1];
    f.out2 = X[o2];
    set_inj(f.a, C, 0, nsrc, nsrc > 0 ? wavelet + (int64_t)(n + 1) * nsrc : nullptr);
    if (nsrc > 0) {
      f.etile_beg = C.at<int>(C.L.epts.tile_beg);
      f.eent = C.at<InjEntry>(C.L.epts.ent);
      f.ecsr_idx = C.at<int>(C.L.epts.csr_idx);
      f.ecsr_w = C.at<float>(C.L.epts.csr_w);
      f.etrace_row = wavelet + (int64_t)n * nsrc;
    }
    set_samp(f.a, C, 1, nrec, n >= 2 && nrec > 0 ? rec_out + (int64_t)(n - 1) * nrec : nullptr);
    f.samp_out2 = n >= 2 && nrec > 0 ? rec_out + (int64_t)(n - 2) * nrec : nullptr;
    LL.fused2(f, r, C.nt);
    const int oc = cur, op = prv;
    cur = o2;
    prv = o1;
    o1 = op;
    o2 = oc;
  }
  // Levels now: X[cur] = u^n, X[prv] = u^{n-1}.
  if (nrec > 0 && n >= 2)  // d^{n-2}, before a single step overwrites u^{n-1}
    LL.sample(X[prv], ST_F32, LevelMeta{}, 0, C.at<int>(PR.samp_idx), C.at<float>(PR.samp_w), nrec,
              rec_out + (int64_t)(n - 2) * nrec);
  int last = cur;
  if (n < g->nt) {
    StepArgs a = base_args(C);
    a.cur = X[cur];
    a.prev = X[prv];
    a.out = X[prv];
    set_inj(a, C, 0, nsrc, nsrc > 0 ? wavelet + (int64_t)n * nsrc : nullptr);
    set_samp(a, C, 1, nrec, n >= 1 && nrec > 0 ? rec_out + (int64_t)(n - 1) * nrec : nullptr);
    LL.step(a, r, false, ST_F32, false, C.nt);
    last = prv;
  } else if (nrec > 0 && n >= 1) {  // d^{n-1} = R u^n (even step count)
    LL.sample(X[cur], ST_F32, LevelMeta{}, 0, C.at<int>(PR.samp_idx), C.at<float>(PR.samp_w), nrec,
              rec_out + (int64_t)(n - 1) * nrec);
  }
  if (nrec > 0 && n < g->nt)  // d^{nt-1} = R u^{nt} after the final single step
    LL.sample(X[last], ST_F32, LevelMeta{}, 0, C.at<int>(PR.samp_idx), C.at<float>(PR.samp_w), nrec,
              rec_out + (int64_t)(g->nt - 1) * nrec);
  if (u_final != nullptr) LL.unpack(X[last], u_final, C.G);
  HIP_TRY(LL.run(C.s, C.path));
  return WAVE_OK;
}

// Forward solve behind wave_forward (basic = false) and the unfactorised ablation
// (basic = true: FP32 storage, SO 8/12/16/24, one step per launch). noalloc: the
// workspace is the device's static scratch (one-step layout, tables staged in heap
// memory); workspace and ws_bytes are ignored.
int forward_impl(const wave_grid* g, const float* vel, const float* wavelet,
                 const double* src_xyz_h, int nsrc, const double* rec_xyz_h, int nrec,
                 float* rec_out, const float* u0, const float* um1, float* u_final, float* ckpt,
                 int ckpt_every, void* workspace, size_t ws_bytes, void* hip_stream, bool basic,
                 bool noalloc = false) {
  int st = validate(g);
  if (st) return st;
  if (vel == nullptr || nsrc < 0 || nrec < 0) return WAVE_EINVAL;
  if (nsrc > 0 && wavelet == nullptr && g->nt > 0) return WAVE_EINVAL;
  if (nrec > 0 && rec_out == nullptr && g->nt > 0) return WAVE_EINVAL;
  if (!points_ok(g, src_xyz_h, nsrc) || !points_ok(g, rec_xyz_h, nrec)) return WAVE_EINVAL;
  if (ckpt != nullptr && ckpt_every <= 0) return WAVE_EINVAL;
  if (ckpt != nullptr && store_kind(g) != WAVE_STORE_F32) return WAVE_EINVAL;
  if (basic && (g->storage != WAVE_STORE_F32 ||
                (g->so != 8 && g->so != 12 && g->so != 16 && g->so != 24)))
    return WAVE_EINVAL;
  if (noalloc) {
    if (ckpt != nullptr || (g->path & WAVE_PATH_TWO_STEP)) return WAVE_EINVAL;
    if (make_layout(g, nsrc, nrec, WAVE_MODE_FORWARD, 0, false).total > kScratchBytes)
      return WAVE_ELIMIT;
    st = scratch_address(&workspace);
    if (st) return st;
    ws_bytes = kScratchBytes;
  }
  int fz = 0;
  const bool fused = !basic && !noalloc && ckpt == nullptr && want_fused(g, &fz);
  Ctx C;
  st = setup(C, g, vel, src_xyz_h, nsrc, rec_xyz_h, nrec, WAVE_MODE_FORWARD, 0, workspace,
             ws_bytes, hip_stream, fused ? fz : 0, noalloc);
  if (st) return st;
  if (store_kind(g) != WAVE_STORE_F32)
    return forward_reduced(C, wavelet, nsrc, nrec, rec_out, u0, um1, u_final);
  if (fused && fused_tiling_ok(C))
    return forward_fused(C, wavelet, nsrc, nrec, rec_out, u0, um1, u_final);
  float* X[2] = {C.at<float>(C.L.u[0]), C.at<float>(C.L.u[1])};
  LaunchList LL;
  LL.pack(u0, X[0], C.G);
  LL.pack(um1, X[1], C.G);
  const int64_t N = (int64_t)g->nx * g->ny * g->nz;
  StepArgs a = base_args(C);
  const int r = g->so / 2;
  for (int n = 0; n < g->nt; ++n) {
    float* cur = X[n & 1];
    float* prev = X[(n + 1) & 1];
    if (ckpt != nullptr && n % ckpt_every == 0) {
      const int64_t k = n / ckpt_every;
      LL.unpack(cur, ckpt + (2 * k) * N, C.G);
      LL.unpack(prev, ckpt + (2 * k + 1) * N, C.G);
    }
    a.cur = cur;
    a.prev = prev;
    a.out = prev;
    set_inj(a, C, 0, nsrc, nsrc > 0 ? wavelet + (int64_t)n * nsrc : nullptr);
    set_samp(a, C, 1, nrec, n >= 1 && nrec > 0 ? rec_out + (int64_t)(n - 1) * nrec : nullptr);
    if (basic)
      LL.step_basic(a, r);
    else
      LL.step(a, r, false, ST_F32, false, C.nt);
  }
  if (nrec > 0 && g->nt > 0) {
    const PointTables& P = C.L.pts[1];
    LL.sample(X[g->nt & 1], ST_F32, LevelMeta{}, g->nt, C.at<int>(P.samp_idx),
              C.at<float>(P.samp_w), nrec, rec_out + (int64_t)(g->nt - 1) * nrec);
  }
  if (u_final != nullptr) LL.unpack(X[g->nt & 1], u_final, C.G);
  // the static-scratch variant never builds graphs (instantiation allocates)
  HIP_TRY(LL.run(C.s, noalloc ? (C.path | WAVE_PATH_DIRECT) & ~WAVE_PATH_GRAPH : C.path));
  return WAVE_OK;
}

int validate(const wave_grid* g) {
  if (!grid_ok(g)) return WAVE_EINVAL;
  const double dtm = wave_cfl_dt_max(g->so, g->vmax, g->hx, g->hy, g->hz);
  if (!(g->dt <= dtm * (1.0 + 1e-12))) return WAVE_ECFL;
  return WAVE_OK;
}

}  // namespace wave

using namespace wave;

extern "C" {

double wave_cfl_dt_max(int so, double vmax, double hx, double hy, double hz) {
  if (so < 2 || so > 2 * MAXR || so % 2 || !(vmax > 0) || !(hx > 0) || !(hy > 0) || !(hz > 0))
    return -1.0;
  double w[MAXR + 1];
  fd_weights(so, w);
  double S = std::fabs(w[0]);
  for (int q = 1; q <= so / 2; ++q) S += 2.0 * std::fabs(w[q]);
  return 2.0 / (vmax * std::sqrt(S * (1.0 / (hx * hx) + 1.0 / (hy * hy) + 1.0 / (hz * hz))));
}

size_t wave_workspace_bytes(const wave_grid* g, int nsrc, int nrec, int mode, int ckpt_every) {
  if (!grid_ok(g) || nsrc < 0 || nrec < 0) return 0;
  if (mode != WAVE_MODE_FORWARD && mode != WAVE_MODE_ADJOINT && mode != WAVE_MODE_GRADIENT)
    return 0;
  return make_layout(g, nsrc, nrec, mode, ckpt_every).total;
}

size_t wave_checkpoint_bytes(const wave_grid* g, int ckpt_every) {
  if (!grid_ok(g) || ckpt_every <= 0) return 0;
  const size_t n = (size_t)g->nx * g->ny * g->nz;
  const size_t nck = g->nt > 0 ? (size_t)(g->nt + ckpt_every - 1) / ckpt_every : 0;
  return nck * 2 * n * sizeof(float);
}

const char* wave_status_string(int status) {
  switch (status) {
    case WAVE_OK: return "ok";
    case WAVE_EINVAL: return "invalid argument";
    case WAVE_ECFL: return "time step above the stability limit";
    case WAVE_ENOMEM: return "workspace too small";
    case WAVE_EDEVICE: return "HIP runtime error";
    case WAVE_EBUSY: return "over the memory budget";
    case WAVE_EAGAIN: return "not ready";
    case WAVE_ELIMIT: return "larger than the static scratch";
    default: return "unknown status";
  }
}

const char* wave_version(void) { return "wave-gfx950 0.1"; }

int wave_forward(const wave_grid* g, const float* vel, const float* wavelet,
                 const double* src_xyz_h, int nsrc, const double* rec_xyz_h, int nrec,
                 float* rec_out, const float* u0, const float* um1, float* u_final, float* ckpt,
                 int ckpt_every, void* workspace, size_t ws_bytes, void* hip_stream) {
  return forward_impl(g, vel, wavelet, src_xyz_h, nsrc, rec_xyz_h, nrec, rec_out, u0, um1,
                      u_final, ckpt, ckpt_every, workspace, ws_bytes, hip_stream, false);
}

int wave_forward_noalloc(const wave_grid* g, const float* vel, const float* wavelet,
                         const double* src_xyz_h, int nsrc, const double* rec_xyz_h, int nrec,
                         float* rec_out, const float* u0, const float* um1, float* u_final,
                         void* hip_stream) {
  return forward_impl(g, vel, wavelet, src_xyz_h, nsrc, rec_xyz_h, nrec, rec_out, u0, um1,
                      u_final, nullptr, 0, nullptr, 0, hip_stream, false, true);
}

size_t wave_noalloc_limit_bytes(void) { return kScratchBytes; }

int wave_forward_unfactorised(const wave_grid* g, const float* vel, const float* wavelet,
                              const double* src_xyz_h, int nsrc, const double* rec_xyz_h,
                              int nrec, float* rec_out, const float* u0, const float* um1,
                              float* u_final, void* workspace, size_t ws_bytes,
                              void* hip_stream) {
  return forward_impl(g, vel, wavelet, src_xyz_h, nsrc, rec_xyz_h, nrec, rec_out, u0, um1,
                      u_final, nullptr, 0, workspace, ws_bytes, hip_stream, true);
}

int wave_adjoint(const wave_grid* g, const float* vel, const float* rec_data,
                 const double* rec_xyz_h, int nrec, const double* src_xyz_h, int nsrc,
                 float* src_out, float* lam_final, void* workspace, size_t ws_bytes,
                 void* hip_stream) {
  int st = validate(g);
  if (st) return st;
  if (vel == nullptr || nsrc < 0 || nrec < 0) return WAVE_EINVAL;
  if (g->storage != WAVE_STORE_F32) return WAVE_EINVAL;
  if (nrec > 0 && rec_data == nullptr && g->nt > 0) return WAVE_EINVAL;
  if (nsrc > 0 && src_out == nullptr && g->nt > 0) return WAVE_EINVAL;
  if (!points_ok(g, src_xyz_h, nsrc) || !points_ok(g, rec_xyz_h, nrec)) return WAVE_EINVAL;
  Ctx C;
  st = setup(C, g, vel, src_xyz_h, nsrc, rec_xyz_h, nrec, WAVE_MODE_ADJOINT, 0, workspace,
             ws_bytes, hip_stream);
  if (st) return st;
  float* X[2] = {C.at<float>(C.L.u[0]), C.at<float>(C.L.u[1])};
  LaunchList LL;
  LL.pack(nullptr, X[0], C.G);
  LL.pack(nullptr, X[1], C.G);
  StepArgs a = base_args(C);
  const int r = g->so / 2;
  const int nt = g->nt;
  for (int n = nt - 1; n >= 0; --n) {
    a.cur = X[(n + 1) & 1];
    a.prev = X[n & 1];
    a.out = X[n & 1];
    set_inj(a, C, 1, nrec, nrec > 0 ? rec_data + (int64_t)n * nrec : nullptr);
    set_samp(a, C, 0, nsrc,
             (n + 1 <= nt - 1 && nsrc > 0) ? src_out + (int64_t)(n + 1) * nsrc : nullptr);
    LL.step(a, r, false, ST_F32, false, C.nt);
  }
  if (nsrc > 0 && nt > 0) {
    const PointTables& P = C.L.pts[0];
    LL.sample(X[0], ST_F32, LevelMeta{}, 0, C.at<int>(P.samp_idx), C.at<float>(P.samp_w), nsrc,
              src_out);
  }
  if (lam_final != nullptr) LL.unpack(X[0], lam_final, C.G);
  HIP_TRY(LL.run(C.s, C.path));
  return WAVE_OK;
}

}  // extern "C"

namespace wave {
// Backward pass shared by the gradient and the image: forward levels from the
// checkpoints (or an internal forward pass), segment recompute, adjoint steps
// driven by rec_adj that accumulate either the velocity gradient (image false)
// or the zero-lag cross-correlation of the two fields (image true) into graw.
int backward_accumulate(const wave_grid* g, const float* vel, const float* wavelet,
                        const double* src_xyz_h, int nsrc, const double* rec_xyz_h, int nrec,
                        const float* rec_grad, const float* ckpt, int ckpt_every, bool image,
                        float* out, float* grad_wavelet, void* workspace, size_t ws_bytes,
                        void* hip_stream) {
  float* grad_vel = out;
  int st = validate(g);
  if (st) return st;
  if (vel == nullptr || grad_vel == nullptr || nsrc < 0 || nrec < 0) return WAVE_EINVAL;
  if (g->storage != WAVE_STORE_F32) return WAVE_EINVAL;
  if (nsrc > 0 && wavelet == nullptr && g->nt > 0) return WAVE_EINVAL;
  if (nrec > 0 && rec_grad == nullptr && g->nt > 0) return WAVE_EINVAL;
  if (ckpt != nullptr && ckpt_every <= 0) return WAVE_EINVAL;
  if (!points_ok(g, src_xyz_h, nsrc) || !points_ok(g, rec_xyz_h, nrec)) return WAVE_EINVAL;
  Ctx C;
  st = setup(C, g, vel, src_xyz_h, nsrc, rec_xyz_h, nrec, WAVE_MODE_GRADIENT, ckpt_every,
             workspace, ws_bytes, hip_stream);
  if (st) return st;
  const int nt = g->nt, Cs = C.L.ckpt_every, r = g->so / 2;
  const int64_t N = (int64_t)g->nx * g->ny * g->nz, F = C.G.nfield;
  float* graw = C.at<float>(C.L.graw);
  float* lam[2] = {C.at<float>(C.L.lam[0]), C.at<float>(C.L.lam[1])};
  float* seg = C.at<float>(C.L.seg);
  float* ick = C.at<float>(C.L.ick);
  LaunchList LL;
  LL.pack(nullptr, graw, C.G);
  LL.pack(nullptr, lam[0], C.G);
  LL.pack(nullptr, lam[1], C.G);
  StepArgs a = base_args(C);
  if (ckpt == nullptr) {
    // internal forward pass keeping (u^{kC}, u^{kC-1}) pitched in the workspace
    float* X[2] = {C.at<float>(C.L.u[0]), C.at<float>(C.L.u[1])};
    LL.pack(nullptr, X[0], C.G);
    LL.pack(nullptr, X[1], C.G);
    set_samp(a, C, 1, 0, nullptr);
    for (int n = 0; n < nt; ++n) {
      float* cur = X[n & 1];
      float* prev = X[(n + 1) & 1];
      if (n % Cs == 0) {
        const int64_t k = n / Cs;
        LL.copy(cur, ick + (2 * k) * F, F);
        LL.copy(prev, ick + (2 * k + 1) * F, F);
      }
      a.cur = cur; a.prev = prev; a.out = prev;
      set_inj(a, C, 0, nsrc, nsrc > 0 ? wavelet + (int64_t)n * nsrc : nullptr);
      LL.step(a, r, false, ST_F32, false, C.nt);
    }
  }
  for (int s = C.L.nseg - 1; s >= 0; --s) {
    const int n0 = s * Cs, n1 = std::min(n0 + Cs, nt);
    // seg slot m holds u^{n0-1+m}
    if (ckpt != nullptr) {
      LL.pack(ckpt + (2 * (int64_t)s) * N, seg + 1 * F, C.G);
      LL.pack(ckpt + (2 * (int64_t)s + 1) * N, seg + 0 * F, C.G);
    } else {
      LL.copy(ick + (2 * (int64_t)s) * F, seg + 1 * F, F);
      LL.copy(ick + (2 * (int64_t)s + 1) * F, seg + 0 * F, F);
    }
    set_samp(a, C, 1, 0, nullptr);
    a.ufwd = nullptr;
    a.grad = nullptr;
    for (int n = n0; n < n1; ++n) {
      a.cur = seg + (int64_t)(n - n0 + 1) * F;
      a.prev = seg + (int64_t)(n - n0) * F;
      a.out = seg + (int64_t)(n - n0 + 2) * F;
      set_inj(a, C, 0, nsrc, nsrc > 0 ? wavelet + (int64_t)n * nsrc : nullptr);
      LL.step(a, r, false, ST_F32, false, C.nt);
    }
    for (int n = n1 - 1; n >= n0; --n) {
      a.cur = lam[(n + 1) & 1];
      a.prev = lam[n & 1];
      a.out = lam[n & 1];
      a.ufwd = seg + (int64_t)(n - n0 + 2) * F;
      a.grad = graw;
      a.acc_image = image ? 1 : 0;
      set_inj(a, C, 1, nrec, nrec > 0 ? rec_grad + (int64_t)n * nrec : nullptr);
      set_samp(a, C, 0, nsrc,
               (grad_wavelet != nullptr && nsrc > 0 && n + 1 <= nt - 1)
                   ? grad_wavelet + (int64_t)(n + 1) * nsrc
                   : nullptr);
      LL.step(a, r, true, ST_F32, false, false);
    }
  }
  if (grad_wavelet != nullptr && nsrc > 0 && nt > 0) {
    const PointTables& P = C.L.pts[0];
    LL.sample(lam[0], ST_F32, LevelMeta{}, 0, C.at<int>(P.samp_idx), C.at<float>(P.samp_w), nsrc,
              grad_wavelet);
  }
  if (image) LL.unpack(graw, out, C.G);
  HIP_TRY(LL.run(C.s, C.path));
  if (!image) {
    // dL/dm = -graw / dt^2  ->  dL/dv = -2 v^-3 dL/dm = (2 / dt^2) graw / v^3
    HIP_TRY(launch_grad_finalize(graw, vel, grad_vel, C.G, 2.0 / (g->dt * g->dt), C.s));
  }
  return WAVE_OK;
}
}  // namespace wave

extern "C" {

int wave_gradient(const wave_grid* g, const float* vel, const float* wavelet,
                  const double* src_xyz_h, int nsrc, const double* rec_xyz_h, int nrec,
                  const float* rec_grad, const float* ckpt, int ckpt_every, float* grad_vel,
                  float* grad_wavelet, void* workspace, size_t ws_bytes, void* hip_stream) {
  return backward_accumulate(g, vel, wavelet, src_xyz_h, nsrc, rec_xyz_h, nrec, rec_grad, ckpt,
                             ckpt_every, false, grad_vel, grad_wavelet, workspace, ws_bytes,
                             hip_stream);
}

int wave_rtm(const wave_grid* g, const float* vel, const float* wavelet,
             const double* src_xyz_h, int nsrc, const double* rec_xyz_h, int nrec,
             const float* rec_data, const float* ckpt, int ckpt_every, float* image,
             void* workspace, size_t ws_bytes, void* hip_stream) {
  return backward_accumulate(g, vel, wavelet, src_xyz_h, nsrc, rec_xyz_h, nrec, rec_data, ckpt,
                             ckpt_every, true, image, nullptr, workspace, ws_bytes, hip_stream);
}


}  // extern "C"
