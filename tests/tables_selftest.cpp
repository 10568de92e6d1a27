// Host-only self-test of the solver's injection and sampling tables, the
// two-step kernel's extended-region tables and the z-chunk policy (paper_1912_00695_amd/csrc/wave_api.cpp, compiled into this test
// with the host compiler; the kernels' launchers resolve against libwave.so but
// none is called). For random point sets -- on grid points, off them, repeated,
// on tile and chunk edges -- the tables are checked against a brute-force
// reference written here from the definition: every point contributes its
// trilinear corners (weights (1-t) or t per axis, corners of weight 0 dropped);
// each distinct grid point becomes one entry of the column (xy tile, plane) that
// holds it, columns numbered (ty * ntile_x + tx) * nz + z, entries ordered by
// (column, index in the tile), with the contributing (point, weight) terms in
// point order; the tables do not depend on the z-chunking. Built and run by tests/test_tables_host.py; exits
// non-zero on failure.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <random>
#include <tuple>
#include <vector>

#include "wave_api.cpp"

using namespace wave;

#define CHECK(c)                                                         \
  do {                                                                   \
    if (!(c)) {                                                          \
      std::fprintf(stderr, "FAILED %s at line %d\n", #c, __LINE__);     \
      std::exit(1);                                                      \
    }                                                                    \
  } while (0)

struct RefTerm {
  int p;
  float w;
};
using RefKey = std::tuple<int, int, int>;  // tile, plane, index in the tile

static void reference(const wave_grid& g, const Geom& G, const Tiling& T,
                      const std::vector<double>& xyz, std::map<RefKey, std::vector<RefTerm>>* ent,
                      std::vector<int>* sidx, std::vector<float>* sw) {
  const int np = (int)xyz.size() / 3;
  sidx->assign((size_t)8 * np, 0);
  sw->assign((size_t)8 * np, 0.f);
  for (int p = 0; p < np; ++p) {
    const double f[3] = {xyz[3 * p] / g.hx, xyz[3 * p + 1] / g.hy, xyz[3 * p + 2] / g.hz};
    int base[3];
    double t[3];
    for (int a = 0; a < 3; ++a) {
      base[a] = (int)std::floor(f[a]);
      t[a] = f[a] - base[a];
    }
    int k = 0;
    for (int c = 0; c < 8; ++c) {  // x fastest, then y, then z
      const int d[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
      double w = 1.0;
      for (int a = 0; a < 3; ++a) w *= d[a] ? t[a] : 1.0 - t[a];
      if (w == 0.0) continue;
      const int i = base[0] + d[0], j = base[1] + d[1], z = base[2] + d[2];
      (*sidx)[8 * p + k] = (int)((int64_t)z * G.plane + (int64_t)j * G.pitch + i);
      (*sw)[8 * p + k] = (float)w;
      ++k;
      const int tile = ((j / TY) * T.ntile_x + i / TX) * G.nz + z;
      (*ent)[RefKey{tile, z, (j % TY) * TX + (i % TX)}].push_back(RefTerm{p, (float)w});
    }
  }
}

static void check_tables(const wave_grid& g, int zchunk, const std::vector<double>& xyz) {
  const Geom G = make_geom(&g);
  const Tiling T = make_tiling(G, g.so / 2, 0, zchunk, WAVE_STORE_F32);
  const int np = (int)xyz.size() / 3;
  const Layout L = make_layout(&g, 0, np, WAVE_MODE_FORWARD, 0);
  const PointTables& P = L.pts[1];
  Blob B;
  B.base = L.tables_beg;
  const size_t size = L.tables_end - L.tables_beg;
  B.bytes = new char[size];  // heap storage (the destructor frees it)
  std::memset(B.bytes, 0xA5, size);  // garbage where nothing is written
  build_point_tables(&g, G, T, xyz.data(), np, P, B);

  std::map<RefKey, std::vector<RefTerm>> ref;
  std::vector<int> sidx;
  std::vector<float> sw;
  reference(g, G, T, xyz, &ref, &sidx, &sw);

  // sampling corners
  CHECK(std::memcmp(B.at<int>(P.samp_idx), sidx.data(), sidx.size() * sizeof(int)) == 0);
  CHECK(std::memcmp(B.at<float>(P.samp_w), sw.data(), sw.size() * sizeof(float)) == 0);
  // entries, terms, tile ranges, plane groups, single-term fields
  const int* tb = B.at<int>(P.tile_beg);
  const InjEntry* ent = B.at<InjEntry>(P.ent);
  const int* cidx = B.at<int>(P.csr_idx);
  const float* cw = B.at<float>(P.csr_w);
  const int ncol = T.ntile_x * T.ntile_y * G.nz;
  CHECK(tb[0] == 0 && tb[ncol] == (int)ref.size());
  int e = 0, c = 0;
  for (const auto& kv : ref) {
    const int tile = std::get<0>(kv.first);
    CHECK(tb[tile] <= e && e < tb[tile + 1]);
    const InjEntry& en = ent[e];
    CHECK(en.z == std::get<1>(kv.first) && en.local == std::get<2>(kv.first));
    CHECK(en.csr_beg == c && en.csr_end == c + (int)kv.second.size());
    for (const RefTerm& t : kv.second) {
      CHECK(cidx[c] == t.p && cw[c] == t.w);
      ++c;
    }
    if (kv.second.size() == 1) {
      CHECK(en.tidx == kv.second[0].p && en.w == kv.second[0].w);
    } else {
      CHECK(en.tidx == -1);
    }
    // the group of en runs to the first entry of the tile on another plane
    int q = e;
    while (q < tb[tile + 1] && ent[q].z == en.z) ++q;
    CHECK(en.grp_end == q);
    ++e;
  }
  for (int t = 0; t < ncol; ++t) CHECK(tb[t] <= tb[t + 1]);
  // uploaded ranges: every written array, within the table region
  size_t covered = 0;
  for (const auto& r : B.used) {
    CHECK(r.first + r.second <= size);
    covered += r.second;
  }
  const size_t want = ((size_t)ncol + 1) * sizeof(int) + (size_t)e * sizeof(InjEntry) +
                      (size_t)c * (sizeof(int) + sizeof(float)) +
                      (size_t)8 * np * (sizeof(int) + sizeof(float));
  CHECK(covered == want);
}

// Extended-region tables of the two-step kernel (build_ext_tables), against a
// reference from the definition: a two-step tile is f2_tiles_y(r) one-step tiles
// stacked along y (TY2 rows); a corner (i, j, z) belongs to every two-step tile
// whose region x in [xt - 4, xt + TX + 4), y in [yt - r, yt + TY2 + r), z in
// [z0 - r, z1 + r) holds it (all tiles scanned), with local index
// (j - yt + r) * (TX + 8) + (i - xt + 4).
static void check_ext_tables(wave_grid g, int zchunk, const std::vector<double>& xyz) {
  const int r = g.so / 2;
  const Geom G = make_geom(&g);
  const Tiling T = make_tiling(G, r, 0, zchunk, WAVE_STORE_F32);
  const int np = (int)xyz.size() / 3;
  const Layout L = make_layout(&g, np, 0, WAVE_MODE_FORWARD, 0, true);
  CHECK(L.fused);
  Blob B;
  B.base = L.tables_beg;
  const size_t size = L.tables_end - L.tables_beg;
  B.bytes = new char[size];
  std::memset(B.bytes, 0xA5, size);
  build_ext_tables(&g, G, T, r, xyz.data(), np, L.epts, B);

  const int TY2 = f2_tiles_y(r) * TY;
  const int nty = (G.ny + TY2 - 1) / TY2;
  const int ntiles = T.ntile_x * nty * T.nchunk;
  std::map<RefKey, std::vector<RefTerm>> ref;
  for (int p = 0; p < np; ++p) {
    const double f[3] = {xyz[3 * p] / g.hx, xyz[3 * p + 1] / g.hy, xyz[3 * p + 2] / g.hz};
    int base[3];
    double t[3];
    for (int a = 0; a < 3; ++a) {
      base[a] = (int)std::floor(f[a]);
      t[a] = f[a] - base[a];
    }
    for (int c = 0; c < 8; ++c) {
      const int d[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
      double w = 1.0;
      for (int a = 0; a < 3; ++a) w *= d[a] ? t[a] : 1.0 - t[a];
      if (w == 0.0) continue;
      const int i = base[0] + d[0], j = base[1] + d[1], z = base[2] + d[2];
      for (int tile = 0; tile < ntiles; ++tile) {
        const int xt = (tile % T.ntile_x) * TX, yt = ((tile / T.ntile_x) % nty) * TY2;
        const int z0 = (tile / (T.ntile_x * nty)) * T.zchunk;
        const int z1 = std::min(z0 + T.zchunk, G.nz);
        if (i < xt - 4 || i >= xt + TX + 4 || j < yt - r || j >= yt + TY2 + r || z < z0 - r ||
            z >= z1 + r)
          continue;
        ref[RefKey{tile, z, (j - yt + r) * (TX + 8) + (i - xt + 4)}].push_back(
            RefTerm{p, (float)w});
      }
    }
  }
  const int* tb = B.at<int>(L.epts.tile_beg);
  const InjEntry* ent = B.at<InjEntry>(L.epts.ent);
  const int* cidx = B.at<int>(L.epts.csr_idx);
  const float* cw = B.at<float>(L.epts.csr_w);
  CHECK(tb[0] == 0 && tb[ntiles] == (int)ref.size());
  int e = 0, c = 0;
  for (const auto& kv : ref) {
    const int tile = std::get<0>(kv.first);
    CHECK(tb[tile] <= e && e < tb[tile + 1]);
    const InjEntry& en = ent[e];
    CHECK(en.z == std::get<1>(kv.first) && en.local == std::get<2>(kv.first));
    CHECK(en.csr_beg == c && en.csr_end == c + (int)kv.second.size());
    for (const RefTerm& q : kv.second) {
      CHECK(cidx[c] == q.p && cw[c] == q.w);
      ++c;
    }
    if (kv.second.size() == 1) {
      CHECK(en.tidx == kv.second[0].p && en.w == kv.second[0].w);
    } else {
      CHECK(en.tidx == -1);
    }
    int q = e;
    while (q < tb[tile + 1] && ent[q].z == en.z) ++q;
    CHECK(en.grp_end == q);
    ++e;
  }
  for (int t = 0; t < ntiles; ++t) CHECK(tb[t] <= tb[t + 1]);
  CHECK((size_t)e <= (size_t)64 * np);  // the layout's bound on entries
}

static wave_grid grid(int nx, int ny, int nz) {
  wave_grid g{};
  g.nx = nx;
  g.ny = ny;
  g.nz = nz;
  g.hx = 10.0;
  g.hy = 12.0;
  g.hz = 9.0;
  g.so = 8;
  g.dt = 1e-3;
  g.nt = 10;
  return g;
}

static void test_tables() {
  std::mt19937_64 rng(7);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  const int shapes[][3] = {{97, 37, 23}, {160, 48, 70}, {64, 16, 9}, {130, 70, 41}};
  int cases = 0;
  for (const auto& s : shapes) {
    const wave_grid g = grid(s[0], s[1], s[2]);
    for (int zc : {0, 1, 5, 8}) {
      for (int kind = 0; kind < 4; ++kind) {
        std::vector<double> xyz;
        const int np = kind == 3 ? 1 : 300 + 200 * kind;
        for (int p = 0; p < np; ++p) {
          double f[3] = {U(rng) * (g.nx - 1), U(rng) * (g.ny - 1), U(rng) * (g.nz - 1)};
          if (kind == 0 || (kind == 2 && p % 2 == 0))
            for (double& v : f) v = std::floor(v);  // on grid points
          if (kind == 1 && p % 5 == 0) {           // on tile and chunk edges
            f[0] = std::min<double>(g.nx - 1, 63 + (p % 3) * 0.5);
            f[1] = std::min<double>(g.ny - 1, 15 + (p % 2) * 0.25);
          }
          if (kind == 2 && p % 7 == 0 && p > 0)    // repeats of the previous point
            for (int a = 0; a < 3; ++a)
              f[a] = xyz[3 * (p - 1) + a] / (a == 0 ? g.hx : a == 1 ? g.hy : g.hz);
          xyz.push_back(f[0] * g.hx);
          xyz.push_back(f[1] * g.hy);
          xyz.push_back(f[2] * g.hz);
        }
        check_tables(g, zc, xyz);
        ++cases;
      }
    }
    // a full plane of receivers in raster order (the presorted path)
    std::vector<double> plane;
    for (int j = 0; j < g.ny; ++j)
      for (int i = 0; i < g.nx; ++i) {
        plane.push_back(i * g.hx);
        plane.push_back(j * g.hy);
        plane.push_back(5 * g.hz);
      }
    check_tables(g, 0, plane);
    // the same plane off the grid points (two planes of corners per tile: the
    // counting-sort path), and shifted across a chunk boundary
    for (const double zf : {5.3, 7.5}) {
      std::vector<double> off;
      for (int j = 0; j + 1 < g.ny; ++j)
        for (int i = 0; i + 1 < g.nx; ++i) {
          off.push_back((i + 0.37) * g.hx);
          off.push_back((j + 0.61) * g.hy);
          off.push_back(zf * g.hz);
        }
      check_tables(g, 8, off);
      cases += 1;
    }
    ++cases;
  }
  // no points
  check_tables(grid(97, 37, 23), 0, {});
  std::printf("tables: %d cases\n", cases + 1);
}

static void test_ext_tables() {
  std::mt19937_64 rng(11);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  const int shapes[][3] = {{97, 37, 23}, {160, 48, 70}, {130, 70, 41}};
  int cases = 0;
  for (const auto& s : shapes) {
    for (int so : {2, 4, 6, 8}) {
      wave_grid g = grid(s[0], s[1], s[2]);
      g.so = so;
      for (int zc : {8, 13}) {
        std::vector<double> xyz;
        for (int p = 0; p < 120; ++p) {
          double f[3] = {U(rng) * (g.nx - 1), U(rng) * (g.ny - 1), U(rng) * (g.nz - 1)};
          if (p % 3 == 0)
            for (double& v : f) v = std::floor(v);  // on grid points
          if (p % 4 == 1) {  // on and next to tile edges: x 63/64, y 15/16 and 31/32
            f[0] = std::min<double>(g.nx - 1, 63 + (p % 3) * 0.5);
            f[1] = std::min<double>(g.ny - 1, (p % 8 < 4 ? 15.0 : 31.0) + (p % 2) * 0.5);
          }
          xyz.push_back(f[0] * g.hx);
          xyz.push_back(f[1] * g.hy);
          xyz.push_back(f[2] * g.hz);
        }
        check_ext_tables(g, zc, xyz);
        ++cases;
      }
    }
  }
  std::printf("ext tables: %d cases\n", cases);
}

static void test_tiling() {
  const auto zc = [](int n, bool naive16, int r = 2, int path = 0) {
    wave_grid g = grid(n, n, n);
    return make_tiling(make_geom(&g), r, path, 0, naive16 ? WAVE_STORE_F16 : WAVE_STORE_F32);
  };
  // about 512 workgroups of one long chunk each
  CHECK(zc(256, false).zchunk == 32 && zc(256, false).nblocks == 512);
  CHECK(zc(320, false).zchunk == 64 && zc(320, false).nblocks == 500);
  CHECK(zc(384, false).zchunk == 128 && zc(384, false).nblocks == 432);
  CHECK(zc(512, false).zchunk == 256 && zc(512, false).nblocks == 512);
  // small grids: short chunks from the same rule (64^3: 4 tiles per plane, 1-plane
  // chunks, 256 workgroups; 128^3: 16 tiles, 4 planes, 512 workgroups)
  CHECK(zc(64, false).zchunk == 1 && zc(64, false).nblocks == 256);
  CHECK(zc(128, false).zchunk == 4 && zc(128, false).nblocks == 512);
  // naive 16-bit storage: chunks of at most 32 planes, ~20 for large grids
  CHECK(zc(256, true).zchunk == 32);
  CHECK(zc(512, true).zchunk == 20);
  // workgroup height of the one-step kernel: 64 x 32 tiles where the radius has
  // them and their count is a multiple of the 256 CUs
  CHECK(zc(256, false).tiles_y == 2);            // radius 2: 4 x 8 x 8 = 256
  CHECK(zc(256, false, 5).tiles_y == 1);         // radius 5: 64 x 16 only
  CHECK(zc(256, false, 4).tiles_y == 2);         // 4 x 8 x 8 = 256 tall workgroups
  CHECK(zc(512, false, 4).tiles_y == 2);         // 8 x 16 x 2 = 256
  CHECK(zc(320, false, 4).tiles_y == 1);         // 5 x 10 x 5 = 250
  CHECK(zc(384, false, 4).tiles_y == 1);         // 6 x 12 x 3 = 216
  CHECK(zc(448, false, 4).tiles_y == 1);         // 7 x 14 x 2 = 196
  CHECK(zc(128, false, 8).tiles_y == 2);         // 2 x 4 x 32 = 256 (4-plane chunks)
  CHECK(zc(96, false, 4).tiles_y == 1);          // 2 x 3 x 32 = 192
  {
    wave_grid g = grid(256, 144, 256);             // 4 x 5 x 14 = 280 (uneven)
    CHECK(make_tiling(make_geom(&g), 4, 0, 0, WAVE_STORE_F32).tiles_y == 1);
    g = grid(256, 256, 512);                       // 4 x 8 x 8 = 256 (64-plane chunks)
    CHECK(make_tiling(make_geom(&g), 4, 0, 0, WAVE_STORE_F32).tiles_y == 2);
    // 16-bit storage keeps 64 x 16 tiles unless asked
    CHECK(make_tiling(make_geom(&g), 4, 0, 0, WAVE_STORE_F16 | WAVE_STORE_DIFF).tiles_y == 1);
    CHECK(make_tiling(make_geom(&g), 4, 0, 0, WAVE_STORE_BF16).tiles_y == 1);
    CHECK(make_tiling(make_geom(&g), 4, WAVE_PATH_TILE32, 0, WAVE_STORE_F16).tiles_y == 2);
  }
  CHECK(zc(256, false, 8).tiles_y == 2 && zc(256, false, 10).tiles_y == 2);
  CHECK(zc(256, false, 6).tiles_y == 1 && zc(256, false, 12).tiles_y == 1);
  CHECK(zc(64, false, 4, WAVE_PATH_TILE32).tiles_y == 2);
  CHECK(zc(64, false, 6, WAVE_PATH_TILE32).tiles_y == 1);  // no 64 x 32 form at radius 6
  CHECK(zc(256, false, 4, WAVE_PATH_TILE16).tiles_y == 1);
  for (int n : {40, 97, 200, 333, 700}) {
    const Tiling T = zc(n, false);
    CHECK(T.zchunk >= 1 && T.zchunk <= MAXZCHUNK && T.zchunk <= n);
    CHECK(T.nchunk * T.zchunk >= n && (T.nchunk - 1) * T.zchunk < n);
  }
  std::printf("tiling: OK\n");
}

int main() {
  test_tables();
  test_ext_tables();
  test_tiling();
  std::printf("OK\n");
  return 0;
}
