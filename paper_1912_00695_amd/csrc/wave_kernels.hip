// wave_kernels.hip -- gfx950 kernels of the acoustic leapfrog solver.
//
// One launch of step_kernel advances one time level of
//   out = ( 2 cur - (1-b) prev + c2 (L_h cur + inj) ) / (1+b),
// evaluated as cur + ((1-b)(cur - prev) + c2 (L_h cur + inj)) / (1+b)
// (the damped leapfrog update of the paper's SO2 listing, Section 2.1,
// generalised to a star Laplacian of order 2r), fused with
//   * point-source injection (inj: per-tile lists of grid points, each with its
//     trilinear terms, summed in a fixed order and scattered through LDS),
//   * sampling of `cur` at receiver points (extra workgroups after the stencil
//     workgroups; `cur` is read-only during the step, so sampling the previous
//     step's result here needs no extra launch),
//   * optionally the gradient accumulation grad += ufwd * c2 (L_h cur + inj), or the
//     imaging condition grad += ufwd * cur.
//
// Memory plan per step (FP32): read cur, prev, c2 and write out once each from
// HBM -- 16 bytes per point; halo re-reads of cur are served by L2. With 16-bit
// wavefield storage (FP16 / BF16, FP32 arithmetic) the naive form moves
// 2+2+4+2 = 10 bytes per point and the difference form (u, u - u_prev) 12.
#include <climits>

#include "wave_device.h"

namespace wave {


// z-sweep variants per radius, chosen from a sweep of the forms over the space
// orders on gfx950: bit R of WAVE_ZUNROLL_MASK runs two planes per loop iteration
// (constant LDS buffer index in each); bit R of WAVE_PF2_MASK issues the loads of
// plane z+2 while plane z is computed (two planes of loads in flight; implies the
// two-plane iteration).
#ifndef WAVE_ZUNROLL_MASK
#define WAVE_ZUNROLL_MASK 0x1FFE  // every radius 1..12
#endif
#ifndef WAVE_PF2_MASK
#define WAVE_PF2_MASK 0x0
#endif
// bit R of WAVE_ZUNROLL4_MASK: four planes per loop iteration, so the register
// queue shifts once per four planes (fewer moves per plane, more code); measured
// at 256^3: +3 % at SO14, SO16 and SO24, none at SO12, -1 % at SO8
#ifndef WAVE_ZUNROLL4_MASK
#define WAVE_ZUNROLL4_MASK 0x1F80  // radius 7..12
#endif
// bit R of WAVE_HRING_MASK: load the xy-halo of each plane R planes ahead (with the
// queue head of the same plane) and park it in LDS until the plane is staged, also
// in launches with non-temporal streams (WAVE_HRING_NT=0: only in those without)
#ifndef WAVE_HRING_MASK
#define WAVE_HRING_MASK 0x1FE  // radius 1..8
#endif
#ifndef WAVE_HRING_NT
#define WAVE_HRING_NT 1
#endif
constexpr bool zunroll2(int r) { return ((WAVE_ZUNROLL_MASK) >> r) & 1; }
constexpr bool prefetch2(int r) { return ((WAVE_PF2_MASK) >> r) & 1; }
constexpr bool zunroll4(int r) { return ((WAVE_ZUNROLL4_MASK) >> r) & 1; }
// bit R of WAVE_BSTORE_MASK: buffer stores of the step's outputs (else predicated
// global stores); measured at 256^3 SO2-24 within +-1 % of the global stores (the
// buffer form saves the per-lane 64-bit address arithmetic: 2-8 % fewer VALU
// instructions per plane)
#ifndef WAVE_BSTORE_MASK
#define WAVE_BSTORE_MASK 0x0
#endif
constexpr bool bstore(int r) { return ((WAVE_BSTORE_MASK) >> r) & 1; }
constexpr bool halo_ring(int r) { return ((WAVE_HRING_MASK) >> r) & 1; }

// One tile of one step: the z-sweep of the TX x TY column block xy (= ty *
// ntile_x + tx) over planes [z0, z1). Shared by the single-shot kernel and the
// batched serving kernel, so a shot's values do not depend on what else is in the
// launch or on how its planes are chunked.
template <int R, bool GRAD, int ST, bool DIFF, bool NT, bool BASIC = false, int K = 1>
__device__ __forceinline__ void step_tile(const StepArgs& a, const int xy, const int z0,
                                          const int z1, const float dec_c, const float dec_p,
                                          const float enc_u, const float enc_d) {
  constexpr int TYK = K * TY;        // rows of the tile (K one-step tiles)
  constexpr int NTH = K * NTHREADS;  // threads of the workgroup
  constexpr int XH = R <= 4 ? 4 : (R <= 8 ? 8 : 12);  // x-halo width (multiple of 4)
  constexpr int XH4 = XH / 4;
  constexpr int LROW4 = NTX + 2 * XH4;  // float4 per LDS row
  constexpr int LROWS = TYK + 2 * R;
  constexpr int NH = 2 * R * NTX + 2 * TYK * XH4;  // halo float4 per plane
  constexpr int NHP = (NH + NTH - 1) / NTH;
  __shared__ float4 lds[2][LROWS * LROW4];
  __shared__ float4 inj[TYK * NTX];
  __shared__ float bzs[MAXZCHUNK];  // z sponge factors of the chunk (read from LDS in the
                                    // sweep, so no vector load there waits on the prefetch)
  // Halo ring: the xy-halo of plane p is read by this workgroup when p is staged,
  // but its bytes are the queue heads of the neighbouring tiles, which those load R
  // planes earlier. Loading it together with this tile's own queue head of plane p
  // (while it is in L2) and parking it in per-thread LDS slots for R+1 planes keeps
  // the halo out of the fabric traffic; loading it one plane ahead put R planes of
  // streaming (about R MB per XCD) between the two reads, more than L2 holds.
  // Measured on MI355X: +2 % (SO4) to +13 % (SO12) at 256^3, where every workgroup
  // of a step is resident at once. With non-temporal streams (grids whose step
  // does not fit the Infinity Cache): 512^3 on 64 x 32 tiles SO2 / SO4 / SO8 / SO16
  // +1.4 / +2.8 / +4.0 / +2.5 %, 384^3 and 448^3 SO8 (64 x 16 tiles) +2.9 and
  // +5.4 %, the FP16 difference form at 512^3 +4 %; only 512^3 SO8 on 64 x 16 tiles
  // lost (-0.7 %).
  constexpr bool HRG = halo_ring(R) && (!NT || WAVE_HRING_NT);
  constexpr bool BSTORE = bstore(R);
  using Raw = typename Store<ST>::Raw;
  __shared__ Raw hbuf[HRG ? R + 1 : 1][HRG ? NH : 1];
  const auto hslot = [](const int p) { return p % (R + 1); };  // p >= 0

  const int tx_t = xy % a.ntile_x;
  const int ty_t = xy / a.ntile_x;  // in tiles of TYK rows
  const int xt = tx_t * TX, yt = ty_t * TYK;
  const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
  const int64_t plane = a.g.plane;
  const int tid = threadIdx.x;
  const int tx = tid % NTX, ty = tid / NTX;
  const int x0 = xt + tx * VX, y = yt + ty;
  const bool colok = (x0 < nx) && (y < ny);
  const int col = y * a.g.pitch + x0;
  const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
  float mx_u = 0.f, mx_d = 0.f;  // running maxima of the written level (reduced precision)

  // Halo items of this thread (fixed for the whole z sweep).
  int hoff[NHP], hlds[NHP];
  bool hok[NHP];
#pragma unroll
  for (int k = 0; k < NHP; ++k) {
    const int i = tid + k * NTH;
    int gy = 0, gx = 0, row = 0, c4 = 0;
    bool in = i < NH;
    if (i < R * NTX) {
      row = i / NTX; c4 = XH4 + i % NTX;
      gy = yt - R + row; gx = xt + 4 * (i % NTX);
    } else if (i < 2 * R * NTX) {
      const int j = i - R * NTX;
      row = R + TYK + j / NTX; c4 = XH4 + j % NTX;
      gy = yt + TYK + j / NTX; gx = xt + 4 * (j % NTX);
    } else if (i < 2 * R * NTX + TYK * XH4) {
      const int j = i - 2 * R * NTX;
      row = R + j / XH4; c4 = j % XH4;
      gy = yt + j / XH4; gx = xt - XH + 4 * (j % XH4);
    } else {
      const int j = i - 2 * R * NTX - TYK * XH4;
      row = R + j / XH4; c4 = XH4 + NTX + j % XH4;
      gy = yt + j / XH4; gx = xt + TX + 4 * (j % XH4);
    }
    hlds[k] = in ? row * LROW4 + c4 : -1;
    hok[k] = in && gy >= 0 && gy < ny && gx >= 0 && gx < nx;
    hoff[k] = hok[k] ? gy * a.g.pitch + gx : 0;
  }

  // Plane resources and per-lane byte offsets of the streamed loads; a plane
  // outside [0, nz) or past the chunk gets a resource with no records.
  constexpr int ES = Store<ST>::kBytes;
  const int pbytes = (int)(plane * ES), pbytes4 = (int)(plane * 4);
  auto rs_at = [&](const void* f, const int zz, const int es, const int bytes, const bool valid) {
    const int zc = min(max(zz, 0), nz - 1);
    return plane_rsrc(f, (int64_t)zc * plane * es, valid ? bytes : 0);
  };
  auto rs_cur = [&](const int zz, const bool valid) { return rs_at(a.cur, zz, ES, pbytes, valid); };
  auto rs_prev = [&](const int zz, const bool valid) { return rs_at(a.prev, zz, ES, pbytes, valid); };
  auto rs_c2 = [&](const int zz, const bool valid) { return rs_at(a.c2, zz, 4, pbytes4, valid); };
  auto rs_f32 = [&](const void* f, const int zz, const bool valid) {
    return rs_at(f, zz, 4, pbytes4, valid);
  };
  const unsigned vo_col = colok ? (unsigned)col * ES : kOOB;
  const unsigned vo_c2 = colok ? (unsigned)col * 4 : kOOB;
  unsigned vo_h[NHP];
#pragma unroll
  for (int k = 0; k < NHP; ++k) vo_h[k] = hok[k] ? (unsigned)hoff[k] * ES : kOOB;

  // Sponge factors: b = bx[x] + by[y] + bz[z].
  const float4 bxv = colok ? ld4(a.bx + x0) : zero4;
  const float byv = y < ny ? gmem(a.by)[y] : 0.f;

  // Loads are kept raw until every load of a batch has been issued, then widened
  // (and decoded) in one go, so that no conversion waits for a single load.
  auto wcur = [&](const Raw& r) {
    const float4 v = Store<ST>::widen(r);
    if constexpr (ST == ST_F32) return v; else return mul4(v, dec_c);
  };
  auto wprev = [&](const Raw& r) {
    const float4 v = Store<ST>::widen(r);
    if constexpr (ST == ST_F32) return v; else return mul4(v, dec_p);
  };

  // Register queue of planes z-R .. z+R for this thread's four points; prev and
  // c2 at the current plane stay raw until the update uses them.
  float4 q[2 * R + 1];
  Raw up;
  f4v cc;
  f4v ufc{}, grc{};  // gradient kernels: forward level and accumulator at the plane
  {
    Raw qr[2 * R + 1], hr[NHP];
#pragma unroll
    for (int s = 0; s <= 2 * R; ++s) {
      const int z = z0 - R + s;
      qr[s] = Store<ST>::template ldb<false>(rs_cur(z, z >= 0 && z < nz), vo_col);
    }
    const auto rh = rs_cur(z0, true);
#pragma unroll
    for (int k = 0; k < NHP; ++k) hr[k] = Store<ST>::template ldb<false>(rh, vo_h[k]);
    Raw hq[HRG ? R : 1][NHP];  // ring: halo of planes z0+1 .. z0+R
    if constexpr (HRG) {
#pragma unroll
      for (int j = 1; j <= R; ++j) {
        const auto rj = rs_cur(z0 + j, z0 + j < z1);
#pragma unroll
        for (int k = 0; k < NHP; ++k) hq[j - 1][k] = Store<ST>::template ldb<false>(rj, vo_h[k]);
      }
    }
    up = Store<ST>::template ldb<NT>(rs_prev(z0, true), vo_col);
    cc = Store<ST_F32>::template ldb<NT>(rs_c2(z0, true), vo_c2);
    if constexpr (GRAD) {
      ufc = Store<ST_F32>::template ldb<false>(rs_f32(a.ufwd, z0, true), vo_c2);
      grc = Store<ST_F32>::template ldb<false>(rs_f32(a.grad, z0, true), vo_c2);
    }
#pragma unroll
    for (int s = 0; s <= 2 * R; ++s) q[s] = wcur(qr[s]);
    lds[0][(ty + R) * LROW4 + XH4 + tx] = q[R];
#pragma unroll
    for (int k = 0; k < NHP; ++k)
      if (hlds[k] >= 0) lds[0][hlds[k]] = wcur(hr[k]);
    if constexpr (HRG) {
#pragma unroll
      for (int j = 1; j <= R; ++j)
#pragma unroll
        for (int k = 0; k < NHP; ++k)
          if (hlds[k] >= 0) hbuf[hslot(z0 + j)][tid + k * NTH] = hq[j - 1][k];
    }
  }
  inj[tid] = zero4;
  if (tid < z1 - z0) bzs[tid] = gmem(a.bz)[z0 + tid];
  __syncthreads();

  // Injection entries of the tile's K one-step tiles on planes [z0, z1) (sorted by
  // plane); ezk[k] is the plane of sub-tile k's next group and ez the nearest of
  // them, kept in registers so the per-plane test needs no load.
  int e[K], e_end[K], ezk[K], eg[K];  // eg[k]: end of sub-tile k's group at ezk[k]
  const auto* ent = gmem(a.ent);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    e[k] = 0;
    e_end[k] = 0;
    ezk[k] = INT_MAX;
    eg[k] = 0;
    const int ty1 = K * ty_t + k;  // one-step tile row
    if (a.tile_beg != nullptr && (K == 1 || ty1 < a.ntile_y)) {
      const int xy1 = ty1 * a.ntile_x + tx_t;
      e[k] = gmem(a.tile_beg)[xy1 * nz + z0];
      e_end[k] = gmem(a.tile_beg)[xy1 * nz + z1];
      if (e[k] < e_end[k]) {
        ezk[k] = ent[e[k]].z;
        eg[k] = ent[e[k]].grp_end;
      }
    }
  }
  int ez = ezk[0];
#pragma unroll
  for (int k = 1; k < K; ++k) ez = min(ez, ezk[k]);

  // Loads that plane zn needs before its own step, kept raw until used: the
  // queue head (plane zn+R), the xy-halo of plane zn (with the halo ring: of plane
  // zn+R, for later), and prev and c2 at plane zn.
  struct Ahead {
    Raw q, up;
    f4v cc, uf, gr;
    Raw h[NHP];
  };
  auto fetch = [&](const int zn, Ahead& f) {
    const bool ok = zn < z1;
    f.q = Store<ST>::template ldb<false>(rs_cur(zn + R, ok && zn + R < nz), vo_col);
    const auto rh = HRG ? rs_cur(zn + R, zn + R < z1) : rs_cur(zn, ok);
#pragma unroll
    for (int k = 0; k < NHP; ++k) f.h[k] = Store<ST>::template ldb<false>(rh, vo_h[k]);
    f.up = Store<ST>::template ldb<NT>(rs_prev(zn, ok), vo_col);
    f.cc = Store<ST_F32>::template ldb<NT>(rs_c2(zn, ok), vo_c2);
    if constexpr (GRAD) {
      f.uf = Store<ST_F32>::template ldb<false>(rs_f32(a.ufwd, zn, ok), vo_c2);
      f.gr = Store<ST_F32>::template ldb<false>(rs_f32(a.grad, zn, ok), vo_c2);
    }
  };
  constexpr bool PF2 = prefetch2(R);

  // One plane of the z-sweep; buf is the LDS buffer that holds plane z, n1 the
  // loads for plane z+1 (issued here, or one plane earlier with PF2, which then
  // issues plane z+2's into n2).
  auto plane_step = [&](const int z, const int buf, Ahead& n1, Ahead& n2) {
    const bool more = z + 1 < z1;
    if constexpr (PF2) fetch(z + 2, n2); else fetch(z + 1, n1);

    // Laplacian of plane z.
    const float4* L = lds[buf];
    const int crow = (ty + R) * LROW4 + XH4 + tx;
    float xv[4 + 2 * XH];  // x0-XH .. x0+3+XH
#pragma unroll
    for (int k = -XH4; k <= XH4; ++k) {
      const float4 v = k == 0 ? q[R] : L[crow + k];
      xv[XH + 4 * k + 0] = v.x; xv[XH + 4 * k + 1] = v.y;
      xv[XH + 4 * k + 2] = v.z; xv[XH + 4 * k + 3] = v.w;
    }
    // Accumulate from the outermost (smallest) weights inwards; the innermost
    // pairs enter as second differences about the centre, (u+1 + u-1) - 2u, and
    // wc = -2 sum_{q>=2} w_q (over the three axes), so a constant field gives
    // exactly zero and no spurious zeroth-order term builds up in FP32.
    float lap[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) lap[p] = BASIC ? 0.f : a.wc * comp(q[R], p);
    if constexpr (!BASIC) {
#pragma unroll
    for (int s = R; s >= 2; --s) {
      const float4 ym = L[crow - s * LROW4];
      const float4 yp = L[crow + s * LROW4];
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        lap[p] = fmaf(a.wx[s], xv[XH + p - s] + xv[XH + p + s], lap[p]);
        lap[p] = fmaf(a.wy[s], comp(ym, p) + comp(yp, p), lap[p]);
        lap[p] = fmaf(a.wz[s], comp(q[R - s], p) + comp(q[R + s], p), lap[p]);
      }
    }
    {
      const float4 ym = L[crow - LROW4];
      const float4 yp = L[crow + LROW4];
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const float u2 = 2.f * comp(q[R], p);
        lap[p] = fmaf(a.wx[1], (xv[XH + p - 1] + xv[XH + p + 1]) - u2, lap[p]);
        lap[p] = fmaf(a.wy[1], (comp(ym, p) + comp(yp, p)) - u2, lap[p]);
        lap[p] = fmaf(a.wz[1], (comp(q[R - 1], p) + comp(q[R + 1], p)) - u2, lap[p]);
      }
    }
    }

    // Fused injection at this plane (uniform branch).
    if (z == ez) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (ezk[k] != z) continue;
        // sub-tile k holds tile rows k*TY .. k*TY+TY-1: local indices offset by k*TY*TX
        for (int i = e[k] + tid; i < eg[k]; i += NTH) {
          const InjEntry en = ent[i];
          const auto* row = gmem(a.trace_row);
          float s = 0.f;
          if (en.tidx >= 0) {  // single term, carried in the entry
            s = fmaf(en.w, row[en.tidx], 0.f);
          } else {
            for (int c = en.csr_beg; c < en.csr_end; ++c)
              s = fmaf(gmem(a.csr_w)[c], row[gmem(a.csr_idx)[c]], s);
          }
          reinterpret_cast<float*>(inj)[k * TY * TX + en.local] = s;
        }
      }
      __syncthreads();
      const float4 iv = inj[tid];
      lap[0] += iv.x; lap[1] += iv.y; lap[2] += iv.z; lap[3] += iv.w;
      inj[tid] = zero4;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (ezk[k] != z) continue;
        e[k] = eg[k];
        ezk[k] = INT_MAX;
        if (e[k] < e_end[k]) {
          ezk[k] = ent[e[k]].z;
          eg[k] = ent[e[k]].grp_end;
        }
      }
      ez = ezk[0];
#pragma unroll
      for (int k = 1; k < K; ++k) ez = min(ez, ezk[k]);
    }

    // Damped leapfrog update in increment form:
    //   out = u + ((1-b)(u - prev) + c2 (L u + inj)) / (1+b)
    // (equal to (2u - (1-b) prev + c2 (L u + inj)) / (1+b)); u - prev is exact for
    // smooth fields, so the only rounding at the magnitude of u is the final add.
    // In the difference form prev already holds d = u^n - u^{n-1} and the new
    // difference is stored beside u^{n+1}.
    const float bzv = bzs[z - z0];
    const float4 upv = wprev(up);
    const float4 ccv = Store<ST_F32>::widen(cc);
    float4 o, dn, src;
    if constexpr (BASIC) {
      // The unfactorised update of the paper's SO2 listing (Section 2.1), every
      // term with its own coefficient and its own division by
      // r0 = dt m + dt^2 damp / 2, with m = dt^2 / c2 and damp = m gamma per point
      // (here lap holds only the injected samples). Ablation only.
      const float dt = a.dt, dt2 = dt * dt, dt3 = dt2 * dt;
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const float c = comp(ccv, p);
        const float b = (comp(bxv, p) + byv) + bzv;
        const float u = comp(q[R], p), um = comp(upv, p);
        const float m = dt2 / c;
        const float damp = m * (2.f * b / dt);
        const float r0 = dt * m + 0.5f * dt2 * damp;
        float acc = -dt * m * um / r0 + dt3 * lap[p] / r0;
#pragma unroll
        for (int s = 1; s <= R; ++s) {
          const float4 ym = L[crow - s * LROW4];
          const float4 yp = L[crow + s * LROW4];
          acc += dt3 * a.wx[s] * xv[XH + p - s] / r0 + dt3 * a.wx[s] * xv[XH + p + s] / r0;
          acc += dt3 * a.wy[s] * comp(ym, p) / r0 + dt3 * a.wy[s] * comp(yp, p) / r0;
          acc += dt3 * a.wz[s] * comp(q[R - s], p) / r0 + dt3 * a.wz[s] * comp(q[R + s], p) / r0;
        }
        acc += 2.f * dt * m * u / r0 + 0.5f * dt2 * damp * um / r0 +
               dt3 * (a.wx[0] + a.wy[0] + a.wz[0]) * u / r0;
        set_comp(o, p, c > 0.f ? acc : 0.f);  // padding columns (c2 = 0) stay zero
      }
    } else {
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const float b = (comp(bxv, p) + byv) + bzv;
      const float u = comp(q[R], p);
      const float d = DIFF ? comp(upv, p) : u - comp(upv, p);
      const float c = comp(ccv, p);
      if constexpr (GRAD) set_comp(src, p, c * lap[p]);
      const float num = fmaf(c, lap[p], fmaf(-b, d, d));
      const float inv = __builtin_amdgcn_rcpf(1.f + b);
      if constexpr (DIFF) {
        const float dd = num * inv;
        set_comp(dn, p, dd);
        set_comp(o, p, u + dd);
      } else {
        set_comp(o, p, fmaf(num, inv, u));
      }
    }
    }
    if constexpr (BSTORE) {
      // buffer stores on every path (lanes outside the grid have offset kOOB): the
      // plane's resource carries the address, no per-lane 64-bit arithmetic
      if constexpr (ST == ST_F32) {
        Store<ST>::template stb<NT>(rs_at(a.out, z, ES, pbytes, true), vo_col, o);
      } else {
        if (colok) {
          mx_u = fmaxf(mx_u, fmaxf(fmaxf(fabsf(o.x), fabsf(o.y)), fmaxf(fabsf(o.z), fabsf(o.w))));
          if constexpr (DIFF)
            mx_d = fmaxf(mx_d, fmaxf(fmaxf(fabsf(dn.x), fabsf(dn.y)), fmaxf(fabsf(dn.z), fabsf(dn.w))));
        }
        if constexpr (DIFF) {
          Store<ST>::template stb<NT>(rs_at(a.out_u, z, ES, pbytes, true), vo_col, mul4(o, enc_u));
          Store<ST>::template stb<NT>(rs_at(a.out, z, ES, pbytes, true), vo_col, mul4(dn, enc_d));
        } else {
          Store<ST>::template stb<NT>(rs_at(a.out, z, ES, pbytes, true), vo_col, mul4(o, enc_u));
        }
      }
      if constexpr (GRAD) {
        const float4 uf = Store<ST_F32>::widen(ufc);
        float4 gv = Store<ST_F32>::widen(grc);
        const float4 f = a.acc_image ? q[R] : src;
        gv.x = fmaf(uf.x, f.x, gv.x); gv.y = fmaf(uf.y, f.y, gv.y);
        gv.z = fmaf(uf.z, f.z, gv.z); gv.w = fmaf(uf.w, f.w, gv.w);
        Store<ST_F32>::template stb<false>(rs_f32(a.grad, z, true), vo_c2, gv);
      }
    } else if (colok) {
      const int64_t at = z * plane + col;
      if constexpr (ST == ST_F32) {
        Store<ST>::template st<NT>(a.out, at, o);
      } else {
        mx_u = fmaxf(mx_u, fmaxf(fmaxf(fabsf(o.x), fabsf(o.y)), fmaxf(fabsf(o.z), fabsf(o.w))));
        if constexpr (DIFF) {
          mx_d = fmaxf(mx_d, fmaxf(fmaxf(fabsf(dn.x), fabsf(dn.y)), fmaxf(fabsf(dn.z), fabsf(dn.w))));
          Store<ST>::template st<NT>(a.out_u, at, mul4(o, enc_u));
          Store<ST>::template st<NT>(a.out, at, mul4(dn, enc_d));
        } else {
          Store<ST>::template st<NT>(a.out, at, mul4(o, enc_u));
        }
      }
      if constexpr (GRAD) {
        const float4 uf = Store<ST_F32>::widen(ufc);
        float4 gv = Store<ST_F32>::widen(grc);
        const float4 f = a.acc_image ? q[R] : src;
        gv.x = fmaf(uf.x, f.x, gv.x); gv.y = fmaf(uf.y, f.y, gv.y);
        gv.z = fmaf(uf.z, f.z, gv.z); gv.w = fmaf(uf.w, f.w, gv.w);
        st4(a.grad + at, gv);
      }
    }

    // Stage plane z+1 into the other LDS buffer (its halo from the ring, which then
    // takes the halo of plane z+1+R).
    if (more) {
      lds[buf ^ 1][crow] = q[R + 1];
#pragma unroll
      for (int k = 0; k < NHP; ++k)
        if (hlds[k] >= 0)
          lds[buf ^ 1][hlds[k]] =
              wcur(HRG ? hbuf[hslot(z + 1)][tid + k * NTH] : n1.h[k]);
    }
    if constexpr (HRG) {
      if (z + 1 + R < z1) {
#pragma unroll
        for (int k = 0; k < NHP; ++k)
          if (hlds[k] >= 0) hbuf[hslot(z + 1 + R)][tid + k * NTH] = n1.h[k];
      }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 2 * R; ++s) q[s] = q[s + 1];
    q[2 * R] = wcur(n1.q);
    up = n1.up;
    cc = n1.cc;
    if constexpr (GRAD) {
      ufc = n1.uf;
      grc = n1.gr;
    }
  };
  // Two planes per iteration give each call a constant LDS buffer index and swap
  // the roles of the two load sets without copies (the barriers inside keep the
  // compiler from unrolling the loop by itself).
  Ahead fa, fb;
  if constexpr (PF2) fetch(z0 + 1, fa);
  int z = z0;
  if constexpr (zunroll4(R) && !PF2) {
    for (; z + 3 < z1; z += 4) {
      plane_step(z, 0, fa, fb);
      plane_step(z + 1, 1, fb, fa);
      plane_step(z + 2, 0, fa, fb);
      plane_step(z + 3, 1, fb, fa);
    }
  }
  if constexpr (PF2 || zunroll2(R) || zunroll4(R)) {
    for (; z + 1 < z1; z += 2) {
      plane_step(z, 0, fa, fb);
      plane_step(z + 1, 1, fb, fa);
    }
    if (z < z1) plane_step(z, 0, fa, fb);
  } else {
    for (; z < z1; ++z) plane_step(z, (z - z0) & 1, fa, fb);
  }
  if constexpr (ST != ST_F32) {
    // Maxima of the level just written, for the next step's scale choice: reduced
    // over the workgroup, then one atomic per workgroup into its slot.
    __shared__ float wm[2][NTH / 64];
    mx_u = wave_max(mx_u);
    if (DIFF) mx_d = wave_max(mx_d);
    if ((tid & 63) == 0) {
      wm[0][tid >> 6] = mx_u;
      wm[1][tid >> 6] = mx_d;
    }
    __syncthreads();
    if (tid == 0) {
      float mu = wm[0][0], md = wm[1][0];
#pragma unroll
      for (int w = 1; w < NTH / 64; ++w) {
        mu = fmaxf(mu, wm[0][w]);
        md = fmaxf(md, wm[1][w]);
      }
      const int slot = (a.level + 2) * kMaxSlots + (int)(blockIdx.x % kMaxSlots);
      atomicMax(a.meta.mu + slot, __float_as_uint(mu));
      if (DIFF) atomicMax(a.meta.md + slot, __float_as_uint(md));
    }
  }
}

// Maximum recorded for bookkeeping entry i (a level index + 1) over its slots.
__device__ __forceinline__ float level_max(const unsigned* arr, int i) {
  unsigned m = 0;
#pragma unroll
  for (int s = 0; s < kMaxSlots; ++s) m = max(m, arr[i * kMaxSlots + s]);
  return __uint_as_float(m);
}

// K one-step tiles per workgroup along y (the launch passes a.tiles_y == K)
template <int R, bool GRAD, int ST, bool DIFF, bool NT, bool BASIC, int K>
__global__ void __launch_bounds__(K * NTHREADS) step_kernel(const StepArgs a) {
  constexpr int NTH = K * NTHREADS;
  // Per-level scales of reduced-precision storage: decode cur and prev, choose
  // the encode scales of the level written here from the previous maxima.
  float dec_c = 1.f, dec_p = 1.f, enc_u = 1.f, enc_d = 1.f;
  if constexpr (ST != ST_F32) {
    const int n = a.level;
    dec_c = ldexpf(1.f, -a.meta.eu[n + 1]);
    dec_p = ldexpf(1.f, DIFF ? -a.meta.ed[n + 1] : -a.meta.eu[n]);
    const float mun = level_max(a.meta.mu, n + 1);
    const float injb = a.meta.injb[n];
    int eu, ed = 0;
    if constexpr (DIFF) {
      // |d^{n+1}| <= |d^n| + c2 |L u^n| + inj, c2 |L| <= 4 under the CFL limit
      const float bd = level_max(a.meta.md, n + 1) + 4.f * mun + injb;
      ed = scale_exp(bd);
      eu = scale_exp(mun + bd);
    } else {
      eu = scale_exp(8.f * fmaxf(mun, level_max(a.meta.mu, n)) + injb);
    }
    enc_u = ldexpf(1.f, eu);
    enc_d = ldexpf(1.f, ed);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.meta.eu[n + 2] = eu;
      if (DIFF) a.meta.ed[n + 2] = ed;
    }
  }
  const int bid = blockIdx.x;
  if (bid >= a.nstencil_blocks) {
    const int r = (bid - a.nstencil_blocks) * NTH + threadIdx.x;
    if (a.samp_out != nullptr && r < a.nsamp)
      a.samp_out[r] = sample_point<ST>(a.cur, dec_c, a.samp_idx, a.samp_w, r);
    return;
  }
  // logical tile t = (chunk * ntile_yK + ty) * ntile_x + tx, in tiles of K one-step
  // tiles along y
  const int t = a.xcd_remap ? remap_tile(bid, a.nstencil_blocks) : bid;
  const int bxy = a.ntile_x * ((a.ntile_y + K - 1) / K);
  const int z0 = (t / bxy) * a.zchunk;
  step_tile<R, GRAD, ST, DIFF, NT, BASIC, K>(a, t % bxy, z0, min(z0 + a.zchunk, a.g.nz), dec_c,
                                             dec_p, enc_u, enc_d);
}

// Serving: one launch advances every active shot of one space order by a step.
// Block b (after the XCD remap) takes table entry b = (shot, xy tile, planes
// [z0, z1)); xy < 0 is sampling block -1-xy of that shot (the host chooses each
// group's chunking when it builds the table). The shot's step n is read from its
// parity-indexed counter cnts[2 * shot + parity] (launches alternate parity), so
// the same captured launch sequence replays for any mix of shots at any steps. A
// shot whose n reached nt only samples its last level; past nt it does nothing.
// The descriptors are read-only here (the counters are a separate array): with a
// descriptor that the kernel also wrote, the compiler held its arguments in 19-38
// more VGPRs than the single-shot kernel's (133 against 114 at r = 4, three waves per
// SIMD instead of four); read-only, the two kernels use the same registers. K is the
// launch's workgroup height in one-step tiles (the table's xy then counts K-tall
// tiles). The table lists every stencil block before the sampling blocks, and only the
// stencil blocks take the XCD remap, so the light sampling blocks are dispatched last
// (a stencil block dispatched after every CU got one would run beside another on one
// CU and hold up the launch: measured 6.7 % at SO8, 15 % at SO4 on 64 x 32 tiles).
template <int R, int K>
__global__ void __launch_bounds__(K * NTHREADS) batched_step_kernel(const ShotDesc* __restrict__ shots,
                                                                    int* __restrict__ cnts,
                                                                    const BatchEntry* __restrict__ table,
                                                                    int nstencil, int parity) {
  const int b = (int)blockIdx.x < nstencil ? remap_tile(blockIdx.x, nstencil) : (int)blockIdx.x;
  const BatchEntry e = table[b];
  const ShotDesc* sd = shots + e.shot;
  const int n = cnts[2 * e.shot + parity];
  const int nt = sd->nt;
  if (e.xy == 0 && e.z0 == 0 && threadIdx.x == 0)  // the shot's first stencil block
    cnts[2 * e.shot + (parity ^ 1)] = n <= nt ? n + 1 : n;
  if (n > nt) return;
  StepArgs a = sd->a;
  a.cur = sd->buf[n & 1];
  a.prev = sd->buf[(n + 1) & 1];
  a.out = sd->buf[(n + 1) & 1];
  if (sd->nsrc > 0 && n < nt) {
    a.trace_row = sd->wavelet + (int64_t)n * sd->nsrc;
  } else {
    a.tile_beg = nullptr;
    a.trace_row = nullptr;
  }
  a.samp_out = (n >= 1 && sd->nrec > 0) ? sd->traces + (int64_t)(n - 1) * sd->nrec : nullptr;
  if (e.xy < 0) {
    const int r = (-1 - e.xy) * (K * NTHREADS) + threadIdx.x;
    if (a.samp_out != nullptr && r < a.nsamp)
      a.samp_out[r] = sample_point<ST_F32>(a.cur, 1.f, a.samp_idx, a.samp_w, r);
    return;
  }
  if (n < nt)
    step_tile<R, false, ST_F32, false, false, false, K>(a, e.xy, e.z0, e.z1, 1.f, 1.f, 1.f, 1.f);
}

// Copy each listed shot's counter of parity 0 into out (host read-back after a replay).
__global__ void gather_counters_kernel(const int* cnts, const int* slots, int n, int* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = cnts[2 * slots[i]];
}

template <int ST>
__global__ void sample_kernel(const void* f, LevelMeta meta, int m, const int* idx,
                              const float* w, int n, float* out) {
  float dec = 1.f;
  if constexpr (ST != ST_F32) dec = ldexpf(1.f, -meta.eu[m + 1]);
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) out[r] = sample_point<ST>(f, dec, idx, w, r);
}

__global__ void pack_kernel(const float* src, float* dst, Geom g) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < g.nfield; p += stride) {
    const int i = (int)(p % g.pitch);
    const int64_t row = p / g.pitch;  // k*ny + j
    dst[p] = (src != nullptr && i < g.nx) ? src[row * g.nx + i] : 0.f;
  }
}

__global__ void unpack_kernel(const float* src, float* dst, Geom g) {
  const int64_t n = (int64_t)g.nx * g.ny * g.nz;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
    const int64_t row = p / g.nx;
    const int i = (int)(p - row * g.nx);
    dst[p] = src[row * g.pitch + i];
  }
}

__global__ void prep_c2_kernel(const float* vel, float* c2, Geom g, double dt2) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < g.nfield; p += stride) {
    const int i = (int)(p % g.pitch);
    const int64_t row = p / g.pitch;
    float v = 0.f;
    if (i < g.nx) {
      const double vv = (double)vel[row * g.nx + i];
      v = (float)(vv * vv * dt2);
    }
    c2[p] = v;
  }
}

__global__ void grad_finalize_kernel(const float* graw, const float* vel, float* gv, Geom g,
                                     double scale) {
  const int64_t n = (int64_t)g.nx * g.ny * g.nz;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
    const int64_t row = p / g.nx;
    const int i = (int)(p - row * g.nx);
    const double v = (double)vel[p];
    gv[p] = (float)(scale * (double)graw[row * g.pitch + i] / (v * v * v));
  }
}

__global__ void copy_kernel(const float* src, float* dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride)
    dst[p] = src[p];
}

__global__ void zero_words_kernel(unsigned* p, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0u;
}

// One block per time step: injb[k] = c2max * 8 * max_j |trace[k][j]| (a point gets
// trilinear contributions from at most 8 traces, weights <= 1).
__global__ void inj_bound_kernel(const float* trace, int ntr, float c2max, float* injb) {
  __shared__ float red[256];
  const int k = blockIdx.x;
  float m = 0.f;
  for (int j = threadIdx.x; j < ntr; j += blockDim.x)
    m = fmaxf(m, fabsf(trace[(int64_t)k * ntr + j]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) injb[k] = c2max * 8.f * red[0];
}

// Maxima of initial levels: slot_a <- max|a|, slot_b <- max|a - b| (diff) or max|b|.
__global__ void initial_max_kernel(const float* a, const float* b, bool diff, unsigned* slot_a,
                                   unsigned* slot_b, int64_t n) {
  __shared__ float ra[256], rb[256];
  float ma = 0.f, mb = 0.f;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
    const float va = a != nullptr ? a[p] : 0.f, vb = b != nullptr ? b[p] : 0.f;
    ma = fmaxf(ma, fabsf(va));
    mb = fmaxf(mb, fabsf(diff ? va - vb : vb));
  }
  ra[threadIdx.x] = ma;
  rb[threadIdx.x] = mb;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if ((int)threadIdx.x < o) {
      ra[threadIdx.x] = fmaxf(ra[threadIdx.x], ra[threadIdx.x + o]);
      rb[threadIdx.x] = fmaxf(rb[threadIdx.x], rb[threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicMax(slot_a, __float_as_uint(ra[0]));
    atomicMax(slot_b, __float_as_uint(rb[0]));
  }
}

// Scale exponents of the initial levels (one thread).
__global__ void initial_scales_kernel(LevelMeta meta, int m, bool diff) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  meta.eu[m + 1] = scale_exp(level_max(meta.mu, m + 1));
  if (diff)
    meta.ed[m + 1] = scale_exp(level_max(meta.md, m + 1));
  else
    meta.eu[m] = scale_exp(level_max(meta.mu, m));
}

// Encode initial levels into pitched stores (padding columns zero).
template <int ST>
__global__ void encode_initial_kernel(const float* a, const float* b, void* ua, void* ub,
                                      bool diff, LevelMeta meta, int m, Geom g) {
  const float ea = ldexpf(1.f, meta.eu[m + 1]);
  const float eb = ldexpf(1.f, diff ? meta.ed[m + 1] : meta.eu[m]);
  const int64_t n4 = g.nfield / 4;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n4; q += stride) {
    const int64_t p = 4 * q;
    const int i = (int)(p % g.pitch);
    const int64_t row = p / g.pitch;
    float va[4], vb[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const bool in = i + k < g.nx;
      const float x = (in && a != nullptr) ? a[row * g.nx + i + k] : 0.f;
      const float y = (in && b != nullptr) ? b[row * g.nx + i + k] : 0.f;
      va[k] = x;
      vb[k] = diff ? x - y : y;
    }
    Store<ST>::template st<false>(ua, p, make_float4(va[0] * ea, va[1] * ea, va[2] * ea, va[3] * ea));
    Store<ST>::template st<false>(ub, p, make_float4(vb[0] * eb, vb[1] * eb, vb[2] * eb, vb[3] * eb));
  }
}

template <int ST>
__global__ void decode_kernel(const void* src, LevelMeta meta, int m, float* dst, Geom g) {
  const float dec = ldexpf(1.f, -meta.eu[m + 1]);
  const int64_t n = (int64_t)g.nx * g.ny * g.nz;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
    const int64_t row = p / g.nx;
    const int i = (int)(p - row * g.nx);
    dst[p] = Store<ST>::ld1(src, row * g.pitch + i) * dec;
  }
}

namespace {
int elementwise_blocks(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (int)b;
}

template <int R, bool GRAD, int ST, bool DIFF, bool NT, bool BASIC, int K>
hipError_t launch_k(const StepArgs& a, hipStream_t s) {
  constexpr int nth = K * NTHREADS;
  const int nsamp_blocks = a.samp_out != nullptr ? (a.nsamp + nth - 1) / nth : 0;
  const dim3 grid(a.nstencil_blocks + nsamp_blocks), block(nth);
  hipLaunchKernelGGL((step_kernel<R, GRAD, ST, DIFF, NT, BASIC, K>), grid, block, 0, s, a);
  return hipGetLastError();
}

// the workgroup height the host chose (a.tiles_y), instantiated where tall_tiles_ok
template <int R, bool GRAD, int ST, bool DIFF, bool NT, bool BASIC = false>
hipError_t launch_r(const StepArgs& a, hipStream_t s) {
  if constexpr (tall_tiles_ok(R)) {
    if (a.tiles_y == 2) return launch_k<R, GRAD, ST, DIFF, NT, BASIC, 2>(a, s);
  }
  if (a.tiles_y != 1) return hipErrorInvalidValue;
  return launch_k<R, GRAD, ST, DIFF, NT, BASIC, 1>(a, s);
}

template <int R, int ST, bool DIFF>
hipError_t launch_nt(const StepArgs& a, bool nt, hipStream_t s) {
  return nt ? launch_r<R, false, ST, DIFF, true>(a, s) : launch_r<R, false, ST, DIFF, false>(a, s);
}

template <int R>
hipError_t launch_variant(const StepArgs& a, bool grad, int st, bool diff, bool nt,
                          hipStream_t s) {
  if (st == ST_F32) {
    if (diff) return hipErrorInvalidValue;
    return grad ? launch_r<R, true, ST_F32, false, false>(a, s)
                : launch_nt<R, ST_F32, false>(a, nt, s);
  }
  if (grad) return hipErrorInvalidValue;
  if (st == ST_F16)
    return diff ? launch_nt<R, ST_F16, true>(a, nt, s) : launch_nt<R, ST_F16, false>(a, nt, s);
  if (st == ST_BF16)
    return diff ? launch_nt<R, ST_BF16, true>(a, nt, s) : launch_nt<R, ST_BF16, false>(a, nt, s);
  return hipErrorInvalidValue;
}
}  // namespace

hipError_t launch_step_basic(const StepArgs& a, int r, hipStream_t s) {
  switch (r) {
    case 4: return launch_r<4, false, ST_F32, false, false, true>(a, s);
    case 6: return launch_r<6, false, ST_F32, false, false, true>(a, s);
    case 8: return launch_r<8, false, ST_F32, false, false, true>(a, s);
    case 12: return launch_r<12, false, ST_F32, false, false, true>(a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_step(const StepArgs& a, int r, bool grad, int st, bool diff, bool nt,
                       hipStream_t s) {
  switch (r) {
    case 1: return launch_variant<1>(a, grad, st, diff, nt, s);
    case 2: return launch_variant<2>(a, grad, st, diff, nt, s);
    case 3: return launch_variant<3>(a, grad, st, diff, nt, s);
    case 4: return launch_variant<4>(a, grad, st, diff, nt, s);
    case 5: return launch_variant<5>(a, grad, st, diff, nt, s);
    case 6: return launch_variant<6>(a, grad, st, diff, nt, s);
    case 7: return launch_variant<7>(a, grad, st, diff, nt, s);
    case 8: return launch_variant<8>(a, grad, st, diff, nt, s);
    case 9: return launch_variant<9>(a, grad, st, diff, nt, s);
    case 10: return launch_variant<10>(a, grad, st, diff, nt, s);
    case 11: return launch_variant<11>(a, grad, st, diff, nt, s);
    case 12: return launch_variant<12>(a, grad, st, diff, nt, s);
    default: return hipErrorInvalidValue;
  }
}

namespace {
template <int R, int K>
hipError_t launch_batched_k(const ShotDesc* shots, int* cnts, const BatchEntry* table, int nentries,
                            int nstencil, int parity, hipStream_t s) {
  const dim3 grid(nentries), block(K * NTHREADS);
  hipLaunchKernelGGL((batched_step_kernel<R, K>), grid, block, 0, s, shots, cnts, table, nstencil,
                     parity);
  return hipGetLastError();
}
template <int R>
hipError_t launch_batched_r(const ShotDesc* shots, int* cnts, const BatchEntry* table, int nentries,
                            int nstencil, int tiles_y, int parity, hipStream_t s) {
  if constexpr (tall_tiles_ok(R)) {
    if (tiles_y == 2) return launch_batched_k<R, 2>(shots, cnts, table, nentries, nstencil, parity, s);
  }
  if (tiles_y != 1) return hipErrorInvalidValue;
  return launch_batched_k<R, 1>(shots, cnts, table, nentries, nstencil, parity, s);
}
}  // namespace

hipError_t launch_batched(const ShotDesc* shots, int* cnts, const BatchEntry* table, int nentries,
                          int nstencil, int r, int tiles_y, int parity, hipStream_t s) {
  if (nentries <= 0) return hipSuccess;
  if (nstencil < 0 || nstencil > nentries) return hipErrorInvalidValue;
  switch (r) {
    case 1: return launch_batched_r<1>(shots, cnts, table, nentries, nstencil, tiles_y, parity, s);
    case 2: return launch_batched_r<2>(shots, cnts, table, nentries, nstencil, tiles_y, parity, s);
    case 3: return launch_batched_r<3>(shots, cnts, table, nentries, nstencil, tiles_y, parity, s);
    case 4: return launch_batched_r<4>(shots, cnts, table, nentries, nstencil, tiles_y, parity, s);
    case 5: return launch_batched_r<5>(shots, cnts, table, nentries, nstencil, tiles_y, parity, s);
    case 6: return launch_batched_r<6>(shots, cnts, table, nentries, nstencil, tiles_y, parity, s);
    case 7: return launch_batched_r<7>(shots, cnts, table, nentries, nstencil, tiles_y, parity, s);
    case 8: return launch_batched_r<8>(shots, cnts, table, nentries, nstencil, tiles_y, parity, s);
    case 9: return launch_batched_r<9>(shots, cnts, table, nentries, nstencil, tiles_y, parity, s);
    case 10: return launch_batched_r<10>(shots, cnts, table, nentries, nstencil, tiles_y, parity, s);
    case 11: return launch_batched_r<11>(shots, cnts, table, nentries, nstencil, tiles_y, parity, s);
    case 12: return launch_batched_r<12>(shots, cnts, table, nentries, nstencil, tiles_y, parity, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_gather_counters(const int* cnts, const int* slots, int n, int* out,
                                  hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_counters_kernel, dim3((n + 255) / 256), dim3(256), 0, s, cnts, slots,
                     n, out);
  return hipGetLastError();
}

hipError_t launch_sample(const void* field, int st, LevelMeta meta, int m, const int* idx,
                         const float* w, int n, float* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const dim3 grid((n + 255) / 256), block(256);
  if (st == ST_F32)
    hipLaunchKernelGGL(sample_kernel<ST_F32>, grid, block, 0, s, field, meta, m, idx, w, n, out);
  else if (st == ST_F16)
    hipLaunchKernelGGL(sample_kernel<ST_F16>, grid, block, 0, s, field, meta, m, idx, w, n, out);
  else
    hipLaunchKernelGGL(sample_kernel<ST_BF16>, grid, block, 0, s, field, meta, m, idx, w, n, out);
  return hipGetLastError();
}

hipError_t launch_pack(const float* src, float* dst, Geom g, hipStream_t s) {
  hipLaunchKernelGGL(pack_kernel, dim3(elementwise_blocks(g.nfield)), dim3(256), 0, s, src, dst,
                     g);
  return hipGetLastError();
}

hipError_t launch_unpack(const float* src, float* dst, Geom g, hipStream_t s) {
  hipLaunchKernelGGL(unpack_kernel, dim3(elementwise_blocks((int64_t)g.nx * g.ny * g.nz)),
                     dim3(256), 0, s, src, dst, g);
  return hipGetLastError();
}

hipError_t launch_prep_c2(const float* vel, float* c2, Geom g, double dt, hipStream_t s) {
  hipLaunchKernelGGL(prep_c2_kernel, dim3(elementwise_blocks(g.nfield)), dim3(256), 0, s, vel, c2,
                     g, dt * dt);
  return hipGetLastError();
}

hipError_t launch_grad_finalize(const float* graw, const float* vel, float* grad_vel, Geom g,
                                double scale, hipStream_t s) {
  hipLaunchKernelGGL(grad_finalize_kernel, dim3(elementwise_blocks((int64_t)g.nx * g.ny * g.nz)),
                     dim3(256), 0, s, graw, vel, grad_vel, g, scale);
  return hipGetLastError();
}

hipError_t launch_copy(const float* src, float* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(copy_kernel, dim3(elementwise_blocks(n)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_zero_words(unsigned* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_words_kernel, dim3(elementwise_blocks(n)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_inj_bound(const float* trace, int nt, int ntr, float c2max, float* injb,
                            hipStream_t s) {
  if (nt <= 0 || ntr <= 0 || trace == nullptr) return hipSuccess;
  hipLaunchKernelGGL(inj_bound_kernel, dim3(nt), dim3(256), 0, s, trace, ntr, c2max, injb);
  return hipGetLastError();
}

hipError_t launch_encode_initial(const float* a, const float* b, void* ua, void* ub, int st,
                                 bool diff, LevelMeta meta, int m, Geom g, hipStream_t s) {
  const int64_t n = (int64_t)g.nx * g.ny * g.nz;
  // slot 0 of the entries of levels m and m-1
  unsigned* slot_b = diff ? meta.md + (m + 1) * kMaxSlots : meta.mu + m * kMaxSlots;
  hipLaunchKernelGGL(initial_max_kernel, dim3(elementwise_blocks(n)), dim3(256), 0, s, a, b, diff,
                     meta.mu + (m + 1) * kMaxSlots, slot_b, n);
  hipLaunchKernelGGL(initial_scales_kernel, dim3(1), dim3(64), 0, s, meta, m, diff);
  const dim3 grid(elementwise_blocks(g.nfield / 4)), block(256);
  if (st == ST_F16)
    hipLaunchKernelGGL(encode_initial_kernel<ST_F16>, grid, block, 0, s, a, b, ua, ub, diff, meta,
                       m, g);
  else
    hipLaunchKernelGGL(encode_initial_kernel<ST_BF16>, grid, block, 0, s, a, b, ua, ub, diff,
                       meta, m, g);
  return hipGetLastError();
}

hipError_t launch_decode(const void* src, int st, LevelMeta meta, int m, float* dst, Geom g,
                         hipStream_t s) {
  const dim3 grid(elementwise_blocks((int64_t)g.nx * g.ny * g.nz)), block(256);
  if (st == ST_F16)
    hipLaunchKernelGGL(decode_kernel<ST_F16>, grid, block, 0, s, src, meta, m, dst, g);
  else
    hipLaunchKernelGGL(decode_kernel<ST_BF16>, grid, block, 0, s, src, meta, m, dst, g);
  return hipGetLastError();
}

}  // namespace wave
