// wave_fused.hip -- two leapfrog steps per pass over HBM (temporal blocking in
// z-streaming form) for the FP32 forward solve, space orders 2..8.
//
// The single-step kernel moves 16 bytes per point and step (read u^n, u^{n-1},
// c2; write u^{n+1}) and is bandwidth-bound at every space order. This kernel
// reads u^n, u^{n-1} and c2 once and writes u^{n+1} and u^{n+2}: 20 bytes per
// point for two steps. Each workgroup owns a tile of TX x TY2 points (TY2 = K TY,
// K = f2_tiles_y(r) one-step tiles stacked along y) and a z-chunk and runs two
// pipelined stages down the chunk:
//   stage A  v = u^{n+1} at plane za on the tile extended by XH columns and R rows
//            on each side (the region E), from a register queue of u^n planes
//            za-R..za+R and an LDS copy of plane za with a further ring;
//   stage B  u^{n+2} at plane zb = za - R on the tile, from a register queue of v
//            planes zb-R..zb+R and an LDS copy of v at plane zb on E.
// Stage A runs R planes beyond the chunk at both ends (and stage B needs u^n
// beyond that), so each chunk recomputes 2R planes of v and re-reads 4R planes of
// u^n; the extended region costs (TX+2XH)(TY2+2R)/(TX TY2) times the stage-A work
// (1.69 at K = 1, r = 4; 1.41 at K = 2).
// Both are paid in arithmetic and L2 traffic, which this bandwidth-bound scheme
// has to spare. Every point's update is the same expression, in the same order,
// as in the single-step kernel.
//
// Loads are cached (u^n, u^{n-1} and c2 are read by neighbouring workgroups and,
// for c2, again by stage B); with NT the two outputs are stored non-temporally.
//
// Injection: stage A adds step n's source terms at every point of E (per-tile
// lists over E, which overlap neighbouring tiles), stage B adds step n+1's at the
// tile's points. Sampling: the two input levels are read-only in the pass, so
// extra workgroups sample u^n and u^{n-1} (the previous pass's outputs).
#include <climits>

#include "wave_device.h"

namespace wave {

namespace {

constexpr int F2_XH = 4;                 // x extension of E (>= R, multiple of 4)
constexpr int F2_XH4 = F2_XH / 4;
constexpr int F2_EX4 = NTX + 2 * F2_XH4;  // float4 columns of E per row
constexpr int F2_UROW4 = NTX + 4 * F2_XH4;  // float4 per row of the LDS copy of u^n

template <int R, bool NT>
__device__ __forceinline__ void fused2_tile(const Fused2Args& f, const int t) {
  const StepArgs& a = f.a;
  constexpr int K = f2_tiles_y(R);                  // one-step tiles per tile, along y
  constexpr int TY2 = K * TY;                       // rows of the tile
  constexpr int NTH = f2_threads(R);
  constexpr int EY = TY2 + 2 * R;                   // rows of E
  constexpr int NE = F2_EX4 * EY;                   // E columns (threads with a column)
  constexpr int UROWS = TY2 + 4 * R;                // rows of the LDS copy of u^n
  constexpr int NRING = 2 * R * F2_UROW4 + EY * 2 * F2_XH4;  // u^n items around E
  static_assert(TX + 2 * F2_XH == 4 * F2_EX4, "E rows hold whole float4");
  static_assert(R <= F2_XH && NE <= NTH && NRING <= NTH, "fused tile shape");
  __shared__ float4 ulds[2][UROWS * F2_UROW4];
  __shared__ float4 vlds[EY * F2_EX4];
  __shared__ float4 inj[EY * F2_EX4];
  __shared__ float bzs[MAXZCHUNK + 2 * F2_XH];
  // Per-thread slots (written and read by the same thread, no barrier needed) for
  // R+1 planes: the u^n ring item of planes za+1 .. za+1+R, loaded in the same
  // iteration as the neighbouring workgroups load those columns as their queue
  // heads (so the ring is served by L2); and c2 of the tile columns at planes
  // za-R .. za for stage B (stage A's own load, reused).
  __shared__ float4 ringbuf[R + 1][NRING];
  __shared__ float4 cring[R + 1][TY2 * NTX];
  const auto slot = [](const int z) { return ((z % (R + 1)) + (R + 1)) % (R + 1); };

  const int tx_t = t % a.ntile_x;
  const int rest = t / a.ntile_x;
  const int ty_t = rest % a.ntile_y;
  const int zc = rest / a.ntile_y;
  const int xt = tx_t * TX, yt = ty_t * TY2;
  const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
  const int64_t plane = a.g.plane;
  const int z0 = zc * a.zchunk;
  const int z1 = min(z0 + a.zchunk, nz);
  const int za0 = z0 - R, za1 = z1 + R;  // stage-A planes [za0, za1)
  const int tid = threadIdx.x;
  const bool act = tid < NE;
  const int ex = act ? tid % F2_EX4 : 0, ey = act ? tid / F2_EX4 : 0;
  const int x0 = xt - F2_XH + 4 * ex, y = yt - R + ey;
  const bool colok = act && x0 >= 0 && x0 < nx && y >= 0 && y < ny;
  const bool inner = act && ex >= F2_XH4 && ex < F2_XH4 + NTX && ey >= R && ey < R + TY2;
  const int col = colok ? y * a.g.pitch + x0 : 0;
  const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);

  // The ring of u^n around E that stage A's x/y neighbours need (one item per thread).
  int hl = -1;
  unsigned vo_h = kOOB;
  if (tid < NRING) {
    int row, c4;
    if (tid < R * F2_UROW4) {
      row = tid / F2_UROW4; c4 = tid % F2_UROW4;
    } else if (tid < 2 * R * F2_UROW4) {
      const int j = tid - R * F2_UROW4;
      row = R + EY + j / F2_UROW4; c4 = j % F2_UROW4;
    } else {
      const int j = tid - 2 * R * F2_UROW4;
      const int side = j % (2 * F2_XH4);
      row = R + j / (2 * F2_XH4);
      c4 = side < F2_XH4 ? side : F2_XH4 + F2_EX4 + (side - F2_XH4);
    }
    const int gy = yt - 2 * R + row, gx = xt - 2 * F2_XH + 4 * c4;
    hl = row * F2_UROW4 + c4;
    if (gy >= 0 && gy < ny && gx >= 0 && gx < nx) vo_h = (unsigned)(gy * a.g.pitch + gx) * 4u;
  }
  const unsigned vo = colok ? (unsigned)col * 4u : kOOB;
  const int pbytes = (int)(plane * 4);
  auto rs = [&](const void* base, const int zz, const bool valid) {
    const int zcl = min(max(zz, 0), nz - 1);
    return plane_rsrc(base, (int64_t)zcl * plane * 4, valid && zz >= 0 && zz < nz ? pbytes : 0);
  };
  auto ld = [&](const void* base, const int zz, const bool valid, const unsigned off) {
    return Store<ST_F32>::template ldb<false>(rs(base, zz, valid), off);
  };
  const auto W = [](const f4v& r) { return Store<ST_F32>::widen(r); };

  const float4 bxv = (colok) ? ld4(a.bx + x0) : zero4;
  const float byv = (act && y >= 0 && y < ny) ? a.by[y] : 0.f;

  // Prologue: u^n queue for za0 (planes za0-R .. za0+R), the LDS copy of plane za0,
  // prev and c2 at za0, c2 at the first stage-B plane.
  float4 q[2 * R + 1], vq[2 * R + 1];
  f4v up, cc;
  {
    f4v qr[2 * R + 1];
#pragma unroll
    for (int s = 0; s <= 2 * R; ++s) qr[s] = ld(a.cur, za0 - R + s, true, vo);
    const f4v hr0 = ld(a.cur, za0, true, vo_h);
    up = ld(a.prev, za0, true, vo);
    cc = ld(a.c2, za0, true, vo);
#pragma unroll
    for (int s = 0; s <= 2 * R; ++s) q[s] = W(qr[s]);
    if (act) ulds[0][(ey + R) * F2_UROW4 + ex + F2_XH4] = q[R];
    if (hl >= 0) ulds[0][hl] = W(hr0);
  }
  {
    // ring items of planes za0+1 .. za0+R into their slots
    f4v hr[R];
#pragma unroll
    for (int j = 0; j < R; ++j) hr[j] = ld(a.cur, za0 + 1 + j, true, vo_h);
    if (hl >= 0) {
#pragma unroll
      for (int j = 0; j < R; ++j) ringbuf[slot(za0 + 1 + j)][tid] = W(hr[j]);
    }
  }
#pragma unroll
  for (int s = 0; s <= 2 * R; ++s) vq[s] = zero4;
  if (act) inj[tid] = zero4;
  for (int i = tid; i < za1 - za0; i += NTH) {
    const int zz = za0 + i;
    bzs[i] = (zz >= 0 && zz < nz) ? a.bz[zz] : 0.f;
  }
  __syncthreads();

  // Injection entries (sorted by plane) of the extended tile (stage A) and of the
  // K one-step tiles that make up the tile (stage B, from the one-step tables);
  // eza / ezb[k] hold the plane of the next group of each, so the per-plane tests
  // need no load.
  int ea = 0, ea_end = 0, eza = INT_MAX, ega = 0;  // ega: end of the group at eza
  int eb[K], eb_end[K], ezb[K], egb[K];
  if (f.etile_beg != nullptr) {
    ea = f.etile_beg[t];
    ea_end = f.etile_beg[t + 1];
    if (ea < ea_end) {
      eza = f.eent[ea].z;
      ega = f.eent[ea].grp_end;
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    eb[k] = 0;
    eb_end[k] = 0;
    ezb[k] = INT_MAX;
    egb[k] = 0;
    const int ty1 = K * ty_t + k;
    if (a.tile_beg != nullptr && ty1 < f.ntile_y1) {  // column tables of xy tile xy1
      const int xy1 = ty1 * a.ntile_x + tx_t;
      eb[k] = a.tile_beg[xy1 * nz + z0];
      eb_end[k] = a.tile_beg[xy1 * nz + z1];
      if (eb[k] < eb_end[k]) {
        ezb[k] = a.ent[eb[k]].z;
        egb[k] = a.ent[eb[k]].grp_end;
      }
    }
  }

  // Laplacian of four consecutive points from a z-queue and an LDS plane (row
  // stride LR4 float4, centre at crow), accumulated in the single-step kernel's
  // order.
  auto laplacian = [&](const float4* Q, const float4* L, const int crow, const int LR4,
                       float lap[4]) {
    float xv[4 + 2 * F2_XH];
#pragma unroll
    for (int k = -F2_XH4; k <= F2_XH4; ++k) {
      const float4 v = k == 0 ? Q[R] : L[crow + k];
      xv[F2_XH + 4 * k + 0] = v.x; xv[F2_XH + 4 * k + 1] = v.y;
      xv[F2_XH + 4 * k + 2] = v.z; xv[F2_XH + 4 * k + 3] = v.w;
    }
#pragma unroll
    for (int p = 0; p < 4; ++p) lap[p] = a.wc * comp(Q[R], p);
#pragma unroll
    for (int s = R; s >= 2; --s) {
      const float4 ym = L[crow - s * LR4];
      const float4 yp = L[crow + s * LR4];
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        lap[p] = fmaf(a.wx[s], xv[F2_XH + p - s] + xv[F2_XH + p + s], lap[p]);
        lap[p] = fmaf(a.wy[s], comp(ym, p) + comp(yp, p), lap[p]);
        lap[p] = fmaf(a.wz[s], comp(Q[R - s], p) + comp(Q[R + s], p), lap[p]);
      }
    }
    {
      const float4 ym = L[crow - LR4];
      const float4 yp = L[crow + LR4];
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const float u2 = 2.f * comp(Q[R], p);
        lap[p] = fmaf(a.wx[1], (xv[F2_XH + p - 1] + xv[F2_XH + p + 1]) - u2, lap[p]);
        lap[p] = fmaf(a.wy[1], (comp(ym, p) + comp(yp, p)) - u2, lap[p]);
        lap[p] = fmaf(a.wz[1], (comp(Q[R - 1], p) + comp(Q[R + 1], p)) - u2, lap[p]);
      }
    }
  };
  // Damped leapfrog update in the single-step kernel's form:
  //   out = u + ((1-b)(u - prev) + c2 (L u + inj)) / (1+b)
  auto update = [&](const float4& u4, const float4& p4, const float4& c4, const float bzv,
                    const float lap[4]) {
    float4 o;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const float b = (comp(bxv, p) + byv) + bzv;
      const float u = comp(u4, p);
      const float d = u - comp(p4, p);
      const float num = fmaf(comp(c4, p), lap[p], fmaf(-b, d, d));
      const float inv = __builtin_amdgcn_rcpf(1.f + b);
      set_comp(o, p, fmaf(num, inv, u));
    }
    return o;
  };
  // Scatter one plane's injection entries [e, eg) into inj and return the
  // thread's four values at float4 slot `slot` (cleared after); advance e to the
  // next group, with its plane ez and end eg.
  auto inject = [&](const InjEntry* ent, const int* cidx, const float* cw, const float* row,
                    int& e, const int e_end, int& ez, int& eg, const bool mine,
                    const int slot) {
    for (int i = e + tid; i < eg; i += NTH) {
      const InjEntry en = ent[i];
      float s = 0.f;
      if (en.tidx >= 0) {  // single term, carried in the entry
        s = fmaf(en.w, row[en.tidx], 0.f);
      } else {
        for (int c = en.csr_beg; c < en.csr_end; ++c) s = fmaf(cw[c], row[cidx[c]], s);
      }
      reinterpret_cast<float*>(inj)[en.local] = s;
    }
    __syncthreads();
    float4 iv = zero4;
    if (mine) {
      iv = inj[slot];
      inj[slot] = zero4;
    }
    e = eg;
    ez = INT_MAX;
    if (e < e_end) {
      ez = ent[e].z;
      eg = ent[e].grp_end;
    }
    return iv;
  };

  const int crowA = (ey + R) * F2_UROW4 + ex + F2_XH4;
  const int crowB = ey * F2_EX4 + ex;
  // tile-layout slot of an inner thread (TX floats per row); 0 for the others, which
  // read a valid slot but store nothing
  const int slotB = inner ? (ey - R) * NTX + (ex - F2_XH4) : 0;

  auto plane_step = [&](const int za, const int buf) {
    const int zb = za - R;
    const bool moreA = za + 1 < za1;
    // Loads for the next plane.
    const f4v nq = ld(a.cur, za + 1 + R, moreA, vo);
    const f4v nh = ld(a.cur, za + 1 + R, za + 1 + R < za1, vo_h);  // ring, R planes ahead
    const f4v nup = ld(a.prev, za + 1, moreA, vo);
    const f4v ncc = ld(a.c2, za + 1, moreA, vo);

    // Stage A: v = u^{n+1} at plane za on E.
    float lap[4];
    laplacian(q, ulds[buf], crowA, F2_UROW4, lap);
    if (za == eza) {
      const float4 iv =
          inject(f.eent, f.ecsr_idx, f.ecsr_w, f.etrace_row, ea, ea_end, eza, ega, act, tid);
      lap[0] += iv.x; lap[1] += iv.y; lap[2] += iv.z; lap[3] += iv.w;
    }
    const float4 ccv = W(cc);
    if (inner) cring[slot(za)][slotB] = ccv;  // c2 at za for stage B, R planes later
    const float4 v = update(q[R], W(up), ccv, bzs[za - za0], lap);
    // stores on every path: planes outside the chunk get a resource with no
    // records, lanes outside the tile or the grid an out-of-range offset
    Store<ST_F32>::template stb<NT>(rs(a.out, za, za >= z0 && za < z1), inner ? vo : kOOB, v);
#pragma unroll
    for (int s = 0; s < 2 * R; ++s) vq[s] = vq[s + 1];
    vq[2 * R] = v;
    if (act) vlds[crowB] = vq[R];
    __syncthreads();

    // Stage B: u^{n+2} at plane zb on the tile.
    const bool doB = zb >= z0 && zb < z1;
    float4 w = zero4;
    if (doB) {
      float lapb[4] = {0.f, 0.f, 0.f, 0.f};
      if (inner) laplacian(vq, vlds, crowB, F2_EX4, lapb);
      bool injb = false;
#pragma unroll
      for (int k = 0; k < K; ++k) injb = injb || zb == ezb[k];
      if (injb) {  // uniform
        // scatter the plane's groups of every sub-tile (sub-tile k holds tile rows
        // k*TY .. k*TY+TY-1, so its local indices are offset by k*TY*TX)
#pragma unroll
        for (int k = 0; k < K; ++k) {
          if (zb != ezb[k]) continue;
          for (int i = eb[k] + tid; i < egb[k]; i += NTH) {
            const InjEntry en = a.ent[i];
            float s = 0.f;
            if (en.tidx >= 0) {
              s = fmaf(en.w, a.trace_row[en.tidx], 0.f);
            } else {
              for (int c = en.csr_beg; c < en.csr_end; ++c)
                s = fmaf(a.csr_w[c], a.trace_row[a.csr_idx[c]], s);
            }
            reinterpret_cast<float*>(inj)[k * TY * TX + en.local] = s;
          }
        }
        __syncthreads();
        if (inner) {
          const float4 iv = inj[slotB];
          inj[slotB] = zero4;
          lapb[0] += iv.x; lapb[1] += iv.y; lapb[2] += iv.z; lapb[3] += iv.w;
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
          if (zb != ezb[k]) continue;
          eb[k] = egb[k];
          ezb[k] = INT_MAX;
          if (eb[k] < eb_end[k]) {
            ezb[k] = a.ent[eb[k]].z;
            egb[k] = a.ent[eb[k]].grp_end;
          }
        }
      }
      w = update(vq[R], q[0], cring[slot(zb)][slotB], bzs[max(zb - za0, 0)], lapb);
    }
    Store<ST_F32>::template stb<NT>(rs(f.out2, zb, doB), inner ? vo : kOOB, w);

    // Stage plane za+1 of u^n into the other LDS buffer.
    if (moreA) {
      if (act) ulds[buf ^ 1][crowA] = q[R + 1];
      if (hl >= 0) ulds[buf ^ 1][hl] = ringbuf[slot(za + 1)][tid];
    }
    if (hl >= 0 && za + 1 + R < za1) ringbuf[slot(za + 1 + R)][tid] = W(nh);
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 2 * R; ++s) q[s] = q[s + 1];
    q[2 * R] = W(nq);
    up = nup;
    cc = ncc;
  };
  int za = za0;
  for (; za + 1 < za1; za += 2) {
    plane_step(za, 0);
    plane_step(za + 1, 1);
  }
  if (za < za1) plane_step(za, 0);
}

// Occupancy per radius: at r = 3 the kernel needs 129 VGPRs unconstrained and fits 128
// without spilling when asked for 4 waves per SIMD, which lets two 512-thread
// workgroups share a CU (LDS 58.5 KB each): measured on MI355X, 100 steps, SO6:
// 512^3 322 -> 382 Gpt/s, 448^3 295 -> 349 (one-step kernel 346 / 332). At r = 4
// (158 VGPRs) the same request spills 72 bytes per lane and runs at 170-215 Gpt/s.
constexpr int f2_waves_per_eu(int r) { return r == 3 ? 4 : 1; }
template <int R, bool NT>
__global__ void __launch_bounds__(f2_threads(R))
__attribute__((amdgpu_waves_per_eu(f2_waves_per_eu(R))))
fused2_kernel(const Fused2Args f) {
  const StepArgs& a = f.a;
  const int bid = blockIdx.x;
  if (bid >= a.nstencil_blocks) {
    const int r = (bid - a.nstencil_blocks) * f2_threads(R) + threadIdx.x;
    if (r < a.nsamp) {
      if (a.samp_out != nullptr)
        a.samp_out[r] = sample_point<ST_F32>(a.cur, 1.f, a.samp_idx, a.samp_w, r);
      if (f.samp_out2 != nullptr)
        f.samp_out2[r] = sample_point<ST_F32>(a.prev, 1.f, a.samp_idx, a.samp_w, r);
    }
    return;
  }
  const int t = a.xcd_remap ? remap_tile(bid, a.nstencil_blocks) : bid;
  fused2_tile<R, NT>(f, t);
}

template <int R>
hipError_t launch_fused2_r(const Fused2Args& f, bool nt, hipStream_t s) {
  constexpr int nth = f2_threads(R);
  const int nsb = (f.a.nsamp + nth - 1) / nth;
  const dim3 grid(f.a.nstencil_blocks + (f.a.nsamp > 0 ? nsb : 0)), block(nth);
  if (nt)
    hipLaunchKernelGGL((fused2_kernel<R, true>), grid, block, 0, s, f);
  else
    hipLaunchKernelGGL((fused2_kernel<R, false>), grid, block, 0, s, f);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_fused2(const Fused2Args& f, int r, bool nt, hipStream_t s) {
  switch (r) {
    case 1: return launch_fused2_r<1>(f, nt, s);
    case 2: return launch_fused2_r<2>(f, nt, s);
    case 3: return launch_fused2_r<3>(f, nt, s);
    case 4: return launch_fused2_r<4>(f, nt, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace wave
