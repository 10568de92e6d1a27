/*
 * wave.h -- C ABI of the MI355X (gfx950) acoustic finite-difference solver.
 *
 * The solver integrates the isotropic acoustic wave equation with a source term
 * and zero initial state (paper Section 2.1, Eq. (1)), m = 1/v^2, extended by the
 * damping term of the paper's damped SO2 propagation listing (Section 2.1):
 *
 *     m u_tt + m gamma u_t - lap(u) = q_s .
 *
 * Discretisation (second-order leapfrog in time, the listing's form divided by
 * its denominator r0):
 *
 *     u^{n+1} = ( 2u^n - (1-b) u^{n-1} + dt^2 v^2 ( L_h u^n + P^T s^n ) ) / (1+b)
 *     b = dt gamma / 2,     d^n = R u^{n+1}
 *
 * L_h: star Laplacian of even space order SO = 2r (2..24), weights of the centred
 * second-derivative stencil, values outside the grid are zero (an r-wide zero
 * halo). gamma = gamma_x(i) + gamma_y(j) + gamma_z(k); on a face of width nbl the
 * d-th point from the outside (d = 0..nbl-1) has p = (nbl-d)/nbl and
 * gamma = gmax (p - sin(2 pi p)/(2 pi)), gmax = 3 vmax ln(1000) / (2 nbl h).
 * P / R: trilinear injection / interpolation at off-grid points (exact on
 * grid points). Source sample s^n (t = n dt) drives the equation that produces
 * u^{n+1}; receivers record d^n = R u^{n+1}, n = 0..nt-1.
 *
 * Backward propagation (paper's conclusion, future work there) is the exact
 * transpose of the forward map s -> d; the gradient is that of a loss L(d) given
 * dL/dd, with respect to velocity (and to the wavelet).
 *
 * Conventions for every entry point:
 *  - Arrays are x-fastest: element (i,j,k) of an nx*ny*nz field is at
 *    (k*ny + j)*nx + i; grid point (i,j,k) sits at (i*hx, j*hy, k*hz) metres.
 *  - Pointers named *_h are host memory, read only during the call. All other
 *    array pointers are device memory owned by the caller.
 *  - The caller owns the workspace (device, 256-byte aligned, at least
 *    wave_workspace_bytes()). Solver calls allocate no device memory. Each call
 *    builds its source/receiver tables on the host in a page-locked staging
 *    buffer taken from a process-wide pool (hipHostMalloc on first need, kept
 *    for the life of the process; sized like the workspace's table region, at
 *    most 384 B per source or receiver point plus 4 B per 64x16 tile and plane)
 *    and uploads them asynchronously on `hip_stream`; the buffer returns to the
 *    pool when the upload has run.
 *  - Work is enqueued on `hip_stream` (a hipStream_t, NULL = the default
 *    stream) and the call returns; outputs are valid after that stream
 *    synchronises. Calls on distinct (workspace, stream) pairs may run
 *    concurrently; calls sharing a workspace must be ordered on one stream.
 *  - Validation is synchronous and happens before anything is enqueued; on
 *    error nothing is enqueued and no output is touched. No exception crosses
 *    the ABI.
 */
#ifndef WAVE_H
#define WAVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes (int return values). */
#define WAVE_OK 0
#define WAVE_EINVAL (-1)  /* bad argument: sizes, space order, null pointer, point off grid */
#define WAVE_ECFL (-2)    /* dt above the stability limit wave_cfl_dt_max()                 */
#define WAVE_ENOMEM (-3)  /* workspace smaller than wave_workspace_bytes()                  */
#define WAVE_EDEVICE (-4) /* a HIP runtime call failed                                      */
#define WAVE_EBUSY (-5)   /* serving engine: request exceeds the memory budget              */
#define WAVE_EAGAIN (-6)  /* serving engine: result not ready yet                           */
#define WAVE_ELIMIT (-7)  /* problem larger than the static scratch of wave_forward_noalloc */

/* Wavefield storage formats (arithmetic is FP32 in every format). The 16-bit
 * formats store each level as value * 2^e with a power-of-two scale e chosen per
 * level on the device from the previous level's maximum (with headroom), and
 * apply only to wave_forward. WAVE_STORE_DIFF (or-ed onto F16 / BF16) stores
 * u^n and the difference u^n - u^{n-1} instead of u^n and u^{n-1}: 12 instead
 * of 10 bytes moved per point and step, much smaller rounding error. */
#define WAVE_STORE_F32 0
#define WAVE_STORE_F16 1
#define WAVE_STORE_BF16 2
#define WAVE_STORE_DIFF 16
/* WAVE_STORE_BF16 without WAVE_STORE_DIFF is diagnostic only: BF16 keeps 8 bits of
 * mantissa and storing two rounded levels turns each rounding into a velocity error,
 * so over long runs the error exceeds the signal (measured rel-L2 above 1 against
 * the FP64 oracle after 1000 steps of a 160^3 SO8 case). It is accepted so that
 * its error can be measured and stated. */

/* Execution-path flags (wave_grid.path). They choose kernels, launch shapes and
 * cache hints, never the arithmetic: every path evaluates each point's update with
 * the same expression (one-step and two-step kernels agree to FP32 contraction
 * differences, every other choice is bitwise neutral). 0 lets the library choose. */
#define WAVE_PATH_ONE_STEP 1  /* never the two-step kernel                            */
#define WAVE_PATH_TWO_STEP 2  /* the two-step kernel wherever it applies (FP32 storage,
                                 SO <= 8, no checkpoints, z-chunks of >= SO planes)    */
#define WAVE_PATH_STREAM 4    /* non-temporal hints on the streamed arrays             */
#define WAVE_PATH_CACHED 8    /* no non-temporal hints                                 */
#define WAVE_PATH_LINEAR 16   /* workgroups in plain tile order (no XCD-aware order)   */
/* The time loop's launches are recorded per call. By default a call whose launches
 * equal (same arguments, same device) those of an earlier call is captured into a
 * HIP graph, kept in a cache of the library (16 graphs, least recently used
 * replaced; the HIP runtime holds their memory), and replayed on hip_stream from
 * then on. The replay runs the same kernels with the same arguments. */
#define WAVE_PATH_GRAPH 32    /* capture and replay from the first call               */
#define WAVE_PATH_DIRECT 64   /* always launch directly (no graph)                     */
/* Workgroup tile of the one-step kernel: 64 x 16 points, or 64 x 32 at SO 2, 4, 6, 8,
 * 16 and 20 (the orders that have it). By default the taller tile is taken at those
 * orders with FP32 storage when its workgroups fill the GPU's 256 CUs evenly (a
 * multiple of 256). */
#define WAVE_PATH_TILE16 128  /* 64 x 16 tiles                                         */
#define WAVE_PATH_TILE32 256  /* 64 x 32 tiles at SO 2, 4, 6, 8, 16 and 20             */

/* Workspace modes for wave_workspace_bytes(). */
#define WAVE_MODE_FORWARD 0
#define WAVE_MODE_ADJOINT 1
#define WAVE_MODE_GRADIENT 2

typedef struct {
  int32_t nx, ny, nz;  /* grid points per axis, sponge included; with the row pitch
                          px = nx rounded up to a multiple of 32, px*ny*nz < 2^31 and
                          px*ny*4 < 2^31 (else WAVE_EINVAL)                          */
  double hx, hy, hz;   /* spacing [m]                                                 */
  int32_t so;          /* space order, even, 2..24 (stencil radius so/2)              */
  double dt;           /* time step [s], at most wave_cfl_dt_max(so, vmax, hx, hy, hz) */
  int32_t nt;          /* number of time steps (>= 0)                                 */
  int32_t nbl[6];      /* sponge width per face: x-, x+, y-, y+, z-, z+ (0 = none)    */
  double vmax;         /* velocity bound [m/s]: max(vel) <= vmax is the caller's
                          promise; sets the sponge strength and the dt check         */
  int32_t storage;     /* WAVE_STORE_F32 | WAVE_STORE_F16 | WAVE_STORE_BF16, the last two
                          optionally | WAVE_STORE_DIFF                               */
  int32_t path;        /* WAVE_PATH_* flags (0 = chosen by the library); ONE_STEP with
                          TWO_STEP, STREAM with CACHED, GRAPH with DIRECT, TILE16 with
                          TILE32, or unknown bits: WAVE_EINVAL                       */
  int32_t zchunk;      /* planes per z-chunk of the stencil sweep, 1..256 (0 = chosen
                          by the library: about 512 workgroups; 64 planes for the
                          two-step kernel, 32-128 at SO8); results do not depend on it */
} wave_grid;

/* Largest stable dt of the leapfrog scheme (von Neumann):
 * 2 / (vmax sqrt(S (hx^-2 + hy^-2 + hz^-2))), S = |w0| + 2 sum_q |w_q| the
 * stencil's symbol at the Nyquist wavenumber. Returns a negative value for an
 * invalid space order or non-positive arguments. */
double wave_cfl_dt_max(int so, double vmax, double hx, double hy, double hz);

/* Device workspace bytes needed by one call of the given mode for this grid,
 * number of sources and receivers, and checkpoint interval (mode GRADIENT
 * only; <= 0 means the interval used internally, 50). Returns 0 for an
 * invalid grid. */
size_t wave_workspace_bytes(const wave_grid* g, int nsrc, int nrec, int mode, int ckpt_every);

/* Bytes of the checkpoint buffer that wave_forward fills and wave_gradient
 * reads: ceil(nt / ckpt_every) pairs (u^{kC}, u^{kC-1}) of nx*ny*nz floats.
 * Returns 0 when ckpt_every <= 0 or the grid is invalid. */
size_t wave_checkpoint_bytes(const wave_grid* g, int ckpt_every);

/* Forward propagation (Eq. (1) with damping, source injection and receiver
 * sampling).
 *   vel       [nz][ny][nx] velocity m/s (device, FP32)
 *   wavelet   [nt][nsrc] source samples (device; may be NULL when nsrc == 0)
 *   src_xyz_h [nsrc][3] source positions in metres (host FP64)
 *   rec_xyz_h [nrec][3] receiver positions in metres (host FP64)
 *   rec_out   [nt][nrec] receives d^n (device; may be NULL when nrec == 0)
 *   u0, um1   optional initial levels u^0, u^{-1} [nz][ny][nx] (NULL = 0)
 *   u_final   optional [nz][ny][nx] receives u^{nt}
 *   ckpt      optional checkpoint buffer (wave_checkpoint_bytes) receiving
 *             (u^{kC}, u^{kC-1}) for k = 0..ceil(nt/C)-1, C = ckpt_every
 *             (FP32 storage only)
 * With 16-bit storage the levels are rounded to the storage format after every
 * step (the error against FP32 storage is a property of the format; the FP32
 * arithmetic is unchanged).
 * Execution: one launch per step, or, for FP32 storage without checkpoints on
 * large grids (SO2 from 3e7, SO4 from 6e7, SO6 from 8e7 points), two fused steps
 * per launch (temporal blocking); both evaluate every point's update with the same
 * expression. For FP32 storage at SO <= 8 the forward workspace holds two extra
 * levels for that kernel. g->path and g->zchunk select among the paths; nothing
 * else (no environment variable) does.
 * Returns WAVE_OK or a negative status. */
int wave_forward(const wave_grid* g, const float* vel, const float* wavelet,
                 const double* src_xyz_h, int nsrc, const double* rec_xyz_h, int nrec,
                 float* rec_out, const float* u0, const float* um1, float* u_final,
                 float* ckpt, int ckpt_every, void* workspace, size_t ws_bytes,
                 void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): wave_forward without a
 * workspace argument. Its workspace is a static device array of the library
 * (wave_noalloc_limit_bytes(), 64 MiB, one per device, held until the process
 * ends), so the call makes no hipMalloc/hipFree or other allocating HIP call:
 * its tables are staged in ordinary host heap memory and uploaded with
 * asynchronous copies on hip_stream. The caller still passes inputs and outputs.
 * Runs on the current device, one step per launch (the one-step layout of
 * wave_forward: v^2 dt^2, the levels and the tables must fit the array, else
 * WAVE_ELIMIT before anything is enqueued; FP32 storage fits grids up to about
 * 5.5e6 points, e.g. 160^3). No checkpoints; WAVE_PATH_TWO_STEP gives
 * WAVE_EINVAL. Every call on a device shares that device's array and leaves its
 * contents behind (each call re-initialises everything it reads): calls that
 * overlap on one device race, so order them on one stream. Results are bitwise
 * those of wave_forward with WAVE_PATH_ONE_STEP. */
int wave_forward_noalloc(const wave_grid* g, const float* vel, const float* wavelet,
                         const double* src_xyz_h, int nsrc, const double* rec_xyz_h, int nrec,
                         float* rec_out, const float* u0, const float* um1, float* u_final,
                         void* hip_stream);
/* Size in bytes of the static device array behind wave_forward_noalloc. */
size_t wave_noalloc_limit_bytes(void);

/* Ablation of the paper's basic-versus-aggressive experiment (Section 4, Tables 2
 * and 3): the forward solve of wave_forward with the update evaluated in the
 * unfactorised form of the paper's SO2 listing (Section 2.1), generalised to the
 * star stencil of order SO: every term with its own coefficient and its own
 * division by r0 = dt m + dt^2 damp / 2, m = 1/v^2, damp = m gamma. Same
 * mathematics as wave_forward, more FP32 roundings and one division per term.
 * FP32 storage, SO 8, 12, 16 or 24, no checkpoints (else WAVE_EINVAL); one launch
 * per step; workspace as for wave_forward (WAVE_MODE_FORWARD). Arguments as for
 * wave_forward. */
int wave_forward_unfactorised(const wave_grid* g, const float* vel, const float* wavelet,
                              const double* src_xyz_h, int nsrc, const double* rec_xyz_h,
                              int nrec, float* rec_out, const float* u0, const float* um1,
                              float* u_final, void* workspace, size_t ws_bytes,
                              void* hip_stream);

/* Backward propagation: the exact transpose of wave_forward's map from
 * wavelet to receiver data (zero initial state). Runs
 *   lambda^n = (2 l^{n+1} - (1-b) l^{n+2} + dt^2 v^2 (L_h l^{n+1} + R^T d^n)) / (1+b)
 * for n = nt-1..0 from lambda^{nt} = lambda^{nt+1} = 0 and samples
 * src_out^n = P lambda^n. FP32 storage only.
 *   rec_data  [nt][nrec] (device), src_out [nt][nsrc] (device, may be NULL
 *   when nsrc == 0), lam_final optional [nz][ny][nx] receives lambda^0. */
int wave_adjoint(const wave_grid* g, const float* vel, const float* rec_data,
                 const double* rec_xyz_h, int nrec, const double* src_xyz_h, int nsrc,
                 float* src_out, float* lam_final, void* workspace, size_t ws_bytes,
                 void* hip_stream);

/* Gradient of a loss L(d) of the forward receiver data d, given
 * rec_grad = dL/dd [nt][nrec] (for the least-squares misfit: d - d_obs).
 * With lambda from wave_adjoint driven by rec_grad,
 *   dL/dm = -sum_n lambda^n ( (u^{n+1} - 2u^n + u^{n-1})/dt^2
 *                             + gamma (u^{n+1} - u^{n-1})/(2 dt) ),
 *   grad_vel = dL/dv = -2 v^-3 dL/dm     (gamma held fixed),
 *   grad_wavelet^n = dL/ds^n = P lambda^n (optional, may be NULL).
 * Forward levels come from ckpt (filled by wave_forward with the same
 * ckpt_every) or, when ckpt is NULL, from an internal forward pass that keeps
 * checkpoints in the workspace; each segment of ckpt_every steps is recomputed
 * before its adjoint steps. FP32 storage only. */
int wave_gradient(const wave_grid* g, const float* vel, const float* wavelet,
                  const double* src_xyz_h, int nsrc, const double* rec_xyz_h, int nrec,
                  const float* rec_grad, const float* ckpt, int ckpt_every,
                  float* grad_vel, float* grad_wavelet, void* workspace, size_t ws_bytes,
                  void* hip_stream);

/* Reverse-time-migration image (the imaging condition on the forward and the
 * backward fields; the paper names RTM among the seismic inversion workloads
 * in its introduction): the zero-lag cross-correlation
 *   image = sum_{n=1..nt} u^n lambda^n
 * of the forward field u (wavelet at the sources, zero initial state) with the
 * backward field lambda of wave_adjoint driven by rec_data [nt][nrec] at the
 * receivers (lambda^{nt} = 0). Forward levels come from ckpt / ckpt_every as in
 * wave_gradient (NULL: internal forward pass); workspace as for
 * WAVE_MODE_GRADIENT. image [nz][ny][nx] (device). FP32 storage only. */
int wave_rtm(const wave_grid* g, const float* vel, const float* wavelet,
             const double* src_xyz_h, int nsrc, const double* rec_xyz_h, int nrec,
             const float* rec_data, const float* ckpt, int ckpt_every, float* image,
             void* workspace, size_t ws_bytes, void* hip_stream);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of independent forward shots on one GPU.
 *
 * An engine owns a device memory pool of hbm_budget_bytes, allocated once by
 * wave_engine_create, and a worker thread. Submitted requests are admitted
 * first-come first-served (later requests that fit may overtake one that does
 * not) whenever a slot and pool space are free; resident shots of each space
 * order advance together, one batched launch per step, replayed as captured
 * HIP graphs while other requests upload. A shot's result is bitwise identical
 * to the same request alone on the engine and to wave_forward of the request.
 * FP32 storage only. Each request is the forward problem of wave_forward (zero
 * initial state). */
typedef struct {
  wave_grid grid;
  const float* vel_h;        /* [nz][ny][nx] m/s (host; copied at submit)           */
  const float* wavelet_h;    /* [nt][nsrc] (host; copied at submit)                 */
  const double* src_xyz_h;   /* [nsrc][3] metres (host; copied at submit)           */
  int32_t nsrc;
  const double* rec_xyz_h;   /* [nrec][3] metres (host; copied at submit)           */
  int32_t nrec;
  float* rec_out_h;          /* [nt][nrec] host buffer filled by the engine when the
                                request completes; must stay valid until then      */
} wave_request;

typedef struct {
  int32_t status;            /* WAVE_OK done, WAVE_EAGAIN queued/running, else error */
  double t_submit, t_admit, t_done;  /* engine clock [s] (steady clock)              */
} wave_result;

typedef struct {
  uint64_t submitted, admitted, completed, rejected, queued, resident;
  double p50_latency_s, p99_latency_s, mean_latency_s, max_latency_s;  /* submit->done */
  double total_gpt;          /* grid-point updates of completed shots / 1e9          */
  double busy_s;             /* time with at least one shot resident                 */
  double span_s;             /* first submit to last completion                      */
  uint64_t graph_builds, replays, max_resident;
  size_t max_pool_bytes;     /* high-water mark of pool bytes in use                 */
} wave_stats;

/* Create an engine with a device pool of hbm_budget_bytes (allocated here, on the
 * current device) and at most max_slots resident shots. Resident shots advance in
 * groups of one space order whose per-step arrays fit the Infinity Cache together
 * (224 MB unless wave_engine_set_group_bytes says otherwise), several steps of a
 * group back to back; a shot's results do not depend on the grouping or on the
 * other shots. A request's zchunk fixes its z-chunk length in the engine; 0 lets the
 * engine choose per group (the longest of 32, 24, ..., 1 planes that gives the
 * group 512 workgroups). */
int wave_engine_create(size_t hbm_budget_bytes, int max_slots, void** engine);
/* Per-step bytes (two FP32 levels and v^2 dt^2) of the shots stepped together in
 * one group; 0 restores the default. Applies from the next change of the set of
 * resident shots. */
int wave_engine_set_group_bytes(void* engine, size_t bytes);
/* Queue a request; its inputs are copied. WAVE_EBUSY if it can never fit the
 * budget; validation errors as for wave_forward. *id identifies it. */
int wave_engine_submit(void* engine, const wave_request* req, uint64_t* id);
/* Non-blocking: the request's status (WAVE_EAGAIN until done), times in *res. */
int wave_engine_poll(void* engine, uint64_t id, wave_result* res);
/* Counters and latency percentiles (nearest rank) over completed requests. */
int wave_engine_stats(void* engine, wave_stats* st);
/* Block until nothing is queued or resident, or timeout_s passes (WAVE_EAGAIN). */
int wave_engine_drain(void* engine, double timeout_s);
/* Pool bytes one request of this shape occupies while resident (0 if invalid). */
size_t wave_engine_request_bytes(const wave_grid* g, int nsrc, int nrec);
/* Stop the worker, wait for the device, free the pool. */
void wave_engine_destroy(void* engine);

/* Human-readable name of a status code (static string). */
const char* wave_status_string(int status);

/* Library version string (static). */
const char* wave_version(void);

#ifdef __cplusplus
}
#endif

#endif /* WAVE_H */
