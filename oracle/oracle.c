/*
 * oracle.c -- plain FP64 CPU oracle for the damped acoustic leapfrog scheme.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark load this library. It shares no source, header, table or
 * helper with the HIP library: every coefficient below is computed here, from the
 * mathematics, in double precision, in the natural loop order.
 *
 * What it computes (paper: Section 2.1, Eq. (1) and the damped SO2 update printed
 * as the Devito-generated C code in Section 2.1; future-work paragraph of the
 * conclusion for receivers and backward propagation):
 *
 *   m u_tt + m*gamma*u_t - lap(u) = q_s,   m = 1/v^2,  u = u_t = 0 at t = 0
 *
 * discretised as
 *
 *   u^{n+1} = ( 2u^n - (1-b) u^{n-1} + dt^2 v^2 (L_h u^n + P^T s^n) ) / (1+b),
 *   b = dt*gamma/2,   d^n = R u^{n+1},
 *
 * with L_h the star Laplacian of even space order SO = 2r (Fornberg weights,
 * zero values outside the grid), gamma the sum of three 1D sponge profiles, P / R
 * trilinear injection / interpolation. The adjoint runs the same update backwards
 * in time with R^T d^n injected and P sampled; the gradient with respect to
 * m = v^-2 is  g_m = -sum_n lambda^n (u^{n+1}-2u^n+u^{n-1})/dt^2
 *                          + gamma (u^{n+1}-u^{n-1})/(2dt) ),
 * chained to velocity as g_v = -2 v^-3 g_m.
 *
 * A periodic halo (oracle-only test mode) replaces the zero halo so that the
 * discrete standing wave is an exact eigenvector of L_h.
 *
 * Layout: index (k*ny + j)*nx + i, x fastest; grid point (i,j,k) sits at
 * (i*hx, j*hy, k*hz) metres.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXR 16

typedef struct {
  int64_t nx, ny, nz;
  double hx, hy, hz;
  int64_t so;        /* even space order, r = so/2                       */
  double dt;
  int64_t nt;
  int64_t nbl[6];    /* sponge widths: x-, x+, y-, y+, z-, z+           */
  double vmax;       /* reference velocity of the sponge strength       */
  int64_t periodic;  /* 1: periodic halo (test mode), 0: zero halo      */
} ogrid;

/* ------------------------------------------------------------------------ */
/* Finite-difference weights: Fornberg's recursion (Math. Comp. 51, 1988) for
 * the second derivative at 0 on the nodes 0, 1, -1, 2, -2, ..., r, -r.
 * Output w[0..r]: w[0] centre, w[q] the (symmetric) weight of nodes +-q.     */
int oracle_fd_weights(int64_t so, double *w) {
  if (so < 2 || so % 2 || so / 2 > OR_MAXR) return -1;
  int r = (int)(so / 2), N = 2 * r; /* nodes 0..N */
  double x[2 * OR_MAXR + 1];
  x[0] = 0.0;
  for (int q = 1; q <= r; ++q) { x[2 * q - 1] = q; x[2 * q] = -q; }
  const int M = 2; /* highest derivative order */
  double c[2 * OR_MAXR + 1][3];
  memset(c, 0, sizeof c);
  double c1 = 1.0, c4 = x[0];
  c[0][0] = 1.0;
  for (int i = 1; i <= N; ++i) {
    int mn = i < M ? i : M;
    double c2 = 1.0, c5 = c4;
    c4 = x[i];
    for (int j = 0; j < i; ++j) {
      double c3 = x[i] - x[j];
      c2 *= c3;
      if (j == i - 1) {
        for (int k = mn; k >= 1; --k)
          c[i][k] = c1 * (k * c[i - 1][k - 1] - c5 * c[i - 1][k]) / c2;
        c[i][0] = -c1 * c5 * c[i - 1][0] / c2;
      }
      for (int k = mn; k >= 1; --k) c[j][k] = (c4 * c[j][k] - k * c[j][k - 1]) / c3;
      c[j][0] = c4 * c[j][0] / c3;
    }
    c1 = c2;
  }
  w[0] = c[0][2];
  for (int q = 1; q <= r; ++q) w[q] = c[2 * q - 1][2];
  return 0;
}

/* Largest stable dt (von Neumann for leapfrog): dt^2 v^2 max(symbol(-L_h)) <= 4,
 * the maximum being at the Nyquist wavenumber on every axis where the symbol
 * equals S = |w0| + 2 sum_q |w_q| per unit h^-2.                              */
double oracle_cfl_dt_max(int64_t so, double vmax, double hx, double hy, double hz) {
  double w[OR_MAXR + 1];
  if (oracle_fd_weights(so, w)) return -1.0;
  double S = fabs(w[0]);
  for (int q = 1; q <= so / 2; ++q) S += 2.0 * fabs(w[q]);
  double sum = 1.0 / (hx * hx) + 1.0 / (hy * hy) + 1.0 / (hz * hz);
  return 2.0 / (vmax * sqrt(S * sum));
}

/* One axis of the sponge: for the d-th point of a face of width nbl (d = 0 the
 * outermost), p = (nbl-d)/nbl and gamma = gmax (p - sin(2 pi p)/(2 pi)),
 * gmax = 3 vmax ln(1/R) / (2 nbl h), R = 1e-3; zero in the interior. The two
 * faces add.                                                                  */
void oracle_sponge_1d(int64_t n, int64_t lo, int64_t hi, double h, double vmax, double *g) {
  const double pi = 3.14159265358979323846, R = 1e-3;
  for (int64_t i = 0; i < n; ++i) g[i] = 0.0;
  for (int face = 0; face < 2; ++face) {
    int64_t nbl = face == 0 ? lo : hi;
    if (nbl <= 0) continue;
    double gmax = 3.0 * vmax * log(1.0 / R) / (2.0 * (double)nbl * h);
    for (int64_t d = 0; d < nbl && d < n; ++d) {
      double p = (double)(nbl - d) / (double)nbl;
      int64_t i = face == 0 ? d : n - 1 - d;
      g[i] += gmax * (p - sin(2.0 * pi * p) / (2.0 * pi));
    }
  }
}

/* Full 3D gamma field (sum of the three axis profiles).                      */
void oracle_sponge_3d(const ogrid *g, double *gamma) {
  double *gx = malloc(sizeof(double) * g->nx), *gy = malloc(sizeof(double) * g->ny),
         *gz = malloc(sizeof(double) * g->nz);
  oracle_sponge_1d(g->nx, g->nbl[0], g->nbl[1], g->hx, g->vmax, gx);
  oracle_sponge_1d(g->ny, g->nbl[2], g->nbl[3], g->hy, g->vmax, gy);
  oracle_sponge_1d(g->nz, g->nbl[4], g->nbl[5], g->hz, g->vmax, gz);
  for (int64_t k = 0; k < g->nz; ++k)
    for (int64_t j = 0; j < g->ny; ++j)
      for (int64_t i = 0; i < g->nx; ++i)
        gamma[(k * g->ny + j) * g->nx + i] = gx[i] + gy[j] + gz[k];
  free(gx); free(gy); free(gz);
}

/* Value at (i,j,k) honouring the halo rule.                                   */
static double at(const ogrid *g, const double *u, int64_t i, int64_t j, int64_t k) {
  if (g->periodic) {
    i = ((i % g->nx) + g->nx) % g->nx;
    j = ((j % g->ny) + g->ny) % g->ny;
    k = ((k % g->nz) + g->nz) % g->nz;
  } else if (i < 0 || i >= g->nx || j < 0 || j >= g->ny || k < 0 || k >= g->nz) {
    return 0.0;
  }
  return u[(k * g->ny + j) * g->nx + i];
}

/* L_h u = sum over axes a of h_a^-2 ( w0 u + sum_q w_q (u(+q e_a) + u(-q e_a)) ). */
int oracle_laplacian(const ogrid *g, const double *u, double *out) {
  double w[OR_MAXR + 1];
  if (oracle_fd_weights(g->so, w)) return -1;
  int r = (int)(g->so / 2);
  double ix = 1.0 / (g->hx * g->hx), iy = 1.0 / (g->hy * g->hy), iz = 1.0 / (g->hz * g->hz);
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < g->nz; ++k)
    for (int64_t j = 0; j < g->ny; ++j)
      for (int64_t i = 0; i < g->nx; ++i) {
        double c = at(g, u, i, j, k);
        double lx = w[0] * c, ly = w[0] * c, lz = w[0] * c;
        for (int q = 1; q <= r; ++q) {
          lx += w[q] * (at(g, u, i + q, j, k) + at(g, u, i - q, j, k));
          ly += w[q] * (at(g, u, i, j + q, k) + at(g, u, i, j - q, k));
          lz += w[q] * (at(g, u, i, j, k + q) + at(g, u, i, j, k - q));
        }
        out[(k * g->ny + j) * g->nx + i] = ix * lx + iy * ly + iz * lz;
      }
  return 0;
}

/* Trilinear corners of a point given in metres: up to 8 (index, weight) pairs;
 * corners of weight exactly zero are dropped. Returns the count, or -1 when the
 * point lies outside [0,(n-1)h] on some axis.                                */
int oracle_trilinear(const ogrid *g, const double *xyz, int64_t *idx, double *wt) {
  double f[3] = {xyz[0] / g->hx, xyz[1] / g->hy, xyz[2] / g->hz};
  int64_t n[3] = {g->nx, g->ny, g->nz}, i0[3];
  double t[3];
  for (int a = 0; a < 3; ++a) {
    if (!(f[a] >= 0.0) || f[a] > (double)(n[a] - 1)) return -1;
    i0[a] = (int64_t)floor(f[a]);
    t[a] = f[a] - (double)i0[a];
  }
  int cnt = 0;
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        double w = (dx ? t[0] : 1.0 - t[0]) * (dy ? t[1] : 1.0 - t[1]) * (dz ? t[2] : 1.0 - t[2]);
        if (w == 0.0) continue;
        int64_t i = i0[0] + dx, j = i0[1] + dy, k = i0[2] + dz;
        idx[cnt] = (k * g->ny + j) * g->nx + i;
        wt[cnt] = w;
        ++cnt;
      }
  return cnt;
}

/* Sparse point operator: for each of np points, its corners.                 */
typedef struct { int np; int *cnt; int64_t *idx; double *w; } opoints;

static int points_make(const ogrid *g, const double *xyz, int np, opoints *p) {
  p->np = np;
  p->cnt = calloc(np > 0 ? np : 1, sizeof(int));
  p->idx = calloc(8 * (np > 0 ? np : 1), sizeof(int64_t));
  p->w = calloc(8 * (np > 0 ? np : 1), sizeof(double));
  for (int s = 0; s < np; ++s) {
    int c = oracle_trilinear(g, xyz + 3 * s, p->idx + 8 * s, p->w + 8 * s);
    if (c < 0) return -1;
    p->cnt[s] = c;
  }
  return 0;
}
static void points_free(opoints *p) { free(p->cnt); free(p->idx); free(p->w); }

/* q += P^T a  (spread amplitudes a[np] onto the grid)                        */
static void points_spread(const opoints *p, const double *a, double *q) {
  for (int s = 0; s < p->np; ++s)
    for (int c = 0; c < p->cnt[s]; ++c) q[p->idx[8 * s + c]] += p->w[8 * s + c] * a[s];
}
/* out = P u  (interpolate the field at the points)                           */
static void points_gather(const opoints *p, const double *u, double *out) {
  for (int s = 0; s < p->np; ++s) {
    double acc = 0.0;
    for (int c = 0; c < p->cnt[s]; ++c) acc += p->w[8 * s + c] * u[p->idx[8 * s + c]];
    out[s] = acc;
  }
}

static int check_grid(const ogrid *g) {
  if (g->nx < 1 || g->ny < 1 || g->nz < 1) return -1;
  if (g->so < 2 || g->so % 2 || g->so / 2 > OR_MAXR) return -1;
  if (!(g->hx > 0 && g->hy > 0 && g->hz > 0 && g->dt > 0) || g->nt < 0) return -1;
  return 0;
}

/* One leapfrog step:  unext = (2 u - (1-b) uprev + C2 (L_h u + q)) / (1+b).
 * unext may alias uprev (each point reads only its own previous value).      */
static void leapfrog(const ogrid *g, const double *C2, const double *b, const double *u,
                     const double *uprev, const double *q, double *lap, double *unext) {
  int64_t N = g->nx * g->ny * g->nz;
  oracle_laplacian(g, u, lap);
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < N; ++p)
    unext[p] = (2.0 * u[p] - (1.0 - b[p]) * uprev[p] + C2[p] * (lap[p] + q[p])) / (1.0 + b[p]);
}

/* Shared set-up: C2 = v^2 dt^2 and b = dt gamma / 2.                          */
static void coefficients(const ogrid *g, const double *vel, double *C2, double *b) {
  int64_t N = g->nx * g->ny * g->nz;
  oracle_sponge_3d(g, b);
  for (int64_t p = 0; p < N; ++p) {
    C2[p] = vel[p] * vel[p] * g->dt * g->dt;
    b[p] = 0.5 * g->dt * b[p];
  }
}

/* Forward solve. wavelet [nt][nsrc], rec_out [nt][nrec] (d^n = R u^{n+1}).
 * u0 / um1: initial levels u^0, u^{-1} (NULL = zero). u_final / um_final
 * receive u^{nt} and u^{nt-1} when not NULL.                                 */
int oracle_forward(const ogrid *g, const double *vel, const double *wavelet,
                   const double *src_xyz, int nsrc, const double *rec_xyz, int nrec,
                   double *rec_out, const double *u0, const double *um1, double *u_final,
                   double *um_final) {
  if (check_grid(g)) return -1;
  int64_t N = g->nx * g->ny * g->nz;
  opoints ps, pr;
  if (points_make(g, src_xyz, nsrc, &ps) || points_make(g, rec_xyz, nrec, &pr)) return -2;
  double *C2 = malloc(sizeof(double) * N), *b = malloc(sizeof(double) * N);
  double *u = calloc(N, sizeof(double)), *um = calloc(N, sizeof(double));
  double *lap = malloc(sizeof(double) * N), *q = malloc(sizeof(double) * N);
  coefficients(g, vel, C2, b);
  if (u0) memcpy(u, u0, sizeof(double) * N);
  if (um1) memcpy(um, um1, sizeof(double) * N);
  for (int64_t n = 0; n < g->nt; ++n) {
    memset(q, 0, sizeof(double) * N);
    if (nsrc) points_spread(&ps, wavelet + n * nsrc, q);
    leapfrog(g, C2, b, u, um, q, lap, um); /* um now holds u^{n+1} */
    double *t = u; u = um; um = t;         /* u = u^{n+1}, um = u^n  */
    if (nrec) points_gather(&pr, u, rec_out + n * nrec);
  }
  if (u_final) memcpy(u_final, u, sizeof(double) * N);
  if (um_final) memcpy(um_final, um, sizeof(double) * N);
  free(C2); free(b); free(u); free(um); free(lap); free(q);
  points_free(&ps); points_free(&pr);
  return 0;
}

/* Adjoint solve: lambda^n for n = nt-1..0 from lambda^{nt} = lambda^{nt+1} = 0,
 *   lambda^n = (2 l^{n+1} - (1-b) l^{n+2} + C2 (L_h l^{n+1} + R^T d^n)) / (1+b),
 * src_out[n] = P lambda^n. rec_data [nt][nrec], src_out [nt][nsrc].
 * lam_final receives lambda^0 when not NULL.                                 */
int oracle_adjoint(const ogrid *g, const double *vel, const double *rec_data,
                   const double *rec_xyz, int nrec, const double *src_xyz, int nsrc,
                   double *src_out, double *lam_final) {
  if (check_grid(g)) return -1;
  int64_t N = g->nx * g->ny * g->nz;
  opoints ps, pr;
  if (points_make(g, src_xyz, nsrc, &ps) || points_make(g, rec_xyz, nrec, &pr)) return -2;
  double *C2 = malloc(sizeof(double) * N), *b = malloc(sizeof(double) * N);
  double *l1 = calloc(N, sizeof(double)), *l2 = calloc(N, sizeof(double));
  double *lap = malloc(sizeof(double) * N), *q = malloc(sizeof(double) * N);
  coefficients(g, vel, C2, b);
  for (int64_t n = g->nt - 1; n >= 0; --n) {
    memset(q, 0, sizeof(double) * N);
    if (nrec) points_spread(&pr, rec_data + n * nrec, q);
    leapfrog(g, C2, b, l1, l2, q, lap, l2); /* l2 now holds lambda^n */
    double *t = l1; l1 = l2; l2 = t;        /* l1 = lambda^n, l2 = lambda^{n+1} */
    if (nsrc) points_gather(&ps, l1, src_out + n * nsrc);
  }
  if (lam_final) memcpy(lam_final, l1, sizeof(double) * N);
  free(C2); free(b); free(l1); free(l2); free(lap); free(q);
  points_free(&ps); points_free(&pr);
  return 0;
}

/* Gradient of a loss L(d) given dL/dd = rec_grad [nt][nrec], zero initial state.
 * Forward levels are kept every ckpt_every steps (as the pair u^{kC}, u^{kC-1})
 * and each segment is recomputed exactly before its adjoint steps; ckpt_every
 * <= 0 keeps every level. Outputs (each may be NULL): grad_m = dL/dm,
 * grad_vel = -2 v^-3 grad_m, grad_wavelet [nt][nsrc] = P lambda^n, and the
 * zero-lag cross-correlation image = sum_{n=1..nt} u^n lambda^n of the forward
 * field with the adjoint field driven by rec_grad (lambda^{nt} = 0).          */
int oracle_gradient_image(const ogrid *g, const double *vel, const double *wavelet,
                          const double *src_xyz, int nsrc, const double *rec_xyz, int nrec,
                          const double *rec_grad, int64_t ckpt_every, double *grad_m,
                          double *grad_vel, double *grad_wavelet, double *image) {
  if (check_grid(g)) return -1;
  int64_t N = g->nx * g->ny * g->nz, nt = g->nt;
  int64_t C = (ckpt_every <= 0 || ckpt_every > nt) ? (nt > 0 ? nt : 1) : ckpt_every;
  int64_t nseg = (nt + C - 1) / C;
  opoints ps, pr;
  if (points_make(g, src_xyz, nsrc, &ps) || points_make(g, rec_xyz, nrec, &pr)) return -2;
  double *C2 = malloc(sizeof(double) * N), *b = malloc(sizeof(double) * N);
  double *gam = malloc(sizeof(double) * N);
  double *lap = malloc(sizeof(double) * N), *q = malloc(sizeof(double) * N);
  double *gm = calloc(N, sizeof(double));
  double *img = calloc(N, sizeof(double));
  coefficients(g, vel, C2, b);
  oracle_sponge_3d(g, gam);
  /* checkpoints: ck[s] = (u^{sC}, u^{sC-1}) */
  double *ck = calloc((size_t)(2 * nseg) * N, sizeof(double));
  {
    double *u = calloc(N, sizeof(double)), *um = calloc(N, sizeof(double));
    for (int64_t n = 0; n < nt; ++n) {
      if (n % C == 0) {
        memcpy(ck + (2 * (n / C)) * N, u, sizeof(double) * N);
        memcpy(ck + (2 * (n / C) + 1) * N, um, sizeof(double) * N);
      }
      memset(q, 0, sizeof(double) * N);
      if (nsrc) points_spread(&ps, wavelet + n * nsrc, q);
      leapfrog(g, C2, b, u, um, q, lap, um);
      double *t = u; u = um; um = t;
    }
    free(u); free(um);
  }
  /* segment store: lev[m] = u^{n0-1+m}, m = 0..C+1 */
  double *lev = malloc(sizeof(double) * (size_t)(C + 2) * N);
  double *l1 = calloc(N, sizeof(double)), *l2 = calloc(N, sizeof(double));
  for (int64_t s = nseg - 1; s >= 0; --s) {
    int64_t n0 = s * C, n1 = n0 + C < nt ? n0 + C : nt;
    memcpy(lev + 1 * N, ck + (2 * s) * N, sizeof(double) * N);
    memcpy(lev + 0 * N, ck + (2 * s + 1) * N, sizeof(double) * N);
    for (int64_t n = n0; n < n1; ++n) { /* recompute u^{n+1} into lev[n-n0+2] */
      memset(q, 0, sizeof(double) * N);
      if (nsrc) points_spread(&ps, wavelet + n * nsrc, q);
      leapfrog(g, C2, b, lev + (n - n0 + 1) * N, lev + (n - n0) * N, q, lap,
               lev + (n - n0 + 2) * N);
    }
    for (int64_t n = n1 - 1; n >= n0; --n) {
      /* image term j = n+1: u^{n+1} lambda^{n+1} (l1 still holds lambda^{n+1}) */
      const double *ujp = lev + (n - n0 + 2) * N;
      for (int64_t p = 0; p < N; ++p) img[p] += ujp[p] * l1[p];
      memset(q, 0, sizeof(double) * N);
      if (nrec) points_spread(&pr, rec_grad + n * nrec, q);
      leapfrog(g, C2, b, l1, l2, q, lap, l2);
      double *t = l1; l1 = l2; l2 = t; /* l1 = lambda^n */
      if (nsrc && grad_wavelet) points_gather(&ps, l1, grad_wavelet + n * nsrc);
      const double *up = lev + (n - n0 + 2) * N, *uc = lev + (n - n0 + 1) * N,
                   *um = lev + (n - n0) * N;
      double idt2 = 1.0 / (g->dt * g->dt), i2dt = 1.0 / (2.0 * g->dt);
#pragma omp parallel for schedule(static)
      for (int64_t p = 0; p < N; ++p)
        gm[p] -= l1[p] * ((up[p] - 2.0 * uc[p] + um[p]) * idt2 + gam[p] * (up[p] - um[p]) * i2dt);
    }
  }
  if (grad_m) memcpy(grad_m, gm, sizeof(double) * N);
  if (image) memcpy(image, img, sizeof(double) * N);
  if (grad_vel)
    for (int64_t p = 0; p < N; ++p) grad_vel[p] = -2.0 * gm[p] / (vel[p] * vel[p] * vel[p]);
  free(C2); free(b); free(gam); free(lap); free(q); free(gm); free(img); free(ck); free(lev);
  free(l1); free(l2);
  points_free(&ps); points_free(&pr);
  return 0;
}

int oracle_gradient(const ogrid *g, const double *vel, const double *wavelet,
                    const double *src_xyz, int nsrc, const double *rec_xyz, int nrec,
                    const double *rec_grad, int64_t ckpt_every, double *grad_m,
                    double *grad_vel, double *grad_wavelet) {
  return oracle_gradient_image(g, vel, wavelet, src_xyz, nsrc, rec_xyz, nrec, rec_grad,
                               ckpt_every, grad_m, grad_vel, grad_wavelet, NULL);
}

/* Number of threads OpenMP would use (for reporting), and a way to change it
 * (a single-thread timing beside the all-core one).                         */
#ifdef _OPENMP
#include <omp.h>
int oracle_num_threads(void) { return omp_get_max_threads(); }
void oracle_set_num_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
#else
int oracle_num_threads(void) { return 1; }
void oracle_set_num_threads(int n) { (void)n; }
#endif
