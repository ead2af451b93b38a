/*
 * Plain C, FP64 oracle routines -- TEST INFRASTRUCTURE ONLY (see
 * oracle/__init__.py).  The same definitions as oracle/fwi.py and
 * oracle/svgd.py, written as loops, for sizes where NumPy is too slow.
 * Shares no code with the HIP library.
 *
 * Scheme (readings of the paper's FD method, section 4.2):
 *   u^{n+1} = g (2 u^n + c (L u^n + f^n) - g u^{n-1}),  c = v_pad^2 dt^2,
 *   (L u)_ij = sum_{o=-2..2} w_o (u_{i+o,j}/dz^2 + u_{i,j+o}/dx^2), u = 0 off the grid,
 *   g = gamma(delta_z) gamma(delta_x), gamma(delta) = exp(-(alpha delta)^2),
 *   f^n = w(t_n)/(dx dz) at the source node, traces d^n_r = u^n(x_r).
 * Adjoint (z = g c lambda):
 *   z^n = g (2 z^{n+1} + c (L z^{n+1} + R^T rho^n) - g z^{n+2}),  n = nt-1 .. 1,
 *   dJ/dv_pad = (2 / v_pad) sum_{n=0}^{nt-2} z^{n+1} (L u^n + f^n).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

static const double W[5] = {-1.0 / 12.0, 4.0 / 3.0, -5.0 / 2.0, 4.0 / 3.0, -1.0 / 12.0};

static double gam(int k, int n, int nb, double alpha) {
  int d1 = nb - k, d2 = k - (nb + n - 1);
  int delta = d1 > d2 ? d1 : d2;
  if (delta < 0) delta = 0;
  double a = alpha * (double)delta;
  return exp(-a * a);
}

/* L u with u = 0 on two ghost layers: u is first copied into the interior of
 * a zero-bordered (NZ+4) x (NX+4) array p. */
static void laplacian(const double *u, double *out, double *p, int NZ, int NX, double dz,
                      double dx) {
  const double iz2 = 1.0 / (dz * dz), ix2 = 1.0 / (dx * dx);
  const int PW = NX + 4;
  for (int i = 0; i < NZ; ++i) memcpy(p + (size_t)(i + 2) * PW + 2, u + (size_t)i * NX, NX * sizeof(double));
  for (int i = 0; i < NZ; ++i) {
    const double *c = p + (size_t)(i + 2) * PW + 2;
    for (int j = 0; j < NX; ++j) {
      double s = 0.0;
      for (int o = -2; o <= 2; ++o) s += W[o + 2] * (c[j + o * PW] * iz2 + c[j + o] * ix2);
      out[(size_t)i * NX + j] = s;
    }
  }
}

typedef struct {
  int nz, nx, nb, nt, NZ, NX;
  double dx, dz, dt, alpha;
  double *vpad, *c, *g;
} problem;

static int setup(problem *P, int nz, int nx, int nb, int nt, double dx, double dz, double dt,
                 double alpha, const double *vel) {
  P->nz = nz; P->nx = nx; P->nb = nb; P->nt = nt;
  P->NZ = nz + 2 * nb; P->NX = nx + 2 * nb;
  P->dx = dx; P->dz = dz; P->dt = dt; P->alpha = alpha;
  size_t N = (size_t)P->NZ * P->NX;
  P->vpad = malloc(N * sizeof(double));
  P->c = malloc(N * sizeof(double));
  P->g = malloc(N * sizeof(double));
  if (!P->vpad || !P->c || !P->g) return -1;
  for (int i = 0; i < P->NZ; ++i)
    for (int j = 0; j < P->NX; ++j) {
      int iz = i - nb, ix = j - nb;
      if (iz < 0) iz = 0;
      if (iz > nz - 1) iz = nz - 1;
      if (ix < 0) ix = 0;
      if (ix > nx - 1) ix = nx - 1;
      double v = vel[iz * nx + ix];
      P->vpad[i * P->NX + j] = v;
      P->c[i * P->NX + j] = v * v * dt * dt;
      P->g[i * P->NX + j] = gam(i, nz, nb, alpha) * gam(j, nx, nb, alpha);
    }
  return 0;
}

static void release(problem *P) {
  free(P->vpad);
  free(P->c);
  free(P->g);
}

/* Forward of one shot.  traces [nt][nr]; hist (optional) [nt-1][N] = L u^n + f^n;
 * snaps (optional) [nsnap][N] = u^n at the steps snap_n[k], ascending. */
static int forward(const problem *P, int src_iz, int src_ix, int nr, const int *rec_iz,
                   const int *rec_ix, const double *wavelet, double *traces, double *hist,
                   int nsnap, const int *snap_n, double *snaps) {
  const int NZ = P->NZ, NX = P->NX;
  const size_t N = (size_t)NZ * NX;
  double *um = calloc(N, sizeof(double)), *u = calloc(N, sizeof(double));
  double *up = malloc(N * sizeof(double)), *a = malloc(N * sizeof(double));
  double *pad = calloc((size_t)(NZ + 4) * (NX + 4), sizeof(double));
  if (!um || !u || !up || !a || !pad) return -1;
  const int s = (src_iz + P->nb) * NX + src_ix + P->nb;
  const double area = P->dx * P->dz;
  for (int r = 0; r < nr; ++r) traces[r] = 0.0;
  int ks = 0;
  while (ks < nsnap && snap_n[ks] == 0) memset(snaps + (size_t)ks++ * N, 0, N * sizeof(double));
  for (int n = 0; n <= P->nt - 2; ++n) {
    laplacian(u, a, pad, NZ, NX, P->dz, P->dx);
    a[s] += wavelet[n] / area;
    for (size_t i = 0; i < N; ++i)
      up[i] = P->g[i] * (2.0 * u[i] + P->c[i] * a[i] - P->g[i] * um[i]);
    for (int r = 0; r < nr; ++r)
      traces[(size_t)(n + 1) * nr + r] = up[(rec_iz[r] + P->nb) * NX + rec_ix[r] + P->nb];
    if (hist) memcpy(hist + (size_t)n * N, a, N * sizeof(double));
    while (ks < nsnap && snap_n[ks] == n + 1) memcpy(snaps + (size_t)ks++ * N, up, N * sizeof(double));
    double *t = um;
    um = u;
    u = up;
    up = t;
  }
  free(um); free(u); free(up); free(a); free(pad);
  return 0;
}

int cref_shot_forward(int nz, int nx, int nb, int nt, double dx, double dz, double dt,
                      double alpha, const double *vel, int src_iz, int src_ix, int nr,
                      const int *rec_iz, const int *rec_ix, const double *wavelet,
                      double *traces) {
  problem P;
  if (setup(&P, nz, nx, nb, nt, dx, dz, dt, alpha, vel)) return -1;
  int st = forward(&P, src_iz, src_ix, nr, rec_iz, rec_ix, wavelet, traces, NULL, 0, NULL, NULL);
  release(&P);
  return st;
}

/* Wavefields u^n [nsnap][NZ][NX] of one shot at the steps snap_n (ascending,
 * 0 <= n <= nt-1), and its traces [nt][nr]. */
int cref_shot_snapshots(int nz, int nx, int nb, int nt, double dx, double dz, double dt,
                        double alpha, const double *vel, int src_iz, int src_ix, int nr,
                        const int *rec_iz, const int *rec_ix, const double *wavelet,
                        int nsnap, const int *snap_n, double *snaps, double *traces) {
  for (int k = 0; k < nsnap; ++k)
    if (snap_n[k] < 0 || snap_n[k] > nt - 1 || (k > 0 && snap_n[k] <= snap_n[k - 1])) return -2;
  problem P;
  if (setup(&P, nz, nx, nb, nt, dx, dz, dt, alpha, vel)) return -1;
  int st = forward(&P, src_iz, src_ix, nr, rec_iz, rec_ix, wavelet, traces, NULL, nsnap, snap_n,
                   snaps);
  release(&P);
  return st;
}

/* Misfit J = 1/2 sum (d - dobs)^2 / sigma^2 of one shot and dJ/dv_pad [NZ][NX]. */
int cref_shot_gradient(int nz, int nx, int nb, int nt, double dx, double dz, double dt,
                       double alpha, const double *vel, int src_iz, int src_ix, int nr,
                       const int *rec_iz, const int *rec_ix, const double *wavelet,
                       const double *dobs, double sigma, double *J_out, double *grad_pad) {
  problem P;
  if (setup(&P, nz, nx, nb, nt, dx, dz, dt, alpha, vel)) return -1;
  const int NZ = P.NZ, NX = P.NX;
  const size_t N = (size_t)NZ * NX;
  double *traces = malloc((size_t)nt * nr * sizeof(double));
  double *hist = malloc((size_t)(nt - 1) * N * sizeof(double));
  if (!traces || !hist) return -1;
  if (forward(&P, src_iz, src_ix, nr, rec_iz, rec_ix, wavelet, traces, hist, 0, NULL, NULL))
    return -1;
  double J = 0.0;
  for (size_t e = 0; e < (size_t)nt * nr; ++e) {
    double r = traces[e] - dobs[e];
    J += r * r;
    traces[e] = r / (sigma * sigma);   /* residual rho */
  }
  *J_out = 0.5 * J / (sigma * sigma);
  double *z2 = calloc(N, sizeof(double)), *z1 = calloc(N, sizeof(double));
  double *z = malloc(N * sizeof(double)), *b = malloc(N * sizeof(double));
  double *img = calloc(N, sizeof(double));
  double *pad = calloc((size_t)(NZ + 4) * (NX + 4), sizeof(double));
  if (!z2 || !z1 || !z || !b || !img || !pad) return -1;
  for (int n = nt - 1; n >= 1; --n) {
    laplacian(z1, b, pad, NZ, NX, P.dz, P.dx);
    for (int r = 0; r < nr; ++r)
      b[(rec_iz[r] + nb) * NX + rec_ix[r] + nb] += traces[(size_t)n * nr + r];
    for (size_t i = 0; i < N; ++i) z[i] = P.g[i] * (2.0 * z1[i] + P.c[i] * b[i] - P.g[i] * z2[i]);
    const double *a = hist + (size_t)(n - 1) * N;
    for (size_t i = 0; i < N; ++i) img[i] += z[i] * a[i];
    double *t = z2;
    z2 = z1;
    z1 = z;
    z = t;
  }
  for (size_t i = 0; i < N; ++i) grad_pad[i] = 2.0 / P.vpad[i] * img[i];
  free(traces); free(hist); free(z2); free(z1); free(z); free(b); free(img); free(pad);
  release(&P);
  return 0;
}

/* D[i][j] = sum_a (X[i][a] - X[j][a])^2 for rows i in [i0, i1), all j. */
void cref_sqdist_rows(int n, long long d, const double *X, int i0, int i1, double *D) {
  for (int i = i0; i < i1; ++i)
    for (int j = 0; j < n; ++j) {
      const double *xi = X + (size_t)i * d, *xj = X + (size_t)j * d;
      double s = 0.0;
      for (long long a = 0; a < d; ++a) {
        double t = xi[a] - xj[a];
        s += t * t;
      }
      D[(size_t)i * n + j] = s;
    }
}
