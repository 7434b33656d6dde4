/*
 * FP64 CPU oracle for wave-equation Born modelling and its exact discrete
 * adjoint, the operator pair inside block-row recursive least-squares
 * migration (Kazemi & Sacchi, "Block row recursive least squares migration",
 * CSEG 2015, arXiv 1801.00819).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the plain, slow, obviously correct
 * definition that the GPU library is checked against. It shares no code with
 * the GPU library; only tests, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.
 *
 * The paper fixes the method (eqs. 1-4: d = A m + n, migration = A^T,
 * damped least squares; eqs. 10-11: sliding windows, warm start) but not the
 * operator: its examples use one-way split-step operators with no formulas
 * given (Examples section). The operator here is the two-way acoustic
 * constant-density Born operator on a regular grid, defined as follows, and
 * the oracle computes exactly that definition in double precision.
 *
 *  Grid.   Model nz x ny x nx (ny = 1 in 2-D), spacing h, padded by nb cells
 *          on every face (all faces absorbing). Velocity is edge-replicated
 *          into the padding. The model vector m lives on the unpadded part
 *          only (P = zero extension, P^T = restriction).
 *  Medium. W = v^2 dt^2. Sponge eta = eta_max * sum_axes (d_a/nb)^2 with d_a
 *          the number of cells into the sponge along axis a, and
 *          eta_max = 3 v_max ln(1000) / (2 nb h).
 *          C1 = 1/(1 + eta dt/2), C2 = (1 - eta dt/2)/(1 + eta dt/2).
 *  Stencil L = sum over axes of the 8th-order central second difference with
 *          weights (-205/72, 8/5, -1/5, 8/315, -1/560)/h^2, zero outside the
 *          padded grid (so L is symmetric).
 *  Source. Ricker of peak frequency f0 delayed by t0 = 1.5/f0, sampled at
 *          t_n = n dt, injected at one grid point.
 *  F1 background: u^{-1} = u^0 = 0,
 *          u^{n+1} = C1 (2u^n + W L u^n) - C2 u^{n-1} + e_s C1 W f(t_n).
 *  F2 Born source: D2u0^n = u0^{n+1} - 2 u0^n + u0^{n-1}, n = 0..nt-2.
 *  F3 Born field: du^{-1} = du^0 = 0,
 *          du^{n+1} = C1 (2du^n + W L du^n) - C2 du^{n-1} - C1 (Pm) D2u0^n,
 *          data d^n = du^n at the receivers, n = 0..nt-1.
 *  A1 adjoint (the literal transpose of F3):
 *          lam^{nt} = lam^{nt+1} = 0; for k = nt-1 .. 1:
 *          lam^k = R^T r^k + 2 C1 lam^{k+1} + L(W C1 lam^{k+1}) - C2 lam^{k+2}
 *          A^T r = P^T sum_{n=0}^{nt-2} (-D2u0^n) C1 lam^{n+1}.
 *
 * m is the relative perturbation of squared slowness: under
 * W -> W/(1 + eps P m), F3 is the derivative of F1 at eps = 0.
 *
 * Layout: row-major [z][y][x], x fastest. Shot data [n][rec].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_RADIUS 4

/* 8th-order central second-derivative weights, offsets 0..4. */
static const double ORC_C[ORC_RADIUS + 1] = {
    -205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};

typedef struct {
  int ndim;
  int nz, ny, nx; /* model */
  int nb;
  int pz, py, px; /* padded */
  double h, dt;
} orc_dims;

static orc_dims make_dims(int ndim, int nz, int ny, int nx, int nb, double h,
                          double dt) {
  orc_dims g;
  g.ndim = ndim;
  g.nz = nz;
  g.ny = (ndim == 3) ? ny : 1;
  g.nx = nx;
  g.nb = nb;
  g.pz = nz + 2 * nb;
  g.py = (ndim == 3) ? ny + 2 * nb : 1;
  g.px = nx + 2 * nb;
  g.h = h;
  g.dt = dt;
  return g;
}

static size_t npad(const orc_dims* g) {
  return (size_t)g->pz * g->py * g->px;
}
static size_t nmodel(const orc_dims* g) {
  return (size_t)g->nz * g->ny * g->nx;
}
static size_t pidx(const orc_dims* g, int z, int y, int x) {
  return ((size_t)z * g->py + y) * g->px + x;
}

/* Number of cells point i lies inside the sponge along one axis (0 inside the
 * model region). */
static int sponge_depth(int i, int nb, int n) {
  if (i < nb) return nb - i;
  if (i >= nb + n) return i - (nb + n - 1);
  return 0;
}

static int clampi(int i, int lo, int hi) {
  return i < lo ? lo : (i > hi ? hi : i);
}

int orc_padded_size(int ndim, int nz, int ny, int nx, int nb, int64_t* out3) {
  orc_dims g = make_dims(ndim, nz, ny, nx, nb, 1.0, 1.0);
  out3[0] = g.pz;
  out3[1] = g.py;
  out3[2] = g.px;
  return 0;
}

/* Medium coefficients on the padded grid from a model-grid velocity. */
int orc_medium(int ndim, int nz, int ny, int nx, int nb, double h, double dt,
               const double* vel, double* W, double* C1, double* C2) {
  if (nb < 1) return -1;
  orc_dims g = make_dims(ndim, nz, ny, nx, nb, h, dt);
  double vmax = 0.0;
  for (size_t i = 0; i < nmodel(&g); i++)
    if (vel[i] > vmax) vmax = vel[i];
  double eta_max = 3.0 * vmax * log(1000.0) / (2.0 * nb * h);
  for (int z = 0; z < g.pz; z++)
    for (int y = 0; y < g.py; y++)
      for (int x = 0; x < g.px; x++) {
        int mz = clampi(z - nb, 0, nz - 1);
        int my = (ndim == 3) ? clampi(y - nb, 0, ny - 1) : 0;
        int mx = clampi(x - nb, 0, nx - 1);
        double v = vel[((size_t)mz * g.ny + my) * g.nx + mx];
        double dz = sponge_depth(z, nb, nz) / (double)nb;
        double dx = sponge_depth(x, nb, nx) / (double)nb;
        double dy = (ndim == 3) ? sponge_depth(y, nb, ny) / (double)nb : 0.0;
        double eta = eta_max * (dz * dz + dy * dy + dx * dx);
        size_t i = pidx(&g, z, y, x);
        W[i] = v * v * dt * dt;
        C1[i] = 1.0 / (1.0 + eta * dt / 2.0);
        C2[i] = (1.0 - eta * dt / 2.0) / (1.0 + eta * dt / 2.0);
      }
  return 0;
}

/* Ricker wavelet, peak frequency f0, delay t0 = 1.5/f0, at t_n = n dt. */
int orc_ricker(int nt, double dt, double f0, double* out) {
  double t0 = 1.5 / f0;
  for (int n = 0; n < nt; n++) {
    double t = n * dt - t0;
    double a = M_PI * M_PI * f0 * f0 * t * t;
    out[n] = (1.0 - 2.0 * a) * exp(-a);
  }
  return 0;
}

/* Value of u at padded point (z,y,x), zero outside the padded grid. */
static double at(const orc_dims* g, const double* u, int z, int y, int x) {
  if (z < 0 || z >= g->pz || y < 0 || y >= g->py || x < 0 || x >= g->px)
    return 0.0;
  return u[pidx(g, z, y, x)];
}

/* out = L u on the padded grid. */
static void laplacian(const orc_dims* g, const double* u, double* out) {
  double ih2 = 1.0 / (g->h * g->h);
#pragma omp parallel for schedule(static)
  for (int z = 0; z < g->pz; z++)
    for (int y = 0; y < g->py; y++)
      for (int x = 0; x < g->px; x++) {
        double c = u[pidx(g, z, y, x)];
        double sz = ORC_C[0] * c, sx = ORC_C[0] * c, sy = 0.0;
        for (int k = 1; k <= ORC_RADIUS; k++) {
          sz += ORC_C[k] * (at(g, u, z + k, y, x) + at(g, u, z - k, y, x));
          sx += ORC_C[k] * (at(g, u, z, y, x + k) + at(g, u, z, y, x - k));
        }
        if (g->ndim == 3) {
          sy = ORC_C[0] * c;
          for (int k = 1; k <= ORC_RADIUS; k++)
            sy += ORC_C[k] * (at(g, u, z, y + k, x) + at(g, u, z, y - k, x));
        }
        out[pidx(g, z, y, x)] = (sz + sy + sx) * ih2;
      }
}

int orc_laplacian(int ndim, int nz, int ny, int nx, int nb, double h,
                  const double* u, double* out) {
  orc_dims g = make_dims(ndim, nz, ny, nx, nb, h, 1.0);
  laplacian(&g, u, out);
  return 0;
}

/* Padded index of a model-grid position (z,y,x). */
static size_t model_to_pad(const orc_dims* g, int z, int y, int x) {
  int py = (g->ndim == 3) ? y + g->nb : 0;
  return pidx(g, z + g->nb, py, x + g->nb);
}

static int check_pos(const orc_dims* g, int z, int y, int x) {
  if (z < 0 || z >= g->nz || x < 0 || x >= g->nx) return -1;
  if (g->ndim == 3 && (y < 0 || y >= g->ny)) return -1;
  return 0;
}

/* One step of F1's recursion applied to any field: next = C1(2cur + W L cur)
 * - C2 prev, using tmp for L cur. */
static void leapfrog(const orc_dims* g, const double* W, const double* C1,
                     const double* C2, const double* prev, const double* cur,
                     double* next, double* tmp) {
  laplacian(g, cur, tmp);
  size_t N = npad(g);
#pragma omp parallel for schedule(static)
  for (size_t i = 0; i < N; i++)
    next[i] = C1[i] * (2.0 * cur[i] + W[i] * tmp[i]) - C2[i] * prev[i];
}

/*
 * F1 background for one shot. Optional outputs (NULL to skip):
 *   d2u0   [nt-1][nz][ny][nx]: F2 Born source on the model region;
 *   u0_rec [nt][nrec]: u0 sampled at the receivers.
 */
int orc_background(int ndim, int nz, int ny, int nx, int nb, double h,
                   double dt, const double* W, const double* C1,
                   const double* C2, int sz, int sy, int sx,
                   const double* wavelet, int nt, int nrec, const int* rec,
                   double* d2u0, double* u0_rec) {
  orc_dims g = make_dims(ndim, nz, ny, nx, nb, h, dt);
  if (nt < 1 || check_pos(&g, sz, sy, sx)) return -1;
  for (int j = 0; j < nrec; j++)
    if (check_pos(&g, rec[3 * j], rec[3 * j + 1], rec[3 * j + 2])) return -1;
  size_t N = npad(&g), M = nmodel(&g);
  double* prev = calloc(N, sizeof(double));
  double* cur = calloc(N, sizeof(double));
  double* next = calloc(N, sizeof(double));
  double* tmp = calloc(N, sizeof(double));
  if (!prev || !cur || !next || !tmp) return -2;
  size_t s = model_to_pad(&g, sz, sy, sx);
  if (u0_rec)
    for (int j = 0; j < nrec; j++) u0_rec[j] = 0.0;
  for (int n = 0; n + 1 < nt; n++) {
    leapfrog(&g, W, C1, C2, prev, cur, next, tmp);
    next[s] += C1[s] * W[s] * wavelet[n];
    if (d2u0) {
      double* out = d2u0 + (size_t)n * M;
      for (int z = 0; z < nz; z++)
        for (int y = 0; y < g.ny; y++)
          for (int x = 0; x < nx; x++) {
            size_t i = model_to_pad(&g, z, y, x);
            out[((size_t)z * g.ny + y) * nx + x] =
                next[i] - 2.0 * cur[i] + prev[i];
          }
    }
    if (u0_rec)
      for (int j = 0; j < nrec; j++)
        u0_rec[(size_t)(n + 1) * nrec + j] =
            next[model_to_pad(&g, rec[3 * j], rec[3 * j + 1], rec[3 * j + 2])];
    double* t = prev;
    prev = cur;
    cur = next;
    next = t;
  }
  free(prev);
  free(cur);
  free(next);
  free(tmp);
  return 0;
}

/* F3: Born data of one shot, d [nt][nrec], for model perturbation m. The
 * background and Born fields are advanced together, so no history is kept. */
int orc_born(int ndim, int nz, int ny, int nx, int nb, double h, double dt,
             const double* W, const double* C1, const double* C2, int sz,
             int sy, int sx, const double* wavelet, int nt, int nrec,
             const int* rec, const double* m, double* d) {
  orc_dims g = make_dims(ndim, nz, ny, nx, nb, h, dt);
  if (nt < 1 || check_pos(&g, sz, sy, sx)) return -1;
  for (int j = 0; j < nrec; j++)
    if (check_pos(&g, rec[3 * j], rec[3 * j + 1], rec[3 * j + 2])) return -1;
  size_t N = npad(&g);
  double* b[3];
  double* f[3];
  double* tmp = calloc(N, sizeof(double));
  double* pm = calloc(N, sizeof(double));
  for (int i = 0; i < 3; i++) {
    b[i] = calloc(N, sizeof(double));
    f[i] = calloc(N, sizeof(double));
    if (!b[i] || !f[i]) return -2;
  }
  if (!tmp || !pm) return -2;
  /* P m: zero extension of the model into the padding. */
  for (int z = 0; z < nz; z++)
    for (int y = 0; y < g.ny; y++)
      for (int x = 0; x < nx; x++)
        pm[model_to_pad(&g, z, y, x)] = m[((size_t)z * g.ny + y) * nx + x];
  size_t s = model_to_pad(&g, sz, sy, sx);
  double *bp = b[0], *bc = b[1], *bn = b[2];
  double *fp = f[0], *fc = f[1], *fn = f[2];
  for (int j = 0; j < nrec; j++) d[j] = 0.0; /* du^0 = 0 */
  for (int n = 0; n + 1 < nt; n++) {
    leapfrog(&g, W, C1, C2, bp, bc, bn, tmp);
    bn[s] += C1[s] * W[s] * wavelet[n];
    leapfrog(&g, W, C1, C2, fp, fc, fn, tmp);
#pragma omp parallel for schedule(static)
    for (size_t i = 0; i < N; i++) {
      double d2 = bn[i] - 2.0 * bc[i] + bp[i];
      fn[i] -= C1[i] * pm[i] * d2;
    }
    for (int j = 0; j < nrec; j++)
      d[(size_t)(n + 1) * nrec + j] =
          fn[model_to_pad(&g, rec[3 * j], rec[3 * j + 1], rec[3 * j + 2])];
    double* t = bp;
    bp = bc;
    bc = bn;
    bn = t;
    t = fp;
    fp = fc;
    fc = fn;
    fn = t;
  }
  for (int i = 0; i < 3; i++) {
    free(b[i]);
    free(f[i]);
  }
  free(tmp);
  free(pm);
  return 0;
}

/* A1: adjoint of orc_born for one shot. r [nt][nrec] -> g [nz][ny][nx]
 * (overwritten). Keeps the whole F2 history of the model region. */
int orc_adjoint(int ndim, int nz, int ny, int nx, int nb, double h, double dt,
                const double* W, const double* C1, const double* C2, int sz,
                int sy, int sx, const double* wavelet, int nt, int nrec,
                const int* rec, const double* r, double* gout) {
  orc_dims g = make_dims(ndim, nz, ny, nx, nb, h, dt);
  size_t N = npad(&g), M = nmodel(&g);
  for (size_t i = 0; i < M; i++) gout[i] = 0.0;
  if (nt < 2) return 0;
  double* hist = malloc((size_t)(nt - 1) * M * sizeof(double));
  if (!hist) return -2;
  int rc = orc_background(ndim, nz, ny, nx, nb, h, dt, W, C1, C2, sz, sy, sx,
                          wavelet, nt, nrec, rec, hist, NULL);
  if (rc) {
    free(hist);
    return rc;
  }
  /* lam[0] = lam^{k+2}, lam[1] = lam^{k+1}, lam[2] = lam^k */
  double* l2 = calloc(N, sizeof(double));
  double* l1 = calloc(N, sizeof(double));
  double* l0 = calloc(N, sizeof(double));
  double* t = calloc(N, sizeof(double));
  double* lt = calloc(N, sizeof(double));
  if (!l2 || !l1 || !l0 || !t || !lt) return -2;
  for (int k = nt - 1; k >= 1; k--) {
#pragma omp parallel for schedule(static)
    for (size_t i = 0; i < N; i++) t[i] = W[i] * C1[i] * l1[i];
    laplacian(&g, t, lt);
#pragma omp parallel for schedule(static)
    for (size_t i = 0; i < N; i++)
      l0[i] = 2.0 * C1[i] * l1[i] + lt[i] - C2[i] * l2[i];
    for (int j = 0; j < nrec; j++)
      l0[model_to_pad(&g, rec[3 * j], rec[3 * j + 1], rec[3 * j + 2])] +=
          r[(size_t)k * nrec + j];
    /* image term n = k-1 */
    const double* d2 = hist + (size_t)(k - 1) * M;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; z++)
      for (int y = 0; y < g.ny; y++)
        for (int x = 0; x < nx; x++) {
          size_t mi = ((size_t)z * g.ny + y) * nx + x;
          size_t pi = model_to_pad(&g, z, y, x);
          gout[mi] += -d2[mi] * C1[pi] * l0[pi];
        }
    double* tt = l2;
    l2 = l1;
    l1 = l0;
    l0 = tt;
  }
  free(hist);
  free(l2);
  free(l1);
  free(l0);
  free(t);
  free(lt);
  return 0;
}
