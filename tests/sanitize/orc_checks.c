/* Runs every entry point of the oracle (oracle/orc.c) on small 2-D and 3-D
 * grids, including positions on the grid's edges and refused ones, so that
 * a build with AddressSanitizer and UndefinedBehaviorSanitizer sees every
 * loop of it. Test infrastructure: built and run by
 * tests/test_sanitizers.py. Exit status 0 when every call returned what it
 * should. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int orc_padded_size(int ndim, int nz, int ny, int nx, int nb, int64_t* out3);
int orc_medium(int ndim, int nz, int ny, int nx, int nb, double h, double dt,
               const double* vel, double* W, double* C1, double* C2);
int orc_ricker(int nt, double dt, double f0, double* out);
int orc_laplacian(int ndim, int nz, int ny, int nx, int nb, double h,
                  const double* u, double* out);
int orc_background(int ndim, int nz, int ny, int nx, int nb, double h,
                   double dt, const double* W, const double* C1,
                   const double* C2, int sz, int sy, int sx,
                   const double* wavelet, int nt, int nrec, const int* rec,
                   double* d2u0, double* u0_rec);
int orc_born(int ndim, int nz, int ny, int nx, int nb, double h, double dt,
             const double* W, const double* C1, const double* C2, int sz,
             int sy, int sx, const double* wavelet, int nt, int nrec,
             const int* rec, const double* m, double* d);
int orc_adjoint(int ndim, int nz, int ny, int nx, int nb, double h, double dt,
                const double* W, const double* C1, const double* C2, int sz,
                int sy, int sx, const double* wavelet, int nt, int nrec,
                const int* rec, const double* r, double* gout);

static int failures = 0;
#define EXPECT(cond, what)                    \
  do {                                        \
    if (!(cond)) {                            \
      fprintf(stderr, "FAILED: %s\n", what);  \
      ++failures;                             \
    }                                         \
  } while (0)

static void run(int ndim, int nz, int ny, int nx, int nb) {
  const double h = 10.0, dt = 1e-3;
  const int nt = 40;
  int64_t p[3];
  orc_padded_size(ndim, nz, ny, nx, nb, p);
  const size_t np = (size_t)(p[0] * p[1] * p[2]);
  const size_t nm = (size_t)nz * (ndim == 3 ? ny : 1) * nx;
  double* vel = malloc(nm * sizeof(double));
  double* m = malloc(nm * sizeof(double));
  double* g = malloc(nm * sizeof(double));
  double* W = malloc(np * sizeof(double));
  double* C1 = malloc(np * sizeof(double));
  double* C2 = malloc(np * sizeof(double));
  double* u = malloc(np * sizeof(double));
  double* lu = malloc(np * sizeof(double));
  double* wav = malloc(nt * sizeof(double));
  for (size_t i = 0; i < nm; ++i) {
    vel[i] = 1800.0 + (double)(i % 7) * 10.0;
    m[i] = (i % 5 == 0) ? 0.05 : 0.0;
  }
  for (size_t i = 0; i < np; ++i) u[i] = (double)(i % 11) - 5.0;
  EXPECT(orc_medium(ndim, nz, ny, nx, nb, h, dt, vel, W, C1, C2) == 0,
         "medium");
  EXPECT(orc_medium(ndim, nz, ny, nx, 0, h, dt, vel, W, C1, C2) != 0,
         "medium refuses nb = 0");
  EXPECT(orc_ricker(nt, dt, 25.0, wav) == 0, "ricker");
  EXPECT(orc_laplacian(ndim, nz, ny, nx, nb, h, u, lu) == 0, "laplacian");
  /* receivers on every corner of the model grid */
  const int yl = ndim == 3 ? ny - 1 : 0;
  int rec[4 * 3] = {0, 0, 0, nz - 1, yl, nx - 1, 0, yl, nx - 1, nz - 1, 0, 0};
  const int nrec = 4;
  double* d2 = malloc((size_t)(nt - 1) * nm * sizeof(double));
  double* urec = malloc((size_t)nt * nrec * sizeof(double));
  double* d = malloc((size_t)nt * nrec * sizeof(double));
  EXPECT(orc_background(ndim, nz, ny, nx, nb, h, dt, W, C1, C2, 0, 0, 0, wav,
                        nt, nrec, rec, d2, urec) == 0,
         "background, source on a corner");
  EXPECT(orc_born(ndim, nz, ny, nx, nb, h, dt, W, C1, C2, nz - 1, yl, nx - 1,
                  wav, nt, nrec, rec, m, d) == 0,
         "born, source on the far corner");
  EXPECT(orc_adjoint(ndim, nz, ny, nx, nb, h, dt, W, C1, C2, nz / 2,
                     ndim == 3 ? ny / 2 : 0, nx / 2, wav, nt, nrec, rec, d,
                     g) == 0,
         "adjoint");
  /* positions outside the model are refused */
  EXPECT(orc_born(ndim, nz, ny, nx, nb, h, dt, W, C1, C2, nz, 0, 0, wav, nt,
                  nrec, rec, m, d) != 0,
         "born refuses a source below the model");
  int bad[3] = {0, 0, nx};
  EXPECT(orc_adjoint(ndim, nz, ny, nx, nb, h, dt, W, C1, C2, 0, 0, 0, wav, nt,
                     1, bad, d, g) != 0,
         "adjoint refuses a receiver right of the model");
  free(vel); free(m); free(g); free(W); free(C1); free(C2); free(u);
  free(lu); free(wav); free(d2); free(urec); free(d);
}

int main(void) {
  run(2, 9, 1, 13, 5);
  run(3, 6, 5, 7, 4);
  if (failures) return 1;
  printf("oracle checks passed\n");
  return 0;
}
