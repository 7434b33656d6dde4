// Background wavefield of a shot in float64, storing its Born-source frames
// in float32 (2-D and 3-D, stored-source strategy).
//
// The background u0 (eq. 1's reference wavefield: the source's field in the
// migration velocity) is computed once per shot that enters the window and
// feeds every Born and adjoint application of every CG iteration through its
// stored frames D2u0^n = u0^{n+1} - 2u0^n + u0^{n-1} (model region). Carried
// in float32, its rounding over thousands of steps is the largest error of
// the operator pair; in float64 the frames are exact up to their final
// rounding to float32. The step is the one the float32 kernels take, in
// difference form: v^{n+1} = C2 v^n + C1 W'(h^2 L u^n + h^2 f(t_n) e_s),
// u^{n+1} = u^n + v^{n+1}, frame n = W'(h^2 L u^n + h^2 f(t_n) e_s) (where
// C1 = C2 = 1, i.e. on the model region).
//
// The 4-cell zero ring around the padded grid (same storage layout as the
// float32 fields, float64 elements) supplies the Dirichlet boundary, so no
// load is bounds-checked. 3-D: one thread per padded point, neighbour reuse
// left to the caches; 2-D: a thread marches a column (k_background64_2d).
// These kernels run nt - 1 times per shot entering the window, not per CG
// iteration.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "layout.h"

namespace brls {

namespace {

__device__ __forceinline__ int depth(int i, int nb, int n) {
  return i < nb ? nb - i : (i >= nb + n ? i - (nb + n - 1) : 0);
}

}  // namespace

// blockDim (64, 4); grid (ceil(px / 64), ceil(pz * py / 4), nshots).
__global__ void __launch_bounds__(256)
    k_background64(Bg64Args a, const Bg64Shot* tab, int n) {
  const Bg64Shot sd = tab[blockIdx.z];
  if (n >= sd.nt - 1) return;
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int row = blockIdx.y * 4 + threadIdx.y;
  const int py = a.ndim == 3 ? a.py : 1;
  if (x >= a.px || row >= a.pz * py) return;
  const int z = row / py, y = row - (row / py) * py;
  const int64_t sz = a.ndim == 3 ? a.plane : a.pitch;  // stride of z
  const int64_t i = (int64_t)(z + kGhost) * sz +
                    (a.ndim == 3 ? (int64_t)(y + kGhost) * a.pitch : 0) + x +
                    a.xoff;
  const double* u = sd.u[n & 1];
  const double c = u[i];
  // h^2 L u on differences, largest offset first
  double lap = 0.0;
  for (int k = 4; k >= 1; --k) {
    double t = (u[i + k * sz] - c) + (u[i - k * sz] - c);
    t += (u[i + k] - c) + (u[i - k] - c);
    if (a.ndim == 3)
      t += (u[i + k * (int64_t)a.pitch] - c) +
           (u[i - k * (int64_t)a.pitch] - c);
    lap = fma(a.w[k - 1], t, lap);
  }
  const bool src = z == sd.src_z && x == sd.src_x &&
                   (a.ndim != 3 || y == sd.src_y);
  const double inc = a.wp[i] * (lap + (src ? sd.wav[n] : 0.0));
  const int dz = depth(z, a.nb, a.nz), dx = depth(x, a.nb, a.nx);
  const int dy = a.ndim == 3 ? depth(y, a.nb, a.ny) : 0;
  const double damp = a.eta_scale * (double)(dz * dz + dx * dx + dy * dy);
  const double C1 = 1.0 / (1.0 + damp), C2 = (1.0 - damp) * C1;
  const double vn = C2 * sd.v[i] + C1 * inc;
  sd.v[i] = vn;
  sd.u[(n + 1) & 1][i] = c + vn;
  if (dz == 0 && dx == 0 && dy == 0) {
    const int64_t mi =
        ((int64_t)(z - a.nb) * (a.ndim == 3 ? a.ny : 1) +
         (a.ndim == 3 ? y - a.nb : 0)) * a.nx + (x - a.nb);
    sd.d2[(int64_t)n * a.mplane + mi] = (float)inc;
  }
}

// 2-D form: each thread marches one column down a chunk of kBgRows rows,
// keeping the column's nine u values the z-stencil needs in registers (one
// new row loaded per point), the x-neighbours read from the same row (the
// block's neighbouring columns: cache hits). Same arithmetic, in the same
// order, as k_background64.
constexpr int kBgRows = 32;

__global__ void __launch_bounds__(256)
    k_background64_2d(Bg64Args a, const Bg64Shot* tab, int n) {
  const Bg64Shot sd = tab[blockIdx.z];
  if (n >= sd.nt - 1) return;
  const int x = blockIdx.x * 256 + threadIdx.x;
  if (x >= a.px) return;
  const int z0 = blockIdx.y * kBgRows;
  const int z1 = min(z0 + kBgRows, a.pz);
  const int64_t sz = a.pitch;
  const double* u = sd.u[n & 1];
  double* uo = sd.u[(n + 1) & 1];
  const int dx = depth(x, a.nb, a.nx);
  const bool inx = dx == 0;
  // q[k]: u at row z - 4 + k, k = 0..8
  double q[9];
  int64_t i = (int64_t)(z0 + kGhost - 4) * sz + x + a.xoff;
#pragma unroll
  for (int k = 0; k < 8; ++k) q[k] = u[i + k * sz];
  i += 4 * sz;  // row z0
  for (int z = z0; z < z1; ++z, i += sz) {
    q[8] = u[i + 4 * sz];
    const double c = q[4];
    double lap = 0.0;
#pragma unroll
    for (int k = 4; k >= 1; --k) {
      double t = (q[4 + k] - c) + (q[4 - k] - c);
      t += (u[i + k] - c) + (u[i - k] - c);
      lap = fma(a.w[k - 1], t, lap);
    }
    const bool src = z == sd.src_z && x == sd.src_x;
    const double inc = a.wp[i] * (lap + (src ? sd.wav[n] : 0.0));
    const int dz = depth(z, a.nb, a.nz);
    const double damp = a.eta_scale * (double)(dz * dz + dx * dx);
    const double C1 = 1.0 / (1.0 + damp), C2 = (1.0 - damp) * C1;
    const double vn = C2 * sd.v[i] + C1 * inc;
    sd.v[i] = vn;
    uo[i] = c + vn;
    if (dz == 0 && inx)
      sd.d2[(int64_t)n * a.mplane + (int64_t)(z - a.nb) * a.nx + (x - a.nb)] =
          (float)inc;
#pragma unroll
    for (int k = 0; k < 8; ++k) q[k] = q[k + 1];
  }
}

hipError_t launch_background64(const Bg64Args& a, const Bg64Shot* tab,
                               int nshots, int n, hipStream_t st) {
  if (nshots <= 0) return hipSuccess;
  if (a.ndim == 2) {
    const dim3 grid((a.px + 255) / 256, (a.pz + kBgRows - 1) / kBgRows,
                    nshots);
    hipLaunchKernelGGL(k_background64_2d, grid, dim3(256), 0, st, a, tab, n);
    return hipGetLastError();
  }
  const int rows = a.pz * a.py;
  const dim3 grid((a.px + 63) / 64, (rows + 3) / 4, nshots);
  hipLaunchKernelGGL(k_background64, grid, dim3(64, 4), 0, st, a, tab, n);
  return hipGetLastError();
}

}  // namespace brls
