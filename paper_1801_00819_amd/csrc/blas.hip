// Vector kernels of the CG solver: fills, axpy-type updates and dot
// products of float32 vectors accumulated in float64, and the same for the
// solver's float64 vectors.
//
// Dot products run in two fixed-order stages (kDotBlocks per-block partial
// sums, then a single block), so a result does not depend on scheduling and
// repeated runs are bitwise identical.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "layout.h"

namespace brls {

__global__ void k_fill_f32(float* p, int64_t n, float v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_u32(unsigned* p, int64_t n, unsigned v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_f64(double* p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Block-wide float64 sum in LDS (256 threads), result in thread 0.
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[256];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  return red[0];
}

__global__ void __launch_bounds__(256)
    k_dot_partial(const float* a, const float* b, int64_t n, double* part) {
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    s += (double)a[i] * (double)b[i];
  const double t = block_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void __launch_bounds__(256)
    k_sum_final(const double* part, int np, double* out) {
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) s += part[i];
  const double t = block_sum(s);
  if (threadIdx.x == 0) out[0] = t;
}

__global__ void k_axpy(float* y, const float* x, double alpha, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (float)((double)y[i] + alpha * (double)x[i]);
}

__global__ void k_xpby(float* p, const float* s, double beta, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = (float)((double)s[i] + beta * (double)p[i]);
}

__global__ void k_sub(float* r, const float* d, const float* q, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    r[i] = d[i] - q[i];
}

__global__ void __launch_bounds__(256)
    k_grad_norm(float* s, const float* g, const float* m, double lambda,
                int64_t n, double* part) {
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float v = (float)((double)g[i] - lambda * (double)m[i]);
    s[i] = v;
    acc += (double)v * (double)v;
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void k_nonfinite(const float* x, int64_t n, int* flag) {
  int bad = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    bad |= !isfinite(x[i]);
  if (bad) atomicOr(flag, 1);
}

// out[i] = sum over frames f of x[f][i]^2 (float64 sum), x [nframes][n].
__global__ void k_sumsq_frames(const float* x, int64_t nframes, int64_t n,
                               float* out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    const float* p = x + i;
    for (int64_t f = 0; f < nframes; ++f, p += n) {
      const double v = (double)__builtin_nontemporal_load(p);
      acc += v * v;
    }
    out[i] = (float)acc;
  }
}

__global__ void k_mul(float* z, const float* a, const float* b, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    z[i] = a[i] * b[i];
}

__global__ void k_scale_segments(float* y, const float* x, const float* w,
                                 int64_t seg, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = w[i / seg] * x[i];
}

__global__ void k_recip_shift(float* y, const float* x, double shift,
                              int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (float)(1.0 / ((double)x[i] + shift));
}

__global__ void __launch_bounds__(256)
    k_sum_partial(const float* a, int64_t n, double* part) {
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    s += (double)a[i];
  const double t = block_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// ---- float64 CG vectors ----------------------------------------------------
#define GRID_STRIDE(i, n)                                                   \
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (n); \
       i += (int64_t)gridDim.x * blockDim.x)

__global__ void k_cvt_f2d(double* y, const float* x, int64_t n) {
  GRID_STRIDE(i, n) y[i] = (double)x[i];
}

__global__ void k_cvt_d2f(float* y, const double* x, const float* w,
                          int64_t seg, int64_t n) {
  if (w) {
    GRID_STRIDE(i, n) y[i] = (float)((double)w[i / seg] * x[i]);
  } else {
    GRID_STRIDE(i, n) y[i] = (float)x[i];
  }
}

__global__ void k_sub_d(double* r, const float* d, const float* q,
                        int64_t n) {
  GRID_STRIDE(i, n) r[i] = (double)d[i] - (double)q[i];
}

__global__ void k_axpy_dd(double* y, const double* x, double alpha,
                          int64_t n) {
  GRID_STRIDE(i, n) y[i] = fma(alpha, x[i], y[i]);
}

__global__ void k_axpy_df(double* y, const float* x, double alpha,
                          int64_t n) {
  GRID_STRIDE(i, n) y[i] = fma(alpha, (double)x[i], y[i]);
}

__global__ void k_xpby_d(double* p, const double* s, double beta,
                         int64_t n) {
  GRID_STRIDE(i, n) p[i] = fma(beta, p[i], s[i]);
}

__global__ void __launch_bounds__(256)
    k_grad_norm_d(double* s, const double* g, const double* m, double lambda,
                  int64_t n, double* part) {
  double acc = 0.0;
  GRID_STRIDE(i, n) {
    const double v = g[i] - lambda * m[i];
    s[i] = v;
    acc = fma(v, v, acc);
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void __launch_bounds__(256)
    k_dot_partial_d(const double* a, const double* b, int64_t n,
                    double* part) {
  double acc = 0.0;
  GRID_STRIDE(i, n) acc = fma(a[i], b[i], acc);
  const double t = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void k_mul_fd(double* z, const float* a, const double* b,
                         int64_t n) {
  GRID_STRIDE(i, n) z[i] = (double)a[i] * b[i];
}
#undef GRID_STRIDE

static int grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (int)b;
}

hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f32, dim3(grid_for(n)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned* p, int64_t n, unsigned v,
                           hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(n)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_dot(const float* a, const float* b, int64_t n,
                      double* partial, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_dot_partial, dim3(kDotBlocks), dim3(256), 0, st, a, b,
                     n, partial);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, st, partial,
                     kDotBlocks, out);
  return hipGetLastError();
}

hipError_t launch_axpy(float* y, const float* x, double alpha, int64_t n,
                       hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpy, dim3(grid_for(n)), dim3(256), 0, st, y, x, alpha,
                     n);
  return hipGetLastError();
}

hipError_t launch_xpby(float* p, const float* s, double beta, int64_t n,
                       hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_xpby, dim3(grid_for(n)), dim3(256), 0, st, p, s, beta,
                     n);
  return hipGetLastError();
}

hipError_t launch_sub(float* r, const float* d, const float* q, int64_t n,
                      hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sub, dim3(grid_for(n)), dim3(256), 0, st, r, d, q, n);
  return hipGetLastError();
}

hipError_t launch_grad_norm(float* s, const float* g, const float* m,
                            double lambda, int64_t n, double* partial,
                            double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_grad_norm, dim3(kDotBlocks), dim3(256), 0, st, s, g, m,
                     lambda, n, partial);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, st, partial,
                     kDotBlocks, out);
  return hipGetLastError();
}

hipError_t launch_sumsq_frames(const float* x, int64_t nframes, int64_t n,
                               float* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sumsq_frames, dim3(grid_for(n)), dim3(256), 0, st, x,
                     nframes, n, out);
  return hipGetLastError();
}

hipError_t launch_mul(float* z, const float* a, const float* b, int64_t n,
                      hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mul, dim3(grid_for(n)), dim3(256), 0, st, z, a, b, n);
  return hipGetLastError();
}

hipError_t launch_scale_segments(float* y, const float* x, const float* w,
                                 int64_t seg, int64_t n, hipStream_t st) {
  if (n <= 0 || seg <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale_segments, dim3(grid_for(n)), dim3(256), 0, st, y,
                     x, w, seg, n);
  return hipGetLastError();
}

hipError_t launch_recip_shift(float* y, const float* x, double shift,
                              int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_recip_shift, dim3(grid_for(n)), dim3(256), 0, st, y, x,
                     shift, n);
  return hipGetLastError();
}

hipError_t launch_sum(const float* x, int64_t n, double* partial, double* out,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_sum_partial, dim3(kDotBlocks), dim3(256), 0, st, x, n,
                     partial);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, st, partial,
                     kDotBlocks, out);
  return hipGetLastError();
}

hipError_t launch_nonfinite(const float* x, int64_t n, int* flag,
                            hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_nonfinite, dim3(grid_for(n)), dim3(256), 0, st, x, n,
                     flag);
  return hipGetLastError();
}

hipError_t launch_cvt_f2d(double* y, const float* x, int64_t n,
                          hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cvt_f2d, dim3(grid_for(n)), dim3(256), 0, st, y, x, n);
  return hipGetLastError();
}

hipError_t launch_cvt_d2f(float* y, const double* x, const float* w,
                          int64_t seg, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cvt_d2f, dim3(grid_for(n)), dim3(256), 0, st, y, x, w,
                     seg, n);
  return hipGetLastError();
}

hipError_t launch_sub_d(double* r, const float* d, const float* q, int64_t n,
                        hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sub_d, dim3(grid_for(n)), dim3(256), 0, st, r, d, q, n);
  return hipGetLastError();
}

hipError_t launch_axpy_dd(double* y, const double* x, double alpha, int64_t n,
                          hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpy_dd, dim3(grid_for(n)), dim3(256), 0, st, y, x,
                     alpha, n);
  return hipGetLastError();
}

hipError_t launch_axpy_df(double* y, const float* x, double alpha, int64_t n,
                          hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpy_df, dim3(grid_for(n)), dim3(256), 0, st, y, x,
                     alpha, n);
  return hipGetLastError();
}

hipError_t launch_xpby_d(double* p, const double* s, double beta, int64_t n,
                         hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_xpby_d, dim3(grid_for(n)), dim3(256), 0, st, p, s,
                     beta, n);
  return hipGetLastError();
}

hipError_t launch_grad_norm_d(double* s, const double* g, const double* m,
                              double lambda, int64_t n, double* partial,
                              double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_grad_norm_d, dim3(kDotBlocks), dim3(256), 0, st, s, g,
                     m, lambda, n, partial);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, st, partial,
                     kDotBlocks, out);
  return hipGetLastError();
}

hipError_t launch_dot_d(const double* a, const double* b, int64_t n,
                        double* partial, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_dot_partial_d, dim3(kDotBlocks), dim3(256), 0, st, a,
                     b, n, partial);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, st, partial,
                     kDotBlocks, out);
  return hipGetLastError();
}

hipError_t launch_mul_fd(double* z, const float* a, const double* b,
                         int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mul_fd, dim3(grid_for(n)), dim3(256), 0, st, z, a, b,
                     n);
  return hipGetLastError();
}

// dst[dat_off + (n + 1) nrec + r] = u^{n+1} at receiver r of every window
// shot with n + 1 < nt: the background level n + 1 sits in field b[(n+1)&1]
// (one-step kernels keep u of even and odd levels there; the two-step
// kernels' field set s holds its u in f[s], and a background launch writes
// set (n+1)&1).
__global__ void k_gather_receivers(const ShotDev* tab, int n, float* dst) {
  const ShotDev& s = tab[blockIdx.y];
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (n + 1 >= s.nt || r >= s.nrec) return;
  dst[s.dat_off + (int64_t)(n + 1) * s.nrec + r] =
      s.b[(n + 1) & 1][s.rsidx[r]];
}

hipError_t launch_gather_receivers(const ShotDev* tab, int nshots,
                                   int nrec_max, int n, float* dst,
                                   hipStream_t st) {
  if (nshots <= 0 || nrec_max <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_receivers, dim3((nrec_max + 255) / 256, nshots),
                     dim3(256), 0, st, tab, n, dst);
  return hipGetLastError();
}

}  // namespace brls
