// Device-side arguments and launchers of the split-step Fourier kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace brls {

// One window shot as the kernels see it.
struct SsfShotDev {
  int slot;   // storage slot: Born weights, receivers, data segment
  int xs;     // source column
  int nrec;   // receivers
};

struct SsfArgs {
  int nz;            // depth levels
  int log2n;         // log2 of the columns (the FFT length)
  int nw;            // frequencies
  int k0;            // DFT index of the first one
  double dw;         // 2 pi df (rad/s per DFT index)
  double dz;
  double kx_unit;    // 2 pi / (nx dx)
  int nrec_max;
  int64_t seg;       // floats per slot of a frequency-domain data vector
  const double* s0;     // [nz] reference slowness
  const double* theta;  // [nz][nx] split-step times (s)
  const float* tau;     // [nx] lateral taper
  const float2* tw;     // [nx] e^{-2 pi i m / nx}
  const double2* tw64;  // the same in double (source march)
  const double2* wav;   // [q_max][nw] source spectra
  float2* W;            // [q_max][nw][nz][nx] Born weights
  const float2* ptab;   // [nw][nz][nx] wavenumber-domain phase / nx
  const float2* sstab;  // [nw][nz][nx] split-step phase times taper
  const double2* ptab64;   // [nw][nz][nx] e^{-i kz dz} (source march)
  const double2* sstab64;  // [nw][nz][nx] e^{-i w theta} (source march)
  const int* rec;       // [q_max][nrec_max] receiver columns
  const int* colptr;    // [q_max][nx + 1] receivers per column (CSR)
  const int* cidx;      // [q_max][nrec_max] receiver index per CSR entry
  const SsfShotDev* tab;  // window shots
  int nshots;
};

// The phase tables of the medium (once per context): float ones for A and
// A^T, double ones for the source march.
hipError_t launch_ssf_tables(const SsfArgs& a, float2* ptab, float2* sstab,
                             double2* ptab64, double2* sstab64,
                             hipStream_t st);
// Born weights of the listed shots (slot and source column of each) for
// every frequency and level.
hipError_t launch_ssf_source(const SsfArgs& a, const SsfShotDev* pend,
                             int npend, hipStream_t st);
// d (slot layout) = A m over the window's shots.
hipError_t launch_ssf_born(const SsfArgs& a, const float* m, float* d,
                           hipStream_t st);
// Per-(shot, frequency) image contributions of A^T d, [items][nz][nx].
hipError_t launch_ssf_adjoint(const SsfArgs& a, const float* d, float* part,
                              hipStream_t st);
// out = the window's source illumination: sum over its shots and
// frequencies of |W_j(x)|^2 (float64 sums, fixed order).
hipError_t launch_ssf_illumination(const SsfArgs& a, float* out,
                                   hipStream_t st);
// img = sum over items of part in a fixed order (npts a multiple of 4;
// psum: kSsfSumGroups * npts doubles of scratch).
constexpr int kSsfSumGroups = 16;
hipError_t launch_ssf_image_sum(const float* part, int items, int64_t npts,
                                float* img, double* psum, hipStream_t st);
// X[k][r] (re, im) = sum_n x[n][r] e^{-i w_k n dt} dt for one shot.
hipError_t launch_ssf_data_dft(const float* x, int nt, int nrec, double dt,
                               int nw, int k0, double dw, float* X,
                               hipStream_t st);

}  // namespace brls
