// Host-side launchers of the library's kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "layout.h"

namespace brls {

struct TileShape {
  int tx, tz, ntz;  // tile width (x), tile height (z), thread rows
                    // (z-marching: rows of loads in flight ahead)
  int pipe;         // 0: staged tile; 1: staged, next shot's loads issued
                    // before computing the current; 2: z-marching; 3: two
                    // steps per launch, one chunk per work item; 4: two
                    // steps per launch, a segment of tz rows per wavefront
};

int tile_shape_count();
TileShape tile_shape(int variant);

struct TileShape3 {
  int tx, ty;  // XY tile (threads)
  int sb;      // shots per block, advanced together plane by plane
};
int tile_shape3_count();
TileShape3 tile_shape3(int variant);
hipError_t launch_step3d(int variant, int mode, const StepArgs& a,
                         hipStream_t st);
hipError_t launch_adj_finalize3(const double* acc, int ngroups,
                                const Geo3D& g, const float* wp, float* out,
                                double* out64, hipStream_t st);

// Blocks of `kernel` (launched with `threads` per block) that fit on the
// current device at once.
int resident_blocks(const void* kernel, int threads);

// z-marching 2-D step over chunks of cz rows (8, 12, 16 or 32), the loads of
// `ahead` rows (2 or 4) in flight ahead of the row computed.
hipError_t launch_march2d(int cz, int ahead, int mode, const StepArgs& a,
                          hipStream_t st);

// Two time steps per launch (a.nsub of them), 2-D, chunks of cz = 16 rows,
// the loads of `ahead` rows (2 or 4) in flight; background, Born and
// adjoint modes.
hipError_t launch_march2t(int cz, int ahead, int mode, const StepArgs& a,
                          hipStream_t st);

// Two time steps per launch, 2-D, a wavefront marching a segment of seg
// output rows (16, 20, 24 or 32) of a 56-column strip for one shot, the
// loads of `ahead` rows in flight; blocks of per_block wavefronts on one
// segment.
hipError_t launch_march2s(int seg, int ahead, int mode, const StepArgs& a,
                          hipStream_t st);

// Persistent form (Born and adjoint): one launch runs every two-step
// launch of an operator application in turn, with a grid barrier between
// them, on a grid no larger than what is resident at once.
struct PersistArgs {
  unsigned* counter;  // barrier arrivals; zero before the launch
  int* error;         // set to 1 when a barrier wait gave up
  int nlaunch;        // two-step launches
  int k_hi, k_lo;     // adjoint: output levels k_hi down to k_lo
  int nt_max;         // Born: input levels 0 .. nt_max - 2
  int spin_limit;     // polls before a barrier wait gives up
};
hipError_t launch_march2s_persistent(int seg, int ahead, int mode,
                                     const StepArgs& a, const PersistArgs& p,
                                     hipStream_t st);
// Blocks of the persistent kernel resident at once on the current device.
int march2s_persistent_capacity(int seg, int ahead, int mode, int per_block);
// Fill n unsigned ints with v (a kernel, so a graph can replay it).
hipError_t launch_fill_u32(unsigned* p, int64_t n, unsigned v,
                           hipStream_t st);

// One time step for all shots of `a` (mode: StepMode).
hipError_t launch_step2d(int variant, int mode, const StepArgs& a,
                         hipStream_t st);
// d^{nt-1} of every shot (two_step: the last level sits in field set
// ceil((nt-1)/2) mod 2, else (nt-1) mod 2).
hipError_t launch_born_last(const ShotDev* tab, int nshots, int nrec_max,
                            float* dat, int two_step, hipStream_t st);
// out (and out64 unless NULL) = sum of the accumulators / W' on the model
// region.
hipError_t launch_adj_finalize(const double* acc, int ngroups,
                               const Geo2D& g, const float* wp, float* out,
                               double* out64, hipStream_t st);
// Background checkpoint save (restore = 0) / restore (1) for all shots.
hipError_t launch_ckpt(const ShotDev* tab, int nshots, int n0, int seg,
                       int64_t fs, int restore, hipStream_t st);

// Vector kernels (blas.hip). Sums are accumulated in float64 in a fixed
// order (per-block partials, then one block), so results are deterministic.
constexpr int kDotBlocks = 1024;
hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t st);
hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t st);
// partial[0..kDotBlocks) of sum(a*b); then out[0] = sum(partial)
hipError_t launch_dot(const float* a, const float* b, int64_t n,
                      double* partial, double* out, hipStream_t st);
// y += alpha * x (alpha applied in float64)
hipError_t launch_axpy(float* y, const float* x, double alpha, int64_t n,
                       hipStream_t st);
// p = s + beta * p
hipError_t launch_xpby(float* p, const float* s, double beta, int64_t n,
                       hipStream_t st);
// r = d - q
hipError_t launch_sub(float* r, const float* d, const float* q, int64_t n,
                      hipStream_t st);
// s = g - lambda * m, and out[0] = ||s||^2 (float64)
hipError_t launch_grad_norm(float* s, const float* g, const float* m,
                            double lambda, int64_t n, double* partial,
                            double* out, hipStream_t st);
// out[i] = sum_f x[f][i]^2 over nframes frames of n floats (float64 sums)
hipError_t launch_sumsq_frames(const float* x, int64_t nframes, int64_t n,
                               float* out, hipStream_t st);
// z = a * b elementwise
hipError_t launch_mul(float* z, const float* a, const float* b, int64_t n,
                      hipStream_t st);
// y[i] = w[i / seg] * x[i]: one weight per data segment of seg floats
// (n a multiple of seg; y may alias x)
hipError_t launch_scale_segments(float* y, const float* x, const float* w,
                                 int64_t seg, int64_t n, hipStream_t st);
// y = 1 / (x + shift) (float64 arithmetic; y may alias x)
hipError_t launch_recip_shift(float* y, const float* x, double shift,
                              int64_t n, hipStream_t st);
// partial sums, then out[0] = sum(x) (float64, fixed order)
hipError_t launch_sum(const float* x, int64_t n, double* partial, double* out,
                      hipStream_t st);
// Receiver samples of background level n + 1 of every window shot into
// its segment of a data vector (see k_gather_receivers).
hipError_t launch_gather_receivers(const ShotDev* tab, int nshots,
                                   int nrec_max, int n, float* dst,
                                   hipStream_t st);
// Float64 background of shots entering the window (bg64.hip), stored-source
// strategy: per shot, u of even / odd levels and v in float64 on the
// wavefield storage layout, the float32 Born-source frames written on the
// model region.
struct Bg64Shot {
  double* u[2];        // u of even / odd levels
  double* v;           // u^n - u^{n-1}, updated in place
  float* d2;           // Born-source frames [nt - 1][model]
  const double* wav;   // h^2 * source wavelet [nt]
  int nt;
  int src_z, src_y, src_x;  // padded grid position of the source
};
struct Bg64Args {
  int ndim;
  int pz, py, px;      // padded grid (py = 1 in 2-D)
  int nz, ny, nx, nb;  // model grid, sponge width
  int pitch, xoff;     // storage row pitch and column of padded x = 0
  int64_t plane;       // 3-D: storage elements per z-plane
  int64_t mplane;      // model points (frame size)
  double eta_scale;    // eta_max * dt / 2 / nb^2
  double w[4];         // 8th-order weights of offsets 1..4
  const double* wp;    // W' = v^2 dt^2 / h^2, storage layout
};
// Advance level n -> n + 1 for every shot of tab with n < nt - 1 and store
// frame n.
hipError_t launch_background64(const Bg64Args& a, const Bg64Shot* tab,
                               int nshots, int n, hipStream_t st);

// Float64 CG vectors (blas.hip).
// y = (double)x
hipError_t launch_cvt_f2d(double* y, const float* x, int64_t n,
                          hipStream_t st);
// y = (float)x, or with w != NULL y[i] = (float)(w[i / seg] * x[i])
hipError_t launch_cvt_d2f(float* y, const double* x, const float* w,
                          int64_t seg, int64_t n, hipStream_t st);
// r = (double)d - (double)q
hipError_t launch_sub_d(double* r, const float* d, const float* q, int64_t n,
                        hipStream_t st);
// y += alpha * x
hipError_t launch_axpy_dd(double* y, const double* x, double alpha, int64_t n,
                          hipStream_t st);
hipError_t launch_axpy_df(double* y, const float* x, double alpha, int64_t n,
                          hipStream_t st);
// p = s + beta * p
hipError_t launch_xpby_d(double* p, const double* s, double beta, int64_t n,
                         hipStream_t st);
// s = g - lambda * m, and out[0] = ||s||^2
hipError_t launch_grad_norm_d(double* s, const double* g, const double* m,
                              double lambda, int64_t n, double* partial,
                              double* out, hipStream_t st);
// out[0] = sum a * b (fixed order)
hipError_t launch_dot_d(const double* a, const double* b, int64_t n,
                        double* partial, double* out, hipStream_t st);
// z = (double)a * b
hipError_t launch_mul_fd(double* z, const float* a, const double* b,
                         int64_t n, hipStream_t st);

// flag[0] = 1 if any entry of x is NaN or Inf (flag must start at 0)
hipError_t launch_nonfinite(const float* x, int64_t n, int* flag,
                            hipStream_t st);

}  // namespace brls
