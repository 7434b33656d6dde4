/*
 * brrlsm_ssf — the split-step Fourier shot-profile operator pair inside the
 * same block-row recursion, on MI355X (gfx950).
 *
 * The paper's examples (Kazemi & Sacchi, arXiv 1801.00819, Examples section)
 * use shot-profile wave-equation de-migration and migration with a
 * split-step correction as A and A^T, and give no formulas for them. This
 * context implements that family, defined as follows (2-D):
 *
 *   - grid: nz depth levels (spacing dz) by nx columns (spacing dx); nx is a
 *     power of two, the lateral FFT length, and includes the taper zone;
 *     slowness s = 1/v, reference slowness s0_j = row mean of s at level j,
 *     split-step time theta_j(x) = (s_j(x) - s0_j) dz;
 *   - frequencies: the DFT grid of nt samples at dt (df = 1/(nt dt))
 *     restricted to [fmin, fmax]: w_k = 2 pi (k0 + k) df, k = 0 .. nw-1,
 *     k0 = ceil(fmin/df); time series enter as X(w) = sum_n x_n e^{-i w n dt} dt;
 *   - one depth step E_j: FFT over x, times e^{-i kz dz} with
 *     kz = sqrt(w^2 s0_j^2 - kx^2) (e^{-|kz| dz} where evanescent), inverse
 *     FFT, times e^{-i w theta_j(x)}, times a lateral cosine taper of ntap
 *     cells per side (time runs as e^{+i w t}: every step adds traveltime);
 *   - source at column xs of level 0: S_0 = F(w) (-i / (2 w s)) there, F
 *     the spectrum of a Ricker wavelet (peak f0, delay 1.5/f0) and s the
 *     slowness at the source (the one-way form of a 2-D point source: the
 *     field below it is dx F times the outgoing Helmholtz Green's
 *     function); S_{j+1} = E_j S_j; Born weights
 *     W_j = -i (w dz/2) s_j S_j (first-order change of the split-step phase
 *     for a relative squared-slowness perturbation m);
 *   - A (de-migration, eq. 1): R_{nz-1} = W_{nz-1} m_{nz-1},
 *     R_j = W_j m_j + E_j R_{j+1}, data = R_0 at the receiver columns;
 *   - A^T (migration, eq. 2): the receivers' data placed in their columns,
 *     continued down by E_j^H; image_j = Re sum_w conj(W_j) Q_j (zero-lag
 *     cross-correlation imaging condition). It is the exact adjoint of A
 *     under the real inner product of the data's (re, im) pairs.
 *
 * Each window solves min ||A_w m - d_w||^2 + lambda ||m||^2 (eq. 10) by CG
 * on the least-squares form, warm-started from the previous image (eq. 11),
 * exactly as the finite-difference context does.
 *
 * Conventions (as in brrlsm.h): every function returns BRLS_OK or a negative
 * BRLS_E* code, the last message is in brls_ssf_last_error; images are
 * [nz][nx] float32; time-domain shot data are [nt][nrec] float32;
 * frequency-domain window data are, per shot in window order,
 * [nw][nrec][2] float32 (re, im); pointers to data and images are host
 * pointers unless the grid's flags hold BRLS_DEVICE_PTRS (then device
 * pointers valid on the context's stream); velocity and receiver lists are
 * host pointers; every input is copied at call time and the caller keeps
 * ownership. A context is bound to the current device and the given stream
 * and is not thread-safe.
 */
#ifndef BRRLSM_SSF_H
#define BRRLSM_SSF_H

#include "brrlsm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct brls_ssf_ctx brls_ssf_ctx;

typedef struct {
  int32_t nz, nx;     /* depth levels; columns, a power of two in [64, 2048] */
  double dx, dz;      /* spacings (m) */
  int32_t nt;         /* time samples of every shot's data, >= 2 */
  double dt;          /* sample interval (s) */
  double fmin, fmax;  /* frequency band (Hz), 0 < fmin <= fmax < 1/(2 dt) */
  int32_t ntap;       /* taper cells per lateral side, 0 <= ntap < nx/2 */
  int32_t nrec_max;   /* largest number of receivers of any shot */
  int32_t q_max;      /* largest number of shots held at once */
  double lambda;      /* damping of eq. 3, absolute */
  uint32_t flags;     /* BRLS_DEVICE_PTRS */
} brls_ssf_grid;

typedef struct {
  int64_t id;          /* caller's key, unique within the window */
  int32_t xs;          /* source column (level 0) */
  int32_t nrec;        /* 1 <= nrec <= nrec_max */
  double f0;           /* Ricker peak frequency (Hz), > 0 */
  const int32_t* rec;  /* host [nrec] receiver columns (level 0); repeats allowed */
  const float* data;   /* time-domain data [nt][nrec], or NULL for zeros */
} brls_ssf_shot;

/* Create a context. g: copied. vel: host [nz][nx] velocity (m/s), all > 0.
 * stream: hipStream_t to order work on, or NULL for a private stream.
 * Errors: BRLS_EINVAL (sizes, band, taper; nz * nx or nt * nrec_max of
 * 2^30 or more), BRLS_ENOMEM, BRLS_EDEVICE. */
int brls_ssf_open(const brls_ssf_grid* g, const float* vel, void* stream,
                  brls_ssf_ctx** out);
void brls_ssf_close(brls_ssf_ctx* ctx);
const char* brls_ssf_last_error(const brls_ssf_ctx* ctx);

/* The frequency band: first DFT index k0, count nw, spacing df (Hz). */
int brls_ssf_band(const brls_ssf_ctx* ctx, int32_t* k0, int32_t* nw,
                  double* df);

/* Rank-one update (the paper's window update after eq. 10, Fig. 1): add a
 * shot to the window. Transforms its data to the band; its Born weights W_j
 * for every level and frequency (nw*nz*nx complex floats) are built, with
 * those of every other shot added since, at the next application of A or
 * A^T (one launch for a whole slide).
 * Errors: BRLS_EFULL, BRLS_EDUP, BRLS_EINVAL (columns, sizes),
 * BRLS_ENONFINITE (data hold NaN/Inf). */
int brls_ssf_update(brls_ssf_ctx* ctx, const brls_ssf_shot* shot);

/* Rank-one downdate: remove a shot. Errors: BRLS_ENOSHOT. */
int brls_ssf_downdate(brls_ssf_ctx* ctx, int64_t id);

/* Window shot ids in window order; *n receives the count (ids may be NULL
 * when cap is 0). */
int brls_ssf_window(const brls_ssf_ctx* ctx, int64_t* ids, int32_t cap,
                    int32_t* n);

/* Floats of a frequency-domain window data vector: sum of 2*nw*nrec. */
int brls_ssf_window_data_size(const brls_ssf_ctx* ctx, int64_t* n);

/* d_out = A_w m (eq. 1) in the frequency-domain window layout. */
int brls_ssf_apply_born(brls_ssf_ctx* ctx, const float* m, float* d_out);

/* m_out = A_w^T d (eq. 2) for d in the frequency-domain window layout. */
int brls_ssf_apply_adjoint(brls_ssf_ctx* ctx, const float* d, float* m_out);

/* The window's observed data, as transformed at update, in the
 * frequency-domain window layout. */
int brls_ssf_observed(brls_ssf_ctx* ctx, float* d_out);

/* Damped CG on the window (eq. 10) from the current image (eq. 11): stops
 * after max_iter iterations or once ||A^T r - lambda m|| <= rtol ||A^T d||
 * (rtol <= 0: iteration count only). stats may be NULL.
 * Errors: BRLS_EBREAKDOWN, BRLS_ENONFINITE. */
int brls_ssf_solve_window(brls_ssf_ctx* ctx, int32_t max_iter, double rtol,
                          brls_stats* stats);

/* Preconditioner of the window CG (the paper asks each window for one,
 * after eq. 11, and names none): 0 none (default); 1 the diagonal
 * M = I + 0.01 mean(I), I the window's source illumination (below), the
 * search directions following M^{-1} s; the stop test stays on ||s||.
 * Other modes: BRLS_EINVAL. */
int brls_ssf_set_precond(brls_ssf_ctx* ctx, int32_t mode);
int brls_ssf_get_precond(const brls_ssf_ctx* ctx, int32_t* mode);

/* The window's source illumination [nz][nx]: at each point the sum over its
 * shots and frequencies of |W_j(x)|^2 (the diagonal of A^T A were the
 * receivers recording every column of the scatterer's own level).
 * out: host or device per flags. */
int brls_ssf_illumination(brls_ssf_ctx* ctx, float* out);

/* Damping of each window's solve (eq. 10, and the two readings of eq. 11):
 * 0 (default) lambda ||m||^2; 1 lambda ||m - m_start||^2, m_start the
 * image the solve starts from (the previous window's), which keeps the
 * memory of earlier windows. Other modes: BRLS_EINVAL. */
int brls_ssf_set_regularization(brls_ssf_ctx* ctx, int32_t mode);
int brls_ssf_get_regularization(const brls_ssf_ctx* ctx, int32_t* mode);

/* Misfit weight of one window shot (default 1, reset by brls_ssf_update),
 * as brls_set_shot_weight: the solve minimises
 * sum_j w_j ||A_j m - d_j||^2 + the damping term; w_j = beta^age gives the
 * exponentially weighted (forgetting-factor) window. Errors: BRLS_ENOSHOT;
 * BRLS_EINVAL for a negative or non-finite weight. */
int brls_ssf_set_shot_weight(brls_ssf_ctx* ctx, int64_t id, double w);
int brls_ssf_get_shot_weight(const brls_ssf_ctx* ctx, int64_t id, double* w);

/* Copy the current image out / set it (the next solve starts there). */
int brls_ssf_image(brls_ssf_ctx* ctx, float* out);
int brls_ssf_set_image(brls_ssf_ctx* ctx, const float* m);

/* Event timing of every kernel launch (off by default) and its summary:
 * families "ssf_data_dft", "ssf_source", "ssf_born", "ssf_adjoint",
 * "ssf_image_sum". Reading the summary clears it. */
int brls_ssf_kernel_timing(brls_ssf_ctx* ctx, int32_t enable);
int brls_ssf_kernel_stats(brls_ssf_ctx* ctx, brls_kstat* out, int32_t cap,
                          int32_t* n);

/* Device bytes held by the context. */
int brls_ssf_memory_bytes(const brls_ssf_ctx* ctx, int64_t* bytes);

/* Wait for all work on the context's stream. */
int brls_ssf_sync(brls_ssf_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* BRRLSM_SSF_H */
