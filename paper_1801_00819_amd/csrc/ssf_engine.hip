// Host engine and C ABI of the split-step Fourier context: tables of the
// medium, the window of shots (update / downdate with their Born weights),
// the operator pair over the window, and the damped CG solve of each window
// (eqs. 10-11 of Kazemi & Sacchi, arXiv 1801.00819), with the operator of
// the paper's examples as defined in brrlsm_ssf.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "brrlsm_ssf.h"
#include "kernels.h"
#include "ssf_kernels.h"

using namespace brls;

namespace {

thread_local std::string g_ssf_open_error;

struct SsfTimer {
  int kind;
  hipEvent_t a, b;
};

enum SsfTimerKind { kSDft, kSSource, kSBorn, kSAdjoint, kSSum, kSNumKinds };
const char* kSsfTimerNames[kSNumKinds] = {"ssf_data_dft", "ssf_source",
                                          "ssf_born", "ssf_adjoint",
                                          "ssf_image_sum"};

struct SsfSlot {
  bool used = false;
  bool w_ready = false;  // Born weights built
  int64_t id = 0;
  int xs = 0, nrec = 0;
  double f0 = 0.0;
  float weight = 1.f;  // the shot's misfit weight in the window CG
};

}  // namespace

struct brls_ssf_ctx {
  brls_ssf_grid g{};
  hipStream_t st = nullptr;
  bool own_stream = false;
  int log2n = 0, N = 0, nz = 0;
  int k0 = 0, nw = 0;
  double df = 0.0;
  int64_t M = 0;      // model points nz * nx
  std::vector<double> slow0;  // slowness of the top level (sources)
  // band spectra of the Ricker wavelet, by peak frequency
  std::map<double, std::vector<double2>> ricker_spectra;
  int64_t seg = 0;    // floats per slot of a data vector: 2 nw nrec_max
  SsfArgs args{};
  // medium tables
  double *s0 = nullptr, *theta = nullptr;
  float* tau = nullptr;
  float2* tw = nullptr;
  double2* tw64 = nullptr;
  // per slot
  float2* W = nullptr;
  double2* wav = nullptr;
  float2 *ptab = nullptr, *sstab = nullptr;  // phase tables
  double2 *ptab64 = nullptr, *sstab64 = nullptr;  // the same in double
  int *rec = nullptr, *colptr = nullptr, *cidx = nullptr;
  SsfShotDev* tab = nullptr;
  SsfShotDev* pend = nullptr;  // shots whose Born weights are pending
  bool tab_dirty = true;
  // vectors
  float* part = nullptr;
  float *m = nullptr, *p = nullptr, *s = nullptr, *gbuf = nullptr,
        *min = nullptr;
  int precond = 0;     // 1: diagonal illumination preconditioner
  int regularize = 0;  // 1: damp the correction to the starting image
  float *minv = nullptr, *z = nullptr, *dm = nullptr;
  float* wslot = nullptr;      // [q_max] per-slot misfit weights (device)
  std::vector<float> wslot_h;  // their host copy, uploaded by the solve
  float *dobs = nullptr, *r = nullptr, *q = nullptr, *dscr = nullptr,
        *dtime = nullptr;
  double *partial = nullptr, *scal = nullptr;
  double* psum = nullptr;  // image-sum partials
  int* flag = nullptr;
  std::vector<SsfSlot> slots;
  std::vector<int> order;
  std::string err;
  bool timing = false;
  std::vector<SsfTimer> timers;
  int64_t mem_bytes = 0;
  std::vector<void*> allocs;
};

namespace {

int sfail(brls_ssf_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c)
    c->err = buf;
  else
    g_ssf_open_error = buf;
  return code;
}

#define SCHECK(ctx, call)                                                    \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess)                                                    \
      return sfail(ctx, BRLS_EDEVICE, "%s: %s (%s:%d)", #call,               \
                   hipGetErrorString(e_), __FILE__, __LINE__);               \
  } while (0)

template <class T>
int salloc(brls_ssf_ctx* c, T** p, int64_t count) {
  *p = nullptr;
  if (count <= 0) count = 1;
  const size_t bytes = (size_t)count * sizeof(T);
  if (hipMalloc((void**)p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return sfail(c, BRLS_ENOMEM, "device allocation of %zu bytes failed",
                 bytes);
  }
  c->allocs.push_back(*p);
  c->mem_bytes += (int64_t)bytes;
  return BRLS_OK;
}

bool dev_ptrs(const brls_ssf_ctx* c) { return c->g.flags & BRLS_DEVICE_PTRS; }
hipMemcpyKind in_kind(const brls_ssf_ctx* c) {
  return dev_ptrs(c) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
}
hipMemcpyKind out_kind(const brls_ssf_ctx* c) {
  return dev_ptrs(c) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
}

int timed_begin(brls_ssf_ctx* c, int kind, SsfTimer* t) {
  if (!c->timing) return BRLS_OK;
  t->kind = kind;
  SCHECK(c, hipEventCreate(&t->a));
  SCHECK(c, hipEventCreate(&t->b));
  SCHECK(c, hipEventRecord(t->a, c->st));
  return BRLS_OK;
}
int timed_end(brls_ssf_ctx* c, SsfTimer* t) {
  if (!c->timing) return BRLS_OK;
  SCHECK(c, hipEventRecord(t->b, c->st));
  c->timers.push_back(*t);
  return BRLS_OK;
}

// Ricker wavelet of peak f0 delayed by 1.5 / f0.
double ricker(double t, double f0) {
  const double a = M_PI * f0 * (t - 1.5 / f0);
  return (1.0 - 2.0 * a * a) * std::exp(-a * a);
}

int find_slot(const brls_ssf_ctx* c, int64_t id) {
  for (int i = 0; i < (int)c->slots.size(); ++i)
    if (c->slots[i].used && c->slots[i].id == id) return i;
  return -1;
}

int read_scalars(brls_ssf_ctx* c, double* out, int n) {
  SCHECK(c, hipMemcpyAsync(out, c->scal, sizeof(double) * n,
                           hipMemcpyDeviceToHost, c->st));
  SCHECK(c, hipStreamSynchronize(c->st));
  return BRLS_OK;
}

// Born weights of every window shot added since the last application, in
// one launch (a slide adds several shots; one launch keeps the chip full).
int ensure_weights(brls_ssf_ctx* c) {
  std::vector<SsfShotDev> h;
  for (int sidx : c->order)
    if (!c->slots[sidx].w_ready)
      h.push_back(SsfShotDev{sidx, c->slots[sidx].xs, c->slots[sidx].nrec});
  if (h.empty()) return BRLS_OK;
  SCHECK(c, hipMemcpyAsync(c->pend, h.data(), h.size() * sizeof(SsfShotDev),
                           hipMemcpyHostToDevice, c->st));
  int rc;
  SsfTimer t{};
  if ((rc = timed_begin(c, kSSource, &t))) return rc;
  SCHECK(c, launch_ssf_source(c->args, c->pend, (int)h.size(), c->st));
  if ((rc = timed_end(c, &t))) return rc;
  // the pending list must be on the device before the host vector goes
  SCHECK(c, hipStreamSynchronize(c->st));
  for (const auto& e : h) c->slots[e.slot].w_ready = true;
  return BRLS_OK;
}

int ensure_tab(brls_ssf_ctx* c) {
  int rc;
  if ((rc = ensure_weights(c))) return rc;
  if (!c->tab_dirty) return BRLS_OK;
  std::vector<SsfShotDev> h;
  for (int sidx : c->order) {
    const SsfSlot& sl = c->slots[sidx];
    h.push_back(SsfShotDev{sidx, sl.xs, sl.nrec});
  }
  if (!h.empty())
    SCHECK(c, hipMemcpyAsync(c->tab, h.data(), h.size() * sizeof(SsfShotDev),
                             hipMemcpyHostToDevice, c->st));
  // the table must be on the device before the host vector goes away
  SCHECK(c, hipStreamSynchronize(c->st));
  c->args.tab = c->tab;
  c->args.nshots = (int)h.size();
  c->tab_dirty = false;
  return BRLS_OK;
}

// q (slot layout) = A m
int born_of(brls_ssf_ctx* c, const float* m_dev) {
  int rc;
  if ((rc = ensure_tab(c))) return rc;
  SsfTimer t{};
  if ((rc = timed_begin(c, kSBorn, &t))) return rc;
  SCHECK(c, launch_ssf_born(c->args, m_dev, c->q, c->st));
  return timed_end(c, &t);
}

// gbuf = A^T d (d in slot layout)
int adjoint_of(brls_ssf_ctx* c, const float* d_dev) {
  int rc;
  if ((rc = ensure_tab(c))) return rc;
  SsfTimer t{};
  if ((rc = timed_begin(c, kSAdjoint, &t))) return rc;
  SCHECK(c, launch_ssf_adjoint(c->args, d_dev, c->part, c->st));
  if ((rc = timed_end(c, &t))) return rc;
  if ((rc = timed_begin(c, kSSum, &t))) return rc;
  SCHECK(c, launch_ssf_image_sum(c->part, c->args.nshots * c->nw, c->M,
                                 c->gbuf, c->psum, c->st));
  return timed_end(c, &t);
}

// Stabiliser of the illumination preconditioner, relative to its mean.
constexpr double kIllumEps = 0.01;

int window_illumination(brls_ssf_ctx* c, float* out) {
  int rc;
  if ((rc = ensure_tab(c))) return rc;
  SCHECK(c, launch_ssf_illumination(c->args, out, c->st));
  return BRLS_OK;
}

// minv = 1 / (I + kIllumEps * mean(I)), I the window illumination.
int build_minv(brls_ssf_ctx* c) {
  int rc;
  if ((rc = window_illumination(c, c->minv))) return rc;
  SCHECK(c, launch_sum(c->minv, c->M, c->partial, c->scal, c->st));
  double sum = 0.0;
  if ((rc = read_scalars(c, &sum, 1))) return rc;
  const double shift = kIllumEps * sum / (double)c->M;
  if (!(shift > 0.0))
    return sfail(c, BRLS_EBREAKDOWN,
                 "preconditioner: the window's shots illuminate nothing");
  SCHECK(c, launch_recip_shift(c->minv, c->minv, shift, c->M, c->st));
  return BRLS_OK;
}

int64_t shot_floats(const brls_ssf_ctx* c, int slot) {
  return 2LL * c->nw * c->slots[slot].nrec;
}

// window layout (shots packed in window order) <-> slot layout
int to_slots(brls_ssf_ctx* c, const float* win, float* slots, hipMemcpyKind k) {
  int64_t off = 0;
  for (int sidx : c->order) {
    const int64_t n = shot_floats(c, sidx);
    SCHECK(c, hipMemcpyAsync(slots + (int64_t)sidx * c->seg, win + off,
                             n * 4, k, c->st));
    off += n;
  }
  return BRLS_OK;
}
int from_slots(brls_ssf_ctx* c, const float* slots, float* win,
               hipMemcpyKind k) {
  int64_t off = 0;
  for (int sidx : c->order) {
    const int64_t n = shot_floats(c, sidx);
    SCHECK(c, hipMemcpyAsync(win + off, slots + (int64_t)sidx * c->seg,
                             n * 4, k, c->st));
    off += n;
  }
  if (k == hipMemcpyDeviceToHost) SCHECK(c, hipStreamSynchronize(c->st));
  return BRLS_OK;
}

int zero_slot(brls_ssf_ctx* c, int sidx) {
  for (float* v : {c->dobs, c->r, c->q, c->dscr})
    SCHECK(c, launch_fill_f32(v + (int64_t)sidx * c->seg, c->seg, 0.f,
                              c->st));
  return BRLS_OK;
}

void release(brls_ssf_ctx* c) {
  for (auto& t : c->timers) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  if (c->st) (void)hipStreamSynchronize(c->st);
  for (void* p : c->allocs) (void)hipFree(p);
  if (c->own_stream && c->st) (void)hipStreamDestroy(c->st);
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int brls_ssf_open(const brls_ssf_grid* gin, const float* vel, void* stream,
                  brls_ssf_ctx** out) {
  if (!out) return BRLS_EINVAL;
  *out = nullptr;
  g_ssf_open_error.clear();
  if (!gin || !vel) return sfail(nullptr, BRLS_EINVAL, "NULL argument");
  const brls_ssf_grid g = *gin;
  int log2n = 0;
  while ((1 << log2n) < g.nx) ++log2n;
  if (g.nx < 64 || g.nx > 2048 || (1 << log2n) != g.nx)
    return sfail(nullptr, BRLS_EINVAL,
                 "nx = %d: must be a power of two in [64, 2048]", g.nx);
  if (g.nz < 1) return sfail(nullptr, BRLS_EINVAL, "nz = %d", g.nz);
  if (!(g.dx > 0) || !(g.dz > 0) || !(g.dt > 0) || g.nt < 2)
    return sfail(nullptr, BRLS_EINVAL, "spacings and nt must be positive");
  if (g.ntap < 0 || 2 * g.ntap >= g.nx)
    return sfail(nullptr, BRLS_EINVAL, "ntap = %d outside [0, nx/2)", g.ntap);
  if (g.q_max < 1 || g.nrec_max < 1)
    return sfail(nullptr, BRLS_EINVAL, "q_max and nrec_max must be >= 1");
  if (!(g.lambda >= 0)) return sfail(nullptr, BRLS_EINVAL, "lambda < 0");
  const double df = 1.0 / (g.nt * g.dt);
  if (!(g.fmin > 0) || !(g.fmax >= g.fmin) || !(g.fmax < 0.5 / g.dt))
    return sfail(nullptr, BRLS_EINVAL,
                 "band [%g, %g] Hz must satisfy 0 < fmin <= fmax < %g",
                 g.fmin, g.fmax, 0.5 / g.dt);
  const int k0 = (int)std::ceil(g.fmin / df - 1e-9);
  const int k1 = (int)std::floor(g.fmax / df + 1e-9);
  if (k1 < k0)
    return sfail(nullptr, BRLS_EINVAL, "no DFT frequency in [%g, %g] Hz",
                 g.fmin, g.fmax);
  const int64_t M = (int64_t)g.nz * g.nx;
  if (M >= ((int64_t)1 << 30) || (int64_t)g.nt * g.nrec_max > ((int64_t)1 << 30))
    return sfail(nullptr, BRLS_EINVAL,
                 "nz * nx and nt * nrec_max must stay below 2^30");
  for (int64_t i = 0; i < M; ++i)
    if (!(vel[i] > 0.f) || !std::isfinite(vel[i]))
      return sfail(nullptr, BRLS_EINVAL, "velocity must be positive and finite");

  auto* c = new brls_ssf_ctx();
  c->g = g;
  c->log2n = log2n;
  c->N = g.nx;
  c->nz = g.nz;
  c->k0 = k0;
  c->nw = k1 - k0 + 1;
  c->df = df;
  c->M = M;
  c->seg = 2LL * c->nw * g.nrec_max;
  c->slots.resize(g.q_max);
  int rc = BRLS_OK;
  auto bail = [&](int code) {
    g_ssf_open_error = c->err;
    release(c);
    delete c;
    return code;
  };
  if (stream) {
    c->st = (hipStream_t)stream;
  } else {
    if (hipStreamCreate(&c->st) != hipSuccess)
      return bail(sfail(c, BRLS_EDEVICE, "hipStreamCreate failed"));
    c->own_stream = true;
  }
  const int N = c->N, nz = c->nz;
  // medium tables (double where they feed phase angles)
  std::vector<double> s0(nz), theta(M);
  std::vector<float> tau(N, 1.f);
  std::vector<float2> tw(N);
  std::vector<double2> tw64(N);
  c->slow0.resize(N);
  for (int x = 0; x < N; ++x) c->slow0[x] = 1.0 / (double)vel[x];
  for (int j = 0; j < nz; ++j) {
    double sum = 0.0;
    for (int x = 0; x < N; ++x) sum += 1.0 / (double)vel[(int64_t)j * N + x];
    s0[j] = sum / N;
    for (int x = 0; x < N; ++x) {
      const double sv = 1.0 / (double)vel[(int64_t)j * N + x];
      theta[(int64_t)j * N + x] = (sv - s0[j]) * g.dz;
    }
  }
  for (int d = 0; d < g.ntap; ++d) {
    const float v =
        (float)(0.5 * (1.0 - std::cos(M_PI * (d + 1) / (g.ntap + 1.0))));
    tau[d] = std::min(tau[d], v);
    tau[N - 1 - d] = std::min(tau[N - 1 - d], v);
  }
  for (int m = 0; m < N; ++m) {
    const double a = -2.0 * M_PI * m / N;
    tw64[m] = make_double2(std::cos(a), std::sin(a));
    tw[m] = make_float2((float)tw64[m].x, (float)tw64[m].y);
  }
  const int64_t items = (int64_t)g.q_max * c->nw;
  const int64_t D = (int64_t)g.q_max * c->seg;
  if ((rc = salloc(c, &c->s0, nz)) || (rc = salloc(c, &c->theta, M)) ||
      (rc = salloc(c, &c->tau, N)) || (rc = salloc(c, &c->tw, N)) ||
      (rc = salloc(c, &c->tw64, N)) ||
      (rc = salloc(c, &c->W, items * M)) ||
      (rc = salloc(c, &c->ptab, (int64_t)c->nw * M)) ||
      (rc = salloc(c, &c->sstab, (int64_t)c->nw * M)) ||
      (rc = salloc(c, &c->ptab64, (int64_t)c->nw * M)) ||
      (rc = salloc(c, &c->sstab64, (int64_t)c->nw * M)) ||
      (rc = salloc(c, &c->wav, items)) ||
      (rc = salloc(c, &c->rec, (int64_t)g.q_max * g.nrec_max)) ||
      (rc = salloc(c, &c->colptr, (int64_t)g.q_max * (N + 1))) ||
      (rc = salloc(c, &c->cidx, (int64_t)g.q_max * g.nrec_max)) ||
      (rc = salloc(c, &c->tab, g.q_max)) ||
      (rc = salloc(c, &c->pend, g.q_max)) ||
      (rc = salloc(c, &c->part, items * M)) || (rc = salloc(c, &c->m, M)) ||
      (rc = salloc(c, &c->p, M)) || (rc = salloc(c, &c->s, M)) ||
      (rc = salloc(c, &c->gbuf, M)) || (rc = salloc(c, &c->min, M)) ||
      (rc = salloc(c, &c->minv, M)) || (rc = salloc(c, &c->z, M)) ||
      (rc = salloc(c, &c->dm, M)) ||
      (rc = salloc(c, &c->dobs, D)) || (rc = salloc(c, &c->r, D)) ||
      (rc = salloc(c, &c->q, D)) || (rc = salloc(c, &c->dscr, D)) ||
      (rc = salloc(c, &c->wslot, (int64_t)g.q_max)) ||
      (rc = salloc(c, &c->dtime, (int64_t)g.nt * g.nrec_max)) ||
      (rc = salloc(c, &c->partial, kDotBlocks)) ||
      (rc = salloc(c, &c->scal, 4)) || (rc = salloc(c, &c->flag, 1)) ||
      (rc = salloc(c, &c->psum, kSsfSumGroups * M)))
    return bail(rc);
  auto up = [&](void* dst, const void* src, size_t bytes) {
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->st);
  };
  if (up(c->s0, s0.data(), nz * 8) != hipSuccess ||
      up(c->theta, theta.data(), M * 8) != hipSuccess ||
      up(c->tau, tau.data(), N * 4) != hipSuccess ||
      up(c->tw, tw.data(), N * 8) != hipSuccess ||
      up(c->tw64, tw64.data(), N * 16) != hipSuccess ||
      launch_fill_f32(c->m, M, 0.f, c->st) != hipSuccess ||
      launch_fill_f32(c->dobs, D, 0.f, c->st) != hipSuccess ||
      launch_fill_f32(c->r, D, 0.f, c->st) != hipSuccess ||
      launch_fill_f32(c->q, D, 0.f, c->st) != hipSuccess ||
      launch_fill_f32(c->dscr, D, 0.f, c->st) != hipSuccess ||
      hipStreamSynchronize(c->st) != hipSuccess)
    return bail(sfail(c, BRLS_EDEVICE, "upload of the medium tables failed"));
  SsfArgs& a = c->args;
  a.nz = nz;
  a.log2n = log2n;
  a.nw = c->nw;
  a.k0 = k0;
  a.dw = 2.0 * M_PI * df;
  a.dz = g.dz;
  a.kx_unit = 2.0 * M_PI / (N * g.dx);
  a.nrec_max = g.nrec_max;
  a.seg = c->seg;
  a.s0 = c->s0;
  a.theta = c->theta;
  a.tau = c->tau;
  a.tw = c->tw;
  a.tw64 = c->tw64;
  a.wav = c->wav;
  a.W = c->W;
  a.rec = c->rec;
  a.colptr = c->colptr;
  a.cidx = c->cidx;
  a.tab = c->tab;
  a.nshots = 0;
  a.ptab = c->ptab;
  a.sstab = c->sstab;
  a.ptab64 = c->ptab64;
  a.sstab64 = c->sstab64;
  if (launch_ssf_tables(a, c->ptab, c->sstab, c->ptab64, c->sstab64,
                        c->st) != hipSuccess ||
      hipStreamSynchronize(c->st) != hipSuccess)
    return bail(sfail(c, BRLS_EDEVICE, "building the phase tables failed"));
  *out = c;
  return BRLS_OK;
}

void brls_ssf_close(brls_ssf_ctx* c) {
  if (!c) return;
  release(c);
  delete c;
}

const char* brls_ssf_last_error(const brls_ssf_ctx* c) {
  return c ? c->err.c_str() : g_ssf_open_error.c_str();
}

int brls_ssf_band(const brls_ssf_ctx* c, int32_t* k0, int32_t* nw,
                  double* df) {
  if (!c) return BRLS_EINVAL;
  if (k0) *k0 = c->k0;
  if (nw) *nw = c->nw;
  if (df) *df = c->df;
  return BRLS_OK;
}

int brls_ssf_update(brls_ssf_ctx* c, const brls_ssf_shot* sh) {
  if (!c || !sh) return BRLS_EINVAL;
  if (find_slot(c, sh->id) >= 0)
    return sfail(c, BRLS_EDUP, "shot %lld is already in the window",
                 (long long)sh->id);
  int sidx = -1;
  for (int i = 0; i < (int)c->slots.size(); ++i)
    if (!c->slots[i].used) {
      sidx = i;
      break;
    }
  if (sidx < 0)
    return sfail(c, BRLS_EFULL, "window already holds q_max = %d shots",
                 c->g.q_max);
  const int N = c->N;
  if (sh->xs < 0 || sh->xs >= N)
    return sfail(c, BRLS_EINVAL, "source column %d outside [0, %d)", sh->xs,
                 N);
  if (sh->nrec < 1 || sh->nrec > c->g.nrec_max || !sh->rec)
    return sfail(c, BRLS_EINVAL, "nrec = %d outside [1, %d]", sh->nrec,
                 c->g.nrec_max);
  if (!(sh->f0 > 0))
    return sfail(c, BRLS_EINVAL, "f0 must be positive");
  std::vector<int> rec(sh->rec, sh->rec + sh->nrec);
  for (int v : rec)
    if (v < 0 || v >= N)
      return sfail(c, BRLS_EINVAL, "receiver column %d outside [0, %d)", v,
                   N);
  // receivers per column, in receiver order
  std::vector<int> colptr(N + 1, 0), cidx(sh->nrec);
  for (int v : rec) colptr[v + 1]++;
  for (int x = 0; x < N; ++x) colptr[x + 1] += colptr[x];
  {
    std::vector<int> fill(colptr.begin(), colptr.end() - 1);
    for (int i = 0; i < sh->nrec; ++i) cidx[fill[rec[i]]++] = i;
  }
  // source spectrum: the DFT of the sampled Ricker over the band (the
  // kernel e^{-i w n dt} advanced by rotation, exact every 64 samples; kept
  // per peak frequency), times -i / (2 w s) at the source: the one-way form
  // of a 2-D point source
  const int nt = c->g.nt;
  const double dt = c->g.dt;
  auto it = c->ricker_spectra.find(sh->f0);
  if (it == c->ricker_spectra.end()) {
    std::vector<double2> F(c->nw);
    std::vector<double> f(nt);
    for (int n = 0; n < nt; ++n) f[n] = ricker(n * dt, sh->f0);
    for (int k = 0; k < c->nw; ++k) {
      const double w = 2.0 * M_PI * (c->k0 + k) * c->df;
      const double rc = std::cos(w * dt), rs = -std::sin(w * dt);
      double re = 0.0, im = 0.0;
      for (int n0 = 0; n0 < nt; n0 += 64) {
        double ec = std::cos(w * dt * n0), es = -std::sin(w * dt * n0);
        const int n1 = std::min(nt, n0 + 64);
        for (int n = n0; n < n1; ++n) {
          re += f[n] * ec;
          im += f[n] * es;
          const double t = ec * rc - es * rs;
          es = ec * rs + es * rc;
          ec = t;
        }
      }
      F[k] = make_double2(re * dt, im * dt);
    }
    it = c->ricker_spectra.emplace(sh->f0, std::move(F)).first;
  }
  std::vector<double2> wav(c->nw);
  for (int k = 0; k < c->nw; ++k) {
    const double w = 2.0 * M_PI * (c->k0 + k) * c->df;
    // (re + i im) (-i / (2 w s)) = (im, -re) / (2 w s)
    const double g = 1.0 / (2.0 * w * c->slow0[sh->xs]);
    wav[k] = make_double2(it->second[k].y * g, -it->second[k].x * g);
  }
  int rc;
  if ((rc = zero_slot(c, sidx))) return rc;
  SCHECK(c, hipMemcpyAsync(c->rec + (int64_t)sidx * c->g.nrec_max, rec.data(),
                           rec.size() * 4, hipMemcpyHostToDevice, c->st));
  SCHECK(c, hipMemcpyAsync(c->colptr + (int64_t)sidx * (N + 1), colptr.data(),
                           (N + 1) * 4, hipMemcpyHostToDevice, c->st));
  SCHECK(c, hipMemcpyAsync(c->cidx + (int64_t)sidx * c->g.nrec_max,
                           cidx.data(), cidx.size() * 4,
                           hipMemcpyHostToDevice, c->st));
  SCHECK(c, hipMemcpyAsync(c->wav + (int64_t)sidx * c->nw, wav.data(),
                           wav.size() * 16, hipMemcpyHostToDevice, c->st));
  if (sh->data) {
    const int64_t n = (int64_t)nt * sh->nrec;
    SCHECK(c, hipMemcpyAsync(c->dtime, sh->data, n * 4, in_kind(c), c->st));
    SCHECK(c, hipMemsetAsync(c->flag, 0, sizeof(int), c->st));
    SCHECK(c, launch_nonfinite(c->dtime, n, c->flag, c->st));
    int h = 0;
    SCHECK(c, hipMemcpyAsync(&h, c->flag, sizeof(int), hipMemcpyDeviceToHost,
                             c->st));
    SCHECK(c, hipStreamSynchronize(c->st));
    if (h) return sfail(c, BRLS_ENONFINITE, "shot data hold NaN or Inf");
    SsfTimer t{};
    if ((rc = timed_begin(c, kSDft, &t))) return rc;
    SCHECK(c, launch_ssf_data_dft(c->dtime, nt, sh->nrec, dt, c->nw, c->k0,
                                  2.0 * M_PI * c->df,
                                  c->dobs + (int64_t)sidx * c->seg, c->st));
    if ((rc = timed_end(c, &t))) return rc;
  }
  // the host vectors above must outlive the asynchronous copies
  SCHECK(c, hipStreamSynchronize(c->st));
  SsfSlot& sl = c->slots[sidx];
  sl.used = true;
  sl.weight = 1.f;
  sl.w_ready = false;
  sl.id = sh->id;
  sl.xs = sh->xs;
  sl.nrec = sh->nrec;
  sl.f0 = sh->f0;
  c->order.push_back(sidx);
  c->tab_dirty = true;
  return BRLS_OK;
}

int brls_ssf_downdate(brls_ssf_ctx* c, int64_t id) {
  if (!c) return BRLS_EINVAL;
  const int sidx = find_slot(c, id);
  if (sidx < 0)
    return sfail(c, BRLS_ENOSHOT, "no shot %lld in the window",
                 (long long)id);
  c->slots[sidx].used = false;
  c->order.erase(std::find(c->order.begin(), c->order.end(), sidx));
  c->tab_dirty = true;
  return zero_slot(c, sidx);
}

int brls_ssf_window(const brls_ssf_ctx* c, int64_t* ids, int32_t cap,
                    int32_t* n) {
  if (!c || !n) return BRLS_EINVAL;
  *n = (int32_t)c->order.size();
  for (int i = 0; i < (int)c->order.size() && i < cap && ids; ++i)
    ids[i] = c->slots[c->order[i]].id;
  return BRLS_OK;
}

int brls_ssf_window_data_size(const brls_ssf_ctx* c, int64_t* n) {
  if (!c || !n) return BRLS_EINVAL;
  int64_t t = 0;
  for (int sidx : c->order) t += shot_floats(c, sidx);
  *n = t;
  return BRLS_OK;
}

int brls_ssf_apply_born(brls_ssf_ctx* c, const float* m, float* d_out) {
  if (!c || !m || !d_out) return sfail(c, BRLS_EINVAL, "NULL argument");
  int rc;
  SCHECK(c, hipMemcpyAsync(c->min, m, c->M * 4, in_kind(c), c->st));
  if ((rc = born_of(c, c->min))) return rc;
  return from_slots(c, c->q, d_out, out_kind(c));
}

int brls_ssf_apply_adjoint(brls_ssf_ctx* c, const float* d, float* m_out) {
  if (!c || !d || !m_out) return sfail(c, BRLS_EINVAL, "NULL argument");
  int rc;
  if ((rc = to_slots(c, d, c->dscr, in_kind(c)))) return rc;
  if ((rc = adjoint_of(c, c->dscr))) return rc;
  SCHECK(c, hipMemcpyAsync(m_out, c->gbuf, c->M * 4, out_kind(c), c->st));
  if (!dev_ptrs(c)) SCHECK(c, hipStreamSynchronize(c->st));
  return BRLS_OK;
}

int brls_ssf_observed(brls_ssf_ctx* c, float* d_out) {
  if (!c || !d_out) return sfail(c, BRLS_EINVAL, "NULL argument");
  return from_slots(c, c->dobs, d_out, out_kind(c));
}

int brls_ssf_solve_window(brls_ssf_ctx* c, int32_t max_iter, double rtol,
                          brls_stats* stats) {
  if (!c) return BRLS_EINVAL;
  const auto t_start = std::chrono::steady_clock::now();
  brls_stats st{};
  auto finish = [&](int code) {
    st.seconds = std::chrono::duration<double>(
                     std::chrono::steady_clock::now() - t_start)
                     .count();
    if (stats) *stats = st;
    return code;
  };
  if (c->order.empty()) return finish(BRLS_OK);
  const double lam = c->g.lambda;
  const int64_t M = c->M, D = (int64_t)c->g.q_max * c->seg;
  double sc[2];
  int rc;
  // r = d - A m; s = A^T r - lambda m (correction mode: - lambda (m -
  // m_start)); gamma = ||s||^2
  const bool corr = c->regularize == 1;
  if (corr) SCHECK(c, launch_fill_f32(c->dm, M, 0.f, c->st));
  const float* damped = corr ? c->dm : c->m;
  // per-shot misfit weights W (all 1 unless set): the adjoint takes W r and
  // delta = <q, W q> + ...
  c->wslot_h.assign(c->g.q_max, 1.f);
  bool weighted = false;
  for (int i = 0; i < (int)c->slots.size(); ++i)
    if (c->slots[i].used) {
      c->wslot_h[i] = c->slots[i].weight;
      weighted |= c->slots[i].weight != 1.f;
    }
  if (weighted)
    SCHECK(c, hipMemcpyAsync(c->wslot, c->wslot_h.data(),
                             (size_t)c->g.q_max * 4, hipMemcpyHostToDevice,
                             c->st));
  auto adjoint_w = [&](const float* x) -> int {
    if (!weighted) return adjoint_of(c, x);
    SCHECK(c, launch_scale_segments(c->dscr, x, c->wslot, c->seg, D, c->st));
    return adjoint_of(c, c->dscr);
  };
  if ((rc = born_of(c, c->m))) return finish(rc);
  SCHECK(c, launch_sub(c->r, c->dobs, c->q, D, c->st));
  if ((rc = adjoint_w(c->r))) return finish(rc);
  SCHECK(c, launch_grad_norm(c->s, c->gbuf, damped, lam, M, c->partial,
                             c->scal, c->st));
  if ((rc = read_scalars(c, sc, 1))) return finish(rc);
  double gamma = sc[0];
  if (!std::isfinite(gamma))
    return finish(sfail(c, BRLS_ENONFINITE, "non-finite gradient norm"));
  st.s0_norm = st.s_norm = std::sqrt(gamma);
  double snorm = st.s0_norm;
  double ref = 0.0;
  if (rtol > 0) {
    if ((rc = adjoint_w(c->dobs))) return finish(rc);
    SCHECK(c, launch_dot(c->gbuf, c->gbuf, M, c->partial, c->scal, c->st));
    if ((rc = read_scalars(c, sc, 1))) return finish(rc);
    ref = std::sqrt(sc[0]);
    st.ref_norm = ref;
  }
  // preconditioned form: directions follow z = M^{-1} s and gamma =
  // <s, z>; the stop test stays on ||s||
  const bool pre = c->precond != 0;
  if (pre) {
    if ((rc = build_minv(c))) return finish(rc);
    SCHECK(c, launch_mul(c->z, c->minv, c->s, M, c->st));
    SCHECK(c, launch_dot(c->s, c->z, M, c->partial, c->scal, c->st));
    if ((rc = read_scalars(c, sc, 1))) return finish(rc);
    gamma = sc[0];
  }
  SCHECK(c, hipMemcpyAsync(c->p, pre ? c->z : c->s, M * 4,
                           hipMemcpyDeviceToDevice, c->st));
  for (int it = 0; it < max_iter; ++it) {
    if (gamma == 0.0) break;
    if (rtol > 0 && snorm <= rtol * ref) break;
    if ((rc = born_of(c, c->p))) return finish(rc);
    if (weighted)
      SCHECK(c, launch_scale_segments(c->dscr, c->q, c->wslot, c->seg, D,
                                      c->st));
    SCHECK(c, launch_dot(c->q, weighted ? c->dscr : c->q, D, c->partial,
                         c->scal, c->st));
    SCHECK(c, launch_dot(c->p, c->p, M, c->partial, c->scal + 1, c->st));
    if ((rc = read_scalars(c, sc, 2))) return finish(rc);
    const double delta = sc[0] + lam * sc[1];
    if (!std::isfinite(delta))
      return finish(sfail(c, BRLS_ENONFINITE, "non-finite CG scalar delta"));
    if (!(delta > 0.0))
      return finish(sfail(c, BRLS_EBREAKDOWN, "CG breakdown: delta = %g",
                          delta));
    const double alpha = gamma / delta;
    SCHECK(c, launch_axpy(c->m, c->p, alpha, M, c->st));
    if (corr) SCHECK(c, launch_axpy(c->dm, c->p, alpha, M, c->st));
    SCHECK(c, launch_axpy(c->r, c->q, -alpha, D, c->st));
    if ((rc = adjoint_w(c->r))) return finish(rc);
    SCHECK(c, launch_grad_norm(c->s, c->gbuf, damped, lam, M, c->partial,
                               c->scal, c->st));
    if (pre) {
      SCHECK(c, launch_mul(c->z, c->minv, c->s, M, c->st));
      SCHECK(c, launch_dot(c->s, c->z, M, c->partial, c->scal + 1, c->st));
    }
    if ((rc = read_scalars(c, sc, pre ? 2 : 1))) return finish(rc);
    const double gnew = pre ? sc[1] : sc[0];
    if (!std::isfinite(sc[0]) || !std::isfinite(gnew))
      return finish(sfail(c, BRLS_ENONFINITE, "non-finite gradient norm"));
    const double beta = gnew / gamma;
    SCHECK(c, launch_xpby(c->p, pre ? c->z : c->s, beta, M, c->st));
    gamma = gnew;
    snorm = std::sqrt(sc[0]);
    st.iters = it + 1;
    st.s_norm = snorm;
  }
  SCHECK(c, launch_dot(c->r, c->r, D, c->partial, c->scal, c->st));
  if ((rc = read_scalars(c, sc, 1))) return finish(rc);
  st.r_norm = std::sqrt(sc[0]);
  return finish(BRLS_OK);
}

int brls_ssf_set_precond(brls_ssf_ctx* c, int32_t mode) {
  if (!c) return BRLS_EINVAL;
  if (mode != 0 && mode != 1)
    return sfail(c, BRLS_EINVAL, "preconditioner mode %d: 0 or 1", mode);
  c->precond = mode;
  return BRLS_OK;
}

int brls_ssf_get_precond(const brls_ssf_ctx* c, int32_t* mode) {
  if (!c || !mode) return BRLS_EINVAL;
  *mode = c->precond;
  return BRLS_OK;
}

int brls_ssf_set_regularization(brls_ssf_ctx* c, int32_t mode) {
  if (!c) return BRLS_EINVAL;
  if (mode != 0 && mode != 1)
    return sfail(c, BRLS_EINVAL, "regularization mode %d: 0 or 1", mode);
  c->regularize = mode;
  return BRLS_OK;
}

int brls_ssf_get_regularization(const brls_ssf_ctx* c, int32_t* mode) {
  if (!c || !mode) return BRLS_EINVAL;
  *mode = c->regularize;
  return BRLS_OK;
}

int brls_ssf_set_shot_weight(brls_ssf_ctx* c, int64_t id, double w) {
  if (!c) return BRLS_EINVAL;
  const int i = find_slot(c, id);
  if (i < 0)
    return sfail(c, BRLS_ENOSHOT, "no shot %lld in the window",
                 (long long)id);
  if (!(w >= 0.0) || !std::isfinite(w))
    return sfail(c, BRLS_EINVAL, "shot weight %g: must be finite and >= 0",
                 w);
  c->slots[i].weight = (float)w;
  return BRLS_OK;
}

int brls_ssf_get_shot_weight(const brls_ssf_ctx* c, int64_t id, double* w) {
  if (!c || !w) return BRLS_EINVAL;
  const int i = find_slot(c, id);
  if (i < 0) return BRLS_ENOSHOT;
  *w = c->slots[i].weight;
  return BRLS_OK;
}

int brls_ssf_illumination(brls_ssf_ctx* c, float* out) {
  if (!c || !out) return sfail(c, BRLS_EINVAL, "NULL argument");
  int rc;
  if ((rc = window_illumination(c, c->gbuf))) return rc;
  SCHECK(c, hipMemcpyAsync(out, c->gbuf, c->M * 4, out_kind(c), c->st));
  if (!dev_ptrs(c)) SCHECK(c, hipStreamSynchronize(c->st));
  return BRLS_OK;
}

int brls_ssf_image(brls_ssf_ctx* c, float* out) {
  if (!c || !out) return sfail(c, BRLS_EINVAL, "NULL argument");
  SCHECK(c, hipMemcpyAsync(out, c->m, c->M * 4, out_kind(c), c->st));
  if (!dev_ptrs(c)) SCHECK(c, hipStreamSynchronize(c->st));
  return BRLS_OK;
}

int brls_ssf_set_image(brls_ssf_ctx* c, const float* m) {
  if (!c || !m) return sfail(c, BRLS_EINVAL, "NULL argument");
  SCHECK(c, hipMemcpyAsync(c->m, m, c->M * 4, in_kind(c), c->st));
  if (!dev_ptrs(c)) SCHECK(c, hipStreamSynchronize(c->st));
  return BRLS_OK;
}

int brls_ssf_kernel_timing(brls_ssf_ctx* c, int32_t enable) {
  if (!c) return BRLS_EINVAL;
  c->timing = enable != 0;
  return BRLS_OK;
}

int brls_ssf_kernel_stats(brls_ssf_ctx* c, brls_kstat* out, int32_t cap,
                          int32_t* n) {
  if (!c || !n) return BRLS_EINVAL;
  SCHECK(c, hipStreamSynchronize(c->st));
  int64_t cnt[kSNumKinds] = {0};
  double tot[kSNumKinds] = {0};
  for (auto& t : c->timers) {
    float ms = 0.f;
    SCHECK(c, hipEventElapsedTime(&ms, t.a, t.b));
    cnt[t.kind]++;
    tot[t.kind] += ms;
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  c->timers.clear();
  int k = 0;
  for (int i = 0; i < kSNumKinds; ++i) {
    if (!cnt[i]) continue;
    if (out && k < cap) {
      std::snprintf(out[k].name, sizeof out[k].name, "%s", kSsfTimerNames[i]);
      out[k].launches = cnt[i];
      out[k].total_ms = tot[i];
    }
    ++k;
  }
  *n = k;
  return BRLS_OK;
}

int brls_ssf_memory_bytes(const brls_ssf_ctx* c, int64_t* bytes) {
  if (!c || !bytes) return BRLS_EINVAL;
  *bytes = c->mem_bytes;
  return BRLS_OK;
}

int brls_ssf_sync(brls_ssf_ctx* c) {
  if (!c) return BRLS_EINVAL;
  SCHECK(c, hipStreamSynchronize(c->st));
  return BRLS_OK;
}

}  // extern "C"
