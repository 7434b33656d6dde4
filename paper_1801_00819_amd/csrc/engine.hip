// Host engine and C ABI of the library: window of shots (update/downdate),
// background wavefields, the operator pair A / A^T over the window in three
// execution modes, and the damped CG solve of each window.
//
// Method: Kazemi & Sacchi, "Block row recursive least squares migration"
// (arXiv 1801.00819). Each window solves min ||A_w m - d_w||^2 + lambda||m||^2
// (eq. 10, the windowed form of eq. 3) by CG on the least-squares form,
// warm-started from the previous window's image (eq. 11); windows change by
// adding new shots and removing the oldest (rank-K update and downdate).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "brrlsm.h"
#include "kernels.h"
#include "layout.h"

using namespace brls;

namespace {

// A roctx range over a scope (window solves, CG iterations, window
// updates, background builds, operator applications): visible in a
// rocprofv3 trace with --marker-trace, a no-op otherwise.
struct Range {
  explicit Range(const char* what) { roctxRangePushA(what); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

// 8th-order central second-derivative weights (offsets 1..4); the
// difference-form stencil needs no centre weight.
constexpr double kW1 = 8.0 / 5.0, kW2 = -1.0 / 5.0, kW3 = 8.0 / 315.0,
                 kW4 = -1.0 / 560.0;
// Largest stable Courant number v dt / h in 2-D for this stencil with the
// second-order time step: the symbol of h^2 L per axis peaks at
// S = 205/72 + 2 (8/5 + 1/5 + 8/315 + 1/560) at the Nyquist wavenumber, and
// leapfrog needs C^2 * 2S <= 4, i.e. C <= 2 / sqrt(2 S).
constexpr double kCfl2D = 0.5546;
// Same for 3-D: C <= 2 / sqrt(3 S).
constexpr double kCfl3D = 0.4529;

thread_local std::string g_open_error;

// Device scratch of brls_apply_adjoint_static, which allocates nothing: the
// adjoint's float64 image accumulators, [groups][model]. Each device the
// library runs on holds its own copy until the process ends. Host code
// reaches it only through the per-device address from hipGetSymbolAddress
// (scratch_dev), never through the symbol itself.
constexpr int64_t kScratchBytes = (int64_t)16 << 20;
static __device__ __align__(256) double scratch[kScratchBytes / 8];
constexpr int kMaxDevices = 64;
double* g_scratch_dev[kMaxDevices] = {};
std::mutex g_scratch_mu;

// Address of the current device's copy of `scratch`, looked up once per
// device (brls_open). Null when the lookup failed.
double* scratch_dev(int dev, hipError_t* err) {
  *err = hipSuccess;
  if (dev < 0 || dev >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    *err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (*err != hipSuccess) return nullptr;
    g_scratch_dev[dev] = static_cast<double*>(p);
  }
  return g_scratch_dev[dev];
}

struct Slot {
  bool used = false;
  int64_t id = 0;
  int64_t seq = 0;
  int nt = 0, nrec = 0;
  int sz = 0, sy = 0, sx = 0;
  double f0 = 0.0;
  std::vector<int32_t> rec;  // host copy (z, y, x)
  bool bg_ready = false;
  float* fields = nullptr;   // u0 | u1 | v
  float* bgf = nullptr;      // background u0 | u1 | v (checkpoint mode)
  float* d2 = nullptr;       // [nt_max-1][nz][nx] (cache mode)
  float* ck = nullptr;       // [nseg][u | v][field] (checkpoint mode)
  float* segd2 = nullptr;    // [ckpt_k][nz][nx] (checkpoint mode)
  float* wav = nullptr;      // [nt_max]
  double* wav64 = nullptr;   // [nt_max] (float64 background)
  float* illum = nullptr;    // [nz][nx] sum of squared Born sources (cache)
  bool illum_ready = false;  // illum holds this shot's sum
  int* rptr = nullptr;       // [ntiles_max + 1]
  int2* rent = nullptr;      // [nrec_max]
  int* rsidx = nullptr;      // [nrec_max]
  int64_t dat_off = 0;
  float weight = 1.f;        // the shot's misfit weight in the window CG
};

struct Timer {
  int kind;
  hipEvent_t a, b;
};

enum TimerKind { kTBackground, kTBorn, kTAdjoint, kTBornGraph, kTAdjGraph,
                 kTNumKinds };
const char* kTimerNames[kTNumKinds] = {"background_step", "born_step",
                                       "adjoint_step", "born_graph",
                                       "adjoint_graph"};

// op, shots, shots per block, tile variant, time steps, resident grid,
// execution mode, chains
using GraphKey = std::tuple<int, int, int, int, int, int, int, int>;

}  // namespace

struct brls_ctx {
  brls_grid g{};
  hipStream_t st = nullptr;
  bool own_stream = false;
  // batched operator launches in two concurrent chains of shot groups:
  // the second chain's stream, the fork and join events, the stream the
  // next launch goes to (null: st) and the chain count (1 or 2)
  hipStream_t st2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipStream_t lst = nullptr;
  int chains = 2;
  int device = 0;
  int ndim = 2;
  Geo2D geo{};
  Geo3D geo3{};
  int variant = 0;
  int bins_variant = 0;  // tile variant the slots' receiver bins are for
  int per_block = 4;      // Born and background launches
  int resident_grid = 0;
  int adj_per_block = 4;  // adjoint launches
  int adj_resident_grid = 0;
  int tune_nt = 0;      // > 0 while autotuning: time steps per trial
  int zchunk = 32;      // 3-D: z planes per work item
  int exec = BRLS_EXEC_GRAPH;
  int rows_alloc = 0;
  int64_t fs = 0;      // floats per field buffer
  int64_t mplane = 0;  // model points
  int64_t seg = 0;     // floats per shot segment of data vectors
  int ntiles_max = 0;
  int ckpt_k = 0;       // 0: cache every Born-source frame; else interval
  int nseg_max = 0;     // checkpoints per shot
  float* wp = nullptr;
  float* fields_all = nullptr;
  float *m = nullptr, *p = nullptr, *s = nullptr, *gbuf = nullptr,
        *born_in = nullptr;
  int precond = 0;        // 1: diagonal illumination preconditioner
  float *minv = nullptr, *z = nullptr;  // its inverse; preconditioned s
  int regularize = 0;     // 0: damp the image; 1: damp the correction to
                          // the image the solve starts from
  float* dm = nullptr;    // that correction (mode 1)
  double* acc = nullptr;
  // persistent execution: grid barrier arrivals and failure flag
  unsigned* pcounter = nullptr;
  int* perror = nullptr;
  int spin_limit = 1 << 20;  // barrier polls before a wait gives up
  // precision (brls_set_precision): float64 background of new shots (stored
  // Born sources only) and float64 CG vectors
  int bg64 = 1;
  int vec64 = 1;
  double eta_scale64 = 0.0;  // eta_max * dt / 2 / nb^2
  double* wp64 = nullptr;     // W' in float64, storage layout
  double* bgf64 = nullptr;    // [q_max][u even | u odd | v] float64 fields
  Bg64Shot* bg64tab_dev = nullptr;
  double *m64 = nullptr, *p64 = nullptr, *s64 = nullptr, *g64 = nullptr,
         *dm64 = nullptr, *z64 = nullptr, *r64 = nullptr;
  float *dobs = nullptr, *r = nullptr, *q = nullptr, *dscr = nullptr;
  float* wslot = nullptr;  // [q_max] per-slot misfit weights (device)
  std::vector<float> wslot_h;  // their host copy, uploaded by the solve
  std::vector<double> hist;    // last solve: (alpha, beta, ||s||) per iter
  double *partial = nullptr, *scal = nullptr;
  int* flag = nullptr;
  ShotDev* tab_dev = nullptr;
  ShotDev* bgtab_dev = nullptr;
  bool tab_dirty = true;
  std::vector<Slot> slots;
  std::vector<int> order;  // slot indices in window order
  int64_t next_seq = 0;
  std::string err;
  bool timing = false;
  std::vector<Timer> timers;
  std::map<GraphKey, std::pair<hipGraph_t, hipGraphExec_t>> graphs;
  int64_t mem_bytes = 0;
  std::vector<void*> allocs;
};

namespace {

int fail(brls_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c)
    c->err = buf;
  else
    g_open_error = buf;
  return code;
}

#define HIPCHECK(ctx, call)                                                  \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess)                                                    \
      return fail(ctx, BRLS_EDEVICE, "%s: %s (%s:%d)", #call,                \
                  hipGetErrorString(e_), __FILE__, __LINE__);                \
  } while (0)

template <class T>
int dalloc(brls_ctx* c, T** p, int64_t count) {
  *p = nullptr;
  if (count <= 0) count = 1;
  const size_t bytes = (size_t)count * sizeof(T);
  if (hipMalloc((void**)p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(c, BRLS_ENOMEM, "device allocation of %zu bytes failed",
                bytes);
  }
  c->allocs.push_back(*p);
  c->mem_bytes += (int64_t)bytes;
  return BRLS_OK;
}

bool dev_ptrs(const brls_ctx* c) { return (c->g.flags & BRLS_DEVICE_PTRS); }

hipMemcpyKind in_kind(const brls_ctx* c) {
  return dev_ptrs(c) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
}
hipMemcpyKind out_kind(const brls_ctx* c) {
  return dev_ptrs(c) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
}

int round_up(int v, int m) { return (v + m - 1) / m * m; }

// Propagated-field buffers per slot: u, u, v, and in 2-D with stored Born
// sources a second v (the two-step kernels alternate between two sets).
int fields_per_slot(const brls_ctx* c) {
  return (c->ndim == 2 && !c->ckpt_k) ? 4 : 3;
}


int variant_count(const brls_ctx* c) {
  return c->ndim == 3 ? tile_shape3_count() : tile_shape_count();
}

void set_variant_geo(brls_ctx* c, int v) {
  if (c->ndim == 3) {
    const TileShape3 ts = tile_shape3(v);
    Geo3D& g = c->geo3;
    g.ntx = (g.px - g.x_org + ts.tx - 1) / ts.tx;
    g.nty = (g.py + ts.ty - 1) / ts.ty;
    g.tzc = c->zchunk;
    g.ntz = (g.pz + g.tzc - 1) / g.tzc;
    g.ntiles = g.ntx * g.nty * g.ntz;
  } else {
    const TileShape ts = tile_shape(v);
    Geo2D& g = c->geo;
    g.ntx = (g.px - g.x_org + ts.tx - 1) / ts.tx;
    g.ntz = (g.pz + ts.tz - 1) / ts.tz;
    g.ntiles = g.ntx * g.ntz;
  }
  c->variant = v;
}

// CSR bins of the receiver lists for the current tile shape.
int receiver_bins(const brls_ctx* c) {
  if (c->ndim == 3) return c->geo3.ntx * c->geo3.nty * c->geo3.pz;
  return c->geo.ntiles;
}

// Per-tile receiver lists of one slot for the current tile shape. 2-D: one
// bin per tile, local index lz * TX + lx. 3-D: one bin per (XY tile, padded
// z), local index ly * TX + lx.
int build_receiver_tiles(brls_ctx* c, Slot& sl) {
  const int nbins = receiver_bins(c);
  struct Entry {
    int bin, loc, rec;
  };
  std::vector<Entry> ms;  // (bin, local index, receiver) memberships
  ms.reserve(sl.nrec);
  for (int j = 0; j < sl.nrec; ++j) {
    if (c->ndim == 3) {
      const TileShape3 ts = tile_shape3(c->variant);
      const Geo3D& g = c->geo3;
      const int pz = sl.rec[3 * j] + g.nb, py = sl.rec[3 * j + 1] + g.nb,
                px = sl.rec[3 * j + 2] + g.nb;
      const int tyi = py / ts.ty, txi = (px - g.x_org) / ts.tx;
      ms.push_back({(tyi * g.ntx + txi) * g.pz + pz,
                    (py - tyi * ts.ty) * ts.tx + (px - g.x_org - txi * ts.tx),
                    j});
      continue;
    }
    const TileShape ts = tile_shape(c->variant);
    const Geo2D& g = c->geo;
    const int pz = sl.rec[3 * j] + g.nb, px = sl.rec[3 * j + 2] + g.nb;
    if (ts.pipe < 3) {
      const int tzi = pz / ts.tz, txi = (px - g.x_org) / ts.tx;
      ms.push_back({tzi * g.ntx + txi,
                    (pz - tzi * ts.tz) * ts.tx + (px - g.x_org - txi * ts.tx),
                    j});
      continue;
    }
    // two-step tiles: every tile whose outputs widened by the 4-cell ring
    // hold the receiver; local index (row - (z0 - 4)) * 64 +
    // (column - (x0 - 4))
    const int xr = px - g.x_org;
    for (int tzi = std::max(0, pz / ts.tz - 1); tzi < g.ntz; ++tzi) {
      const int z0 = tzi * ts.tz;
      if (pz < z0 - kRadius) break;
      if (pz >= z0 + ts.tz + kRadius) continue;
      for (int txi = std::max(0, xr / ts.tx - 1); txi < g.ntx; ++txi) {
        const int x0 = txi * ts.tx;  // relative to x_org
        if (xr < x0 - kRadius) break;
        if (xr >= x0 + ts.tx + kRadius) continue;
        ms.push_back({tzi * g.ntx + txi,
                      (pz - (z0 - kRadius)) * 64 + (xr - (x0 - kRadius)), j});
      }
    }
  }
  std::vector<int> cnt(nbins + 1, 0);
  for (const Entry& m : ms) cnt[m.bin + 1]++;
  for (int t = 0; t < nbins; ++t) cnt[t + 1] += cnt[t];
  std::vector<int2> ent(std::max<size_t>(ms.size(), 1));
  std::vector<int> fillp(cnt.begin(), cnt.end() - 1);
  for (const Entry& m : ms) {
    int2 e;
    e.x = m.loc;
    e.y = m.rec;
    ent[fillp[m.bin]++] = e;
  }
  // each bin in local-index order (2-D: by row, then column), which the
  // z-marching kernels rely on
  for (int b = 0; b < nbins; ++b)
    std::stable_sort(ent.begin() + cnt[b], ent.begin() + cnt[b + 1],
                     [](const int2& p, const int2& q) { return p.x < q.x; });
  HIPCHECK(c, hipMemcpyAsync(sl.rptr, cnt.data(), sizeof(int) * cnt.size(),
                             hipMemcpyHostToDevice, c->st));
  HIPCHECK(c, hipMemcpyAsync(sl.rent, ent.data(), sizeof(int2) * ms.size(),
                             hipMemcpyHostToDevice, c->st));
  HIPCHECK(c, hipStreamSynchronize(c->st));
  return BRLS_OK;
}

int64_t store_index(const brls_ctx* c, int z, int y, int x) {
  return c->ndim == 3 ? sidx3(c->geo3, z, y, x) : sidx2(c->geo, z, x);
}

ShotDev shot_dev(const brls_ctx* c, const Slot& sl) {
  ShotDev d{};
  d.f[3] = fields_per_slot(c) == 4 ? sl.fields + 3 * c->fs : nullptr;
  for (int k = 0; k < 3; ++k) {
    d.f[k] = sl.fields + k * c->fs;
    d.b[k] = (c->ckpt_k ? sl.bgf : sl.fields) + k * c->fs;
  }
  d.d2 = c->ckpt_k ? sl.segd2 : sl.d2;
  d.ck = sl.ck;
  d.rptr = sl.rptr;
  d.rent = sl.rent;
  d.rsidx = sl.rsidx;
  d.wav = sl.wav;
  d.dat_off = sl.dat_off;
  d.nt = sl.nt;
  d.nrec = sl.nrec;
  d.src_z = sl.sz + c->g.nb;
  d.src_y = c->ndim == 3 ? sl.sy + c->g.nb : 0;
  d.src_x = sl.sx + c->g.nb;
  return d;
}

void rebuild_order(brls_ctx* c) {
  c->order.clear();
  for (int i = 0; i < (int)c->slots.size(); ++i)
    if (c->slots[i].used) c->order.push_back(i);
  std::sort(c->order.begin(), c->order.end(), [c](int a, int b) {
    return c->slots[a].seq < c->slots[b].seq;
  });
  c->tab_dirty = true;
}

int ensure_tab(brls_ctx* c) {
  if (!c->tab_dirty) return BRLS_OK;
  std::vector<ShotDev> tab;
  for (int i : c->order) tab.push_back(shot_dev(c, c->slots[i]));
  HIPCHECK(c, hipStreamSynchronize(c->st));
  if (!tab.empty())
    HIPCHECK(c, hipMemcpy(c->tab_dev, tab.data(), sizeof(ShotDev) * tab.size(),
                          hipMemcpyHostToDevice));
  c->tab_dirty = false;
  return BRLS_OK;
}

int nt_max_of(const brls_ctx* c, const std::vector<int>& idx) {
  int n = 0;
  for (int i : idx) n = std::max(n, c->slots[i].nt);
  return c->tune_nt > 0 ? std::min(n, c->tune_nt) : n;
}

// --- timing ---------------------------------------------------------------
int timed_begin(brls_ctx* c, int kind, Timer* t) {
  if (!c->timing) return BRLS_OK;
  t->kind = kind;
  HIPCHECK(c, hipEventCreate(&t->a));
  HIPCHECK(c, hipEventCreate(&t->b));
  HIPCHECK(c, hipEventRecord(t->a, c->st));
  return BRLS_OK;
}
int timed_end(brls_ctx* c, Timer* t) {
  if (!c->timing) return BRLS_OK;
  HIPCHECK(c, hipEventRecord(t->b, c->st));
  c->timers.push_back(*t);
  return BRLS_OK;
}

StepArgs base_args(const brls_ctx* c) {
  StepArgs a{};
  a.g = c->geo;
  a.g3 = c->geo3;
  a.wp = c->wp;
  a.resident_grid = c->resident_grid;  // step() overrides for the adjoint
  return a;
}

// The persistent form runs the segment-marching two-step kernel (tile kind
// 4), which needs stored Born sources.
bool persistent_ok(const brls_ctx* c, int variant) {
  return c->ndim == 2 && !c->ckpt_k && tile_shape(variant).pipe == 4;
}

// Whether the 2-D tile variant advances two time steps per launch.
bool two_step(const brls_ctx* c) {
  return c->ndim == 2 && tile_shape(c->variant).pipe >= 3;
}

// One time step over `nshots` table entries starting at `tab` (two-step
// variants: `nsub` steps, reading field set `par`).
int step(brls_ctx* c, int mode, int n, const ShotDev* tab, int nshots,
         int per_block, const float* pm, float* dat, double* acc,
         int d2_n0 = 0, int write_d2 = 0, int nsub = 1, int par = 0) {
  StepArgs a = base_args(c);
  a.nsub = nsub;
  a.par = par;
  a.d2_n0 = d2_n0;
  a.write_d2 = write_d2;
  a.tab = tab;
  a.nshots = nshots;
  a.per_block = per_block;
  a.ngroups = (nshots + per_block - 1) / per_block;
  if (mode == kAdjoint) a.resident_grid = c->adj_resident_grid;
  a.n = n;
  a.pm = pm;
  a.dat = dat;
  a.acc = acc;
  Timer t;
  int rc = timed_begin(c, mode == kBackground ? kTBackground
                          : mode == kAdjoint  ? kTAdjoint
                                              : kTBorn,
                       &t);
  if (rc) return rc;
  hipStream_t ls = c->lst ? c->lst : c->st;
  HIPCHECK(c, c->ndim == 3 ? launch_step3d(c->variant, mode, a, ls)
                           : launch_step2d(c->variant, mode, a, ls));
  return timed_end(c, &t);
}

// The time loop of a batched operator application over the window's shot
// groups, in one chain of launches or, with two chains, as two independent
// chains over the first ceil(groups / 2) groups and the rest, the second on
// its own stream (forked from and joined back to the context's stream):
// the two run concurrently, so one chain's launches fill the slots the
// other's leave idle at the end of each launch. body(first, count, group0)
// enqueues the launches for shots first .. first + count - 1 (window
// order), groups from group0 on. Not with per-launch timing (the timers
// bracket launches on the context's stream).
template <typename F>
int in_chains(brls_ctx* c, int nsh, int pb, F&& body) {
  const int ngroups = (nsh + pb - 1) / pb;
  if (c->chains < 2 || ngroups < 2 || c->timing || !c->st2)
    return body(0, nsh, 0);
  const int g0 = (ngroups + 1) / 2;
  const int s0 = g0 * pb;
  HIPCHECK(c, hipEventRecord(c->ev_fork, c->st));
  HIPCHECK(c, hipStreamWaitEvent(c->st2, c->ev_fork, 0));
  int rc = body(0, s0, 0);
  if (!rc) {
    c->lst = c->st2;
    rc = body(s0, nsh - s0, g0);
    c->lst = nullptr;
  }
  HIPCHECK(c, hipEventRecord(c->ev_join, c->st2));
  HIPCHECK(c, hipStreamWaitEvent(c->st, c->ev_join, 0));
  return rc;
}

std::vector<int> order_part(const brls_ctx* c, int first, int count) {
  return std::vector<int>(c->order.begin() + first,
                          c->order.begin() + first + count);
}

int64_t field_floats(const brls_ctx* c) {
  return (int64_t)c->g.q_max * (fields_per_slot(c) + (c->ckpt_k ? 3 : 0)) *
         c->fs;
}

int zero_fields(brls_ctx* c) {
  HIPCHECK(c, launch_fill_f32(c->fields_all, field_floats(c), 0.f, c->st));
  return BRLS_OK;
}

int nseg_of(const brls_ctx* c, int nt) {
  return (nt - 1 + c->ckpt_k - 1) / c->ckpt_k;
}

Bg64Args bg64_args(const brls_ctx* c) {
  Bg64Args a{};
  a.ndim = c->ndim;
  a.nb = c->g.nb;
  a.nz = c->g.nz;
  a.ny = c->ndim == 3 ? c->g.ny : 1;
  a.nx = c->g.nx;
  a.pz = a.nz + 2 * a.nb;
  a.py = c->ndim == 3 ? a.ny + 2 * a.nb : 1;
  a.px = a.nx + 2 * a.nb;
  a.pitch = c->ndim == 3 ? c->geo3.pitch : c->geo.pitch;
  a.xoff = c->ndim == 3 ? c->geo3.xoff : c->geo.xoff;
  a.plane = c->ndim == 3 ? c->geo3.plane : 0;
  a.mplane = c->mplane;
  a.eta_scale = c->eta_scale64;
  a.w[0] = kW1;
  a.w[1] = kW2;
  a.w[2] = kW3;
  a.w[3] = kW4;
  a.wp = c->wp64;
  return a;
}

// Background wavefields (and Born-source caches) of shots that lack them.
int ensure_backgrounds(brls_ctx* c) {
  std::vector<int> todo;
  for (int i : c->order)
    if (!c->slots[i].bg_ready) todo.push_back(i);
  if (todo.empty()) return BRLS_OK;
  Range range("brls background build");
  std::vector<ShotDev> tab;
  for (int i : todo) tab.push_back(shot_dev(c, c->slots[i]));
  HIPCHECK(c, hipStreamSynchronize(c->st));
  HIPCHECK(c, hipMemcpy(c->bgtab_dev, tab.data(), sizeof(ShotDev) * tab.size(),
                        hipMemcpyHostToDevice));
  int rc;
  for (int i : todo) {
    Slot& sl = c->slots[i];
    HIPCHECK(c, launch_fill_f32(c->ckpt_k ? sl.bgf : sl.fields,
                                (c->ckpt_k ? 3 : fields_per_slot(c)) * c->fs,
                                0.f, c->st));
  }
  const int ntm = nt_max_of(c, todo);
  const int nsh = (int)todo.size();
  if (!c->ckpt_k && c->bg64) {
    // float64 background, one batched launch per time step (the fields of
    // the k-th shot to build in the k-th triple of bgf64)
    std::vector<Bg64Shot> bt(nsh);
    for (int k = 0; k < nsh; ++k) {
      const Slot& sl = c->slots[todo[k]];
      double* f = c->bgf64 + (int64_t)k * 3 * c->fs;
      bt[k].u[0] = f;
      bt[k].u[1] = f + c->fs;
      bt[k].v = f + 2 * c->fs;
      bt[k].d2 = sl.d2;
      bt[k].wav = sl.wav64;
      bt[k].nt = sl.nt;
      bt[k].src_z = sl.sz + c->g.nb;
      bt[k].src_y = c->ndim == 3 ? sl.sy + c->g.nb : 0;
      bt[k].src_x = sl.sx + c->g.nb;
    }
    HIPCHECK(c, hipMemcpy(c->bg64tab_dev, bt.data(), sizeof(Bg64Shot) * nsh,
                          hipMemcpyHostToDevice));
    HIPCHECK(c, launch_fill_f64(c->bgf64, (int64_t)nsh * 3 * c->fs, 0.0,
                                c->st));
    const Bg64Args ba = bg64_args(c);
    for (int n = 0; n + 1 < ntm; ++n)
      HIPCHECK(c, launch_background64(ba, c->bg64tab_dev, nsh, n, c->st));
    HIPCHECK(c, hipStreamSynchronize(c->st));
    for (int i : todo) {
      c->slots[i].bg_ready = true;
      c->slots[i].illum_ready = false;
    }
    return BRLS_OK;
  }
  // cache mode: every Born-source frame stored; checkpoint mode: the state
  // every ckpt_k steps
  const int wr = c->ckpt_k ? 0 : 1;
  auto save = [&](const ShotDev* tab, int ns, int n) -> int {
    if (!c->ckpt_k || n % c->ckpt_k) return BRLS_OK;
    HIPCHECK(c, launch_ckpt(tab, ns, n, n / c->ckpt_k, c->fs, 0, c->st));
    return BRLS_OK;
  };
  // (two-step variants take the background one step per launch, the field
  // sets alternating)
  if (c->exec == BRLS_EXEC_PLAIN) {
    for (int k = 0; k < nsh; ++k)
      for (int n = 0; n + 1 < c->slots[todo[k]].nt; ++n)
        if ((rc = save(c->bgtab_dev + k, 1, n)) ||
            (rc = step(c, kBackground, n, c->bgtab_dev + k, 1, 1, nullptr,
                       nullptr, nullptr, 0, wr, 1, n & 1)))
          return rc;
  } else {
    for (int n = 0; n + 1 < ntm; ++n)
      if ((rc = save(c->bgtab_dev, nsh, n)) ||
          (rc = step(c, kBackground, n, c->bgtab_dev, nsh,
                     std::min(c->per_block, nsh), nullptr, nullptr, nullptr,
                     0, wr, 1, n & 1)))
        return rc;
  }
  HIPCHECK(c, hipStreamSynchronize(c->st));
  for (int i : todo) {
    c->slots[i].bg_ready = true;
    c->slots[i].illum_ready = false;
  }
  return BRLS_OK;
}

// Stabiliser of the illumination preconditioner, relative to its mean.
constexpr double kIllumEps = 0.01;

int read_scalars(brls_ctx* c, double* out, int n);

// Window illumination (sum over the window's slots) into out. Each shot's
// own sum of its squared stored Born-source frames is formed the first
// time a window holding it needs it (cache mode only).
int window_illumination(brls_ctx* c, float* out) {
  int rc;
  if ((rc = ensure_tab(c)) || (rc = ensure_backgrounds(c))) return rc;
  for (int i : c->order) {
    Slot& sl = c->slots[i];
    if (sl.illum_ready) continue;
    HIPCHECK(c, launch_sumsq_frames(sl.d2, std::max(sl.nt - 1, 0), c->mplane,
                                    sl.illum, c->st));
    sl.illum_ready = true;
  }
  HIPCHECK(c, launch_fill_f32(out, c->mplane, 0.f, c->st));
  for (int i : c->order)
    HIPCHECK(c, launch_axpy(out, c->slots[i].illum, 1.0, c->mplane, c->st));
  return BRLS_OK;
}

// minv = 1 / (I + kIllumEps * mean(I)), I the window illumination.
int build_minv(brls_ctx* c) {
  int rc;
  if ((rc = window_illumination(c, c->minv))) return rc;
  HIPCHECK(c, launch_sum(c->minv, c->mplane, c->partial, c->scal, c->st));
  double sum = 0.0;
  if ((rc = read_scalars(c, &sum, 1))) return rc;
  const double shift = kIllumEps * sum / (double)c->mplane;
  if (!(shift > 0.0))
    return fail(c, BRLS_EBREAKDOWN,
                "preconditioner: the window's shots illuminate nothing");
  HIPCHECK(c, launch_recip_shift(c->minv, c->minv, shift, c->mplane, c->st));
  return BRLS_OK;
}

// Kernel sequence of one operator application (also what a graph captures).
// Cache mode reads the stored Born-source frames; checkpoint mode advances
// the background alongside (Born) or recomputes it segment by segment from
// its checkpoints (adjoint).
int enqueue_born(brls_ctx* c, int batched) {
  const int nsh = (int)c->order.size();
  const int ntm = nt_max_of(c, c->order);
  const int mode = c->ckpt_k ? kBornFused : kBorn;
  int rc;
  if ((rc = zero_fields(c))) return rc;
  // one step per launch, or two (levels n, n + 1; the field sets alternate)
  const int dn = two_step(c) ? 2 : 1;
  if (batched && c->exec == BRLS_EXEC_PERSISTENT) {
    // one launch for all two-step launches of the application
    StepArgs a = base_args(c);
    a.tab = c->tab_dev;
    a.nshots = nsh;
    a.per_block = std::min(c->per_block, nsh);
    a.ngroups = (nsh + a.per_block - 1) / a.per_block;
    a.pm = c->born_in;
    a.dat = c->q;
    PersistArgs p{};
    p.counter = c->pcounter;
    p.error = c->perror;
    p.nlaunch = (ntm - 1 + 1) / 2;
    p.nt_max = ntm;
    p.spin_limit = c->spin_limit;
    const TileShape ts = tile_shape(c->variant);
    HIPCHECK(c, launch_fill_u32(c->pcounter, 2, 0u, c->st));
    HIPCHECK(c, launch_march2s_persistent(ts.tz, ts.ntz, kBorn, a, p, c->st));
    HIPCHECK(c, launch_born_last(c->tab_dev, nsh, c->g.nrec_max, c->q, 1,
                                 c->st));
    return BRLS_OK;
  }
  auto run = [&](const ShotDev* tab, int ns, int pb, int nt) -> int {
    for (int n = 0, i = 0; n + 1 < nt; n += dn, ++i) {
      const int r = step(c, mode, n, tab, ns, pb, c->born_in, c->q, nullptr,
                         0, 0, std::min(dn, nt - 1 - n), i & 1);
      if (r) return r;
    }
    return BRLS_OK;
  };
  if (!batched) {
    for (int k = 0; k < nsh; ++k)
      if ((rc = run(c->tab_dev + k, 1, 1, nt_max_of(c, {c->order[k]}))))
        return rc;
  } else {
    const int pb = std::min(c->per_block, nsh);
    rc = in_chains(c, nsh, pb, [&](int first, int count, int) {
      return run(c->tab_dev + first, count, pb,
                 count == nsh ? ntm : nt_max_of(c, order_part(c, first, count)));
    });
    if (rc) return rc;
  }
  HIPCHECK(c, launch_born_last(c->tab_dev, nsh, c->g.nrec_max, c->q,
                               two_step(c), c->st));
  return BRLS_OK;
}

// Adjoint steps k = k_hi .. k_lo (descending) of the shots in tab, the
// Born-source frames of levels >= d2_n0 being available.
// Two-step variants take levels k and k - 1 per launch, the field sets
// alternating.
int adjoint_steps(brls_ctx* c, const ShotDev* tab, int nsh, int pb, int k_hi,
                  int k_lo, int d2_n0, double* acc) {
  const int dk = two_step(c) ? 2 : 1;
  int rc;
  for (int k = k_hi, i = 0; k >= k_lo; k -= dk, ++i)
    if ((rc = step(c, kAdjoint, k, tab, nsh, pb, nullptr, c->dscr, acc,
                   d2_n0, 0, std::min(dk, k - k_lo + 1), i & 1)))
      return rc;
  return BRLS_OK;
}

// Checkpoint mode: for each segment, last first, restore the background at
// the segment start, recompute the segment's Born-source frames, then run
// the adjoint steps that consume them.
int adjoint_segments(brls_ctx* c, const ShotDev* tab, int nsh, int pb,
                     int nt, double* acc) {
  int rc;
  for (int seg = nseg_of(c, nt) - 1; seg >= 0; --seg) {
    const int n0 = seg * c->ckpt_k;
    const int n1 = std::min(n0 + c->ckpt_k, nt - 1);
    HIPCHECK(c, launch_ckpt(tab, nsh, n0, seg, c->fs, 1,
                            c->lst ? c->lst : c->st));
    for (int n = n0; n < n1; ++n)
      if ((rc = step(c, kBackground, n, tab, nsh, pb, nullptr, nullptr,
                     nullptr, n0, 1)))
        return rc;
    if ((rc = adjoint_steps(c, tab, nsh, pb, n1, n0 + 1, n0, acc)))
      return rc;
  }
  return BRLS_OK;
}

// Shots per adjoint work item. The two-step adjoint with 4 or 8 shots per
// item runs cooperative blocks of that many wavefronts, one shot each (idle
// where the window holds fewer), so the count is not clamped there.
int adj_pb(const brls_ctx* c, int nsh) {
  const int pb = c->adj_per_block;
  if (two_step(c) && (pb == 4 || pb == 8)) return pb;
  return std::min(pb, nsh);
}

// Float64 image accumulators of the adjoint: [groups][model]. The adjoint
// launches of a window use ceil(shots / shots-per-item) groups.
int64_t adjoint_acc_doubles(const brls_ctx* c, int batched) {
  const int nsh = (int)c->order.size();
  const int pb = batched ? adj_pb(c, nsh) : 1;
  const int ngroups = batched ? (nsh + pb - 1) / pb : 1;
  return (int64_t)ngroups * c->mplane;
}

int enqueue_adjoint(brls_ctx* c, int batched, double* acc) {
  const int nsh = (int)c->order.size();
  const int ntm = nt_max_of(c, c->order);
  const int pb = batched ? adj_pb(c, nsh) : 1;
  const int ngroups = batched ? (nsh + pb - 1) / pb : 1;
  int rc;
  if ((rc = zero_fields(c))) return rc;
  HIPCHECK(c, launch_fill_f64(acc, ngroups * c->mplane, 0.0, c->st));
  if (batched && c->exec == BRLS_EXEC_PERSISTENT) {
    StepArgs a = base_args(c);
    a.resident_grid = c->adj_resident_grid;
    a.tab = c->tab_dev;
    a.nshots = nsh;
    a.per_block = pb;
    a.ngroups = ngroups;
    a.dat = c->dscr;
    a.acc = acc;
    PersistArgs p{};
    p.counter = c->pcounter;
    p.error = c->perror;
    p.k_hi = ntm - 1;
    p.k_lo = 1;
    p.nlaunch = (ntm - 1 + 1) / 2;
    p.spin_limit = c->spin_limit;
    const TileShape ts = tile_shape(c->variant);
    HIPCHECK(c, launch_fill_u32(c->pcounter, 2, 0u, c->st));
    HIPCHECK(c, launch_march2s_persistent(ts.tz, ts.ntz, kAdjoint, a, p,
                                          c->st));
  } else if (!batched) {
    for (int k = 0; k < nsh; ++k) {
      const int nt = nt_max_of(c, {c->order[k]});
      rc = c->ckpt_k
               ? adjoint_segments(c, c->tab_dev + k, 1, 1, nt, acc)
               : adjoint_steps(c, c->tab_dev + k, 1, 1, nt - 1, 1, 0, acc);
      if (rc) return rc;
    }
  } else if (c->ckpt_k) {
    // each chain restores its shots' checkpoints, recomputes their
    // backgrounds segment by segment and runs their adjoint steps (one
    // step per launch: no level pairing to keep)
    rc = in_chains(c, nsh, pb, [&](int first, int count, int group0) {
      const int nt = count == nsh ? ntm
                                  : nt_max_of(c, order_part(c, first, count));
      return adjoint_segments(c, c->tab_dev + first, count, pb, nt,
                              acc + (int64_t)group0 * c->mplane);
    });
    if (rc) return rc;
  } else {
    rc = in_chains(c, nsh, pb, [&](int first, int count, int group0) {
      // a chain of shorter shots starts at its own last level, kept at the
      // parity of the window's so that levels pair into two-step launches
      // exactly as in one chain (the image sums stay bitwise the same)
      const int nt = count == nsh ? ntm
                                  : nt_max_of(c, order_part(c, first, count));
      const int k_hi = nt - 1 + ((ntm - nt) & (two_step(c) ? 1 : 0));
      return adjoint_steps(c, c->tab_dev + first, count, pb, k_hi, 1, 0,
                           acc + (int64_t)group0 * c->mplane);
    });
    if (rc) return rc;
  }
  HIPCHECK(c, c->ndim == 3
                  ? launch_adj_finalize3(acc, ngroups, c->geo3, c->wp,
                                         c->gbuf, c->g64, c->st)
                  : launch_adj_finalize(acc, ngroups, c->geo, c->wp,
                                        c->gbuf, c->g64, c->st));
  return BRLS_OK;
}

int run_op(brls_ctx* c, int op) {
  int rc;
  if ((rc = ensure_tab(c)) || (rc = ensure_backgrounds(c)) ||
      (rc = ensure_tab(c)))
    return rc;
  if (c->order.empty()) return BRLS_OK;
  if (c->exec != BRLS_EXEC_GRAPH && c->exec != BRLS_EXEC_PERSISTENT)
    return op == kBorn
               ? enqueue_born(c, c->exec == BRLS_EXEC_BATCHED)
               : enqueue_adjoint(c, c->exec == BRLS_EXEC_BATCHED, c->acc);
  const int nsh = (int)c->order.size();
  const bool adj = op == kAdjoint;
  const GraphKey key(op, nsh,
                     adj ? adj_pb(c, nsh) : std::min(c->per_block, nsh),
                     c->variant, nt_max_of(c, c->order),
                     adj ? c->adj_resident_grid : c->resident_grid, c->exec,
                     c->chains);
  auto it = c->graphs.find(key);
  if (it == c->graphs.end()) {
    const bool was_timing = c->timing;
    c->timing = false;
    HIPCHECK(c, hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal));
    rc = op == kBorn ? enqueue_born(c, 1) : enqueue_adjoint(c, 1, c->acc);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(c->st, &graph);
    c->timing = was_timing;
    if (rc) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess)
      return fail(c, BRLS_EDEVICE, "graph capture failed: %s",
                  hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    HIPCHECK(c, hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    it = c->graphs.emplace(key, std::make_pair(graph, exec)).first;
  }
  Timer t;
  if ((rc = timed_begin(c, op == kBorn ? kTBornGraph : kTAdjGraph, &t)))
    return rc;
  HIPCHECK(c, hipGraphLaunch(it->second.second, c->st));
  if ((rc = timed_end(c, &t))) return rc;
  if (c->exec == BRLS_EXEC_PERSISTENT) {
    int bad = 0;
    HIPCHECK(c, hipMemcpyAsync(&bad, c->perror, sizeof(int),
                               hipMemcpyDeviceToHost, c->st));
    HIPCHECK(c, hipStreamSynchronize(c->st));
    if (bad)
      return fail(c, BRLS_EDEVICE,
                  "persistent launch: a grid barrier wait gave up after %d "
                  "polls; the operator's result is invalid",
                  c->spin_limit);
  }
  return BRLS_OK;
}

void drop_graphs(brls_ctx* c) {
  for (auto& kv : c->graphs) {
    (void)hipGraphExecDestroy(kv.second.second);
    (void)hipGraphDestroy(kv.second.first);
  }
  c->graphs.clear();
}

int born_of(brls_ctx* c, const float* model_dev) {
  if (model_dev != c->born_in)
    HIPCHECK(c, hipMemcpyAsync(c->born_in, model_dev, c->mplane * 4,
                               hipMemcpyDeviceToDevice, c->st));
  return run_op(c, kBorn);
}

int adjoint_of(brls_ctx* c, const float* data_dev) {
  if (data_dev != c->dscr)
    HIPCHECK(c, hipMemcpyAsync(c->dscr, data_dev,
                               (size_t)c->g.q_max * c->seg * 4,
                               hipMemcpyDeviceToDevice, c->st));
  return run_op(c, kAdjoint);
}

int read_scalars(brls_ctx* c, double* out, int n) {
  HIPCHECK(c, hipMemcpyAsync(out, c->scal, sizeof(double) * n,
                             hipMemcpyDeviceToHost, c->st));
  HIPCHECK(c, hipStreamSynchronize(c->st));
  return BRLS_OK;
}

int find_slot(const brls_ctx* c, int64_t id) {
  for (int i = 0; i < (int)c->slots.size(); ++i)
    if (c->slots[i].used && c->slots[i].id == id) return i;
  return -1;
}

int check_finite(brls_ctx* c, const float* dev, int64_t n, bool* ok) {
  HIPCHECK(c, hipMemsetAsync(c->flag, 0, sizeof(int), c->st));
  HIPCHECK(c, launch_nonfinite(dev, n, c->flag, c->st));
  int h = 0;
  HIPCHECK(c, hipMemcpyAsync(&h, c->flag, sizeof(int), hipMemcpyDeviceToHost,
                             c->st));
  HIPCHECK(c, hipStreamSynchronize(c->st));
  *ok = (h == 0);
  return BRLS_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int brls_open(const brls_grid* gin, const float* vel, void* stream,
              brls_ctx** out) {
  if (!out) return fail(nullptr, BRLS_EINVAL, "out is NULL");
  *out = nullptr;
  if (!gin || !vel) return fail(nullptr, BRLS_EINVAL, "grid or vel is NULL");
  const brls_grid g = *gin;
  if (g.ndim != 2 && g.ndim != 3)
    return fail(nullptr, BRLS_EINVAL, "ndim must be 2 or 3, got %d", g.ndim);
  const int ny = g.ndim == 3 ? g.ny : 1;
  if (g.nz < 1 || ny < 1 || g.nx < 1 || g.nb < 1 || g.nt_max < 2 ||
      g.nrec_max < 1 || g.q_max < 1 || !(g.h > 0) || !(g.dt > 0) ||
      !(g.lambda >= 0))
    return fail(nullptr, BRLS_EINVAL, "invalid grid sizes or spacing");
  // The kernels address one wavefield, the model and a frame with 32-bit
  // byte offsets (signed in 2-D, element index times four in 3-D), and one
  // shot's data segment with 32-bit indices.
  const int64_t lim = g.ndim == 2 ? ((int64_t)1 << 29) : ((int64_t)1 << 30);
  const int64_t mpts = (int64_t)g.nz * ny * g.nx;
  const int64_t ppts = (int64_t)(g.nz + 2 * g.nb) *
                       (g.ndim == 3 ? ny + 2 * g.nb : 1) * (g.nx + 2 * g.nb);
  if (mpts >= lim || ppts >= lim)
    return fail(nullptr, BRLS_EINVAL,
                "padded grid of %lld points is too large (limit %lld)",
                (long long)ppts, (long long)lim);
  if ((int64_t)g.nt_max * g.nrec_max > ((int64_t)1 << 30))
    return fail(nullptr, BRLS_EINVAL,
                "nt_max * nrec_max = %lld exceeds 2^30 samples per shot",
                (long long)g.nt_max * g.nrec_max);
  double vmax = 0.0;
  for (int64_t i = 0; i < mpts; ++i) {
    if (!(vel[i] > 0.f) || !std::isfinite(vel[i]))
      return fail(nullptr, BRLS_EINVAL, "velocity must be finite and > 0");
    vmax = std::max(vmax, (double)vel[i]);
  }
  const double cfl = g.ndim == 3 ? kCfl3D : kCfl2D;
  if (vmax * g.dt / g.h > cfl)
    return fail(nullptr, BRLS_EINVAL,
                "unstable: v_max dt / h = %.4f exceeds %.4f",
                vmax * g.dt / g.h, cfl);
  hipDeviceProp_t prop;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return fail(nullptr, BRLS_EDEVICE, "no HIP device");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(nullptr, BRLS_EDEVICE,
                "library is built for gfx950, device is %s", prop.gcnArchName);

  brls_ctx* c = new brls_ctx();
  c->g = g;
  c->st = (hipStream_t)stream;
  if (!c->st) {
    // The null stream cannot be captured into a graph: use a private stream
    // that still synchronises with the null stream (blocking, default
    // priority).
    if (hipStreamCreate(&c->st) != hipSuccess) {
      delete c;
      return fail(nullptr, BRLS_EDEVICE, "hipStreamCreate failed");
    }
    c->own_stream = true;
  }
  c->device = dev;
  {
    hipError_t e = hipSuccess;
    if (!scratch_dev(dev, &e)) {
      if (c->own_stream) (void)hipStreamDestroy(c->st);
      delete c;
      return fail(nullptr, BRLS_EDEVICE,
                  "hipGetSymbolAddress of the static scratch: %s",
                  hipGetErrorString(e));
    }
  }
  if (hipStreamCreate(&c->st2) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) !=
          hipSuccess ||
      hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) !=
          hipSuccess) {
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->st2) (void)hipStreamDestroy(c->st2);
    if (c->own_stream) (void)hipStreamDestroy(c->st);
    delete c;
    return fail(nullptr, BRLS_EDEVICE, "second stream or its events");
  }
  c->ndim = g.ndim;
  const double eta_max = 3.0 * vmax * std::log(1000.0) / (2.0 * g.nb * g.h);
  c->eta_scale64 = eta_max * g.dt / 2.0 / ((double)g.nb * g.nb);
  const float eta_scale = (float)c->eta_scale64;
  const StencilW sw = {(float)kW1, (float)kW2, (float)kW3, (float)kW4};
  const int x_org = (g.nb % 32 == 0) ? 0 : (g.nb % 32) - 32;
  const int px = g.nx + 2 * g.nb;
  // x: first model column on a 128-byte boundary; room for the tile widths
  // that divide 128 plus the 4-cell ring, and in 2-D 64 columns more (a
  // two-step strip's wavefront and edge fills reach 64 columns past its
  // last output)
  const int pitch = round_up(32 - x_org + round_up(px - x_org, 128) + kGhost +
                                 (g.ndim == 2 ? 64 : 0),
                             32);
  if (g.ndim == 3) {
    Geo3D& geo = c->geo3;
    geo.nz = g.nz;
    geo.ny = ny;
    geo.nx = g.nx;
    geo.nb = g.nb;
    geo.pz = g.nz + 2 * g.nb;
    geo.py = ny + 2 * g.nb;
    geo.px = px;
    geo.x_org = x_org;
    geo.xoff = 32 - x_org;
    geo.pitch = pitch;
    // y: room for tiles of up to 8 rows plus the ring; z: the ring (z chunks
    // stop at the padded grid)
    const int rows = round_up(geo.py, 8) + 2 * kGhost;
    geo.plane = rows * pitch;
    c->rows_alloc = geo.pz + 2 * kGhost;
    c->fs = (int64_t)c->rows_alloc * geo.plane;
    geo.eta_scale = eta_scale;
    geo.w = sw;
  } else {
    Geo2D& geo = c->geo;
    geo.nz = g.nz;
    geo.nx = g.nx;
    geo.nb = g.nb;
    geo.pz = g.nz + 2 * g.nb;
    geo.px = px;
    geo.x_org = x_org;
    geo.xoff = 32 - x_org;
    geo.pitch = pitch;
    // z: room for tiles of up to 64 rows plus the ring, and for chunk
    // heights that do not divide 64 (rows past the grid are read as zeros)
    c->rows_alloc = round_up(geo.pz, 64) + 24;
    c->fs = (int64_t)c->rows_alloc * geo.pitch;
    geo.eta_scale = eta_scale;
    geo.w = sw;
  }
  c->ntiles_max = 0;  // largest receiver-bin count over tile variants
  for (int v = 0; v < variant_count(c); ++v) {
    set_variant_geo(c, v);
    c->ntiles_max = std::max(c->ntiles_max, receiver_bins(c));
  }
  set_variant_geo(c, 0);
  if (g.ndim == 3) c->per_block = c->adj_per_block = tile_shape3(0).sb;
  c->mplane = mpts;
  if (g.ckpt_interval < 0)
    c->ckpt_k = std::max(1, (int)std::ceil(std::sqrt((double)g.nt_max)));
  else
    c->ckpt_k = g.ckpt_interval;
  if (c->ckpt_k) c->nseg_max = (g.nt_max - 1 + c->ckpt_k - 1) / c->ckpt_k;
  if (c->ckpt_k) c->bg64 = 0;  // the background is recomputed in float32
  // two launch chains by default where they measured faster: 2-D with
  // stored Born sources (the 512 x 1024 window pair 128 ms against 150 ms).
  // 3-D launches already hold many work items per shot group (pair
  // 14.83 s with two chains against 14.13 s), and with checkpoints each
  // chain's restore-recompute-adjoint segments serialise on its stream
  // (autograd forward + backward 0.34 s against 0.29 s)
  c->chains = (g.ndim == 2 && c->ckpt_k == 0) ? 2 : 1;
  if (c->fs >= lim) {  // the storage ring and pitch padding on top
    brls_close(c);
    return fail(nullptr, BRLS_EINVAL,
                "wavefield storage of %lld floats is too large (limit %lld)",
                (long long)c->fs, (long long)lim);
  }
  c->seg = round_up((int)((int64_t)g.nt_max * g.nrec_max), 64);

  int rc = BRLS_OK;
#define ALLOC(ptr, n)                               \
  if ((rc = dalloc(c, &(ptr), (n))) != BRLS_OK) {   \
    g_open_error = c->err;                          \
    brls_close(c);                                  \
    return rc;                                      \
  }
  ALLOC(c->wp, c->fs);
  ALLOC(c->fields_all, field_floats(c));
  ALLOC(c->m, mpts);
  ALLOC(c->p, mpts);
  ALLOC(c->s, mpts);
  ALLOC(c->gbuf, mpts);
  ALLOC(c->born_in, mpts);
  ALLOC(c->minv, mpts);
  ALLOC(c->z, mpts);
  ALLOC(c->dm, mpts);
  ALLOC(c->acc, (int64_t)g.q_max * mpts);
  ALLOC(c->m64, mpts);
  ALLOC(c->p64, mpts);
  ALLOC(c->s64, mpts);
  ALLOC(c->g64, mpts);
  ALLOC(c->dm64, mpts);
  ALLOC(c->z64, mpts);
  ALLOC(c->r64, (int64_t)g.q_max * c->seg);
  if (!c->ckpt_k) {
    ALLOC(c->wp64, c->fs);
    ALLOC(c->bgf64, (int64_t)g.q_max * 3 * c->fs);
    ALLOC(c->bg64tab_dev, g.q_max);
  }
  ALLOC(c->dobs, (int64_t)g.q_max * c->seg);
  ALLOC(c->r, (int64_t)g.q_max * c->seg);
  ALLOC(c->q, (int64_t)g.q_max * c->seg);
  ALLOC(c->dscr, (int64_t)g.q_max * c->seg);
  ALLOC(c->wslot, g.q_max);
  ALLOC(c->partial, kDotBlocks);
  ALLOC(c->pcounter, 2);  // [0] arrivals, [1] the failure flag
  c->perror = reinterpret_cast<int*>(c->pcounter + 1);
  ALLOC(c->scal, 16);
  ALLOC(c->flag, 1);
  ALLOC(c->tab_dev, g.q_max);
  ALLOC(c->bgtab_dev, g.q_max);
  c->slots.resize(g.q_max);
  for (int i = 0; i < g.q_max; ++i) {
    Slot& sl = c->slots[i];
    const int nf = fields_per_slot(c);
    sl.fields = c->fields_all + (int64_t)i * nf * c->fs;
    if (c->ckpt_k)
      sl.bgf = c->fields_all + ((int64_t)g.q_max * nf + (int64_t)i * 3) * c->fs;
    sl.dat_off = (int64_t)i * c->seg;
    if (c->ckpt_k) {
      ALLOC(sl.ck, (int64_t)c->nseg_max * 2 * c->fs);
      ALLOC(sl.segd2, (int64_t)c->ckpt_k * mpts);
    } else {
      ALLOC(sl.d2, (int64_t)(g.nt_max - 1) * mpts);
      ALLOC(sl.illum, mpts);
    }
    ALLOC(sl.wav, g.nt_max);
    if (!c->ckpt_k) ALLOC(sl.wav64, g.nt_max);
    ALLOC(sl.rptr, c->ntiles_max + 1);
    // a receiver lies in up to 4 tiles' widened regions (two-step tiles)
    ALLOC(sl.rent, (int64_t)g.nrec_max * (g.ndim == 2 ? 4 : 1));
    ALLOC(sl.rsidx, g.nrec_max);
  }
#undef ALLOC
  // W' = v^2 dt^2 / h^2 on the padded grid (velocity edge-replicated)
  std::vector<float> wh((size_t)c->fs, 0.f);
  std::vector<double> wh64(c->ckpt_k ? 0 : (size_t)c->fs, 0.0);
  const double s2 = g.dt * g.dt / (g.h * g.h);
  const int pz = g.nz + 2 * g.nb, py = g.ndim == 3 ? ny + 2 * g.nb : 1;
  for (int z = 0; z < pz; ++z)
    for (int y = 0; y < py; ++y)
      for (int x = 0; x < px; ++x) {
        const int mz = std::min(std::max(z - g.nb, 0), g.nz - 1);
        const int my = g.ndim == 3 ? std::min(std::max(y - g.nb, 0), ny - 1)
                                   : 0;
        const int mx = std::min(std::max(x - g.nb, 0), g.nx - 1);
        const double v = vel[((int64_t)mz * ny + my) * g.nx + mx];
        wh[store_index(c, z, y, x)] = (float)(v * v * s2);
        if (!wh64.empty()) wh64[store_index(c, z, y, x)] = v * v * s2;
      }
  auto init = [&]() -> int {
    HIPCHECK(c, hipMemcpy(c->wp, wh.data(), sizeof(float) * wh.size(),
                          hipMemcpyHostToDevice));
    HIPCHECK(c, launch_fill_f32(c->fields_all, field_floats(c), 0.f, c->st));
    if (!wh64.empty())
      HIPCHECK(c, hipMemcpy(c->wp64, wh64.data(),
                            sizeof(double) * wh64.size(),
                            hipMemcpyHostToDevice));
    HIPCHECK(c, launch_fill_f32(c->m, mpts, 0.f, c->st));
    HIPCHECK(c, launch_fill_f64(c->m64, mpts, 0.0, c->st));
    for (float* v : {c->dobs, c->r, c->q, c->dscr})
      HIPCHECK(c, launch_fill_f32(v, (int64_t)g.q_max * c->seg, 0.f, c->st));
    HIPCHECK(c, hipStreamSynchronize(c->st));
    return BRLS_OK;
  };
  if ((rc = init()) != BRLS_OK) {
    g_open_error = c->err;
    brls_close(c);
    return rc;
  }
  *out = c;
  return BRLS_OK;
}

void brls_close(brls_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->st);
  drop_graphs(c);
  for (auto& t : c->timers) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (void* p : c->allocs) (void)hipFree(p);
  (void)hipStreamSynchronize(c->st2);
  (void)hipEventDestroy(c->ev_fork);
  (void)hipEventDestroy(c->ev_join);
  (void)hipStreamDestroy(c->st2);
  if (c->own_stream) (void)hipStreamDestroy(c->st);
  delete c;
}

const char* brls_last_error(const brls_ctx* c) {
  return c ? c->err.c_str() : g_open_error.c_str();
}

int brls_update(brls_ctx* c, const brls_shot* sh) {
  if (!c || !sh) return fail(c, BRLS_EINVAL, "NULL argument");
  Range range("brls_update");
  if (find_slot(c, sh->id) >= 0)
    return fail(c, BRLS_EDUP, "shot %lld already in the window",
                (long long)sh->id);
  int free_i = -1;
  for (int i = 0; i < (int)c->slots.size(); ++i)
    if (!c->slots[i].used) {
      free_i = i;
      break;
    }
  if (free_i < 0)
    return fail(c, BRLS_EFULL, "window already holds q_max = %d shots",
                c->g.q_max);
  if (sh->nt < 2 || sh->nt > c->g.nt_max || sh->nrec < 1 ||
      sh->nrec > c->g.nrec_max || !(sh->f0 > 0) || !sh->rec)
    return fail(c, BRLS_EINVAL, "shot %lld: bad nt, nrec, f0 or receivers",
                (long long)sh->id);
  const int ny = c->ndim == 3 ? c->g.ny : 1;
  const int ssy = c->ndim == 3 ? sh->sy : 0;
  if (sh->sz < 0 || sh->sz >= c->g.nz || sh->sx < 0 || sh->sx >= c->g.nx ||
      ssy < 0 || ssy >= ny)
    return fail(c, BRLS_EINVAL, "shot %lld: source outside the model",
                (long long)sh->id);
  for (int j = 0; j < sh->nrec; ++j) {
    const int z = sh->rec[3 * j], x = sh->rec[3 * j + 2];
    const int y = c->ndim == 3 ? sh->rec[3 * j + 1] : 0;
    if (z < 0 || z >= c->g.nz || x < 0 || x >= c->g.nx || y < 0 || y >= ny)
      return fail(c, BRLS_EINVAL, "shot %lld: receiver %d outside the model",
                  (long long)sh->id, j);
  }
  Slot& sl = c->slots[free_i];
  const int64_t nd = (int64_t)sh->nt * sh->nrec;
  float* seg = c->dobs + sl.dat_off;
  HIPCHECK(c, launch_fill_f32(seg, c->seg, 0.f, c->st));
  if (sh->data) {
    HIPCHECK(c, hipMemcpyAsync(seg, sh->data, nd * 4, in_kind(c), c->st));
    bool ok = true;
    int rc = check_finite(c, seg, nd, &ok);
    if (rc) return rc;
    if (!ok) {
      HIPCHECK(c, launch_fill_f32(seg, c->seg, 0.f, c->st));
      return fail(c, BRLS_ENONFINITE, "shot %lld: data hold NaN or Inf",
                  (long long)sh->id);
    }
  }
  sl.id = sh->id;
  sl.nt = sh->nt;
  sl.nrec = sh->nrec;
  sl.sz = sh->sz;
  sl.sy = ssy;
  sl.sx = sh->sx;
  sl.f0 = sh->f0;
  sl.rec.assign(sh->rec, sh->rec + 3 * sh->nrec);
  if (c->ndim != 3)
    for (int j = 0; j < sh->nrec; ++j) sl.rec[3 * j + 1] = 0;
  // h^2 * Ricker(f0), delay 1.5/f0: the point source of strength h^d f(t)
  // scaled to the W' = v^2 dt^2 / h^2 of the kernels.
  std::vector<float> wav(sh->nt);
  std::vector<double> wav64(sh->nt);
  const double t0 = 1.5 / sh->f0, pi = 3.14159265358979323846;
  for (int n = 0; n < sh->nt; ++n) {
    const double t = n * c->g.dt - t0;
    const double a = pi * pi * sh->f0 * sh->f0 * t * t;
    wav64[n] = c->g.h * c->g.h * (1.0 - 2.0 * a) * std::exp(-a);
    wav[n] = (float)wav64[n];
  }
  std::vector<int> rs(sh->nrec);
  for (int j = 0; j < sh->nrec; ++j)
    rs[j] = (int)store_index(c, sl.rec[3 * j] + c->g.nb,
                             sl.rec[3 * j + 1] + (c->ndim == 3 ? c->g.nb : 0),
                             sl.rec[3 * j + 2] + c->g.nb);
  HIPCHECK(c, hipMemcpyAsync(sl.wav, wav.data(), 4 * wav.size(),
                             hipMemcpyHostToDevice, c->st));
  if (sl.wav64)
    HIPCHECK(c, hipMemcpyAsync(sl.wav64, wav64.data(), 8 * wav64.size(),
                               hipMemcpyHostToDevice, c->st));
  HIPCHECK(c, hipMemcpyAsync(sl.rsidx, rs.data(), 4 * rs.size(),
                             hipMemcpyHostToDevice, c->st));
  int rc = build_receiver_tiles(c, sl);  // synchronises
  if (rc) return rc;
  sl.used = true;
  sl.weight = 1.f;
  sl.bg_ready = false;
  sl.seq = c->next_seq++;
  rebuild_order(c);
  return BRLS_OK;
}

int brls_downdate(brls_ctx* c, int64_t id) {
  if (!c) return BRLS_EINVAL;
  Range range("brls_downdate");
  const int i = find_slot(c, id);
  if (i < 0)
    return fail(c, BRLS_ENOSHOT, "no shot %lld in the window", (long long)id);
  Slot& sl = c->slots[i];
  for (float* v : {c->dobs, c->r, c->q, c->dscr})
    HIPCHECK(c, launch_fill_f32(v + sl.dat_off, c->seg, 0.f, c->st));
  sl.used = false;
  sl.bg_ready = false;
  rebuild_order(c);
  return BRLS_OK;
}

int brls_set_data(brls_ctx* c, int64_t id, const float* data) {
  if (!c || !data) return fail(c, BRLS_EINVAL, "NULL argument");
  const int i = find_slot(c, id);
  if (i < 0)
    return fail(c, BRLS_ENOSHOT, "no shot %lld in the window", (long long)id);
  Slot& sl = c->slots[i];
  const int64_t nd = (int64_t)sl.nt * sl.nrec;
  HIPCHECK(c, hipMemcpyAsync(c->dscr, data, nd * 4, in_kind(c), c->st));
  bool ok = true;
  int rc = check_finite(c, c->dscr, nd, &ok);
  if (rc) return rc;
  if (!ok) return fail(c, BRLS_ENONFINITE, "data hold NaN or Inf");
  HIPCHECK(c, hipMemcpyAsync(c->dobs + sl.dat_off, c->dscr, nd * 4,
                             hipMemcpyDeviceToDevice, c->st));
  HIPCHECK(c, hipStreamSynchronize(c->st));
  return BRLS_OK;
}

int brls_window(const brls_ctx* c, int64_t* ids, int32_t cap, int32_t* n) {
  if (!c || !n) return BRLS_EINVAL;
  *n = (int32_t)c->order.size();
  if (ids)
    for (int k = 0; k < *n && k < cap; ++k) ids[k] = c->slots[c->order[k]].id;
  return BRLS_OK;
}

int brls_window_data_size(const brls_ctx* c, int64_t* n) {
  if (!c || !n) return BRLS_EINVAL;
  int64_t s = 0;
  for (int i : c->order) s += (int64_t)c->slots[i].nt * c->slots[i].nrec;
  *n = s;
  return BRLS_OK;
}

namespace {

// brls_solve_window with float64 CG vectors: m, p, s (and the correction,
// the preconditioned direction) on the model, r on the data, all float64;
// the operators take float32 copies of p (or m) and of r (times the shot
// weights), and the adjoint's float64 image sum is taken before rounding.
// Same recurrences and stop test as the float32 form.
int solve_window64(brls_ctx* c, int32_t max_iter, double rtol,
                   brls_stats* st, bool weighted) {
  const double lam = c->g.lambda;
  const int64_t M = c->mplane, D = (int64_t)c->g.q_max * c->seg;
  const float* wts = weighted ? c->wslot : nullptr;
  double sc[2];
  int rc;
  // A x for a float64 model vector x
  auto born64 = [&](const double* x) -> int {
    HIPCHECK(c, launch_cvt_d2f(c->born_in, x, nullptr, 1, M, c->st));
    return born_of(c, c->born_in);
  };
  // A^T W x for a float64 data vector x; the image lands in g64
  auto adjoint64 = [&](const double* x) -> int {
    HIPCHECK(c, launch_cvt_d2f(c->dscr, x, wts, c->seg, D, c->st));
    return adjoint_of(c, c->dscr);
  };
  // r = d - A m (m64 is the image, kept between solves: a warm start is
  // not rounded to float32)
  if ((rc = born64(c->m64))) return rc;
  HIPCHECK(c, launch_sub_d(c->r64, c->dobs, c->q, D, c->st));
  const bool corr = c->regularize == 1;
  if (corr) HIPCHECK(c, launch_fill_f64(c->dm64, M, 0.0, c->st));
  const double* damped = corr ? c->dm64 : c->m64;
  if ((rc = adjoint64(c->r64))) return rc;
  HIPCHECK(c, launch_grad_norm_d(c->s64, c->g64, damped, lam, M, c->partial,
                                 c->scal, c->st));
  if ((rc = read_scalars(c, sc, 1))) return rc;
  double gamma = sc[0];
  if (!std::isfinite(gamma))
    return fail(c, BRLS_ENONFINITE, "non-finite gradient norm");
  st->s0_norm = std::sqrt(gamma);
  st->s_norm = st->s0_norm;
  double ref = 0.0;
  if (rtol > 0) {
    // ||A^T W d||: the observed data are float32 already
    if (weighted) {
      HIPCHECK(c, launch_scale_segments(c->dscr, c->dobs, c->wslot, c->seg, D,
                                        c->st));
      if ((rc = adjoint_of(c, c->dscr))) return rc;
    } else if ((rc = adjoint_of(c, c->dobs))) {
      return rc;
    }
    HIPCHECK(c, launch_dot_d(c->g64, c->g64, M, c->partial, c->scal, c->st));
    if ((rc = read_scalars(c, sc, 1))) return rc;
    ref = std::sqrt(sc[0]);
    st->ref_norm = ref;
  }
  double snorm = std::sqrt(gamma);
  const bool pre = c->precond != 0;
  if (pre) {
    if ((rc = build_minv(c))) return rc;
    HIPCHECK(c, launch_mul_fd(c->z64, c->minv, c->s64, M, c->st));
    HIPCHECK(c, launch_dot_d(c->s64, c->z64, M, c->partial, c->scal, c->st));
    if ((rc = read_scalars(c, sc, 1))) return rc;
    gamma = sc[0];
  }
  HIPCHECK(c, hipMemcpyAsync(c->p64, pre ? c->z64 : c->s64, M * 8,
                             hipMemcpyDeviceToDevice, c->st));
  for (int it = 0; it < max_iter; ++it) {
    if (gamma == 0.0) break;
    if (rtol > 0 && snorm <= rtol * ref) break;
    Range range("brls CG iteration");
    if ((rc = born64(c->p64))) return rc;
    if (weighted)
      HIPCHECK(c, launch_scale_segments(c->dscr, c->q, c->wslot, c->seg, D,
                                        c->st));
    HIPCHECK(c, launch_dot(c->q, weighted ? c->dscr : c->q, D, c->partial,
                           c->scal, c->st));
    HIPCHECK(c, launch_dot_d(c->p64, c->p64, M, c->partial, c->scal + 1,
                             c->st));
    if ((rc = read_scalars(c, sc, 2))) return rc;
    const double delta = sc[0] + lam * sc[1];
    if (!std::isfinite(delta))
      return fail(c, BRLS_ENONFINITE, "non-finite CG scalar delta");
    if (!(delta > 0.0))
      return fail(c, BRLS_EBREAKDOWN, "CG breakdown: delta = %g", delta);
    const double alpha = gamma / delta;
    HIPCHECK(c, launch_axpy_dd(c->m64, c->p64, alpha, M, c->st));
    if (corr) HIPCHECK(c, launch_axpy_dd(c->dm64, c->p64, alpha, M, c->st));
    HIPCHECK(c, launch_axpy_df(c->r64, c->q, -alpha, D, c->st));
    if ((rc = adjoint64(c->r64))) return rc;
    HIPCHECK(c, launch_grad_norm_d(c->s64, c->g64, damped, lam, M,
                                   c->partial, c->scal, c->st));
    if (pre) {
      HIPCHECK(c, launch_mul_fd(c->z64, c->minv, c->s64, M, c->st));
      HIPCHECK(c, launch_dot_d(c->s64, c->z64, M, c->partial, c->scal + 1,
                               c->st));
    }
    if ((rc = read_scalars(c, sc, pre ? 2 : 1))) return rc;
    const double gnew = pre ? sc[1] : sc[0];
    if (!std::isfinite(sc[0]) || !std::isfinite(gnew))
      return fail(c, BRLS_ENONFINITE, "non-finite gradient norm");
    const double beta = gnew / gamma;
    HIPCHECK(c, launch_xpby_d(c->p64, pre ? c->z64 : c->s64, beta, M, c->st));
    gamma = gnew;
    snorm = std::sqrt(sc[0]);
    st->iters = it + 1;
    st->s_norm = snorm;
    c->hist.insert(c->hist.end(), {alpha, beta, snorm});
  }
  HIPCHECK(c, launch_dot_d(c->r64, c->r64, D, c->partial, c->scal, c->st));
  if ((rc = read_scalars(c, sc, 1))) return rc;
  st->r_norm = std::sqrt(sc[0]);
  // the float32 image mirrors the float64 one
  HIPCHECK(c, launch_cvt_d2f(c->m, c->m64, nullptr, 1, M, c->st));
  return BRLS_OK;
}

}  // namespace

int brls_solve_window(brls_ctx* c, int32_t max_iter, double rtol,
                      brls_stats* stats) {
  if (!c) return BRLS_EINVAL;
  Range range("brls_solve_window");
  c->hist.clear();
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
  const int64_t M = c->mplane, D = (int64_t)c->g.q_max * c->seg;
  double sc[2];
  int rc;
  // per-shot misfit weights W (all 1 unless set): the adjoint takes W r
  // (written into the adjoint's input buffer) and delta = <q, W q> + ...
  c->wslot_h.assign(c->g.q_max, 1.f);
  bool weighted = false;
  for (int i = 0; i < (int)c->slots.size(); ++i)
    if (c->slots[i].used) {
      c->wslot_h[i] = c->slots[i].weight;
      weighted |= c->slots[i].weight != 1.f;
    }
  if (weighted)
    HIPCHECK(c, hipMemcpyAsync(c->wslot, c->wslot_h.data(),
                               (size_t)c->g.q_max * 4, hipMemcpyHostToDevice,
                               c->st));
  if (c->vec64) return finish(solve_window64(c, max_iter, rtol, &st, weighted));
  // adjoint of W x (x itself when unweighted)
  auto adjoint_w = [&](const float* x) -> int {
    if (!weighted) return adjoint_of(c, x);
    HIPCHECK(c, launch_scale_segments(c->dscr, x, c->wslot, c->seg, D, c->st));
    return adjoint_of(c, c->dscr);
  };
  // r = d - A m
  if ((rc = born_of(c, c->m))) return finish(rc);
  HIPCHECK(c, launch_sub(c->r, c->dobs, c->q, D, c->st));
  // s = A^T r - lambda m (correction mode: - lambda (m - m_start)),
  // gamma = ||s||^2
  const bool corr = c->regularize == 1;
  if (corr) HIPCHECK(c, launch_fill_f32(c->dm, M, 0.f, c->st));
  const float* damped = corr ? c->dm : c->m;
  if ((rc = adjoint_w(c->r))) return finish(rc);
  HIPCHECK(c, launch_grad_norm(c->s, c->gbuf, damped, lam, M, c->partial,
                               c->scal, c->st));
  if ((rc = read_scalars(c, sc, 1))) return finish(rc);
  double gamma = sc[0];
  if (!std::isfinite(gamma))
    return finish(fail(c, BRLS_ENONFINITE, "non-finite gradient norm"));
  st.s0_norm = std::sqrt(gamma);
  st.s_norm = st.s0_norm;
  double ref = 0.0;
  if (rtol > 0) {
    if ((rc = adjoint_w(c->dobs))) return finish(rc);
    HIPCHECK(c, launch_dot(c->gbuf, c->gbuf, M, c->partial, c->scal, c->st));
    if ((rc = read_scalars(c, sc, 1))) return finish(rc);
    ref = std::sqrt(sc[0]);
    st.ref_norm = ref;
  }
  // preconditioned form (diagonal illumination): directions follow
  // z = M^{-1} s and gamma = <s, z>; the stop test stays on ||s||
  double snorm = std::sqrt(gamma);
  const bool pre = c->precond != 0;
  if (pre) {
    if ((rc = build_minv(c))) return finish(rc);
    HIPCHECK(c, launch_mul(c->z, c->minv, c->s, M, c->st));
    HIPCHECK(c, launch_dot(c->s, c->z, M, c->partial, c->scal, c->st));
    if ((rc = read_scalars(c, sc, 1))) return finish(rc);
    gamma = sc[0];
  }
  HIPCHECK(c, hipMemcpyAsync(c->p, pre ? c->z : c->s, M * 4,
                             hipMemcpyDeviceToDevice, c->st));
  for (int it = 0; it < max_iter; ++it) {
    if (gamma == 0.0) break;
    if (rtol > 0 && snorm <= rtol * ref) break;
    Range range("brls CG iteration");
    if ((rc = born_of(c, c->p))) return finish(rc);
    if (weighted)
      HIPCHECK(c, launch_scale_segments(c->dscr, c->q, c->wslot, c->seg, D,
                                        c->st));
    HIPCHECK(c, launch_dot(c->q, weighted ? c->dscr : c->q, D, c->partial,
                           c->scal, c->st));
    HIPCHECK(c, launch_dot(c->p, c->p, M, c->partial, c->scal + 1, c->st));
    if ((rc = read_scalars(c, sc, 2))) return finish(rc);
    const double delta = sc[0] + lam * sc[1];
    if (!std::isfinite(delta))
      return finish(fail(c, BRLS_ENONFINITE, "non-finite CG scalar delta"));
    if (!(delta > 0.0))
      return finish(fail(c, BRLS_EBREAKDOWN, "CG breakdown: delta = %g",
                         delta));
    const double alpha = gamma / delta;
    HIPCHECK(c, launch_axpy(c->m, c->p, alpha, M, c->st));
    if (corr) HIPCHECK(c, launch_axpy(c->dm, c->p, alpha, M, c->st));
    HIPCHECK(c, launch_axpy(c->r, c->q, -alpha, D, c->st));
    if ((rc = adjoint_w(c->r))) return finish(rc);
    HIPCHECK(c, launch_grad_norm(c->s, c->gbuf, damped, lam, M, c->partial,
                                 c->scal, c->st));
    if (pre) {
      HIPCHECK(c, launch_mul(c->z, c->minv, c->s, M, c->st));
      HIPCHECK(c, launch_dot(c->s, c->z, M, c->partial, c->scal + 1, c->st));
    }
    if ((rc = read_scalars(c, sc, pre ? 2 : 1))) return finish(rc);
    const double gnew = pre ? sc[1] : sc[0];
    if (!std::isfinite(sc[0]) || !std::isfinite(gnew))
      return finish(fail(c, BRLS_ENONFINITE, "non-finite gradient norm"));
    const double beta = gnew / gamma;
    HIPCHECK(c, launch_xpby(c->p, pre ? c->z : c->s, beta, M, c->st));
    gamma = gnew;
    snorm = std::sqrt(sc[0]);
    st.iters = it + 1;
    st.s_norm = snorm;
    c->hist.insert(c->hist.end(), {alpha, beta, snorm});
  }
  HIPCHECK(c, launch_dot(c->r, c->r, D, c->partial, c->scal, c->st));
  if ((rc = read_scalars(c, sc, 1))) return finish(rc);
  st.r_norm = std::sqrt(sc[0]);
  HIPCHECK(c, launch_cvt_f2d(c->m64, c->m, M, c->st));
  return finish(BRLS_OK);
}

int brls_solve_history(brls_ctx* c, int32_t cap, double* alpha,
                       double* beta, double* s_norm, int32_t* n) {
  if (!c || !n || cap < 0) return fail(c, BRLS_EINVAL, "bad argument");
  const int32_t k = (int32_t)(c->hist.size() / 3);
  *n = k;
  for (int32_t i = 0; i < k && i < cap; ++i) {
    if (alpha) alpha[i] = c->hist[3 * i];
    if (beta) beta[i] = c->hist[3 * i + 1];
    if (s_norm) s_norm[i] = c->hist[3 * i + 2];
  }
  return BRLS_OK;
}

int brls_set_shot_weight(brls_ctx* c, int64_t id, double w) {
  if (!c) return BRLS_EINVAL;
  const int i = find_slot(c, id);
  if (i < 0)
    return fail(c, BRLS_ENOSHOT, "no shot %lld in the window", (long long)id);
  if (!(w >= 0.0) || !std::isfinite(w))
    return fail(c, BRLS_EINVAL, "shot weight %g: must be finite and >= 0", w);
  c->slots[i].weight = (float)w;
  return BRLS_OK;
}

int brls_get_shot_weight(const brls_ctx* c, int64_t id, double* w) {
  if (!c || !w) return BRLS_EINVAL;
  const int i = find_slot(c, id);
  if (i < 0) return BRLS_ENOSHOT;
  *w = c->slots[i].weight;
  return BRLS_OK;
}

int brls_image(brls_ctx* c, float* out) {
  if (!c || !out) return fail(c, BRLS_EINVAL, "NULL argument");
  HIPCHECK(c, hipMemcpyAsync(out, c->m, c->mplane * 4, out_kind(c), c->st));
  HIPCHECK(c, hipStreamSynchronize(c->st));
  return BRLS_OK;
}

int brls_set_precond(brls_ctx* c, int32_t mode) {
  if (!c) return BRLS_EINVAL;
  if (mode != 0 && mode != 1)
    return fail(c, BRLS_EINVAL, "preconditioner mode %d unknown", mode);
  if (mode == 1 && c->ckpt_k)
    return fail(c, BRLS_EINVAL,
                "the illumination preconditioner needs stored Born sources "
                "(checkpoint interval 0)");
  c->precond = mode;
  return BRLS_OK;
}

int brls_set_precision(brls_ctx* c, int32_t background, int32_t vectors) {
  if (!c) return BRLS_EINVAL;
  if ((background != 32 && background != 64) ||
      (vectors != 32 && vectors != 64))
    return fail(c, BRLS_EINVAL, "precision %d / %d: each must be 32 or 64",
                background, vectors);
  if (background == 64 && c->ckpt_k)
    return fail(c, BRLS_EINVAL,
                "a float64 background needs stored Born sources (checkpoint "
                "interval 0)");
  const int bg = background == 64;
  if (bg != c->bg64) {  // rebuild the window's stored sources
    for (Slot& sl : c->slots) sl.bg_ready = false;
    c->bg64 = bg;
  }
  c->vec64 = vectors == 64;
  return BRLS_OK;
}

int brls_get_precision(const brls_ctx* c, int32_t* background,
                       int32_t* vectors) {
  if (!c || !background || !vectors) return BRLS_EINVAL;
  *background = c->bg64 ? 64 : 32;
  *vectors = c->vec64 ? 64 : 32;
  return BRLS_OK;
}

int brls_set_regularization(brls_ctx* c, int32_t mode) {
  if (!c) return BRLS_EINVAL;
  if (mode != 0 && mode != 1)
    return fail(c, BRLS_EINVAL, "regularisation mode %d unknown", mode);
  c->regularize = mode;
  return BRLS_OK;
}

int brls_get_regularization(const brls_ctx* c, int32_t* mode) {
  if (!c || !mode) return BRLS_EINVAL;
  *mode = c->regularize;
  return BRLS_OK;
}

int brls_get_precond(const brls_ctx* c, int32_t* mode) {
  if (!c || !mode) return BRLS_EINVAL;
  *mode = c->precond;
  return BRLS_OK;
}

int brls_illumination(brls_ctx* c, float* out) {
  if (!c || !out) return fail(c, BRLS_EINVAL, "NULL argument");
  if (c->ckpt_k)
    return fail(c, BRLS_EINVAL,
                "the illumination needs stored Born sources (checkpoint "
                "interval 0)");
  int rc;
  if ((rc = window_illumination(c, c->gbuf))) return rc;
  HIPCHECK(c, hipMemcpyAsync(out, c->gbuf, c->mplane * 4, out_kind(c), c->st));
  HIPCHECK(c, hipStreamSynchronize(c->st));
  return BRLS_OK;
}

int brls_set_image(brls_ctx* c, const float* m) {
  if (!c || !m) return fail(c, BRLS_EINVAL, "NULL argument");
  HIPCHECK(c, hipMemcpyAsync(c->m, m, c->mplane * 4, in_kind(c), c->st));
  HIPCHECK(c, launch_cvt_f2d(c->m64, c->m, c->mplane, c->st));
  HIPCHECK(c, hipStreamSynchronize(c->st));
  return BRLS_OK;
}

int brls_image64(brls_ctx* c, double* out) {
  if (!c || !out) return fail(c, BRLS_EINVAL, "NULL argument");
  HIPCHECK(c, hipMemcpyAsync(out, c->m64, c->mplane * 8, out_kind(c), c->st));
  HIPCHECK(c, hipStreamSynchronize(c->st));
  return BRLS_OK;
}

int brls_set_image64(brls_ctx* c, const double* m) {
  if (!c || !m) return fail(c, BRLS_EINVAL, "NULL argument");
  HIPCHECK(c, hipMemcpyAsync(c->m64, m, c->mplane * 8, in_kind(c), c->st));
  HIPCHECK(c, launch_cvt_d2f(c->m, c->m64, nullptr, 1, c->mplane, c->st));
  HIPCHECK(c, hipStreamSynchronize(c->st));
  return BRLS_OK;
}

int brls_apply_born(brls_ctx* c, const float* m, float* d_out) {
  if (!c || !m || !d_out) return fail(c, BRLS_EINVAL, "NULL argument");
  Range range("brls_apply_born");
  HIPCHECK(c, hipMemcpyAsync(c->born_in, m, c->mplane * 4, in_kind(c), c->st));
  int rc = born_of(c, c->born_in);
  if (rc) return rc;
  int64_t off = 0;
  for (int i : c->order) {
    const Slot& sl = c->slots[i];
    const int64_t nd = (int64_t)sl.nt * sl.nrec;
    HIPCHECK(c, hipMemcpyAsync(d_out + off, c->q + sl.dat_off, nd * 4,
                               out_kind(c), c->st));
    off += nd;
  }
  HIPCHECK(c, hipStreamSynchronize(c->st));
  return BRLS_OK;
}

int brls_background_window(brls_ctx* c, float* out) {
  if (!c || !out) return fail(c, BRLS_EINVAL, "NULL argument");
  if (c->order.empty()) return BRLS_OK;
  int rc;
  if ((rc = ensure_tab(c))) return rc;
  // one batched background pass over the window's shots from rest, no
  // Born-source frames written (the stored ones stay valid); after each
  // step the receivers' samples of the new level go to their segments
  for (int i : c->order) {
    Slot& sl = c->slots[i];
    HIPCHECK(c, launch_fill_f32(c->ckpt_k ? sl.bgf : sl.fields,
                                (c->ckpt_k ? 3 : fields_per_slot(c)) * c->fs,
                                0.f, c->st));
  }
  HIPCHECK(c, launch_fill_f32(c->dscr, (int64_t)c->g.q_max * c->seg, 0.f,
                              c->st));
  const int nsh = (int)c->order.size();
  const int ntm = nt_max_of(c, c->order);
  for (int n = 0; n + 1 < ntm; ++n) {
    if ((rc = step(c, kBackground, n, c->tab_dev, nsh,
                   std::min(c->per_block, nsh), nullptr, nullptr, nullptr, 0,
                   0, 1, n & 1)))
      return rc;
    HIPCHECK(c, launch_gather_receivers(c->tab_dev, nsh, c->g.nrec_max, n,
                                        c->dscr, c->st));
  }
  int64_t off = 0;
  for (int i : c->order) {
    const Slot& sl = c->slots[i];
    const int64_t nd = (int64_t)sl.nt * sl.nrec;
    HIPCHECK(c, hipMemcpyAsync(out + off, c->dscr + sl.dat_off, nd * 4,
                               out_kind(c), c->st));
    off += nd;
  }
  HIPCHECK(c, hipStreamSynchronize(c->st));
  return BRLS_OK;
}

int brls_apply_adjoint(brls_ctx* c, const float* d, float* m_out) {
  if (!c || !d || !m_out) return fail(c, BRLS_EINVAL, "NULL argument");
  Range range("brls_apply_adjoint");
  HIPCHECK(c, launch_fill_f32(c->dscr, (int64_t)c->g.q_max * c->seg, 0.f,
                              c->st));
  int64_t off = 0;
  for (int i : c->order) {
    const Slot& sl = c->slots[i];
    const int64_t nd = (int64_t)sl.nt * sl.nrec;
    HIPCHECK(c, hipMemcpyAsync(c->dscr + sl.dat_off, d + off, nd * 4,
                               in_kind(c), c->st));
    off += nd;
  }
  int rc = adjoint_of(c, c->dscr);
  if (rc) return rc;
  if (c->order.empty())
    HIPCHECK(c, launch_fill_f32(c->gbuf, c->mplane, 0.f, c->st));
  HIPCHECK(c, hipMemcpyAsync(m_out, c->gbuf, c->mplane * 4, out_kind(c),
                             c->st));
  HIPCHECK(c, hipStreamSynchronize(c->st));
  return BRLS_OK;
}

int brls_apply_adjoint_static(brls_ctx* c, const float* d, float* m_out) {
  if (!c || !d || !m_out) return fail(c, BRLS_EINVAL, "NULL argument");
  hipError_t e = hipSuccess;
  double* acc = scratch_dev(c->device, &e);
  if (!acc)
    return fail(c, BRLS_EDEVICE, "static scratch unavailable: %s",
                hipGetErrorString(e));
  const int64_t need = adjoint_acc_doubles(c, 1);
  if (need * 8 > kScratchBytes)
    return fail(c, BRLS_EINVAL,
                "the window's image accumulators need %lld bytes; the static "
                "scratch holds %lld (fewer shots per window, more shots per "
                "adjoint work item, or brls_apply_adjoint)",
                (long long)(need * 8), (long long)kScratchBytes);
  int rc;
  if ((rc = ensure_tab(c)) || (rc = ensure_backgrounds(c)) ||
      (rc = ensure_tab(c)))
    return rc;
  HIPCHECK(c, launch_fill_f32(c->dscr, (int64_t)c->g.q_max * c->seg, 0.f,
                              c->st));
  int64_t off = 0;
  for (int i : c->order) {
    const Slot& sl = c->slots[i];
    const int64_t nd = (int64_t)sl.nt * sl.nrec;
    HIPCHECK(c, hipMemcpyAsync(c->dscr + sl.dat_off, d + off, nd * 4,
                               in_kind(c), c->st));
    off += nd;
  }
  if (c->order.empty()) {
    HIPCHECK(c, launch_fill_f32(c->gbuf, c->mplane, 0.f, c->st));
  } else {
    // batched launches, no graph (instantiating one may allocate) and no
    // per-launch timing events
    const bool was_timing = c->timing;
    c->timing = false;
    rc = enqueue_adjoint(c, 1, acc);
    c->timing = was_timing;
    if (rc) return rc;
  }
  HIPCHECK(c, hipMemcpyAsync(m_out, c->gbuf, c->mplane * 4, out_kind(c),
                             c->st));
  HIPCHECK(c, hipStreamSynchronize(c->st));
  return BRLS_OK;
}

int brls_set_chains(brls_ctx* c, int32_t n) {
  if (!c) return BRLS_EINVAL;
  if (n != 1 && n != 2)
    return fail(c, BRLS_EINVAL, "launch chains: %d (1 or 2)", n);
  c->chains = n;
  return BRLS_OK;
}

int brls_get_chains(const brls_ctx* c, int32_t* n) {
  if (!c || !n) return BRLS_EINVAL;
  *n = c->chains;
  return BRLS_OK;
}

int brls_set_exec(brls_ctx* c, int32_t mode) {
  if (!c) return BRLS_EINVAL;
  if (mode < BRLS_EXEC_PLAIN || mode > BRLS_EXEC_PERSISTENT)
    return fail(c, BRLS_EINVAL, "unknown exec mode %d", mode);
  if (mode == BRLS_EXEC_PERSISTENT && !persistent_ok(c, c->variant))
    return fail(c, BRLS_EINVAL,
                "persistent execution needs a 2-D context with stored Born "
                "sources and a segment-marching tile variant (kind 4); "
                "variant %d is kind %d",
                c->variant, tile_shape(c->variant).pipe);
  c->exec = mode;
  return BRLS_OK;
}

int brls_set_zchunk(brls_ctx* c, int32_t planes) {
  if (!c) return BRLS_EINVAL;
  if (c->ndim != 3)
    return fail(c, BRLS_EINVAL, "z chunks are a 3-D launch parameter");
  if (planes < 1 || planes > 4096)
    return fail(c, BRLS_EINVAL, "z chunk of %d planes out of range", planes);
  HIPCHECK(c, hipStreamSynchronize(c->st));
  c->zchunk = planes;
  set_variant_geo(c, c->variant);
  drop_graphs(c);
  return BRLS_OK;
}

int brls_get_zchunk(const brls_ctx* c, int32_t* planes) {
  if (!c || !planes) return BRLS_EINVAL;
  *planes = c->zchunk;
  return BRLS_OK;
}

int brls_set_spin_limit(brls_ctx* c, int32_t polls) {
  if (!c) return BRLS_EINVAL;
  if (polls < 0) return fail(c, BRLS_EINVAL, "spin limit %d < 0", polls);
  c->spin_limit = polls;
  drop_graphs(c);  // the limit is a kernel argument baked into graphs
  return BRLS_OK;
}

int brls_tile_count(int32_t* n) {
  if (!n) return BRLS_EINVAL;
  *n = tile_shape_count();
  return BRLS_OK;
}

int brls_tile3_count(int32_t* n) {
  if (!n) return BRLS_EINVAL;
  *n = tile_shape3_count();
  return BRLS_OK;
}

int brls_tile3_info(int32_t v, int32_t* tx, int32_t* ty, int32_t* shots) {
  if (v < 0 || v >= tile_shape3_count()) return BRLS_EINVAL;
  const TileShape3 s = tile_shape3(v);
  if (tx) *tx = s.tx;
  if (ty) *ty = s.ty;
  if (shots) *shots = s.sb;
  return BRLS_OK;
}

int brls_tile_info(int32_t v, int32_t* tx, int32_t* tz, int32_t* rows,
                   int32_t* pipelined) {
  if (v < 0 || v >= tile_shape_count()) return BRLS_EINVAL;
  const TileShape s = tile_shape(v);
  if (tx) *tx = s.tx;
  if (tz) *tz = s.tz;
  if (rows) *rows = s.ntz;
  if (pipelined) *pipelined = s.pipe;
  return BRLS_OK;
}

static int set_tile_impl(brls_ctx* c, int v, int per_block,
                         int adj_per_block) {
  if (v < 0 || v >= variant_count(c))
    return fail(c, BRLS_EINVAL, "tile variant %d out of range", v);
  if (c->ndim == 2 && c->ckpt_k && tile_shape(v).pipe >= 3)
    return fail(c, BRLS_EINVAL,
                "tile variant %d takes two steps per launch and needs stored "
                "Born sources (checkpoint interval 0)",
                v);
  if (c->exec == BRLS_EXEC_PERSISTENT && !persistent_ok(c, v))
    return fail(c, BRLS_EINVAL,
                "tile variant %d cannot run in persistent execution (needs "
                "kind 4)", v);
  if (per_block < 1) per_block = 1;
  if (adj_per_block < 1) adj_per_block = 1;
  // segment-marching variants run one wavefront per shot of a block
  if (c->ndim == 2 && tile_shape(v).pipe == 4 &&
      (per_block > 8 || adj_per_block > 8))
    return fail(c, BRLS_EINVAL,
                "tile variant %d runs at most 8 shots per work item", v);
  // 3-D kernels advance a fixed number of shots per block together
  if (c->ndim == 3) per_block = adj_per_block = tile_shape3(v).sb;
  HIPCHECK(c, hipStreamSynchronize(c->st));
  // the geometry follows the variant and (3-D) the z chunk; captured
  // graphs hold it, the receiver bins follow the variant's tile shape
  const int old_tiles = c->ndim == 3 ? c->geo3.ntiles : c->geo.ntiles;
  const int old_tzc = c->geo3.tzc;
  const bool changed = v != c->variant;
  set_variant_geo(c, v);
  c->per_block = per_block;
  c->adj_per_block = adj_per_block;
  const int new_tiles = c->ndim == 3 ? c->geo3.ntiles : c->geo.ntiles;
  if (changed || new_tiles != old_tiles || c->geo3.tzc != old_tzc)
    drop_graphs(c);
  if (v != c->bins_variant) {
    for (auto& sl : c->slots)
      if (sl.used) {
        int rc = build_receiver_tiles(c, sl);
        if (rc) return rc;
      }
    c->bins_variant = v;
  }
  return BRLS_OK;
}

int brls_set_tile(brls_ctx* c, int32_t variant) {
  if (!c) return BRLS_EINVAL;
  return set_tile_impl(c, variant < 0 ? 0 : variant, c->per_block,
                       c->adj_per_block);
}

int brls_set_shots_per_block(brls_ctx* c, int32_t per_block) {
  if (!c || per_block < 1)
    return fail(c, BRLS_EINVAL, "shots per block must be >= 1");
  if (c->ndim == 3 && per_block != tile_shape3(c->variant).sb)
    return fail(c, BRLS_EINVAL,
                "3-D tile variant %d advances %d shots per block", c->variant,
                tile_shape3(c->variant).sb);
  c->per_block = c->adj_per_block = per_block;
  return BRLS_OK;
}

int brls_autotune(brls_ctx* c, int32_t* best) {
  if (!c) return BRLS_EINVAL;
  int rc;
  if ((rc = ensure_tab(c)) || (rc = ensure_backgrounds(c)) ||
      (rc = ensure_tab(c)))
    return rc;
  const int nsh = (int)c->order.size();
  if (nsh == 0) {
    if (best) *best = c->variant;
    return BRLS_OK;
  }
  const int saved_exec = c->exec;
  const int saved_v = c->variant, saved_pb = c->per_block,
            saved_apb = c->adj_per_block, saved_rg = c->resident_grid,
            saved_arg = c->adj_resident_grid, saved_zc = c->zchunk;
  int best_v = saved_v, best_pb = saved_pb, best_apb = saved_apb,
      best_rg = saved_rg, best_arg = saved_arg, best_zc = saved_zc;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  // time one operator application with the current settings
  auto timed = [&](int op, float* ms) -> int {
    HIPCHECK(c, hipEventRecord(e0, c->st));
    const int r =
        op == kBorn ? enqueue_born(c, 1) : enqueue_adjoint(c, 1, c->acc);
    if (r) return r;
    HIPCHECK(c, hipEventRecord(e1, c->st));
    HIPCHECK(c, hipEventSynchronize(e1));
    HIPCHECK(c, hipEventElapsedTime(ms, e0, e1));
    return BRLS_OK;
  };
  auto trials = [&]() -> int {
    HIPCHECK(c, hipEventCreate(&e0));
    HIPCHECK(c, hipEventCreate(&e1));
    c->exec = BRLS_EXEC_BATCHED;
    // trials run a few hundred time steps (the kernels' cost per step does
    // not depend on the step index)
    c->tune_nt = 400;
    float best_total = 1e30f;
    // 3-D: z planes per work item 8, 16, 32, 64; 2-D: one pass
    const int nzc = c->ndim == 3 ? 4 : 1;
    for (int zi = 0; zi < nzc; ++zi)
    for (int v = 0; v < variant_count(c); ++v) {
      if (c->ndim == 2 && c->ckpt_k && tile_shape(v).pipe >= 3) continue;
      if (saved_exec == BRLS_EXEC_PERSISTENT && !persistent_ok(c, v))
        continue;
      if (c->ndim == 3) c->zchunk = 8 << zi;
      // the tile shape fixes the receiver lists; shots per block and grid
      // shape are chosen per operator
      float bt[2] = {1e30f, 1e30f};
      int bpb[2] = {1, 1}, brg[2] = {0, 0};
      // shots per block 1, 2, 4, 8 x grid shape: one block per item,
      // resident grid, items in launch order (2-D only); two-step 2-D
      // variants also with strips varying fastest (bit 2)
      const bool xf = c->ndim == 2 && tile_shape(v).pipe >= 3;
      static const int kShapes2D[] = {0, 1, 2, 4, 5};
      const int nshape = c->ndim == 3 ? 2 : (xf ? 5 : 3);
      for (int trial = 0; trial < 4 * nshape; ++trial) {
        int pb = 1 << (trial / nshape);
        const int rg = c->ndim == 3 ? trial % nshape
                                    : kShapes2D[trial % nshape];
        if (c->ndim == 3) {  // shots per block fixed by the variant
          if (trial >= nshape) break;
          pb = tile_shape3(v).sb;
        }
        if (pb > nsh && pb > 1) break;
        int r;
        // set_tile_impl sets the geometry for the variant and z chunk and
        // rebuilds the receiver bins when the tile shape changes
        if ((r = set_tile_impl(c, v, pb, pb))) return r;
        c->resident_grid = c->adj_resident_grid = rg;
        for (int k = 0; k < 2; ++k) {
          float ms = 0.f;
          if ((r = timed(k == 0 ? kBorn : kAdjoint, &ms))) return r;
          if (ms < bt[k]) {
            bt[k] = ms;
            bpb[k] = pb;
            brg[k] = rg;
          }
        }
      }
      if (bt[0] + bt[1] < best_total) {
        best_total = bt[0] + bt[1];
        best_v = v;
        best_pb = bpb[0];
        best_apb = bpb[1];
        best_rg = brg[0];
        best_arg = brg[1];
        best_zc = c->zchunk;
      }
    }
    return BRLS_OK;
  };
  rc = trials();
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  c->exec = saved_exec;
  c->tune_nt = 0;
  if (rc) {  // restore the previous choice
    c->resident_grid = saved_rg;
    c->adj_resident_grid = saved_arg;
    c->zchunk = saved_zc;
    (void)set_tile_impl(c, saved_v, saved_pb, saved_apb);
    return rc;
  }
  c->resident_grid = best_rg;
  c->adj_resident_grid = best_arg;
  c->zchunk = best_zc;
  if ((rc = set_tile_impl(c, best_v, best_pb, best_apb))) return rc;
  if (best) *best = best_v;
  return BRLS_OK;
}

int brls_set_tuning(brls_ctx* c, int32_t variant, int32_t born_pb,
                    int32_t born_grid, int32_t adj_pb, int32_t adj_grid) {
  if (!c) return BRLS_EINVAL;
  if (born_pb < 1 || adj_pb < 1)
    return fail(c, BRLS_EINVAL, "shots per block must be >= 1");
  const int rc = set_tile_impl(c, variant, born_pb, adj_pb);
  if (rc) return rc;
  c->resident_grid = born_grid & 7;
  c->adj_resident_grid = adj_grid & 7;
  return BRLS_OK;
}

int brls_get_tuning(const brls_ctx* c, int32_t* variant, int32_t* born_pb,
                    int32_t* born_grid, int32_t* adj_pb, int32_t* adj_grid) {
  if (!c) return BRLS_EINVAL;
  if (variant) *variant = c->variant;
  if (born_pb) *born_pb = c->per_block;
  if (born_grid) *born_grid = c->resident_grid;
  if (adj_pb) *adj_pb = c->adj_per_block;
  if (adj_grid) *adj_grid = c->adj_resident_grid;
  return BRLS_OK;
}

int brls_get_tile(const brls_ctx* c, int32_t* variant, int32_t* per_block) {
  if (!c) return BRLS_EINVAL;
  if (variant) *variant = c->variant;
  if (per_block) *per_block = c->per_block;
  return BRLS_OK;
}

int brls_set_resident_grid(brls_ctx* c, int32_t enable) {
  if (!c) return BRLS_EINVAL;
  c->resident_grid = c->adj_resident_grid = enable != 0;
  return BRLS_OK;
}

int brls_get_resident_grid(const brls_ctx* c, int32_t* enable) {
  if (!c || !enable) return BRLS_EINVAL;
  *enable = c->resident_grid;
  return BRLS_OK;
}

int brls_kernel_timing(brls_ctx* c, int32_t enable) {
  if (!c) return BRLS_EINVAL;
  c->timing = enable != 0;
  return BRLS_OK;
}

int brls_kernel_stats(brls_ctx* c, brls_kstat* out, int32_t cap, int32_t* n) {
  if (!c || !n) return BRLS_EINVAL;
  HIPCHECK(c, hipStreamSynchronize(c->st));
  int64_t cnt[kTNumKinds] = {0};
  double tot[kTNumKinds] = {0};
  for (auto& t : c->timers) {
    float ms = 0.f;
    HIPCHECK(c, hipEventElapsedTime(&ms, t.a, t.b));
    cnt[t.kind]++;
    tot[t.kind] += ms;
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  c->timers.clear();
  int k = 0;
  for (int i = 0; i < kTNumKinds; ++i) {
    if (!cnt[i]) continue;
    if (out && k < cap) {
      std::snprintf(out[k].name, sizeof out[k].name, "%s", kTimerNames[i]);
      out[k].launches = cnt[i];
      out[k].total_ms = tot[i];
    }
    ++k;
  }
  *n = k;
  return BRLS_OK;
}

int brls_memory_bytes(const brls_ctx* c, int64_t* bytes) {
  if (!c || !bytes) return BRLS_EINVAL;
  *bytes = c->mem_bytes;
  return BRLS_OK;
}

int brls_sync(brls_ctx* c) {
  if (!c) return BRLS_EINVAL;
  HIPCHECK(c, hipStreamSynchronize(c->st));
  return BRLS_OK;
}

}  // extern "C"
