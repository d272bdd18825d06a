// Host runtime of the gtod C-ABI: contexts, the HBM budget, resident
// screens and spectral setups, per-stream workspaces, job validation and
// the enqueue of the panel / contraction / 1/f kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/gtod.h"
#include "gtod_internal.h"

using namespace gtod;

namespace {

struct ScreenObj {
  double* pwv = nullptr;
  int64_t nx = 0, ny = 0;
  double dx = 0, dy = 0, ix0 = 0, iy0 = 0, h = 0, wind = 0;
  double vmin = NAN, vmax = NAN;
  size_t bytes = 0;
};

struct SpecObj {
  int F = 0, Fp = 0, K = 0, Kp = 0, n_pwv = 0;
  double pwv0 = 0, dpwv = 0;
  float* tau = nullptr;
  float* E = nullptr;
  float* D = nullptr;
  float* W = nullptr;
  float* Pref = nullptr;
  float* B = nullptr;
  uint16_t* Bh = nullptr;
  uint16_t* Bl = nullptr;
  uint16_t* Bt = nullptr;   // Bh / Bl tiled for the split contraction
  double* c0 = nullptr;
  double* c1 = nullptr;
  int pexp = 0;   // the panel carries spectral powers times 2^pexp
  std::vector<double> nep2ref;
  // FP64 tables kept for the skydip, and its brightness-temperature scale
  double t_atm = 0;
  double* tau64 = nullptr;
  double* E64 = nullptr;
  double* D64 = nullptr;
  double* B0_64 = nullptr;
  double* kel_a = nullptr;
  double* kel_b = nullptr;
  double* kel_ib = nullptr;
  bool has_kelvin = false;
  std::vector<double> kel_ib_h;
  std::vector<void*> allocs;
};

constexpr int kSlots = 8;
constexpr size_t kSlotBytes = 1 << 20;

// Device scratch of gtod_simulate_tod_noalloc: one copy per GPU, resident
// from the library's first use on that device until the process ends.  In
// host code this name is only a stand-in for the symbol; the device
// address comes from hipGetSymbolAddress (scratch_address below).
static __device__ __align__(256) unsigned char scratch[GTOD_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;   // device -> address of its scratch

// Address of `scratch` on `dev`, which must be the current device; looked
// up once per device.
hipError_t scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) {
    *out = it->second;
    return hipSuccess;
  }
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[dev] = p;
  *out = p;
  return hipSuccess;
}

struct StreamWs {
  hipStream_t stream = nullptr;
  float* panel = nullptr;
  size_t panel_bytes = 0;
  float2* pink = nullptr;
  size_t pink_bytes = 0;
  char* h_stage = nullptr;
  char* d_stage = nullptr;
  hipEvent_t ev[kSlots] = {};
  bool ev_used[kSlots] = {};
  int slot = 0;
};

}  // namespace

struct gtod_ctx {
  int device = 0;
  int precision = GTOD_PREC_FP32;
  uint32_t flags = 0;
  uint64_t budget = 0, used = 0, ws_bytes = 0;
  double fs = 0, eta_taper = 0, rho_surf = 0, eta_pol = 0, delta_J = 0,
         eta_pb = 0, t_cmb = 0;
  std::map<int32_t, ScreenObj> screens;
  std::map<int32_t, SpecObj> specs;
  int32_t next_id = 1;
  std::map<void*, size_t> sizes;
  std::map<hipStream_t, StreamWs> ws;
  // gtod_simulate_tod_noalloc: device areas inside the per-GPU scratch,
  // pinned staging and events made at init
  StreamWs na;
  unsigned long long* counters = nullptr;
  hipStream_t sink_streams[2] = {nullptr, nullptr};  // out-of-core runs
  std::string err;
  // profiling
  bool prof = false;
  struct Rec { int kernel; hipEvent_t a, b; double units; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> ev_pool;
  double prof_ms[GTOD_N_KERNELS] = {}, prof_n[GTOD_N_KERNELS] = {},
         prof_units[GTOD_N_KERNELS] = {};
};

namespace {

std::string g_init_err;

gtod_status fail(gtod_ctx* c, gtod_status st, const std::string& msg) {
  if (c) c->err = msg; else g_init_err = msg;
  return st;
}

#define HIP_TRY(ctx, expr)                                                  \
  do {                                                                      \
    hipError_t e_ = (expr);                                                 \
    if (e_ != hipSuccess)                                                   \
      return fail(ctx, GTOD_EDEVICE,                                        \
                  std::string(#expr) + ": " + hipGetErrorString(e_));       \
  } while (0)

gtod_status dev_alloc(gtod_ctx* c, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 256;
  if (c->used + bytes > c->budget)
    return fail(c, GTOD_EBUDGET, "allocation of " + std::to_string(bytes) +
                                     " bytes exceeds the HBM budget");
  if (hipMalloc(p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(c, GTOD_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  c->used += bytes;
  c->sizes[*p] = bytes;
  return GTOD_OK;
}

void dev_free(gtod_ctx* c, void* p) {
  if (!p) return;
  auto it = c->sizes.find(p);
  if (it != c->sizes.end()) {
    c->used -= it->second;
    c->sizes.erase(it);
  }
  (void)hipFree(p);
}

void free_spec(gtod_ctx* c, SpecObj& s) {
  for (void* p : s.allocs) dev_free(c, p);
  s.allocs.clear();
}

void free_ws(gtod_ctx* c, StreamWs& w) {
  dev_free(c, w.panel);
  dev_free(c, w.pink);
  dev_free(c, w.d_stage);
  if (w.h_stage) (void)hipHostFree(w.h_stage);
  for (int i = 0; i < kSlots; ++i)
    if (w.ev[i]) (void)hipEventDestroy(w.ev[i]);
  w = StreamWs{};
}

// Byte sizes of a stream workspace's panel and 1/f areas.
void ws_sizes(const gtod_ctx* c, size_t* panel_bytes, size_t* pink_bytes) {
  *panel_bytes = round_up((int64_t)(c->ws_bytes * 3 / 4), 256);
  *pink_bytes = std::max<int64_t>(round_up((int64_t)(c->ws_bytes - *panel_bytes), 256),
                                  2 * kPinkTableFloat2 * (int64_t)sizeof(float2));
}

gtod_status get_ws(gtod_ctx* c, hipStream_t s, StreamWs** out) {
  auto it = c->ws.find(s);
  if (it != c->ws.end()) {
    *out = &it->second;
    return GTOD_OK;
  }
  StreamWs w;
  w.stream = s;
  ws_sizes(c, &w.panel_bytes, &w.pink_bytes);
  gtod_status st;
  if ((st = dev_alloc(c, (void**)&w.panel, w.panel_bytes)) != GTOD_OK ||
      (st = dev_alloc(c, (void**)&w.pink, w.pink_bytes)) != GTOD_OK ||
      (st = dev_alloc(c, (void**)&w.d_stage, kSlots * kSlotBytes)) != GTOD_OK) {
    free_ws(c, w);
    return st;
  }
  if (hipHostMalloc((void**)&w.h_stage, kSlots * kSlotBytes, hipHostMallocDefault) !=
      hipSuccess) {
    (void)hipGetLastError();
    free_ws(c, w);
    return fail(c, GTOD_ENOMEM, "pinned staging allocation failed");
  }
  for (int i = 0; i < kSlots; ++i) {
    if (hipEventCreateWithFlags(&w.ev[i], hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      free_ws(c, w);
      return fail(c, GTOD_EDEVICE, "event creation failed");
    }
  }
  auto res = c->ws.emplace(s, w);
  *out = &res.first->second;
  return GTOD_OK;
}

static_assert(GTOD_NOALLOC_SCRATCH_BYTES % 256 == 0 &&
                  GTOD_NOALLOC_SCRATCH_BYTES >= 2 * kSlots * kSlotBytes,
              "no-alloc scratch too small for the staging slots");

// Workspace of gtod_simulate_tod_noalloc, set up once by gtod_sim_init:
// the device staging slots at the head of the GPU's scratch, then one
// area that the panel (SIGNAL jobs) and the 1/f transform scratch (PINK
// jobs) share -- the jobs of a call run one after another on one stream,
// and every kernel writes what it later reads.  The pinned host slots and
// their events are made here, so the call itself allocates nothing.
gtod_status init_noalloc(gtod_ctx* c) {
  void* base = nullptr;
  const hipError_t e = scratch_address(c->device, &base);
  if (e != hipSuccess)
    return fail(c, GTOD_EDEVICE,
                std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  StreamWs& w = c->na;
  w.d_stage = static_cast<char*>(base);
  w.panel = reinterpret_cast<float*>(static_cast<char*>(base) + kSlots * kSlotBytes);
  w.panel_bytes = GTOD_NOALLOC_SCRATCH_BYTES - kSlots * kSlotBytes;
  w.pink = reinterpret_cast<float2*>(w.panel);
  w.pink_bytes = w.panel_bytes;
  if (hipHostMalloc((void**)&w.h_stage, kSlots * kSlotBytes, hipHostMallocDefault) !=
      hipSuccess) {
    (void)hipGetLastError();
    w.h_stage = nullptr;
    return fail(c, GTOD_ENOMEM, "pinned staging allocation failed");
  }
  for (int i = 0; i < kSlots; ++i) {
    if (hipEventCreateWithFlags(&w.ev[i], hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      w.ev[i] = nullptr;
      return fail(c, GTOD_EDEVICE, "event creation failed");
    }
  }
  return GTOD_OK;
}

// Releases what init_noalloc made (the device scratch itself stays).
void free_noalloc(StreamWs& w) {
  if (w.h_stage) (void)hipHostFree(w.h_stage);
  for (int i = 0; i < kSlots; ++i)
    if (w.ev[i]) (void)hipEventDestroy(w.ev[i]);
  w = StreamWs{};
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

hipEvent_t pool_event(gtod_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

// Runs launch() on stream s; with profiling on, brackets it by events.
template <class Fn>
void timed(gtod_ctx* c, int kernel, double units, hipStream_t s, Fn launch) {
  if (!c->prof) {
    launch();
    return;
  }
  hipEvent_t a = pool_event(c), b = pool_event(c);
  if (a && b) (void)hipEventRecord(a, s);
  launch();
  if (a && b) {
    (void)hipEventRecord(b, s);
    c->recs.push_back({kernel, a, b, units});
  }
}

void drain_profile(gtod_ctx* c) {
  for (auto& r : c->recs) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      c->prof_ms[r.kernel] += ms;
      c->prof_n[r.kernel] += 1;
      c->prof_units[r.kernel] += r.units;
    } else {
      (void)hipGetLastError();
    }
    c->ev_pool.push_back(r.a);
    c->ev_pool.push_back(r.b);
  }
  c->recs.clear();
}

struct JobPlan {
  const gtod_job* j;
  const ScreenObj* scr;
  const SpecObj* spec;
  int precision;
  size_t off_dphi, off_dtheta, off_scale, off_alpha;
  // SIGNAL: cube-cell buckets, rows per chunk, pixels and samples per chunk
  int n_buckets, cell_shift, n_az_c, pg;
  int64_t rows_cap, Tc_max;
  // PINK: series per batch
  int64_t pink_per;
};

// Chunking of a validated job in areas of the given sizes: how many rows
// (SIGNAL) or series (PINK) one launch takes.  EINVAL when not even the
// smallest unit fits, before anything is enqueued.
gtod_status plan_chunks(gtod_ctx* c, JobPlan* pl, int idx, size_t panel_bytes,
                        size_t pink_bytes, const char* ws_name) {
  const gtod_job& j = *pl->j;
  const SpecObj& f = *pl->spec;
  const std::string at = "job " + std::to_string(idx) + ": ";
  if (j.kind == GTOD_JOB_PINK) {
    int64_t N = 2;
    while (N < j.t_total) N *= 2;
    const int64_t M = N / 2;
    const size_t scratch_bytes = pink_bytes - kPinkTableFloat2 * sizeof(float2);
    const int64_t S = (int64_t)j.n_pix * f.K;
    // a single-pass transform (M <= 2048) needs no scratch
    int64_t per = M > (1 << kPinkLgM2) ? (int64_t)(scratch_bytes / ((size_t)M * sizeof(float2))) : S;
    per = std::min<int64_t>(std::min<int64_t>(per, S), 65535);
    if (per < 1) return fail(c, GTOD_EINVAL, at + "1/f series too long for " + ws_name);
    pl->pink_per = per;
    return GTOD_OK;
  }
  // with a source cube the rows are bucketed by coarse cube cell (at most
  // kPanelMaxBuckets cells); each row then also needs a record, a key and
  // an order slot beside its panel row
  int n_buckets = 1, cell_shift = 0, n_az_c = 0;
  if (j.cube) {
    for (;; ++cell_shift) {
      const int64_t ne = ((int64_t)j.n_el + (1 << cell_shift) - 1) >> cell_shift;
      const int64_t na = ((int64_t)j.n_az + (1 << cell_shift) - 1) >> cell_shift;
      if (ne * na <= kPanelMaxBuckets) {
        n_buckets = (int)(ne * na) + 1;
        n_az_c = (int)na;
        break;
      }
    }
  }
  const int64_t per_row = (int64_t)f.Fp * 4 + (n_buckets > 1 ? kPanelRowInfoBytes + 8 : 0);
  const int64_t hist_bytes = round_up((int64_t)n_buckets * 4, 256);
  const int64_t rows_cap = std::max<int64_t>(
      0, ((int64_t)panel_bytes - hist_bytes - 4 * 256) / per_row);
  int pg;          // pixels per chunk
  int64_t Tc_max;  // samples per chunk
  if ((int64_t)j.n_pix * kRowPad <= rows_cap) {
    pg = j.n_pix;
    Tc_max = std::max<int64_t>(kRowPad, rows_cap / j.n_pix / kRowPad * kRowPad);
  } else {
    pg = (int)std::max<int64_t>(1, rows_cap / kRowPad);
    Tc_max = kRowPad;
  }
  if ((int64_t)pg * kRowPad > rows_cap)
    return fail(c, GTOD_EINVAL, at + "frequency axis too long for " + ws_name);
  Tc_max = std::min<int64_t>(Tc_max, round_up(std::max<int64_t>(j.t_end - j.t_begin, 1), kRowPad));
  pl->n_buckets = n_buckets;
  pl->cell_shift = cell_shift;
  pl->n_az_c = n_az_c;
  pl->rows_cap = rows_cap;
  pl->pg = pg;
  pl->Tc_max = Tc_max;
  return GTOD_OK;
}

gtod_status validate(gtod_ctx* c, const gtod_job& j, int idx, JobPlan* pl) {
  const std::string at = "job " + std::to_string(idx) + ": ";
  if (j.kind != GTOD_JOB_SIGNAL && j.kind != GTOD_JOB_PINK)
    return fail(c, GTOD_EINVAL, at + "unknown kind");
  auto sp = c->specs.find(j.spec_id);
  if (sp == c->specs.end()) return fail(c, GTOD_ENOTFOUND, at + "unknown spec_id");
  pl->spec = &sp->second;
  pl->scr = nullptr;
  if (j.n_pix < 1) return fail(c, GTOD_EINVAL, at + "n_pix < 1");
  if (j.pix0 < 0 || (int64_t)j.pix0 + j.n_pix > ((int64_t)1 << 31))
    return fail(c, GTOD_EINVAL, at + "pix0 out of range");
  if (!j.tod) return fail(c, GTOD_EINVAL, at + "tod is NULL");
  if (j.t_total < 1 || j.t_total > (int64_t)1 << 31)
    return fail(c, GTOD_EINVAL, at + "t_total out of range");
  if (j.flags & ~(GTOD_JOB_PHOTON_NOISE | GTOD_JOB_ACCUMULATE | GTOD_JOB_KELVIN))
    return fail(c, GTOD_EINVAL, at + "unknown flags");
  if ((j.flags & GTOD_JOB_KELVIN) && !pl->spec->has_kelvin)
    return fail(c, GTOD_EINVAL, at + "KELVIN output needs a brightness scale: "
                                     "run gtod_skydip on this spectral setup first");
  const int64_t ot0 = j.out_ld ? j.out_t0 : 0, old = j.out_ld ? j.out_ld : j.t_total;
  if (old < 1 || ot0 < 0) return fail(c, GTOD_EINVAL, at + "bad output window");
  if (j.kind == GTOD_JOB_PINK && (ot0 != 0 || old < j.t_total))
    return fail(c, GTOD_EINVAL, at + "PINK output must hold all t_total samples");
  if (j.kind == GTOD_JOB_SIGNAL && (j.t_begin < ot0 || j.t_end > ot0 + old))
    return fail(c, GTOD_EINVAL, at + "output window does not cover [t_begin, t_end)");
  const int prec = j.precision < 0 ? c->precision : j.precision;
  if (prec != GTOD_PREC_FP32 && prec != GTOD_PREC_SPLIT_BF16)
    return fail(c, GTOD_EINVAL, at + "unknown precision");
  pl->precision = prec;
  if (j.kind == GTOD_JOB_PINK) {
    if (!j.pink_alpha) return fail(c, GTOD_EINVAL, at + "pink_alpha is NULL");
    // the two-pass transform holds up to 4096 x 4096 complex points
    if (j.t_total > ((int64_t)1 << 25))
      return fail(c, GTOD_EINVAL, at + "PINK series longer than 2^25 samples");
    if (!j.pink_A && !finite_pos(j.pink_knee_hz))
      return fail(c, GTOD_EINVAL, at + "pink_knee_hz must be > 0");
    if ((int64_t)j.n_pix * pl->spec->K > ((int64_t)1 << 31))
      return fail(c, GTOD_EINVAL, at + "too many series");
    for (int k = 0; k < pl->spec->K; ++k)
      if (!std::isfinite(j.pink_alpha[k]))
        return fail(c, GTOD_EINVAL, at + "pink_alpha not finite");
    if (j.pink_A)
      for (int k = 0; k < pl->spec->K; ++k)
        if (!(std::isfinite(j.pink_A[k]) && j.pink_A[k] >= 0.0))
          return fail(c, GTOD_EINVAL, at + "pink_A must be finite and >= 0");
    return GTOD_OK;
  }
  auto sc = c->screens.find(j.screen_id);
  if (sc == c->screens.end()) return fail(c, GTOD_ENOTFOUND, at + "unknown screen_id");
  pl->scr = &sc->second;
  if (!j.dphi_rad || !j.dtheta_rad) return fail(c, GTOD_EINVAL, at + "pixel offsets are NULL");
  if (j.t_begin < 0 || j.t_end > j.t_total || j.t_begin > j.t_end)
    return fail(c, GTOD_EINVAL, at + "bad [t_begin, t_end)");
  if (j.scan_kind < 0 || j.scan_kind > 2) return fail(c, GTOD_EINVAL, at + "unknown scan kind");
  if (j.scan_kind == GTOD_SCAN_TRAJ && !j.traj)
    return fail(c, GTOD_EINVAL, at + "TRAJ scan without trajectory");
  if (j.cube) {
    if (j.n_az < 2 || j.n_el < 2) return fail(c, GTOD_EINVAL, at + "source grid needs >= 2 nodes per axis");
    if (j.cube_ld < pl->spec->F) return fail(c, GTOD_EINVAL, at + "cube_ld < F");
    if (!(j.daz_rad > 0) || !(j.del_rad > 0)) return fail(c, GTOD_EINVAL, at + "source grid spacing must be > 0");
  }
  double rmax = 0;
  if (j.scan_kind == GTOD_SCAN_DAISY) {
    rmax = std::fabs(j.scan_params[0]);
    for (int q = 0; q < 3; ++q)
      if (!std::isfinite(j.scan_params[q])) return fail(c, GTOD_EINVAL, at + "daisy parameters not finite");
  }
  double dpmin = 1e300, dpmax = -1e300, dtmin = 1e300, dtmax = -1e300;
  for (int p = 0; p < j.n_pix; ++p) {
    if (!std::isfinite(j.dphi_rad[p]) || !std::isfinite(j.dtheta_rad[p]))
      return fail(c, GTOD_EINVAL, at + "pixel offsets not finite");
    dpmin = std::min(dpmin, j.dphi_rad[p]);
    dpmax = std::max(dpmax, j.dphi_rad[p]);
    dtmin = std::min(dtmin, j.dtheta_rad[p]);
    dtmax = std::max(dtmax, j.dtheta_rad[p]);
  }
  if (j.scan_kind != GTOD_SCAN_TRAJ) {
    const double elo = j.theta0_rad + dtmin - rmax, ehi = j.theta0_rad + dtmax + rmax;
    if (!(elo > 0.0 && ehi < M_PI)) return fail(c, GTOD_EINVAL, at + "elevation leaves (0, pi)");
    if (c->flags & GTOD_INIT_STRICT_RANGE) {
      const ScreenObj& s = *pl->scr;
      const double t0 = j.t_begin / c->fs, t1 = std::max<int64_t>(j.t_end - 1, j.t_begin) / c->fs;
      const double w0 = std::min(s.wind * t0, s.wind * t1), w1 = std::max(s.wind * t0, s.wind * t1);
      const double xlo = s.h * std::tan(dpmin - rmax) + w0, xhi = s.h * std::tan(dpmax + rmax) + w1;
      const double ylo = s.h * std::tan(dtmin - rmax), yhi = s.h * std::tan(dtmax + rmax);
      const double gx0 = xlo / s.dx + s.ix0, gx1 = xhi / s.dx + s.ix0;
      const double gy0 = ylo / s.dy + s.iy0, gy1 = yhi / s.dy + s.iy0;
      if (gx0 < 0 || gx1 > s.nx - 1 || gy0 < 0 || gy1 > s.ny - 1)
        return fail(c, GTOD_ERANGE, at + "pointing leaves the screen");
      const SpecObj& f = *pl->spec;
      if (std::isfinite(s.vmin) &&
          (s.vmin < f.pwv0 || s.vmax > f.pwv0 + (f.n_pwv - 1) * f.dpwv))
        return fail(c, GTOD_ERANGE, at + "screen PWV leaves the table axis");
    }
  }
  return GTOD_OK;
}

}  // namespace

namespace gtod {

int32_t ctx_alloc(gtod_ctx* c, void** p, size_t bytes) { return dev_alloc(c, p, bytes); }
void ctx_free(gtod_ctx* c, void* p) { dev_free(c, p); }
int32_t ctx_fail(gtod_ctx* c, int32_t status, const char* msg) { return fail(c, status, msg); }
int ctx_device(const gtod_ctx* c) { return c->device; }
double ctx_f_sample(const gtod_ctx* c) { return c->fs; }
hipStream_t ctx_sink_stream(gtod_ctx* c, int which) {
  hipStream_t& s = c->sink_streams[which & 1];
  if (!s && hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    s = nullptr;
  }
  return s;
}

int ctx_spec_channels(const gtod_ctx* c, int32_t spec_id) {
  auto it = c->specs.find(spec_id);
  return it == c->specs.end() ? -1 : it->second.K;
}

}  // namespace gtod

extern "C" {

gtod_status gtod_sim_init(const gtod_init_desc* d, gtod_ctx** out) {
  if (!out) return fail(nullptr, GTOD_EINVAL, "out is NULL");
  *out = nullptr;
  if (!d) return fail(nullptr, GTOD_EINVAL, "desc is NULL");
  if (!finite_pos(d->f_sample_hz)) return fail(nullptr, GTOD_EINVAL, "f_sample_hz must be > 0");
  if (!finite_pos(d->eta_pb)) return fail(nullptr, GTOD_EINVAL, "eta_pb must be > 0");
  if (d->precision != GTOD_PREC_FP32 && d->precision != GTOD_PREC_SPLIT_BF16)
    return fail(nullptr, GTOD_EINVAL, "unknown precision");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || d->device < 0 || d->device >= ndev) {
    (void)hipGetLastError();
    return fail(nullptr, GTOD_EINVAL, "no such device");
  }
  if (hipSetDevice(d->device) != hipSuccess) return fail(nullptr, GTOD_EDEVICE, "hipSetDevice failed");
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, d->device) != hipSuccess)
    return fail(nullptr, GTOD_EDEVICE, "hipGetDeviceProperties failed");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(nullptr, GTOD_EUNSUPPORTED, std::string("device is ") + prop.gcnArchName + ", not gfx950");
  auto* c = new gtod_ctx;
  c->device = d->device;
  c->precision = d->precision;
  c->flags = d->flags;
  size_t free_b = 0, total_b = 0;
  (void)hipMemGetInfo(&free_b, &total_b);
  c->budget = d->hbm_budget_bytes ? d->hbm_budget_bytes : (uint64_t)(0.9 * (double)free_b);
  c->ws_bytes = d->workspace_bytes ? d->workspace_bytes : (1ull << 30);
  c->fs = d->f_sample_hz;
  c->eta_taper = d->eta_taper;
  c->rho_surf = d->rho_surf_m;
  c->eta_pol = d->eta_pol;
  c->delta_J = d->delta_J;
  c->eta_pb = d->eta_pb;
  c->t_cmb = d->t_cmb_K;
  gtod_status st = dev_alloc(c, (void**)&c->counters, 4 * sizeof(unsigned long long));
  if (st != GTOD_OK) {
    g_init_err = c->err;
    delete c;
    return st;
  }
  if (hipMemset(c->counters, 0, 4 * sizeof(unsigned long long)) != hipSuccess) {
    dev_free(c, c->counters);
    delete c;
    return fail(nullptr, GTOD_EDEVICE, "hipMemset failed");
  }
  st = init_noalloc(c);
  if (st != GTOD_OK) {
    g_init_err = c->err;
    free_noalloc(c->na);
    dev_free(c, c->counters);
    delete c;
    return st;
  }
  *out = c;
  return GTOD_OK;
}

gtod_status gtod_load_screen(gtod_ctx* c, const gtod_screen_desc* d, int32_t* id) {
  if (!c || !d || !id) return fail(c, GTOD_EINVAL, "NULL argument");
  if (!d->pwv_mm || d->nx < 2 || d->ny < 2) return fail(c, GTOD_EINVAL, "screen needs nx, ny >= 2");
  if (!finite_pos(d->dx_m) || !finite_pos(d->dy_m)) return fail(c, GTOD_EINVAL, "cell size must be > 0");
  if (!std::isfinite(d->h_column_m) || !std::isfinite(d->wind_mps) ||
      !std::isfinite(d->ix0) || !std::isfinite(d->iy0))
    return fail(c, GTOD_EINVAL, "screen parameters not finite");
  if (d->mem_kind != 0 && d->mem_kind != 1) return fail(c, GTOD_EINVAL, "unknown mem_kind");
  HIP_TRY(c, hipSetDevice(c->device));
  ScreenObj s;
  s.nx = d->nx;
  s.ny = d->ny;
  s.dx = d->dx_m;
  s.dy = d->dy_m;
  s.ix0 = d->ix0;
  s.iy0 = d->iy0;
  s.h = d->h_column_m;
  s.wind = d->wind_mps;
  s.bytes = (size_t)s.nx * s.ny * sizeof(double);
  gtod_status st = dev_alloc(c, (void**)&s.pwv, s.bytes);
  if (st != GTOD_OK) return st;
  if (d->mem_kind == 0) {
    double lo = INFINITY, hi = -INFINITY;
    const int64_t n = s.nx * s.ny;
    for (int64_t i = 0; i < n; ++i) {
      lo = std::min(lo, d->pwv_mm[i]);
      hi = std::max(hi, d->pwv_mm[i]);
    }
    s.vmin = lo;
    s.vmax = hi;
  }
  hipError_t e = hipMemcpy(s.pwv, d->pwv_mm, s.bytes,
                           d->mem_kind == 0 ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice);
  if (e != hipSuccess) {
    dev_free(c, s.pwv);
    return fail(c, GTOD_EDEVICE, std::string("screen copy: ") + hipGetErrorString(e));
  }
  *id = c->next_id++;
  c->screens[*id] = s;
  return GTOD_OK;
}

gtod_status gtod_load_filters(gtod_ctx* c, const gtod_spectral_desc* d, int32_t* id) {
  if (!c || !d || !id) return fail(c, GTOD_EINVAL, "NULL argument");
  const int F = d->F, K = d->K;
  if (F < 1 || K < 1 || d->n_pwv < 2) return fail(c, GTOD_EINVAL, "need F >= 1, K >= 1, n_pwv >= 2");
  // the contractions address a response plane, and 256 panel rows, with
  // 32-bit byte offsets
  if (round_up(F, kFPad) * round_up(K, kKPad) * 4 > (int64_t)UINT32_MAX)
    return fail(c, GTOD_EINVAL, "K x F too large: a padded response plane must stay below 4 GiB");
  if (round_up(F, kFPad) * 256 * 4 > (int64_t)UINT32_MAX)
    return fail(c, GTOD_EINVAL, "F too large: 256 padded panel rows must stay below 4 GiB");
  if (!d->nu_hz || !d->w_hz || !d->eta_z) return fail(c, GTOD_EINVAL, "NULL spectral array");
  if (!finite_pos(d->dpwv_mm) || !std::isfinite(d->pwv0_mm)) return fail(c, GTOD_EINVAL, "bad PWV axis");
  if (d->n_stage < 0 || (d->n_stage > 0 && !d->stages)) return fail(c, GTOD_EINVAL, "bad stage list");
  if (d->filter_mode < 0 || d->filter_mode > 2) return fail(c, GTOD_EINVAL, "unknown filter mode");
  if (d->filter_mode == GTOD_FILT_MATRIX ? !d->eta_filt : (!d->f_hz || !d->R || !d->eta_peak))
    return fail(c, GTOD_EINVAL, "missing filter parameters");
  if (!(d->ref_el_rad > 0 && d->ref_el_rad < M_PI)) return fail(c, GTOD_EINVAL, "ref_el_rad outside (0, pi)");
  for (int j = 0; j < F; ++j)
    if (!finite_pos(d->nu_hz[j]) || !finite_pos(d->w_hz[j]))
      return fail(c, GTOD_EINVAL, "nu and w must be positive");
  for (int64_t i = 0; i < (int64_t)d->n_pwv * F; ++i)
    if (!(d->eta_z[i] > 0.0 && d->eta_z[i] <= 1.0))
      return fail(c, GTOD_EINVAL, "eta_z must lie in (0, 1]");
  if (d->filter_mode != GTOD_FILT_MATRIX)
    for (int k = 0; k < K; ++k)
      if (!finite_pos(d->f_hz[k]) || !finite_pos(d->R[k]) || !std::isfinite(d->eta_peak[k]))
        return fail(c, GTOD_EINVAL, "bad channel parameters");

  // optics stages -> passes (a refractive stage is surface, absorption,
  // surface; AR-coated keeps the absorption only)
  std::vector<int> ptype, pcoup, poff;
  std::vector<double> pprm, pT, pool;
  for (int s = 0; s < d->n_stage; ++s) {
    const gtod_stage& g = d->stages[s];
    auto add = [&](int type, int coup, double a0, double a1, double a2, double T, int off) {
      ptype.push_back(type);
      pcoup.push_back(coup);
      poff.push_back(off);
      pprm.push_back(a0);
      pprm.push_back(a1);
      pprm.push_back(a2);
      pT.push_back(T);
    };
    switch (g.kind) {
      case GTOD_STAGE_REFLECT:
      case GTOD_STAGE_ATM_COUPLED: {
        const int coup = g.kind == GTOD_STAGE_ATM_COUPLED;
        if (g.eta) {
          const int off = (int)pool.size();
          pool.insert(pool.end(), g.eta, g.eta + F);
          add(0, coup, 0, 0, 0, g.t_K, off);
        } else {
          add(1, coup, g.eta_const, 0, 0, g.t_K, 0);
        }
        break;
      }
      case GTOD_STAGE_OHMIC:
        if (!finite_pos(g.nu_ref_hz)) return fail(c, GTOD_EINVAL, "Ohmic stage needs nu_ref_hz > 0");
        add(2, 0, g.eps_ref, g.nu_ref_hz, 0, g.t_K, 0);
        break;
      case GTOD_STAGE_REFRACTIVE:
        if (!finite_pos(g.n_index)) return fail(c, GTOD_EINVAL, "refractive stage needs n > 0");
        if (!g.ar_coated) add(4, 0, g.n_index, 0, 0, g.t_refl_K, 0);
        add(3, 0, g.d_m, g.n_index, g.tan_delta, g.t_K, 0);
        if (!g.ar_coated) add(4, 0, g.n_index, 0, 0, g.t_refl_K, 0);
        break;
      default:
        return fail(c, GTOD_EINVAL, "unknown stage kind");
    }
  }
  if (pool.empty()) pool.push_back(0.0);
  const int n_pass = (int)ptype.size();
  std::vector<int> order(K);
  std::iota(order.begin(), order.end(), 0);
  if (d->filter_mode == GTOD_FILT_FILTERBANK)
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return d->f_hz[a] > d->f_hz[b]; });

  HIP_TRY(c, hipSetDevice(c->device));
  SpecObj so;
  so.F = F;
  so.K = K;
  so.Fp = (int)round_up(F, kFPad);
  so.Kp = (int)round_up(K, kKPad);
  so.n_pwv = d->n_pwv;
  so.pwv0 = d->pwv0_mm;
  so.dpwv = d->dpwv_mm;
  so.t_atm = d->t_atm_K;
  const int64_t Fp = so.Fp, Kp = so.Kp;
  gtod_status st = GTOD_OK;
  auto res = [&](void** p, size_t bytes) {
    if (st != GTOD_OK) return;
    st = dev_alloc(c, p, bytes);
    if (st == GTOD_OK) so.allocs.push_back(*p);
  };
  res((void**)&so.tau, (size_t)d->n_pwv * Fp * 4);
  res((void**)&so.E, Fp * 4);
  res((void**)&so.D, Fp * 4);
  res((void**)&so.W, Fp * 4);
  res((void**)&so.Pref, Fp * 4);
  res((void**)&so.B, 3 * Kp * Fp * 4);
  res((void**)&so.Bh, 3 * Kp * Fp * 2);
  res((void**)&so.Bl, 3 * Kp * Fp * 2);
  res((void**)&so.Bt, split_tiled_bytes((int)Kp, (int)Fp));
  res((void**)&so.c0, Kp * 8);
  res((void**)&so.c1, Kp * 8);
  res((void**)&so.tau64, (size_t)d->n_pwv * F * 8);
  res((void**)&so.E64, F * 8);
  res((void**)&so.D64, F * 8);
  res((void**)&so.B0_64, (size_t)F * K * 8);
  // temporaries
  std::vector<void*> tmp;
  auto tmpa = [&](void** p, size_t bytes) {
    if (st != GTOD_OK) return;
    st = dev_alloc(c, p, bytes);
    if (st == GTOD_OK) tmp.push_back(*p);
  };
  double *d_nu, *d_w, *d_eta, *d_pool, *d_prm, *d_T, *d_f = nullptr, *d_R = nullptr,
         *d_pk = nullptr, *d_mat = nullptr, *d_pref64, *d_B64;
  int *d_type, *d_coup, *d_off, *d_order;
  tmpa((void**)&d_nu, F * 8);
  tmpa((void**)&d_w, F * 8);
  tmpa((void**)&d_eta, (size_t)d->n_pwv * F * 8);
  tmpa((void**)&d_pool, pool.size() * 8);
  tmpa((void**)&d_prm, std::max<size_t>(pprm.size(), 1) * 8);
  tmpa((void**)&d_T, std::max<size_t>(pT.size(), 1) * 8);
  tmpa((void**)&d_type, std::max<size_t>(ptype.size(), 1) * 4);
  tmpa((void**)&d_coup, std::max<size_t>(pcoup.size(), 1) * 4);
  tmpa((void**)&d_off, std::max<size_t>(poff.size(), 1) * 4);
  tmpa((void**)&d_order, K * 4);
  tmpa((void**)&d_pref64, Fp * 8);
  tmpa((void**)&d_B64, (size_t)2 * F * K * 8);
  if (d->filter_mode == GTOD_FILT_MATRIX) {
    tmpa((void**)&d_mat, (size_t)F * K * 8);
  } else {
    tmpa((void**)&d_f, K * 8);
    tmpa((void**)&d_R, K * 8);
    tmpa((void**)&d_pk, K * 8);
  }
  auto cleanup = [&]() {
    for (void* p : tmp) dev_free(c, p);
    tmp.clear();
  };
  if (st != GTOD_OK) {
    cleanup();
    free_spec(c, so);
    return st;
  }
  hipError_t e = hipSuccess;
  auto cp = [&](void* dst, const void* src, size_t bytes) {
    if (e == hipSuccess && bytes) e = hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
  };
  cp(d_nu, d->nu_hz, F * 8);
  cp(d_w, d->w_hz, F * 8);
  cp(d_eta, d->eta_z, (size_t)d->n_pwv * F * 8);
  cp(d_pool, pool.data(), pool.size() * 8);
  cp(d_prm, pprm.data(), pprm.size() * 8);
  cp(d_T, pT.data(), pT.size() * 8);
  cp(d_type, ptype.data(), ptype.size() * 4);
  cp(d_coup, pcoup.data(), pcoup.size() * 4);
  cp(d_off, poff.data(), poff.size() * 4);
  cp(d_order, order.data(), K * 4);
  if (d_mat) cp(d_mat, d->eta_filt, (size_t)F * K * 8);
  if (d_f) {
    cp(d_f, d->f_hz, K * 8);
    cp(d_R, d->R, K * 8);
    cp(d_pk, d->eta_peak, K * 8);
  }
  if (e == hipSuccess) e = hipMemset(so.B, 0, 3 * Kp * Fp * 4);
  if (e == hipSuccess) e = hipMemset(so.Bh, 0, 3 * Kp * Fp * 2);
  if (e == hipSuccess) e = hipMemset(so.Bl, 0, 3 * Kp * Fp * 2);
  if (e == hipSuccess) {
    SpecSetupArgs a{};
    a.F = F;
    a.Fp = so.Fp;
    a.K = K;
    a.Kp = so.Kp;
    a.n_pwv = d->n_pwv;
    a.mode = d->filter_mode;
    a.nu = d_nu;
    a.w = d_w;
    a.eta_z = d_eta;
    a.f_hz = d_f;
    a.R = d_R;
    a.eta_peak = d_pk;
    a.order = d_order;
    a.eta_filt = d_mat;
    a.t_atm = d->t_atm_K;
    a.t_cmb = c->t_cmb;
    a.eta_taper = c->eta_taper;
    a.rho_surf = c->rho_surf;
    a.eta_pol = c->eta_pol;
    a.delta_J = c->delta_J;
    a.eta_pb = c->eta_pb;
    a.ref_pwv = d->ref_pwv_mm;
    a.pwv0 = d->pwv0_mm;
    a.dpwv = d->dpwv_mm;
    a.ref_el = d->ref_el_rad;
    a.tau = so.tau;
    a.E = so.E;
    a.D = so.D;
    a.W = so.W;
    a.Pref = so.Pref;
    a.tau64 = so.tau64;
    a.E64 = so.E64;
    a.D64 = so.D64;
    a.Pref64 = d_pref64;
    a.B0_64 = so.B0_64;
    a.B64 = d_B64;
    a.B = so.B;
    a.Bh = so.Bh;
    a.Bl = so.Bl;
    a.c0 = so.c0;
    a.c1 = so.c1;
    PassTable pt{n_pass, d_type, d_coup, d_off, d_prm, d_T, d_pool};
    launch_spec_setup(a, pt, nullptr);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipDeviceSynchronize();
  }
  if (e == hipSuccess) {
    so.nep2ref.resize(K);
    e = hipMemcpy(so.nep2ref.data(), so.c1, K * 8, hipMemcpyDeviceToHost);
  }
  if (e == hipSuccess) {
    // power-of-two scale bringing the largest reference power to [1, 2)
    std::vector<double> pref(Fp);
    e = hipMemcpy(pref.data(), d_pref64, Fp * 8, hipMemcpyDeviceToHost);
    double mx = 0.0;
    for (double v : pref) mx = std::max(mx, std::fabs(v));
    so.pexp = (mx > 0.0 && std::isfinite(mx)) ? -std::ilogb(mx) : 0;
    so.pexp = std::max(-60, std::min(so.pexp, 100));
    if (e == hipSuccess) {
      launch_scale_spectra(so.E, so.D, so.W, so.Pref, so.Fp,
                           std::ldexp(1.0f, so.pexp), nullptr);
      launch_tile_split_responses(so.Bh, so.Bl, so.Bt, so.Kp, so.Fp,
                                  std::ldexp(1.0f, -so.pexp), nullptr);
      e = hipGetLastError();
      if (e == hipSuccess) e = hipDeviceSynchronize();
    }
  }
  cleanup();
  if (e != hipSuccess) {
    free_spec(c, so);
    return fail(c, GTOD_EDEVICE, std::string("spectral setup: ") + hipGetErrorString(e));
  }
  *id = c->next_id++;
  c->specs[*id] = so;
  return GTOD_OK;
}

// Body of gtod_simulate_tod and gtod_simulate_tod_noalloc: the second
// runs in the GPU's static scratch instead of the stream's workspace.
static gtod_status simulate(gtod_ctx* c, const gtod_job* jobs, int32_t n_jobs,
                            void* hip_stream, bool noalloc) {
  if (!c) return GTOD_EINVAL;
  if (n_jobs < 0 || (n_jobs > 0 && !jobs)) return fail(c, GTOD_EINVAL, "bad job array");
  if (n_jobs == 0) return GTOD_OK;
  // the areas the jobs run in: the stream's workspace (made on its first
  // use, with these sizes) or the GPU's static scratch
  size_t panel_bytes = c->na.panel_bytes, pink_bytes = c->na.pink_bytes;
  if (!noalloc) ws_sizes(c, &panel_bytes, &pink_bytes);
  const char* ws_name = noalloc ? "the no-alloc scratch" : "the workspace";
  std::vector<JobPlan> plan(n_jobs);
  size_t stage_bytes = 0;
  for (int i = 0; i < n_jobs; ++i) {
    plan[i] = JobPlan{};
    plan[i].j = &jobs[i];
    gtod_status st = validate(c, jobs[i], i, &plan[i]);
    if (st == GTOD_OK) st = plan_chunks(c, &plan[i], i, panel_bytes, pink_bytes, ws_name);
    if (st != GTOD_OK) return st;
    const gtod_job& j = jobs[i];
    if (j.kind == GTOD_JOB_SIGNAL) {
      plan[i].off_dphi = stage_bytes;
      stage_bytes += round_up((int64_t)j.n_pix * 8, 256);
      plan[i].off_dtheta = stage_bytes;
      stage_bytes += round_up((int64_t)j.n_pix * 8, 256);
    } else {
      const int K = plan[i].spec->K;
      plan[i].off_scale = stage_bytes;
      stage_bytes += round_up((int64_t)K * 4, 256);
      plan[i].off_alpha = stage_bytes;
      stage_bytes += round_up((int64_t)K * 4, 256);
    }
  }
  if (stage_bytes > kSlotBytes) return fail(c, GTOD_EINVAL, "per-call job parameters exceed 1 MiB");
  HIP_TRY(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)hip_stream;
  StreamWs* w = &c->na;
  if (!noalloc) {
    const gtod_status st = get_ws(c, s, &w);
    if (st != GTOD_OK) return st;
  }

  // stage the small per-job arrays through a pinned slot
  const int slot = w->slot;
  w->slot = (w->slot + 1) % kSlots;
  if (w->ev_used[slot]) HIP_TRY(c, hipEventSynchronize(w->ev[slot]));
  char* hs = w->h_stage + (size_t)slot * kSlotBytes;
  char* ds = w->d_stage + (size_t)slot * kSlotBytes;
  for (int i = 0; i < n_jobs; ++i) {
    const gtod_job& j = jobs[i];
    if (j.kind == GTOD_JOB_SIGNAL) {
      std::memcpy(hs + plan[i].off_dphi, j.dphi_rad, (size_t)j.n_pix * 8);
      std::memcpy(hs + plan[i].off_dtheta, j.dtheta_rad, (size_t)j.n_pix * 8);
    } else {
      const SpecObj& f = *plan[i].spec;
      const int64_t N = [&] { int64_t n = 2; while (n < j.t_total) n *= 2; return n; }();
      float* scale = (float*)(hs + plan[i].off_scale);
      float* alpha = (float*)(hs + plan[i].off_alpha);
      const bool kel = (j.flags & GTOD_JOB_KELVIN) != 0;
      for (int k = 0; k < f.K; ++k) {
        const double A = j.pink_A ? j.pink_A[k]
                                  : f.nep2ref[k] * std::pow(j.pink_knee_hz, j.pink_alpha[k]);
        double sc = std::sqrt(A * (double)N * c->fs / 4.0) / (double)N;
        if (kel) sc *= f.kel_ib_h[k];
        scale[k] = (float)sc;
        alpha[k] = (float)j.pink_alpha[k];
      }
    }
  }
  HIP_TRY(c, hipMemcpyAsync(ds, hs, stage_bytes, hipMemcpyHostToDevice, s));

  for (int i = 0; i < n_jobs; ++i) {
    const gtod_job& j = jobs[i];
    const SpecObj& f = *plan[i].spec;
    const uint32_t key0 = (uint32_t)(j.seed & 0xFFFFFFFFull);
    const uint32_t key1 = (uint32_t)(j.seed >> 32);
    const bool acc = (j.flags & GTOD_JOB_ACCUMULATE) != 0;
    if (j.kind == GTOD_JOB_PINK) {
      PinkArgs a{};
      int64_t N = 2;
      while (N < j.t_total) N *= 2;
      const int lgM = (int)std::log2((double)(N / 2));
      a.M = (int)(N / 2);
      // pass-1 transforms of 2048 (two per workgroup, 35 KB of LDS), longer
      // only where pass 2 would exceed 4096 values per column set
      a.lgM2 = std::max(std::min(lgM, kPinkLgM2), lgM - 12);
      a.lgM1 = lgM - a.lgM2;
      a.M1 = 1 << a.lgM1;
      a.M2 = 1 << a.lgM2;
      a.N = (int)N;
      // pass-2 columns per workgroup: 16 while the block fits 4096 values
      a.lgB2 = std::max(0, std::min(kPinkLgB2, 12 - a.lgM1));
      a.fs = c->fs;
      a.K = f.K;
      a.scale = (const float*)(ds + plan[i].off_scale);
      a.alpha = (const float*)(ds + plan[i].off_alpha);
      a.key0 = key0;
      a.key1 = key1;
      a.pix0 = j.pix0;
      a.tod = j.tod;
      a.t_total = j.t_total;
      a.out_ld = j.out_ld ? j.out_ld : j.t_total;
      a.accumulate = acc;
      a.tab = w->pink;
      a.tab_w = w->pink;
      a.scratch = w->pink + kPinkTableFloat2;
      const int64_t S = (int64_t)j.n_pix * f.K;
      const int64_t per = plan[i].pink_per;
      launch_pink_tables(a, s);
      for (int64_t s0 = 0; s0 < S; s0 += per) {
        a.s0 = s0;
        a.n_series = (int)std::min<int64_t>(per, S - s0);
        const double pts = (double)a.n_series * a.M;
        timed(c, GTOD_KERNEL_PINK1, pts, s, [&] { launch_pink_pass1(a, s); });
        if (a.M1 > 1)
          timed(c, GTOD_KERNEL_PINK2, pts, s, [&] { launch_pink_pass2(a, s); });
      }
      continue;
    }
    const ScreenObj& sc = *plan[i].scr;
    const int64_t T = j.t_end - j.t_begin;
    if (T == 0) continue;
    const int n_buckets = plan[i].n_buckets, cell_shift = plan[i].cell_shift;
    const int n_az_c = plan[i].n_az_c, pg = plan[i].pg;
    const int64_t rows_cap = plan[i].rows_cap, Tc_max = plan[i].Tc_max;
    PanelArgs pa{};
    pa.tau = f.tau;
    pa.E = f.E;
    pa.D = f.D;
    pa.W = f.W;
    pa.Pref = f.Pref;
    pa.F = f.F;
    pa.Fp = f.Fp;
    pa.n_pwv = f.n_pwv;
    pa.pwv0 = f.pwv0;
    pa.dpwv = f.dpwv;
    pa.scr = sc.pwv;
    pa.nx = sc.nx;
    pa.ny = sc.ny;
    pa.dx = sc.dx;
    pa.dy = sc.dy;
    pa.ix0 = sc.ix0;
    pa.iy0 = sc.iy0;
    pa.h = sc.h;
    pa.wind = sc.wind;
    pa.scan_kind = j.scan_kind;
    pa.phi0 = j.phi0_rad;
    pa.theta0 = j.theta0_rad;
    pa.r_petal = j.scan_params[0];
    pa.omega = j.scan_params[1];
    pa.Omega = j.scan_params[2];
    pa.traj = j.traj;
    pa.f_s = c->fs;
    pa.dphi = (const double*)(ds + plan[i].off_dphi);
    pa.dtheta = (const double*)(ds + plan[i].off_dtheta);
    pa.cube = j.cube;
    pa.n_az = j.n_az;
    pa.n_el = j.n_el;
    pa.cube_ld = j.cube_ld;
    pa.az0 = j.az0_rad;
    pa.daz = j.daz_rad;
    pa.el0 = j.el0_rad;
    pa.del = j.del_rad;
    pa.panel = w->panel;
    pa.pwv_out = j.pwv;
    pa.out_t0 = j.out_ld ? j.out_t0 : 0;
    pa.out_ld = j.out_ld ? j.out_ld : j.t_total;
    pa.counters = c->counters;
    pa.n_buckets = n_buckets;
    pa.cell_shift = cell_shift;
    pa.n_az_coarse = n_az_c;
    if (n_buckets > 1) {
      char* aux = (char*)w->panel + round_up(rows_cap * f.Fp * 4, 256);
      pa.rinfo = aux;
      aux += round_up(rows_cap * kPanelRowInfoBytes, 256);
      pa.key = (uint32_t*)aux;
      aux += round_up(rows_cap * 4, 256);
      pa.order = (uint32_t*)aux;
      aux += round_up(rows_cap * 4, 256);
      pa.hist = (uint32_t*)aux;
    }
    GemmArgs ga{};
    ga.panel = w->panel;
    ga.B = f.B;
    ga.Bh = f.Bh;
    ga.Bl = f.Bl;
    ga.Bt = f.Bt;
    ga.c0 = f.c0;
    ga.c1 = f.c1;
    ga.Fp = f.Fp;
    ga.K = f.K;
    ga.Kp = f.Kp;
    ga.out_t0 = pa.out_t0;
    ga.out_ld = pa.out_ld;
    ga.fs_half = (float)(0.5 * c->fs);
    ga.pinv = std::ldexp(1.0, -f.pexp);
    ga.pinv_f = std::ldexp(1.0f, -f.pexp);
    ga.key0 = key0;
    ga.key1 = key1;
    ga.pix0 = j.pix0;
    ga.photon = (j.flags & GTOD_JOB_PHOTON_NOISE) != 0;
    ga.accumulate = acc;
    ga.kelvin = (j.flags & GTOD_JOB_KELVIN) != 0;
    ga.kel_a = f.kel_a;
    ga.kel_ib = f.kel_ib;
    ga.tod = j.tod;
    ga.p_kid = j.p_kid;
    ga.sigma = j.sigma;
    for (int p0 = 0; p0 < j.n_pix; p0 += pg) {
      const int np = std::min(pg, j.n_pix - p0);
      for (int64_t tb = j.t_begin; tb < j.t_end; tb += Tc_max) {
        const int Tc = (int)std::min<int64_t>(Tc_max, j.t_end - tb);
        const int Tpad = (int)round_up(Tc, kRowPad);
        pa.p0 = p0;
        pa.n_pix = np;
        pa.t0 = tb;
        pa.Tc = Tc;
        pa.Tpad = Tpad;
        const double rows = (double)np * Tc;
        timed(c, GTOD_KERNEL_PANEL, rows * (20.0 * f.F + 32.0), s,
              [&] { launch_panel(pa, s); });
        const double flop = rows * 6.0 * f.K * f.F;
        ga.p0 = p0;
        ga.n_pix = np;
        ga.t0 = tb;
        ga.Tc = Tc;
        ga.Tpad = Tpad;
        ga.n_tt = (int)((int64_t)np * Tpad / kRowPad);
        if (plan[i].precision == GTOD_PREC_SPLIT_BF16)
          timed(c, GTOD_KERNEL_GEMM_BF16, flop, s, [&] { launch_gemm_bf16(ga, s); });
        else
          timed(c, GTOD_KERNEL_GEMM_F32, flop, s, [&] { launch_gemm_f32(ga, s); });
      }
    }
  }
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipEventRecord(w->ev[slot], s));
  w->ev_used[slot] = true;
  return GTOD_OK;
}

gtod_status gtod_simulate_tod(gtod_ctx* c, const gtod_job* jobs, int32_t n_jobs,
                              void* hip_stream) {
  return simulate(c, jobs, n_jobs, hip_stream, false);
}

gtod_status gtod_simulate_tod_noalloc(gtod_ctx* c, const gtod_job* jobs, int32_t n_jobs,
                                      void* hip_stream) {
  return simulate(c, jobs, n_jobs, hip_stream, true);
}

gtod_status gtod_skydip(gtod_ctx* c, int32_t spec_id, double el_rad, double pwv_lo_mm,
                        double pwv_hi_mm, int32_t n, double* a_out, double* b_out,
                        double* p_kid_out, double* t_b_out) {
  if (!c) return GTOD_EINVAL;
  auto it = c->specs.find(spec_id);
  if (it == c->specs.end()) return fail(c, GTOD_ENOTFOUND, "unknown spec id");
  SpecObj& f = it->second;
  if (!(el_rad > 0.0 && el_rad < M_PI)) return fail(c, GTOD_EINVAL, "el_rad outside (0, pi)");
  if (!std::isfinite(pwv_lo_mm) || !std::isfinite(pwv_hi_mm) || !(pwv_hi_mm > pwv_lo_mm))
    return fail(c, GTOD_EINVAL, "need finite pwv_lo_mm < pwv_hi_mm");
  if (n < 2 || n > GTOD_SKYDIP_MAX_N) return fail(c, GTOD_EINVAL, "n outside [2, GTOD_SKYDIP_MAX_N]");
  const double top = f.pwv0 + (f.n_pwv - 1) * f.dpwv;
  if ((c->flags & GTOD_INIT_STRICT_RANGE) && (pwv_lo_mm < f.pwv0 || pwv_hi_mm > top))
    return fail(c, GTOD_ERANGE, "skydip PWV range leaves the transmission table");
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipDeviceSynchronize());
  gtod_status st = GTOD_OK;
  if (!f.kel_a) {
    auto res = [&](double** p) {
      if (st != GTOD_OK) return;
      st = dev_alloc(c, (void**)p, (size_t)f.Kp * 8);
      if (st == GTOD_OK) f.allocs.push_back(*p);
    };
    res(&f.kel_a);
    res(&f.kel_b);
    res(&f.kel_ib);
    if (st != GTOD_OK) return st;
  }
  double *Pm = nullptr, *Xm = nullptr, *pk = nullptr, *tb = nullptr;
  const size_t nf = (size_t)n * f.F * 8, nk = (size_t)n * f.K * 8;
  st = dev_alloc(c, (void**)&Pm, nf);
  if (st == GTOD_OK) st = dev_alloc(c, (void**)&Xm, nf);
  if (st == GTOD_OK) st = dev_alloc(c, (void**)&pk, nk);
  if (st == GTOD_OK) st = dev_alloc(c, (void**)&tb, nk);
  auto cleanup = [&] {
    dev_free(c, Pm);
    dev_free(c, Xm);
    dev_free(c, pk);
    dev_free(c, tb);
  };
  if (st != GTOD_OK) {
    cleanup();
    return st;
  }
  SkydipArgs a{};
  a.F = f.F;
  a.K = f.K;
  a.n_pwv = f.n_pwv;
  a.n = n;
  a.pwv_lo = pwv_lo_mm;
  a.pwv_hi = pwv_hi_mm;
  a.pwv0 = f.pwv0;
  a.dpwv = f.dpwv;
  a.csc = 1.0 / std::sin(el_rad);
  a.t_atm = f.t_atm;
  a.tau64 = f.tau64;
  a.E64 = f.E64;
  a.D64 = f.D64;
  a.B0 = f.B0_64;
  a.Pm = Pm;
  a.Xm = Xm;
  a.p_kid = pk;
  a.t_b = tb;
  a.a = f.kel_a;
  a.b = f.kel_b;
  a.ib = f.kel_ib;
  launch_skydip(a, nullptr);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipDeviceSynchronize();
  std::vector<double> ib(f.K);
  if (e == hipSuccess) e = hipMemcpy(ib.data(), f.kel_ib, f.K * 8, hipMemcpyDeviceToHost);
  if (e == hipSuccess && a_out) e = hipMemcpy(a_out, f.kel_a, f.K * 8, hipMemcpyDeviceToHost);
  if (e == hipSuccess && b_out) e = hipMemcpy(b_out, f.kel_b, f.K * 8, hipMemcpyDeviceToHost);
  if (e == hipSuccess && p_kid_out) e = hipMemcpy(p_kid_out, pk, nk, hipMemcpyDeviceToHost);
  if (e == hipSuccess && t_b_out) e = hipMemcpy(t_b_out, tb, nk, hipMemcpyDeviceToHost);
  cleanup();
  if (e != hipSuccess) {
    f.has_kelvin = false;
    return fail(c, GTOD_EDEVICE, std::string("skydip: ") + hipGetErrorString(e));
  }
  f.kel_ib_h = ib;
  f.has_kelvin = true;
  return GTOD_OK;
}

gtod_status gtod_reduce(gtod_ctx* c, const gtod_reduce_desc* d, void* hip_stream) {
  if (!c) return GTOD_EINVAL;
  if (!d) return fail(c, GTOD_EINVAL, "NULL descriptor");
  auto it = c->specs.find(d->spec_id);
  if (it == c->specs.end()) return fail(c, GTOD_ENOTFOUND, "unknown spec id");
  const SpecObj& f = it->second;
  const int P = d->n_pix;
  if (P < 1 || !d->dphi_rad || !d->dtheta_rad) return fail(c, GTOD_EINVAL, "need n_pix >= 1 and pixel offsets");
  if (!d->tod) return fail(c, GTOD_EINVAL, "tod is NULL");
  if (d->T < 1 || d->t0 < 0 || d->ld < d->T) return fail(c, GTOD_EINVAL, "bad sample window (T >= 1, t0 >= 0, ld >= T)");
  if (d->scan_kind < 0 || d->scan_kind > 2) return fail(c, GTOD_EINVAL, "unknown scan kind");
  if (d->scan_kind == GTOD_SCAN_TRAJ && (!d->traj || d->t0 + d->T > d->t_total))
    return fail(c, GTOD_EINVAL, "TRAJ scan needs traj covering [t0, t0 + T)");
  if (d->scan_kind == GTOD_SCAN_DAISY)
    for (int q = 0; q < 3; ++q)
      if (!std::isfinite(d->scan_params[q])) return fail(c, GTOD_EINVAL, "daisy parameters not finite");
  if (!std::isfinite(d->theta0_rad)) return fail(c, GTOD_EINVAL, "theta0 not finite");
  if (d->pwv ? (d->pwv_len < 1 || d->pwv_ld < d->pwv_len) : !std::isfinite(d->pwv_mean_mm))
    return fail(c, GTOD_EINVAL, "need a PWV array (pwv_len >= 1, pwv_ld >= pwv_len) or a finite pwv_mean_mm");
  if (!(d->r_out_rad >= 0.0) || !std::isfinite(d->r_out_rad)) return fail(c, GTOD_EINVAL, "r_out_rad must be finite and >= 0");
  const bool maps = d->map || d->weight;
  if (maps && (!d->map || !d->weight)) return fail(c, GTOD_EINVAL, "map and weight must both be set");
  if (!maps && !d->t_star) return fail(c, GTOD_EINVAL, "no output: set t_star, or map and weight");
  if (maps && (d->map_n < 2 || d->map_n > GTOD_MAP_MAX_N || !finite_pos(d->map_half_rad)))
    return fail(c, GTOD_EINVAL, "map_n outside [2, GTOD_MAP_MAX_N] or map_half_rad <= 0");
  std::vector<int> off(P);
  int n_out = 0;
  for (int p = 0; p < P; ++p) {
    if (!std::isfinite(d->dphi_rad[p]) || !std::isfinite(d->dtheta_rad[p]))
      return fail(c, GTOD_EINVAL, "pixel offsets not finite");
    off[p] = std::hypot(d->dphi_rad[p], d->dtheta_rad[p]) > d->r_out_rad;
    n_out += off[p];
  }
  if (n_out == 0) return fail(c, GTOD_EINVAL, "no spaxel lies outside r_out_rad");
  const size_t stage_bytes = (size_t)P * 20 + 64;
  if (stage_bytes > kSlotBytes) return fail(c, GTOD_EINVAL, "too many spaxels");
  HIP_TRY(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)hip_stream;
  StreamWs* w = nullptr;
  gtod_status st = get_ws(c, s, &w);
  if (st != GTOD_OK) return st;
  // workspace: scan table, channel transmissions and mean PWV, then per
  // channel group the common-mode rows and the cell statistics
  const int64_t T = d->T, K = f.K;
  const int64_t C = maps ? (int64_t)d->map_n * d->map_n : 0;
  const int64_t fixed = round_up(T * 16, 256) + round_up(K * 8, 256) + 256;
  const int64_t per_ch = maps ? round_up(T * 8, 256) + (int64_t)P * C * 16 : 0;
  const int64_t avail = (int64_t)w->panel_bytes - fixed;
  int64_t kg = avail > 0 ? K : 0;
  if (maps) kg = avail > 0 ? std::min<int64_t>(K, (avail - 256) / per_ch) : 0;
  if (kg < 1) return fail(c, GTOD_EINVAL, "workspace too small for one channel of the reduction");

  const int slot = w->slot;
  w->slot = (w->slot + 1) % kSlots;
  if (w->ev_used[slot]) HIP_TRY(c, hipEventSynchronize(w->ev[slot]));
  char* hs = w->h_stage + (size_t)slot * kSlotBytes;
  char* ds = w->d_stage + (size_t)slot * kSlotBytes;
  std::memcpy(hs, d->dphi_rad, (size_t)P * 8);
  std::memcpy(hs + (size_t)P * 8, d->dtheta_rad, (size_t)P * 8);
  std::memcpy(hs + (size_t)P * 16, off.data(), (size_t)P * 4);
  HIP_TRY(c, hipMemcpyAsync(ds, hs, (size_t)P * 20, hipMemcpyHostToDevice, s));

  char* ws = (char*)w->panel;
  ReduceArgs a{};
  a.P = P;
  a.K = f.K;
  a.F = f.F;
  a.n_pwv = f.n_pwv;
  a.T = T;
  a.t0 = d->t0;
  a.ld = d->ld;
  a.scan_kind = d->scan_kind;
  a.r_petal = d->scan_params[0];
  a.omega = d->scan_params[1];
  a.Omega = d->scan_params[2];
  a.f_s = c->fs;
  a.theta0 = d->theta0_rad;
  a.traj = d->traj;
  a.dphi = (const double*)ds;
  a.dtheta = (const double*)(ds + (size_t)P * 8);
  a.off = (const int*)(ds + (size_t)P * 16);
  a.n_out = n_out;
  a.tau64 = f.tau64;
  a.B0 = f.B0_64;
  a.pwv0 = f.pwv0;
  a.dpwv = f.dpwv;
  a.pwv = d->pwv;
  a.pwv_ld = d->pwv_ld;
  a.pwv_len = d->pwv_len;
  a.pwv_host = d->pwv_mean_mm;
  a.scan_tab = (double2*)ws;
  a.lnz = (double*)(ws + round_up(T * 16, 256));
  a.pwv_mean = (double*)(ws + round_up(T * 16, 256) + round_up(K * 8, 256));
  a.tod = d->tod;
  a.t_star = d->t_star;
  a.map_n = maps ? d->map_n : 0;
  a.half = d->map_half_rad;
  a.dcell = maps ? 2.0 * d->map_half_rad / (d->map_n - 1) : 0.0;
  a.map = d->map;
  a.weight = d->weight;
  char* grp = ws + fixed;
  a.M = maps ? (double*)grp : nullptr;
  a.stats = maps ? (double2*)(grp + round_up(kg * T * 8, 256)) : nullptr;
  launch_reduce_setup(a, s);
  for (int64_t k0 = 0; k0 < K; k0 += kg) {
    a.k0 = (int)k0;
    a.kg = (int)std::min<int64_t>(kg, K - k0);
    const double samples = (double)P * a.kg * T;
    // with maps the gridding kernel writes T*; the common-mode kernel only M
    const double cm_bytes = samples * ((d->t_star && !maps) ? 8.0 : 4.0) +
                            (maps ? 8.0 * a.kg * T : 0.0);
    timed(c, GTOD_KERNEL_COMMON, cm_bytes, s, [&] { launch_reduce_common(a, s); });
    if (maps) {
      const double gb = samples * (d->t_star ? 8.0 : 4.0) + 8.0 * a.kg * T +
                        16.0 * P * a.kg * C;
      int bad = 0;
      timed(c, GTOD_KERNEL_GRID, gb, s, [&] { bad = launch_reduce_grid(a, s); });
      if (bad) return fail(c, GTOD_EDEVICE, "gridding needs more LDS than the device allows");
      launch_reduce_combine(a, s);
    }
  }
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipEventRecord(w->ev[slot], s));
  w->ev_used[slot] = true;
  return GTOD_OK;
}

}  // extern "C"

namespace {

// Quadrature nodes for the far field of a grid whose largest argument of
// J0 is kr = 2 pi rho_max R / lambda_min.
int beam_nodes(double kr) { return (int)round_up((int64_t)std::ceil(0.6 * kr) + 64, 32); }

// Stages nu (host [F]) through the stream's pinned ring; returns the device
// copy, valid for work enqueued on s before the slot's next reuse.
gtod_status stage_doubles(gtod_ctx* c, StreamWs* w, hipStream_t s, const double* h,
                          int64_t n, const double** dev, int* slot_out) {
  if ((size_t)n * 8 > kSlotBytes) return fail(c, GTOD_EINVAL, "too many frequencies");
  const int slot = w->slot;
  w->slot = (w->slot + 1) % kSlots;
  if (w->ev_used[slot]) HIP_TRY(c, hipEventSynchronize(w->ev[slot]));
  char* hs = w->h_stage + (size_t)slot * kSlotBytes;
  char* ds = w->d_stage + (size_t)slot * kSlotBytes;
  std::memcpy(hs, h, (size_t)n * 8);
  HIP_TRY(c, hipMemcpyAsync(ds, hs, (size_t)n * 8, hipMemcpyHostToDevice, s));
  *dev = (const double*)ds;
  *slot_out = slot;
  return GTOD_OK;
}

gtod_status check_nu(gtod_ctx* c, const double* nu, int32_t F, double* nu_max) {
  if (!nu || F < 1) return fail(c, GTOD_EINVAL, "need F >= 1 frequencies");
  *nu_max = 0.0;
  for (int f = 0; f < F; ++f) {
    if (!finite_pos(nu[f])) return fail(c, GTOD_EINVAL, "frequencies must be positive");
    *nu_max = std::max(*nu_max, nu[f]);
  }
  return GTOD_OK;
}

}  // namespace

extern "C" {

gtod_status gtod_far_field(gtod_ctx* c, const double* nu_hz, int32_t F, int32_t n_a,
                           int32_t n_b, double da, double db, double r_tel,
                           double t_edge_db, float* out, void* hip_stream) {
  if (!c) return GTOD_EINVAL;
  double nu_max;
  gtod_status st = check_nu(c, nu_hz, F, &nu_max);
  if (st != GTOD_OK) return st;
  if (n_a < 1 || n_b < 1 || !(da >= 0.0) || !(db >= 0.0) || !std::isfinite(da) ||
      !std::isfinite(db) || !finite_pos(r_tel) || !std::isfinite(t_edge_db) || !out)
    return fail(c, GTOD_EINVAL, "bad far-field grid or aperture");
  const double rho = std::hypot((n_a - 1) * da, (n_b - 1) * db);
  const double kr = 2.0 * M_PI * rho * r_tel * nu_max / 299792458.0;
  if (kr > 6000.0) return fail(c, GTOD_EINVAL, "far-field grid too oscillatory for the quadrature");
  HIP_TRY(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)hip_stream;
  StreamWs* w = nullptr;
  if ((st = get_ws(c, s, &w)) != GTOD_OK) return st;
  const double* d_nu;
  int slot;
  if ((st = stage_doubles(c, w, s, nu_hz, F, &d_nu, &slot)) != GTOD_OK) return st;
  BeamArgs b{};
  b.n_nodes = beam_nodes(kr);
  b.gl_x = (double*)w->panel;
  b.gl_w = b.gl_x + b.n_nodes;
  b.r_tel = r_tel;
  b.t_edge_db = t_edge_db;
  b.nu = d_nu;
  b.F = F;
  b.n_a = n_a;
  b.n_b = n_b;
  b.da = da;
  b.db = db;
  b.table = out;
  launch_gauss_legendre(b.gl_x, b.gl_w, b.n_nodes, s);
  timed(c, GTOD_KERNEL_BEAM, (double)n_a * n_b * F * b.n_nodes, s,
        [&] { launch_beam_table(b, s); });
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipEventRecord(w->ev[slot], s));
  w->ev_used[slot] = true;
  return GTOD_OK;
}

gtod_status gtod_convolve_source(gtod_ctx* c, const float* in, int32_t n_az, int32_t n_el,
                                 int64_t ld_in, const double* nu_hz, int32_t F,
                                 double daz, double el0, double del, double r_tel,
                                 double t_edge_db, float* out, int64_t ld_out,
                                 void* hip_stream) {
  if (!c) return GTOD_EINVAL;
  double nu_max;
  gtod_status st = check_nu(c, nu_hz, F, &nu_max);
  if (st != GTOD_OK) return st;
  if (!in || !out || n_az < 1 || n_el < 1 || (int64_t)n_az * n_el > kMaxSrcNodes ||
      ld_in < F || ld_out < F)
    return fail(c, GTOD_EINVAL, "bad source grid (n_az n_el <= 20000, ld >= F)");
  if (!finite_pos(daz) || !finite_pos(del) || !std::isfinite(el0) || !finite_pos(r_tel) ||
      !std::isfinite(t_edge_db))
    return fail(c, GTOD_EINVAL, "bad grid spacing, elevation or aperture");
  const int64_t nn = (int64_t)n_az * n_el;
  const char* ib = (const char*)in;
  const char* ob = (const char*)out;
  if (ib < ob + nn * ld_out * 4 && ob < ib + nn * ld_in * 4)
    return fail(c, GTOD_EINVAL, "in and out overlap");
  const double rho = std::hypot((n_az - 1) * daz, (n_el - 1) * del);
  const double kr = 2.0 * M_PI * rho * r_tel * nu_max / 299792458.0;
  if (kr > 6000.0) return fail(c, GTOD_EINVAL, "source grid too oscillatory for the quadrature");
  HIP_TRY(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)hip_stream;
  StreamWs* w = nullptr;
  if ((st = get_ws(c, s, &w)) != GTOD_OK) return st;
  const double* d_nu;
  int slot;
  if ((st = stage_doubles(c, w, s, nu_hz, F, &d_nu, &slot)) != GTOD_OK) return st;
  BeamArgs b{};
  b.n_nodes = beam_nodes(kr);
  b.gl_x = (double*)w->panel;
  b.gl_w = b.gl_x + b.n_nodes;
  const int64_t head = round_up((int64_t)b.n_nodes * 16, 256);
  const int64_t nf_max = ((int64_t)w->panel_bytes - head) / (nn * 4);
  if (nf_max < 1) return fail(c, GTOD_EINVAL, "workspace too small for one far-field table");
  b.r_tel = r_tel;
  b.t_edge_db = t_edge_db;
  b.n_a = n_az;
  b.n_b = n_el;
  b.da = daz;
  b.db = del;
  b.table = (float*)((char*)w->panel + head);
  SrcConvArgs v{};
  v.in = in;
  v.ld_in = ld_in;
  v.ld_out = ld_out;
  v.n_az = n_az;
  v.n_el = n_el;
  v.el0 = el0;
  v.del = del;
  v.scale = M_PI * r_tel * r_tel * daz * del;
  v.table = b.table;
  v.out = out;
  launch_gauss_legendre(b.gl_x, b.gl_w, b.n_nodes, s);
  for (int f0 = 0; f0 < F; f0 += (int)nf_max) {
    const int nf = (int)std::min<int64_t>(nf_max, F - f0);
    b.nu = d_nu + f0;
    b.F = nf;
    timed(c, GTOD_KERNEL_BEAM, (double)nn * nf * b.n_nodes, s, [&] { launch_beam_table(b, s); });
    v.f0 = f0;
    v.nf = nf;
    int bad = 0;
    timed(c, GTOD_KERNEL_SRC_CONV, 2.0 * (double)nn * nn * nf, s,
          [&] { bad = launch_source_conv(v, s); });
    if (bad) return fail(c, GTOD_EDEVICE, "source convolution needs more LDS than the device allows");
  }
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipEventRecord(w->ev[slot], s));
  w->ev_used[slot] = true;
  return GTOD_OK;
}

gtod_status gtod_convolve_screen(gtod_ctx* c, const double* in, int64_t nx, int64_t ny,
                                 double dx, double dy, double r_tel, double t_edge_db,
                                 double* out, void* hip_stream) {
  if (!c) return GTOD_EINVAL;
  if (!in || !out || nx < 1 || ny < 1) return fail(c, GTOD_EINVAL, "bad screen");
  if (!finite_pos(dx) || !finite_pos(dy) || !finite_pos(r_tel) || !std::isfinite(t_edge_db))
    return fail(c, GTOD_EINVAL, "bad cell size or aperture");
  const double fx = std::floor(r_tel / dx), fy = std::floor(r_tel / dy);
  if (fx > kMaxFootprint || fy > kMaxFootprint)
    return fail(c, GTOD_EINVAL, "footprint wider than 32 cells each side");
  const char* ib = (const char*)in;
  const char* ob = (const char*)out;
  if (ib < ob + nx * ny * 8 && ob < ib + nx * ny * 8) return fail(c, GTOD_EINVAL, "in and out overlap");
  HIP_TRY(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)hip_stream;
  StreamWs* w = nullptr;
  gtod_status st;
  if ((st = get_ws(c, s, &w)) != GTOD_OK) return st;
  ScreenConvArgs a{};
  a.in = in;
  a.out = out;
  a.nx = nx;
  a.ny = ny;
  a.rx = (int)fx;
  a.ry = (int)fy;
  a.dx = dx;
  a.dy = dy;
  a.r_tel = r_tel;
  a.t_edge_db = t_edge_db;
  a.w = (double*)w->panel;
  launch_screen_weights(a, s);
  int taps = 0;
  for (int yy = -a.ry; yy <= a.ry; ++yy)
    for (int xx = -a.rx; xx <= a.rx; ++xx)
      taps += std::hypot(xx * dx, yy * dy) < r_tel;
  int bad = 0;
  timed(c, GTOD_KERNEL_SCREEN_CONV, 2.0 * taps * (double)nx * ny, s,
        [&] { bad = launch_screen_conv(a, s); });
  if (bad) return fail(c, GTOD_EDEVICE, "screen convolution needs more LDS than the device allows");
  HIP_TRY(c, hipGetLastError());
  return GTOD_OK;
}

gtod_status gtod_free(gtod_ctx* c, int32_t kind, int32_t id) {
  if (!c) return GTOD_EINVAL;
  (void)hipSetDevice(c->device);
  if (kind == GTOD_OBJ_SCREEN) {
    auto it = c->screens.find(id);
    if (it == c->screens.end()) return fail(c, GTOD_ENOTFOUND, "unknown screen id");
    HIP_TRY(c, hipDeviceSynchronize());
    dev_free(c, it->second.pwv);
    c->screens.erase(it);
    return GTOD_OK;
  }
  if (kind == GTOD_OBJ_SPEC) {
    auto it = c->specs.find(id);
    if (it == c->specs.end()) return fail(c, GTOD_ENOTFOUND, "unknown spec id");
    HIP_TRY(c, hipDeviceSynchronize());
    free_spec(c, it->second);
    c->specs.erase(it);
    return GTOD_OK;
  }
  if (kind == GTOD_OBJ_CTX) {
    (void)hipDeviceSynchronize();
    drain_profile(c);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    for (auto& kv : c->screens) dev_free(c, kv.second.pwv);
    for (auto& kv : c->specs) free_spec(c, kv.second);
    for (auto& kv : c->ws) free_ws(c, kv.second);
    free_noalloc(c->na);
    for (hipStream_t s : c->sink_streams)
      if (s) (void)hipStreamDestroy(s);
    dev_free(c, c->counters);
    delete c;
    return GTOD_OK;
  }
  return fail(c, GTOD_EINVAL, "unknown object kind");
}

const char* gtod_last_error(const gtod_ctx* c) {
  return c ? c->err.c_str() : g_init_err.c_str();
}

gtod_status gtod_memory(const gtod_ctx* c, uint64_t* used, uint64_t* budget) {
  if (!c) return GTOD_EINVAL;
  if (used) *used = c->used;
  if (budget) *budget = c->budget;
  return GTOD_OK;
}

gtod_status gtod_release_stream(gtod_ctx* c, void* hip_stream) {
  if (!c) return GTOD_EINVAL;
  auto it = c->ws.find((hipStream_t)hip_stream);
  if (it == c->ws.end()) return fail(c, GTOD_ENOTFOUND, "stream has no workspace");
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipStreamSynchronize((hipStream_t)hip_stream));
  free_ws(c, it->second);
  c->ws.erase(it);
  return GTOD_OK;
}

gtod_status gtod_get_counters(gtod_ctx* c, uint64_t out[4]) {
  if (!c || !out) return GTOD_EINVAL;
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipDeviceSynchronize());
  unsigned long long h[4];
  HIP_TRY(c, hipMemcpy(h, c->counters, sizeof(h), hipMemcpyDeviceToHost));
  for (int i = 0; i < 4; ++i) out[i] = h[i];
  return GTOD_OK;
}

gtod_status gtod_spec_nep2_ref(gtod_ctx* c, int32_t spec_id, double* out) {
  if (!c || !out) return GTOD_EINVAL;
  auto it = c->specs.find(spec_id);
  if (it == c->specs.end()) return fail(c, GTOD_ENOTFOUND, "unknown spec id");
  std::memcpy(out, it->second.nep2ref.data(), it->second.nep2ref.size() * 8);
  return GTOD_OK;
}

gtod_status gtod_philox(gtod_ctx* c, const uint32_t* ctr, uint32_t* out, int64_t n,
                        uint64_t seed, void* hip_stream) {
  if (!c || n < 0 || (n > 0 && (!ctr || !out))) return fail(c, GTOD_EINVAL, "bad arguments");
  if (n == 0) return GTOD_OK;
  HIP_TRY(c, hipSetDevice(c->device));
  launch_philox(ctr, out, n, (uint32_t)(seed & 0xFFFFFFFFull), (uint32_t)(seed >> 32),
                (hipStream_t)hip_stream);
  HIP_TRY(c, hipGetLastError());
  return GTOD_OK;
}

gtod_status gtod_profile_enable(gtod_ctx* c, int32_t enable) {
  if (!c) return GTOD_EINVAL;
  HIP_TRY(c, hipSetDevice(c->device));
  if (enable) {
    HIP_TRY(c, hipDeviceSynchronize());
    drain_profile(c);
    for (int k = 0; k < GTOD_N_KERNELS; ++k)
      c->prof_ms[k] = c->prof_n[k] = c->prof_units[k] = 0.0;
  }
  c->prof = enable != 0;
  return GTOD_OK;
}

gtod_status gtod_profile_read(gtod_ctx* c, double* out, int32_t n_kernels) {
  if (!c || !out || n_kernels < 0) return GTOD_EINVAL;
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipDeviceSynchronize());
  drain_profile(c);
  for (int k = 0; k < n_kernels && k < GTOD_N_KERNELS; ++k) {
    out[3 * k] = c->prof_ms[k];
    out[3 * k + 1] = c->prof_n[k];
    out[3 * k + 2] = c->prof_units[k];
  }
  return GTOD_OK;
}

void gtod_abi_sizes(int64_t out[6]) {
  out[0] = sizeof(gtod_init_desc);
  out[1] = sizeof(gtod_screen_desc);
  out[2] = sizeof(gtod_stage);
  out[3] = sizeof(gtod_spectral_desc);
  out[4] = sizeof(gtod_job);
  out[5] = sizeof(gtod_reduce_desc);
}

}  // extern "C"
