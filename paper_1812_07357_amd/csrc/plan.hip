// Host runtime of the PSATD library: plans, FFT schedules, workspace, the C ABI.
//
// A plan corresponds to one FFT group of the hybrid solver (Sec. 2.6 of
// arXiv:1812.07357: FFT plans are initialised once per group and the
// exchange protocol is fixed before the time loop).  It owns the twiddles,
// the modified-wavenumber and PSATD coefficient tables (built on the device in
// FP64, Sec. 1.1 / 1.3), the two spectral work arrays and the launch schedule
// of the five passes.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <functional>
#include <map>
#include <mutex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/psatd.h"
#include "internal.hpp"

using namespace psatd;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int check_hip(const char* where) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(PSATD_EHIP, "%s: %s", where, hipGetErrorString(e));
  return PSATD_OK;
}

// Device bytes the library holds (plans, batch descriptors) and an optional
// ceiling on them (psatd_set_device_budget); a request that would pass the
// ceiling fails as if hipMalloc had.
std::atomic<long long> g_live_bytes{0};
std::atomic<long long> g_budget{-1};

hipError_t budget_malloc(void** out, size_t bytes) {
  const long long b = g_budget.load();
  if (b >= 0 && g_live_bytes.load() + (long long)bytes > b) {
    *out = nullptr;
    return hipErrorOutOfMemory;
  }
  const hipError_t e = hipMalloc(out, bytes);
  if (e == hipSuccess) g_live_bytes += (long long)bytes;
  return e;
}

void budget_free(void* q, size_t bytes) {
  if (!q) return;
  (void)hipFree(q);
  g_live_bytes -= (long long)bytes;
}

// LDS a single workgroup may use on the current device (160 KB per workgroup on
// gfx950; 64 KB if the query fails).
size_t lds_limit() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0) {
    (void)hipGetLastError();
    return 64 * 1024;
  }
  return (size_t)v;
}


// Factor n into compiled radices, largest powers of two first.
// Radices with compiled stages, and the VALU instructions per element one stage
// of that radix costs (gfx950, FP32, twiddles included; measured on the stage
// code).  A stage also costs an LDS round trip and two barriers, charged as
// kStageCost; the first stage applies no twiddles.
constexpr int kRadix[] = {36, 32, 24, 20, 18, 17, 16, 13, 12, 11, 10, 9, 8, 7, 6, 5, 4, 3, 2};
double radix_cost(int r) {
  switch (r) {
    case 2: return 26.0;
    case 3: return 28.3;
    case 4: return 25.2;
    case 5: return 31.0;
    case 6: return 30.8;
    case 7: return 34.4;
    case 8: return 27.1;
    case 9: return 35.0;
    case 10: return 34.9;
    case 11: return 41.9;
    case 12: return 31.8;
    case 13: return 45.8;
    case 16: return 30.3;
    case 17: return 53.6;
    case 18: return 39.8;
    case 20: return 37.9;
    case 24: return 36.9;
    case 32: return 34.7;
    case 36: return 42.8;
    default: return 1e9;
  }
}
constexpr double kStageCost = 4.0;
constexpr int kMaxSearchStages = 6;

double schedule_cost(const std::vector<int>& r) {
  double c = 0.0;
  for (size_t i = 0; i < r.size(); ++i) c += radix_cost(r[i]) + kStageCost;
  if (!r.empty()) c -= 8.0 * (r[0] - 1) / r[0];
  return c;
}

// All factorisations of n into compiled radices (non-increasing), at most kMaxSearchStages stages.
void factorisations(int n, int start, std::vector<int>& cur, std::vector<std::vector<int>>& out) {
  if (n == 1) {
    out.push_back(cur);
    return;
  }
  if ((int)cur.size() == kMaxSearchStages) return;
  for (size_t i = start; i < sizeof(kRadix) / sizeof(kRadix[0]); ++i)
    if (n % kRadix[i] == 0) {
      cur.push_back(kRadix[i]);
      factorisations(n / kRadix[i], (int)i, cur, out);
      cur.pop_back();
    }
}

// Radix sequences for n, cheapest first (by schedule_cost), largest radix first
// and, as alternatives, smallest first; at most `cap` of them.
std::vector<std::vector<int>> ranked_schedules(int n, size_t cap) {
  std::vector<std::vector<int>> sets, out;
  std::vector<int> cur;
  if (n > 1) factorisations(n, 0, cur, sets);
  std::sort(sets.begin(), sets.end(), [](const std::vector<int>& x, const std::vector<int>& y) {
    const double cx = schedule_cost(x), cy = schedule_cost(y);
    return cx != cy ? cx < cy : x.size() < y.size();
  });
  for (const auto& s : sets) {
    if (out.size() >= cap) break;
    out.push_back(s);
    std::vector<int> rev(s.rbegin(), s.rend());
    if (rev != s && out.size() < cap) out.push_back(rev);
  }
  return out;
}

bool set_schedule(int n, const std::vector<int>& r, LineSchedule* s) {
  std::memset(s, 0, sizeof *s);
  s->n = n;
  if ((int)r.size() > kMaxStages) return false;
  s->nstages = n == 1 ? 0 : (int)r.size();
  int span = 1;
  for (int i = 0; i < s->nstages; ++i) {
    s->radix[i] = r[i];
    s->bfl[i] = make_fastdiv((uint32_t)(n / r[i]));
    s->ns[i] = make_fastdiv((uint32_t)span);
    span *= r[i];
  }
  return true;
}

// The default schedule of length n: the cheapest factorisation (see ranked_schedules).
bool make_schedule(int n, int emax, LineSchedule* s) {
  (void)emax;
  if (n == 1) return set_schedule(1, {}, s);
  const auto r = ranked_schedules(n, 1);
  return !r.empty() && set_schedule(n, r[0], s);
}

// One transform axis of a box: direct stages over n, or Bluestein over a padded
// length m >= 2n - 1 (the smallest m whose factors all have compiled radices).
struct Axis {
  int n = 0;
  int blue = 0;
  LineSchedule sch{};  // over n, or over m
  void* tw = nullptr;
  void* chirp = nullptr;
  void* filt = nullptr;
};

bool make_axis(int n, int emax, Axis* a) {
  a->n = n;
  a->blue = 0;
  if (make_schedule(n, emax, &a->sch)) return true;
  // Bluestein: among padded lengths 2n - 1 <= m <= 4n, the one whose transform
  // costs least (m times the per-element cost of its best schedule): a slightly
  // longer m with two cheap stages beats the shortest m with three costly ones.
  int best_m = 0;
  double best = 0.0;
  for (int m = 2 * n - 1; m <= 4 * n; ++m) {
    const auto r = ranked_schedules(m, 1);
    if (r.empty()) continue;
    const double c = m * schedule_cost(r[0]);
    if (!best_m || c < best) {
      best = c;
      best_m = m;
    }
  }
  for (int m = 4 * n + 1; !best_m && m <= 8 * n; ++m)
    if (!ranked_schedules(m, 1).empty()) best_m = m;
  if (!best_m || !make_schedule(best_m, emax, &a->sch)) return false;
  a->blue = 1;
  return true;
}

template <typename T>
LineFFT<T> line_fft(const Axis& a) {
  LineFFT<T> L{};
  L.sch = a.sch;
  L.tw = (const Tw<T>*)a.tw;
  L.n = a.n;
  L.blue = a.blue;
  L.fd_n = make_fastdiv((uint32_t)a.n);
  L.fd_m = make_fastdiv((uint32_t)a.sch.n);
  L.chirp = (const Tw<T>*)a.chirp;
  L.filt = (const Tw<T>*)a.filt;
  return L;
}

// Largest line count per tile (<= cap) that fits the register budget and `lds` bytes.
int fit_lines(const LineSchedule& s, int nth, int emax, size_t csize, int cap, size_t lds) {
  for (int nl = cap; nl >= 1; --nl) {
    bool ok = (size_t)nl * lds_line(s.n) * csize <= lds;
    for (int i = 0; i < s.nstages && ok; ++i) {
      const int R = s.radix[i];
      const long long bf = (long long)nl * (s.n / R);
      const long long per = (bf + nth - 1) / nth;
      if (per > std::max(1, emax / R)) ok = false;  // one butterfly per thread above the budget
    }
    if (ok) return nl;
  }
  return 0;
}

template <typename T>
size_t csz() {
  return sizeof(cx<T>);
}

}  // namespace

namespace {
// Default set of passes on two-stage kernels (bit i = P(i+1)): all but the x inverse.
constexpr int kTwoStageDefault = 1 | 2 | 4 | 8;
}  // namespace

struct psatd_plan {
  psatd_plan_desc d{};
  int NX = 0, NY = 0, NZ = 0, NXH = 0;
  long long npts = 0, ncell = 0;
  int fp64 = 0;
  size_t rsize = 0;  // bytes per real
  Axis ax, ay, az;   // transform axes x, y, z
  int ty1 = 0;       // real y-lines per P1 tile
  bool xtab = false; // P1 tiles leave LDS room for the gather table
  int ty5 = 0;       // real y-lines per P5 tile
  int x5threads = 0; // P5 block size
  int nl_y = 0;      // lines per P2/P4 tile
  int zthreads = 0;  // threads of the P3 block
  int zcols = 0;     // (kx, ky) columns per P3 tile
  // Passes (bit i = P(i+1)) that run the compiled two-stage kernel when their
  // schedule has one; the autotuner keeps a pass's bit only if that kernel is the
  // faster of the two.  The x inverse starts on the run-time-schedule kernel.
  int two_stage_mask = kTwoStageDefault;
  double* kd = nullptr;  // FP64 modified k: kx (NXH), ky (NY), kz (NZ)
  void* kw = nullptr;    // same at working precision
  void* kwc = nullptr;   // staggered grids: kappa = k_s exp(i k d / 2) per axis index, complex
  void* coef = nullptr;  // 5 * npts
  void* wsA = nullptr;   // 11 * npts complex
  void* wsB = nullptr;   // 11 * npts complex
  size_t bytes = 0;
  std::vector<std::pair<void*, size_t>> allocs;  // every device allocation of the plan
  int timing = 0;
  std::vector<std::array<hipEvent_t, 6>> events;  // per recorded step
  // Completion of the last step and the stream it ran on: a step on another
  // stream while that one is still in flight would share the workspace.
  hipEvent_t done = nullptr;
  hipStream_t last_stream = nullptr;
  bool in_flight_known = false;
  // Two-step PML (psatd_pml_set): damping factors per axis (NX, NY, NZ values), and
  // six box arrays each for the full fields and for one set of split increments.
  bool pml_ready = false;
  void* pml_wsB = nullptr;  // layout B with 12 fields (P3 writes both split sets)
  void* pml_damp[3] = {nullptr, nullptr, nullptr};
  void* pml_full[6] = {};
  void* pml_inc[6] = {};
};

namespace {

void release_events(psatd_plan* p) {
  for (auto& set : p->events)
    for (hipEvent_t e : set)
      if (e) (void)hipEventDestroy(e);
  p->events.clear();
}

void free_plan(psatd_plan* p) {
  if (!p) return;
  release_events(p);
  if (p->done) (void)hipEventDestroy(p->done);
  for (const auto& a : p->allocs) budget_free(a.first, a.second);
  delete p;
}

int dalloc(psatd_plan* p, void** out, size_t bytes) {
  if (budget_malloc(out, bytes) != hipSuccess) {
    (void)hipGetLastError();
    *out = nullptr;
    return fail(PSATD_ENOMEM, "device allocation of %zu bytes failed", bytes);
  }
  p->allocs.push_back({*out, bytes});
  p->bytes += bytes;
  return PSATD_OK;
}

int validate(const psatd_plan_desc* d) {
  if (!d) return fail(PSATD_EINVAL, "descriptor is NULL");
  if (d->nx <= 0 || d->ny <= 0 || d->nz <= 0) return fail(PSATD_EINVAL, "interior sizes must be positive");
  if (d->ngx < 0 || d->ngy < 0 || d->ngz < 0) return fail(PSATD_EINVAL, "guard widths must be >= 0");
  if (d->order < 0 || (d->order % 2) != 0)
    return fail(PSATD_EINVAL, "order must be 0 (infinite) or an even integer >= 2, got %d", d->order);
  if (!(d->dx > 0) || !(d->dy > 0) || !(d->dz > 0)) return fail(PSATD_EINVAL, "cell sizes must be > 0");
  if (!(d->dt == d->dt) || d->dt == 0) return fail(PSATD_EINVAL, "dt must be non-zero");
  if (!(d->c > 0) || !(d->eps0 > 0)) return fail(PSATD_EINVAL, "c and eps0 must be > 0");
  if (d->precision != PSATD_FP32 && d->precision != PSATD_FP64) return fail(PSATD_EINVAL, "unknown precision");
  if (d->flags & ~(PSATD_FLAG_STAGGERED | PSATD_FLAG_NO_WORKSPACE))
    return fail(PSATD_EINVAL, "unknown flags 0x%x", d->flags);
  const long long bx = (long long)d->nx + 2LL * d->ngx, by = (long long)d->ny + 2LL * d->ngy,
                  bz = (long long)d->nz + 2LL * d->ngz;
  if (bx > (1 << 20) || by > (1 << 20) || bz > (1 << 20)) return fail(PSATD_EINVAL, "box too large");
  if ((bx / 2 + 1) * by * bz > (1LL << 40)) return fail(PSATD_EINVAL, "box too large");
  return PSATD_OK;
}

// Lines per tile: about one block's worth of elements for long lines, more
// lines for short ones (many small boxes), always within LDS and the
// one-butterfly-round-per-radix register budget checked by fit_lines.
int x_line_cap(int n) { return std::max(8, 4608 / n); }   // complex x-lines (pairs of real lines)
// P5 block size and real y-lines per P5 tile: the lines of a P1 tile of ty1
// lines, as far as the butterfly budget of the smaller P5 block allows; the
// P1 block size and tile when not even one line fits it.
int x_inv_tile(psatd_plan* p, const LineSchedule& s, int em, size_t cs, int ty1, size_t lds) {
  const int f = fit_lines(s, kXInvThreads, em, cs, x_line_cap(p->NX), lds);
  p->x5threads = f >= 1 ? kXInvThreads : kLineThreads;
  return f >= 1 ? 2 * std::min(ty1 / 2, f) : ty1;
}
// LDS of the P1 gather table for a box of NX cells along x: one int per column and per real row
// of the largest tile, rounded to 16 bytes.
size_t x_table_bytes(int NX) { return ((size_t)(NX + 2 * x_line_cap(NX)) * 4 + 15) & ~(size_t)15; }
int y_line_cap(int n) { return std::max(16, 5120 / n); }
// LDS a z tile may use: the device limit for one column, 64 KB for several.
size_t z_lds(int cols) { return cols > 1 ? std::min<size_t>(64 * 1024, lds_limit()) : lds_limit(); }

// A z tile of `cols` columns must hold its 11 cols lines in LDS; the block of
// zt threads transforms them in groups, so it only needs room for the
// butterflies of one line per round.
bool z_fits(const LineSchedule& s, int zt, int em, size_t cs, int cols) {
  return (size_t)11 * cols * lds_line(s.n) * cs <= z_lds(cols) && fit_lines(s, zt, em, cs, 1, SIZE_MAX) >= 1;
}
// Lines a block of zt threads transforms per call.
int z_group(const LineSchedule& s, int zt, int em, size_t cs, int nlines) {
  return std::max(1, fit_lines(s, zt, em, cs, nlines, SIZE_MAX));
}

// Columns and threads of a z tile: about 320 points of line per tile, the
// smallest block that fits.
void choose_z_tile(psatd_plan* p, const LineSchedule& szs, int em, size_t cs) {
  p->zthreads = 0;
  p->zcols = 0;
  for (int c = std::max(1, std::min(16, 320 / p->NZ)); c >= 1 && !p->zthreads; --c)
    for (int zt : kZThreads)
      if (z_fits(szs, zt, em, cs, c)) {
        p->zthreads = zt;
        p->zcols = c;
        break;
      }
}

// ---------------------------------------------------------------- static scratch
// psatd_step_g1_noalloc runs the same five passes with their two spectral
// workspaces in a fixed device array instead of the plan's own, so a step
// allocates nothing (for callers that cannot allocate: graph capture, tight
// serving loops).  Every GPU holds its own copy of the array for the life of
// the process; its device address comes from hipGetSymbolAddress, once per
// device, at plan creation (or the first call on a device).  The passes
// overwrite every workspace element before reading it, so no call depends on
// what an earlier call left there.  All calls on one GPU share the array:
// calls that overlap in time on one GPU race (a call on a second stream while
// the previous one is still running is refused with PSATD_ESTATE).
constexpr size_t kScratchBytes = (size_t)256 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct ScratchSlot {
  void* base = nullptr;  // device address of `scratch` on this device
  hipEvent_t done = nullptr;
  hipStream_t last_stream = nullptr;
  bool known = false;
};
ScratchSlot g_scratch[kMaxDevices];
std::mutex g_scratch_mu;

// Bytes of the two workspaces of plan p (each rounded up to 256 bytes).
size_t scratch_half(const psatd_plan* p) { return ((size_t)p->npts * 11 * 2 * p->rsize + 255) & ~(size_t)255; }
size_t scratch_need(const psatd_plan* p) { return 2 * scratch_half(p); }

// The current device's slot, set up on first use: the array's address and the
// event that marks the end of the last call.
int scratch_slot(ScratchSlot** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return check_hip("hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(PSATD_EUNSUPPORTED, "device %d: static scratch slots exhausted", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  ScratchSlot& sl = g_scratch[dev];
  if (!sl.base) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return check_hip("hipGetSymbolAddress");
    if (!sl.done && hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
      sl.done = nullptr;
      return check_hip("hipEventCreateWithFlags");
    }
    sl.base = ptr;
  }
  *out = &sl;
  return PSATD_OK;
}

int build_plan(const psatd_plan_desc* d, psatd_plan** out) {
  int rc = validate(d);
  if (rc) return rc;
  psatd_plan* p = new psatd_plan;
  p->d = *d;
  p->NX = d->nx + 2 * d->ngx;
  p->NY = d->ny + 2 * d->ngy;
  p->NZ = d->nz + 2 * d->ngz;
  p->NXH = p->NX / 2 + 1;
  p->npts = (long long)p->NXH * p->NY * p->NZ;
  p->ncell = (long long)p->NX * p->NY * p->NZ;
  p->fp64 = d->precision == PSATD_FP64;
  p->rsize = p->fp64 ? 8 : 4;
  const int em = p->fp64 ? emax<double>::v : emax<float>::v;
  const size_t cs = 2 * p->rsize;
  if (!make_axis(p->NX, em, &p->ax) || !make_axis(p->NY, em, &p->ay) || !make_axis(p->NZ, em, &p->az)) {
    free_plan(p);
    return fail(PSATD_EUNSUPPORTED, "box %dx%dx%d: no transform schedule", p->NX, p->NY, p->NZ);
  }
  const LineSchedule& sxs = p->ax.sch;
  const LineSchedule& sys = p->ay.sch;
  const LineSchedule& szs = p->az.sch;
  // Tiles of the x and y passes stay within 64 KB (several workgroups per CU);
  // a z tile holds all 11 lines of each of its columns and may use the device
  // limit when it has a single column.
  const size_t lds_small = std::min<size_t>(64 * 1024, lds_limit());
  const int nth = kLineThreads;
  // P1 tiles leave room for the gather table when a tile of at least one line still fits.
  int nc1 = fit_lines(sxs, nth, em, cs, x_line_cap(p->NX), lds_small - x_table_bytes(p->NX));
  p->xtab = nc1 >= 1;
  if (!p->xtab) nc1 = fit_lines(sxs, nth, em, cs, x_line_cap(p->NX), lds_small);
  p->ty1 = 2 * std::max(nc1, 0);
  p->ty5 = x_inv_tile(p, sxs, em, cs, p->ty1, lds_small);
  p->nl_y = fit_lines(sys, nth, em, cs, y_line_cap(p->NY), lds_small);
  choose_z_tile(p, szs, em, cs);
  if (p->ty1 <= 0 || p->ty5 <= 0 || p->nl_y <= 0 || p->zthreads == 0) {
    free_plan(p);
    return fail(PSATD_EUNSUPPORTED, "box %dx%dx%d does not fit the LDS / register tiling of this build", p->NX,
                p->NY, p->NZ);
  }
  // Every array is addressed through 32-bit byte offsets.
  const double field_bytes = (double)p->npts * cs;
  if (field_bytes >= 4294967296.0 || (double)p->ncell * p->rsize >= 4294967296.0) {
    free_plan(p);
    return fail(PSATD_EUNSUPPORTED, "box %dx%dx%d: one field exceeds 4 GiB", p->NX, p->NY, p->NZ);
  }
  const size_t npts = (size_t)p->npts;
  const size_t tws = p->fp64 ? sizeof(Tw<double>) : sizeof(Tw<float>);
  for (Axis* a : {&p->ax, &p->ay, &p->az}) {
    if ((rc = dalloc(p, &a->tw, tws * a->sch.n)) ||
        (a->blue && ((rc = dalloc(p, &a->chirp, tws * a->n)) || (rc = dalloc(p, &a->filt, tws * a->sch.n))))) {
      std::string msg = g_err;
      free_plan(p);
      return fail(rc, "%s", msg.c_str());
    }
  }
  if ((rc = dalloc(p, (void**)&p->kd, 8 * (size_t)(p->NXH + p->NY + p->NZ))) ||
      (rc = dalloc(p, &p->kw, p->rsize * (size_t)(p->NXH + p->NY + p->NZ))) ||
      ((d->flags & PSATD_FLAG_STAGGERED) && (rc = dalloc(p, &p->kwc, 2 * p->rsize * (size_t)(p->NXH + p->NY + p->NZ)))) ||
      (rc = dalloc(p, &p->coef, 5 * p->rsize * npts)) ||
      (!(d->flags & PSATD_FLAG_NO_WORKSPACE) &&
       ((rc = dalloc(p, &p->wsA, 11 * cs * npts)) || (rc = dalloc(p, &p->wsB, 11 * cs * npts))))) {
    std::string msg = g_err;
    free_plan(p);
    return fail(rc, "%s", msg.c_str());
  }
  hipStream_t s = nullptr;
  for (Axis* a : {&p->ax, &p->ay, &p->az}) {
    launch_twiddles(a->tw, a->sch, p->fp64, s);
    if (a->blue) launch_bluestein(a->chirp, a->filt, a->n, a->sch.n, p->fp64, s);
  }
  const int stag = (d->flags & PSATD_FLAG_STAGGERED) ? 1 : 0;
  launch_modk(p->kd, p->NX, p->NXH, d->dx, d->order, stag, s);
  launch_modk(p->kd + p->NXH, p->NY, p->NY, d->dy, d->order, stag, s);
  launch_modk(p->kd + p->NXH + p->NY, p->NZ, p->NZ, d->dz, d->order, stag, s);
  if (stag) {
    char* kc = (char*)p->kwc;
    const size_t cs1 = 2 * p->rsize;
    launch_shifted(p->kd, kc, p->NX, p->NXH, p->fp64, s);
    launch_shifted(p->kd + p->NXH, kc + cs1 * p->NXH, p->NY, p->NY, p->fp64, s);
    launch_shifted(p->kd + p->NXH + p->NY, kc + cs1 * (p->NXH + p->NY), p->NZ, p->NZ, p->fp64, s);
  }
  char* kw = (char*)p->kw;
  launch_coef(p->coef, kw, kw + p->rsize * p->NXH, kw + p->rsize * (p->NXH + p->NY), p->kd, p->kd + p->NXH,
              p->kd + p->NXH + p->NY, p->NXH, p->NY, p->NZ, d->dt, d->c, 1.0 / (double)p->ncell, p->fp64, s);
  if ((rc = check_hip("table kernels")) || hipDeviceSynchronize() != hipSuccess) {
    if (!rc) rc = check_hip("table build");
    if (!rc) rc = fail(PSATD_EHIP, "table build failed");
    free_plan(p);
    return rc;
  }
  if (d->flags & PSATD_FLAG_NO_WORKSPACE) {
    // such a plan steps only through the static scratch: it must fit, and the
    // scratch is located now so that the first step does no set-up
    ScratchSlot* slot = nullptr;
    if (scratch_need(p) > kScratchBytes)
      rc = fail(PSATD_EINVAL, "box %dx%dx%d needs %zu bytes of workspace, above the %zu-byte static scratch", p->NX,
                p->NY, p->NZ, scratch_need(p), kScratchBytes);
    else
      rc = scratch_slot(&slot);
    if (rc) {
      free_plan(p);
      return rc;
    }
  }
  *out = p;
  return PSATD_OK;
}

// ---------------------------------------------------------------- the five passes
struct StepIO {
  void* wsA = nullptr;  // spectral workspaces (layouts A and B, 11 half spectra each)
  void* wsB = nullptr;
  const void* src[11];  // P1 sources
  int gather;
  int GX, GY, GZ, x0, y0, z0;
  long long src_elems;  // elements of each source array
  void* dst[6];         // P5 destinations
  int scatter;
  int ox, oy, oz;
  long long dst_elems;  // elements of each destination array
  int y_lo, y_hi, z_lo, z_hi;  // box lines needed after the inverse
  int pml = 0;                 // two-step PML: P3 writes the twelve split increments (wsB holds 12 fields)
};

// The compiled two-stage z kernel applies when a box's z tiles hold one column,
// its z lines are transformed directly in exactly two stages, the pair of
// radices is one of kZTwoStage and the tile fits the LDS of one workgroup.
void two_stage_radices(const psatd_plan* p, size_t csize, int* ra, int* rb) {
  *ra = *rb = 0;
  const LineSchedule& s = p->az.sch;
  if (p->zcols != 1 || p->az.blue || s.nstages != 2) return;
  for (const auto& pr : kZTwoStage)
    if (pr[0] == s.radix[0] && pr[1] == s.radix[1] &&
        (size_t)11 * two_stage_slots(pr[0], pr[1]) * csize + (size_t)pr[0] * (pr[1] - 1) * 16 <= lds_limit()) {
      *ra = pr[0];
      *rb = pr[1];
      return;
    }
}

// The compiled two-stage x kernels apply to single boxes whose x lines are transformed
// directly in exactly two stages with radices in kXTwoStage, the tile (and P1's
// column table) fitting in a quarter of the LDS a workgroup may use.
void two_stage_x_radices(const psatd_plan* p, size_t csize, int* ra, int* rb) {
  *ra = *rb = 0;
  const LineSchedule& s = p->ax.sch;
  if (p->ax.blue || s.nstages != 2) return;
  for (const auto& pr : kXTwoStage)
    if (pr[0] == s.radix[0] && pr[1] == s.radix[1] &&
        (size_t)kXTwoStageLines * two_stage_slots(pr[0], pr[1]) * csize + (size_t)(p->NX + 3) * sizeof(int) +
                (size_t)pr[0] * (pr[1] - 1) * 16 <=
            lds_limit() / 3) {
      *ra = pr[0];
      *rb = pr[1];
      return;
    }
}

// The compiled two-stage y kernels apply when the y lines are transformed
// directly in exactly two stages whose radices are one of kYTwoStage, and a tile
// of kYTwoStageLines lines fits in LDS with room for a second block per CU.
void two_stage_y_radices(const psatd_plan* p, size_t csize, int* ra, int* rb) {
  *ra = *rb = 0;
  const LineSchedule& s = p->ay.sch;
  if (p->ay.blue || s.nstages != 2) return;
  for (const auto& pr : kYTwoStage)
    if (pr[0] == s.radix[0] && pr[1] == s.radix[1] &&
        (size_t)kYTwoStageLines * two_stage_y_slots(pr[0], pr[1]) * csize + (size_t)pr[0] * (pr[1] - 1) * 16 <=
            lds_limit() / 2) {
      *ra = pr[0];
      *rb = pr[1];
      return;
    }
}

template <typename T>
void set_ypass(YPassParams<T>& y, int nfields) {
  y.utiles = (y.u_hi - y.u_lo + y.nl - 1) / y.nl;
  y.nl_last = (y.u_hi - y.u_lo) - (y.utiles - 1) * y.nl;
  y.ntiles = nfields * y.nouter * y.utiles;
  y.fd_utiles = make_fastdiv(y.utiles);
  y.fd_nouter = make_fastdiv(y.nouter);
  y.fd_n = make_fastdiv(y.n);
  y.fd_nl = make_fastdiv(y.nl);
  y.fd_nl_last = make_fastdiv(y.nl_last);
  y.fd_np = make_fastdiv(y.p_hi - y.p_lo);
}

// Records event `i` of the current step when timing is on.
struct Marks {
  std::array<hipEvent_t, 6>* set = nullptr;
  hipStream_t s = nullptr;
  void mark(int i) {
    if (set) (void)hipEventRecord((*set)[i], s);
  }
};

template <typename T>
struct StepParams {
  XFwdParams<T> x1;
  YPassParams<T> y2;
  ZPushParams<T> z3;
  YPassParams<T> y4;
  XInvParams<T> x5;
};

// Kernel parameters of the five passes of one step of plan p with the given inputs / outputs.
template <typename T>
void build_step(psatd_plan* p, const StepIO& io, StepParams<T>& sp, bool batched = false) {
  const int NX = p->NX, NY = p->NY, NZ = p->NZ, NXH = p->NXH;
  const long long npts = p->npts;
  const uint32_t fbytes = (uint32_t)(npts * (long long)sizeof(cx<T>));
  const int nth = kLineThreads;
  cx<T>* A = (cx<T>*)io.wsA;
  cx<T>* B = (cx<T>*)io.wsB;
  const T* kw = (const T*)p->kw;

  XFwdParams<T>& x1 = sp.x1;
  x1 = XFwdParams<T>{};
  for (int f = 0; f < 11; ++f) x1.src[f] = (const T*)io.src[f];
  x1.src_bytes = (uint32_t)(io.src_elems * (long long)sizeof(T));
  x1.dst = A;
  x1.npts = npts;
  x1.dst_bytes = fbytes;
  x1.NX = NX;
  x1.NY = NY;
  x1.NZ = NZ;
  x1.NXH = NXH;
  x1.ty = p->ty1;
  x1.ytiles = (NY + x1.ty - 1) / x1.ty;
  x1.ntiles = 11 * NZ * x1.ytiles;
  x1.gather = io.gather;
  x1.xtab = io.gather && p->xtab;
  x1.GX = io.GX;
  x1.GY = io.GY;
  x1.GZ = io.GZ;
  x1.x0 = io.x0;
  x1.y0 = io.y0;
  x1.z0 = io.z0;
  x1.fd_ytiles = make_fastdiv(x1.ytiles);
  x1.fd_NZ = make_fastdiv(NZ);
  x1.fd_NX = make_fastdiv(NX);
  x1.fd_nc = make_fastdiv(x1.ty / 2);
  if (io.gather) {
    x1.fd_GX = make_fastdiv(io.GX);
    x1.fd_GY = make_fastdiv(io.GY);
    x1.fd_GZ = make_fastdiv(io.GZ);
  }
  x1.ld_drow = nth / NX;
  x1.ld_dcol = nth % NX;
  x1.wr_drow = nth / (x1.ty / 2);
  x1.wr_dcol = nth % (x1.ty / 2);
  x1.fft = line_fft<T>(p->ax);
  int xra = 0, xrb = 0;
  if (!batched) two_stage_x_radices(p, sizeof(cx<T>), &xra, &xrb);
  if (p->two_stage_mask & 1) {
    x1.ra = xra;
    x1.rb = xrb;
  }
  if (x1.ra) {  // tiles of kXTwoStageLines complex lines
    x1.ty = 2 * kXTwoStageLines;
    x1.ytiles = (NY + x1.ty - 1) / x1.ty;
    x1.ntiles = 11 * NZ * x1.ytiles;
    x1.fd_ytiles = make_fastdiv(x1.ytiles);
    x1.fd_nc = make_fastdiv(x1.ty / 2);
  }

  YPassParams<T>& y2 = sp.y2;
  y2 = YPassParams<T>{};
  y2.in = A;
  y2.out = B;
  y2.fs_in = npts;
  y2.fs_out = npts;
  y2.in_bytes = fbytes;
  y2.out_bytes = fbytes;
  y2.os_in = NY;
  y2.ls_in = NXH * NY;
  y2.ps_in = 1;
  y2.os_out = NY * NZ;
  y2.ls_out = 1;
  y2.ps_out = NZ;
  y2.n = NY;
  y2.nl = p->nl_y;
  int yra = 0, yrb = 0;
  if (!batched) two_stage_y_radices(p, sizeof(cx<T>), &yra, &yrb);
  if (p->two_stage_mask & 2) {
    y2.ra = yra;
    y2.rb = yrb;
  }
  if (y2.ra) y2.nl = kYTwoStageLines;
  y2.u_lo = 0;
  y2.u_hi = NZ;
  y2.nouter = NXH;
  y2.p_lo = 0;
  y2.p_hi = NY;
  set_ypass(y2, 11);
  y2.fft = line_fft<T>(p->ay);

  ZPushParams<T>& z3 = sp.z3;
  z3 = ZPushParams<T>{};
  z3.b = B;
  z3.npts = npts;
  z3.field_bytes = fbytes;
  z3.coef = (const T*)p->coef;
  z3.coef_bytes = (uint32_t)(npts * (long long)sizeof(T));
  z3.kx = kw;
  z3.ky = kw + NXH;
  z3.kz = kw + NXH + NY;
  z3.stag = (p->d.flags & PSATD_FLAG_STAGGERED) ? 1 : 0;
  if (z3.stag) {
    const cx<T>* kc = (const cx<T>*)p->kwc;
    z3.kxc = kc;
    z3.kyc = kc + NXH;
    z3.kzc = kc + NXH + NY;
  }
  z3.NY = NY;
  z3.NZ = NZ;
  z3.NXH = NXH;
  z3.ncol = p->zcols;
  z3.zgroup = z_group(p->az.sch, p->zthreads, emax<T>::v, sizeof(cx<T>), 11 * p->zcols);
  z3.ntiles = (NXH * NY + p->zcols - 1) / p->zcols;
  z3.z_lo = io.z_lo;
  z3.z_hi = io.z_hi;
  z3.c2 = T(p->d.c * p->d.c);
  z3.inv_eps0 = T(1.0 / p->d.eps0);
  z3.fd_NY = make_fastdiv(NY);
  z3.fd_NZ = make_fastdiv(NZ);
  z3.fd_ncol = make_fastdiv(p->zcols);
  z3.fft = line_fft<T>(p->az);
  z3.pml = io.pml;
  z3.dt = T(p->d.dt);
  z3.inv_n = T(1.0 / ((double)NX * NY * NZ));
  if (io.pml) {  // twelve lines per column in LDS: fewer columns per tile if needed
    int nc = p->zcols;
    while (nc > 1 && (size_t)12 * nc * lds_line(p->az.sch.n) * sizeof(cx<T>) > z_lds(nc)) --nc;
    z3.ncol = nc;
    z3.ntiles = (NXH * NY + nc - 1) / nc;
    z3.fd_ncol = make_fastdiv(nc);
    z3.zgroup = z_group(p->az.sch, p->zthreads, emax<T>::v, sizeof(cx<T>), 12 * nc);
  }
  if (!batched && (p->two_stage_mask & 4)) {
    two_stage_radices(p, sizeof(cx<T>), &z3.ra, &z3.rb);
    // PML: the two-stage kernel keeps a twelfth line in LDS
    if (io.pml && z3.ra &&
        (size_t)12 * two_stage_slots(z3.ra, z3.rb) * sizeof(cx<T>) + (size_t)z3.ra * (z3.rb - 1) * 16 > lds_limit())
      z3.ra = z3.rb = 0;
  }

  YPassParams<T>& y4 = sp.y4;
  y4 = YPassParams<T>{};
  y4.in = B;
  y4.out = A;
  y4.fs_in = npts;
  y4.fs_out = npts;
  y4.in_bytes = fbytes;
  y4.out_bytes = fbytes;
  y4.os_in = NY * NZ;
  y4.ls_in = 1;
  y4.ps_in = NZ;
  y4.os_out = NY;
  y4.ls_out = NXH * NY;
  y4.ps_out = 1;
  y4.n = NY;
  y4.nl = p->nl_y;
  if (p->two_stage_mask & 8) {
    y4.ra = yra;
    y4.rb = yrb;
  }
  if (y4.ra) y4.nl = kYTwoStageLines;
  y4.u_lo = io.z_lo;
  y4.u_hi = io.z_hi;
  y4.nouter = NXH;
  y4.p_lo = io.y_lo;
  y4.p_hi = io.y_hi;
  set_ypass(y4, 6);
  y4.fft = line_fft<T>(p->ay);

  XInvParams<T>& x5 = sp.x5;
  x5 = XInvParams<T>{};
  x5.src = A;
  x5.npts = npts;
  x5.src_bytes = fbytes;
  for (int f = 0; f < 6; ++f) x5.dst[f] = (T*)io.dst[f];
  x5.dst_bytes = (uint32_t)(io.dst_elems * (long long)sizeof(T));
  x5.NX = NX;
  x5.NY = NY;
  x5.NZ = NZ;
  x5.NXH = NXH;
  x5.ty = p->ty5;
  x5.y_lo = io.y_lo;
  x5.y_hi = io.y_hi;
  x5.z_lo = io.z_lo;
  x5.z_hi = io.z_hi;
  x5.ytiles = (io.y_hi - io.y_lo + x5.ty - 1) / x5.ty;
  x5.ntiles = 6 * (io.z_hi - io.z_lo) * x5.ytiles;
  x5.scatter = io.scatter;
  x5.GX = io.GX;
  x5.GY = io.GY;
  x5.GZ = io.GZ;
  x5.ox = io.ox;
  x5.oy = io.oy;
  x5.oz = io.oz;
  x5.gx = p->d.ngx;
  x5.gy = p->d.ngy;
  x5.gz = p->d.ngz;
  x5.nx = p->d.nx;
  x5.fd_ytiles = make_fastdiv(x5.ytiles);
  x5.fd_nz = make_fastdiv(io.z_hi - io.z_lo);
  x5.fd_nc = make_fastdiv(x5.ty / 2);
  x5.fd_NX = make_fastdiv(NX);
  if (io.scatter) {
    x5.fd_GX = make_fastdiv(io.GX);
    x5.fd_GY = make_fastdiv(io.GY);
    x5.fd_GZ = make_fastdiv(io.GZ);
  }
  x5.nthreads = p->x5threads;
  x5.fft = line_fft<T>(p->ax);
  if (p->two_stage_mask & 16) {
    x5.ra = xra;
    x5.rb = xrb;
  }
  if (x5.ra) {
    x5.ty = 2 * kXTwoStageLines;
    x5.ytiles = (io.y_hi - io.y_lo + x5.ty - 1) / x5.ty;
    x5.ntiles = 6 * (io.z_hi - io.z_lo) * x5.ytiles;
    x5.fd_ytiles = make_fastdiv(x5.ytiles);
    x5.fd_nc = make_fastdiv(x5.ty / 2);
  }
}

template <typename T>
int run_step(psatd_plan* p, const StepIO& io, hipStream_t s, bool allow_timing = true) {
  Marks mk;
  mk.s = s;
  if (p->timing && allow_timing) {
    std::array<hipEvent_t, 6> set{};
    for (auto& e : set)
      if (hipEventCreate(&e) != hipSuccess) return check_hip("hipEventCreate");
    p->events.push_back(set);
    mk.set = &p->events.back();
  }
  StepParams<T> sp;
  build_step<T>(p, io, sp);
  mk.mark(0);
  launch_xfwd<T>(sp.x1, s);
  mk.mark(1);
  launch_ypass<T>(sp.y2, 0, s);
  mk.mark(2);
  launch_zpush<T>(sp.z3, p->zthreads, s);
  mk.mark(3);
  launch_ypass<T>(sp.y4, 1, s);
  mk.mark(4);
  launch_xinv<T>(sp.x5, s);
  mk.mark(5);
  return check_hip("step kernels");
}

// Two-step PML step on the split parts: forward passes and the z pass once (the z pass
// writes both split sets' increments, 12 fields of layout B), then per set the inverse y
// and x passes into the increment arrays and the damped update of that set's parts.
template <typename T>
int run_pml(psatd_plan* p, const StepIO& io, void* const* parts, hipStream_t s) {
  StepParams<T> sp;
  build_step<T>(p, io, sp);
  launch_xfwd<T>(sp.x1, s);
  launch_ypass<T>(sp.y2, 0, s);
  launch_zpush<T>(sp.z3, p->zthreads, s);
  for (int set = 0; set < 2; ++set) {
    YPassParams<T> y4 = sp.y4;
    y4.in = (const cx<T>*)io.wsB + (i64)6 * set * p->npts;
    launch_ypass<T>(y4, 1, s);
    launch_xinv<T>(sp.x5, s);
    launch_pml_update(parts + 6 * set, p->pml_inc, p->pml_damp, set + 1, p->NX, p->NY, p->NZ, p->fp64, s);
  }
  return check_hip("psatd_pml_step");
}

// Streams: an object (plan or batch) owns its workspace, so a step may start on
// a stream other than the previous step's only once that step has finished.
// Each step records an event at its end; a call on another stream queries it.
// Steps enqueued while the stream is being captured into a graph are left to
// the caller (an event query is not allowed there, and the graph runs later).
bool capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return st != hipStreamCaptureStatusNone;
}

struct StreamGuard {
  hipEvent_t* done;
  hipStream_t* last;
  bool* known;
  // PSATD_ESTATE while the previous step runs on another stream.
  int check(hipStream_t s, const char* what) const {
    if (!*known || *last == s || capturing(s)) return PSATD_OK;
    const hipError_t e = hipEventQuery(*done);
    if (e == hipErrorNotReady)
      return fail(PSATD_ESTATE, "%s: the previous step is still running on another stream", what);
    if (e != hipSuccess) return check_hip(what);
    return PSATD_OK;
  }
  // Records the end of the step just enqueued on s.
  int mark(hipStream_t s, const char* what) const {
    if (capturing(s)) return PSATD_OK;
    if (!*done && hipEventCreateWithFlags(done, hipEventDisableTiming) != hipSuccess) {
      *done = nullptr;
      return check_hip(what);
    }
    if (hipEventRecord(*done, s) != hipSuccess) return check_hip(what);
    *last = s;
    *known = true;
    return PSATD_OK;
  }
};

StreamGuard guard_of(psatd_plan* p) { return StreamGuard{&p->done, &p->last_stream, &p->in_flight_known}; }

int dispatch_step(psatd_plan* p, const StepIO& io, hipStream_t s) {
  const StreamGuard g = guard_of(p);
  int rc = g.check(s, "step");
  if (rc) return rc;
  rc = p->fp64 ? run_step<double>(p, io, s) : run_step<float>(p, io, s);
  if (rc) return rc;
  return g.mark(s, "step");
}

// ---------------------------------------------------------------- autotuner
// For each axis the tuner times the passes that transform along it (x: P1 + P5,
// y: P2 + P4, z: P3) for a few radix factorisations / orders of the line
// length and tile sizes, on the plan's own workspace (contents irrelevant), and
// keeps the fastest.  Results are cached per (precision, axis role, line
// length, the two other box lengths) in memory and optionally in a JSON file.

// Radix sequences the autotuner times for n: the cost model's best few, the
// default first.
std::vector<std::vector<int>> radix_candidates(int n, int emax, size_t cap) {
  (void)emax;
  return ranked_schedules(n, cap);
}

void set_radices(LineSchedule* s, const std::vector<int>& r) {
  const int n = s->n;
  std::memset(s, 0, sizeof *s);
  s->n = n;
  s->nstages = (int)r.size();
  int span = 1;
  for (size_t i = 0; i < r.size(); ++i) {
    s->radix[i] = r[i];
    s->bfl[i] = make_fastdiv((uint32_t)(n / r[i]));
    s->ns[i] = make_fastdiv((uint32_t)span);
    span *= r[i];
  }
}

struct TuneEntry {
  std::vector<int> radix;
  int tile = 0;
  int kern = -1;  // two-stage kernel bits (psatd_plan::two_stage_mask) of the axis's passes, -1 unknown
};
std::map<std::string, TuneEntry>& tune_cache() {
  static std::map<std::string, TuneEntry> c;
  return c;
}

// Version of the cache file format and of the schedule space it describes (the
// compiled radices, tile rules and register budget).  Entries of files written
// under another version are discarded.
constexpr int kTuneSchema = 3;

bool compiled_radix(int r) {
  for (int k : kRadix)
    if (k == r) return true;
  return false;
}

// A radix sequence is usable for a transform of length m when its radices are all
// compiled and multiply to m.
bool valid_radices(const std::vector<int>& r, int m) {
  if (m < 1 || (int)r.size() > kMaxStages || (m > 1 && r.empty())) return false;
  long long prod = 1;
  for (int v : r) {
    if (!compiled_radix(v)) return false;
    prod *= v;
    if (prod > m) return false;
  }
  return prod == m;
}

// Minimal reader of the cache file written by save_tune_file:
//   {"psatd_tune_cache": <schema>, "entries": {"<key>": {"radix": [..], "tile": <int>}, ...}}
// Malformed text ends the scan; entries that fail the checks are counted as rejected.
struct Scanner {
  const std::string& t;
  size_t i = 0;
  void ws() {
    while (i < t.size() && (t[i] == ' ' || t[i] == '\n' || t[i] == '\t' || t[i] == '\r')) ++i;
  }
  bool eat(char c) {
    ws();
    if (i < t.size() && t[i] == c) {
      ++i;
      return true;
    }
    return false;
  }
  bool str(std::string* out) {
    ws();
    if (i >= t.size() || t[i] != '"') return false;
    const size_t e = t.find('"', i + 1);
    if (e == std::string::npos) return false;
    *out = t.substr(i + 1, e - i - 1);
    i = e + 1;
    return true;
  }
  bool num(long long* out) {
    ws();
    size_t j = i;
    if (j < t.size() && t[j] == '-') ++j;
    const size_t d0 = j;
    while (j < t.size() && t[j] >= '0' && t[j] <= '9' && j - d0 < 12) ++j;
    if (j == d0 || (j < t.size() && t[j] >= '0' && t[j] <= '9')) return false;
    *out = std::strtoll(t.c_str() + i, nullptr, 10);
    i = j;
    return true;
  }
};

// Transform length m recorded in a cache key ("...|m=<m>|...").
int key_length(const std::string& key) {
  const size_t k = key.find("|m=");
  if (k == std::string::npos) return -1;
  long long v = 0;
  size_t j = k + 3, d0 = j;
  while (j < key.size() && key[j] >= '0' && key[j] <= '9' && j - d0 < 9) v = 10 * v + (key[j++] - '0');
  return j == d0 ? -1 : (int)v;
}

void load_tune_file(const char* path, int* accepted = nullptr, int* rejected = nullptr) {
  int ok = 0, bad = 0;
  if (accepted) *accepted = 0;
  if (rejected) *rejected = 0;
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  std::string text;
  char buf[4096];
  size_t k;
  while ((k = std::fread(buf, 1, sizeof buf, f)) > 0 && text.size() < (1u << 24)) text.append(buf, k);
  std::fclose(f);
  Scanner sc{text};
  std::string name;
  long long schema = -1;
  if (!sc.eat('{') || !sc.str(&name) || name != "psatd_tune_cache" || !sc.eat(':') || !sc.num(&schema) ||
      !sc.eat(',') || !sc.str(&name) || name != "entries" || !sc.eat(':') || !sc.eat('{')) {
    if (rejected) *rejected = 1;
    return;
  }
  const bool current = schema == kTuneSchema;
  for (bool first = true;; first = false) {
    if (sc.eat('}')) break;
    if (!first && !sc.eat(',')) {
      ++bad;
      break;
    }
    std::string key, field;
    TuneEntry e;
    long long v = 0;
    bool good = sc.str(&key) && sc.eat(':') && sc.eat('{') && sc.str(&field) && field == "radix" && sc.eat(':') &&
                sc.eat('[');
    if (good && !sc.eat(']')) {
      do {
        good = sc.num(&v) && v > 0 && v < 1000 && e.radix.size() < (size_t)kMaxStages;
        if (good) e.radix.push_back((int)v);
      } while (good && sc.eat(','));
      good = good && sc.eat(']');
    }
    good = good && sc.eat(',') && sc.str(&field) && field == "tile" && sc.eat(':') && sc.num(&v);
    e.tile = (int)std::max(-1LL, std::min(v, 1LL << 20));
    if (good && sc.eat(',')) {
      long long kv = -1;
      good = sc.str(&field) && field == "kern" && sc.eat(':') && sc.num(&kv) && kv >= 0 && kv < 32;
      e.kern = (int)kv;
    }
    good = good && sc.eat('}');
    if (!good) {  // malformed: stop reading
      ++bad;
      break;
    }
    if (current && e.tile > 0 && valid_radices(e.radix, key_length(key))) {
      tune_cache()[key] = e;
      ++ok;
    } else {
      ++bad;
    }
  }
  if (accepted) *accepted = ok;
  if (rejected) *rejected = bad;
}

void save_tune_file(const char* path) {
  if (!path) return;
  FILE* f = std::fopen(path, "w");
  if (!f) return;
  std::fprintf(f, "{\n  \"psatd_tune_cache\": %d,\n  \"entries\": {\n", kTuneSchema);
  size_t i = 0;
  for (auto& kv : tune_cache()) {
    std::fprintf(f, "    \"%s\": {\"radix\": [", kv.first.c_str());
    for (size_t j = 0; j < kv.second.radix.size(); ++j)
      std::fprintf(f, "%s%d", j ? ", " : "", kv.second.radix[j]);
    std::fprintf(f, "], \"tile\": %d, \"kern\": %d}%s\n", kv.second.tile, std::max(0, kv.second.kern),
                 ++i < tune_cache().size() ? "," : "");
  }
  std::fprintf(f, "  }\n}\n");
  std::fclose(f);
}

// Mean milliseconds of `reps` runs of the passes of axis `ax` (0 x, 1 y, 2 z) on scratch data.
template <typename T>
float time_axis(psatd_plan* p, int ax, int reps, hipStream_t s) {
  StepIO io{};
  io.wsA = p->wsA;
  io.wsB = p->wsB;
  T* scratch = (T*)p->wsB;  // box-shaped real arrays for P1 inputs / P5 outputs
  for (int f = 0; f < 11; ++f) io.src[f] = scratch;
  for (int f = 0; f < 6; ++f) io.dst[f] = scratch;
  io.src_elems = io.dst_elems = p->ncell;
  io.y_lo = 0;
  io.y_hi = p->NY;
  io.z_lo = 0;
  io.z_hi = p->NZ;
  StepParams<T> sp;
  build_step<T>(p, io, sp);
  if (ax == 0) sp.x5.src = (const cx<T>*)p->wsA;
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  float best = 1e30f;
  for (int pass = 0; pass < 2; ++pass) {  // first pass warms up
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps; ++r) {
      if (ax == 0) {
        launch_xfwd<T>(sp.x1, s);
        launch_xinv<T>(sp.x5, s);
      } else if (ax == 1) {
        launch_ypass<T>(sp.y2, 0, s);
        launch_ypass<T>(sp.y4, 1, s);
      } else {
        launch_zpush<T>(sp.z3, p->zthreads, s);
      }
    }
    (void)hipEventRecord(e1, s);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    best = std::min(best, ms / reps);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return best;
}

// Mean milliseconds of `reps` launches of pass `pass` (0..4 = P1..P5) on scratch data.
template <typename T>
float time_pass(psatd_plan* p, int pass, int reps, hipStream_t s) {
  StepIO io{};
  io.wsA = p->wsA;
  io.wsB = p->wsB;
  T* scratch = (T*)p->wsB;
  for (int f = 0; f < 11; ++f) io.src[f] = scratch;
  for (int f = 0; f < 6; ++f) io.dst[f] = scratch;
  io.src_elems = io.dst_elems = p->ncell;
  io.y_lo = 0;
  io.y_hi = p->NY;
  io.z_lo = 0;
  io.z_hi = p->NZ;
  StepParams<T> sp;
  build_step<T>(p, io, sp);
  if (pass == 4) sp.x5.src = (const cx<T>*)p->wsA;
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  float best = 1e30f;
  for (int rep = 0; rep < 2; ++rep) {  // first round warms up
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps; ++r) {
      switch (pass) {
        case 0: launch_xfwd<T>(sp.x1, s); break;
        case 1: launch_ypass<T>(sp.y2, 0, s); break;
        case 2: launch_zpush<T>(sp.z3, p->zthreads, s); break;
        case 3: launch_ypass<T>(sp.y4, 1, s); break;
        default: launch_xinv<T>(sp.x5, s); break;
      }
    }
    (void)hipEventRecord(e1, s);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    best = std::min(best, ms / reps);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return best;
}

// Whether pass `pass` has a two-stage kernel under the plan's current schedules.
template <typename T>
bool has_two_stage(psatd_plan* p, int pass) {
  int ra = 0, rb = 0;
  const size_t cs = sizeof(cx<T>);
  if (pass == 0 || pass == 4)
    two_stage_x_radices(p, cs, &ra, &rb);
  else if (pass == 1 || pass == 3)
    two_stage_y_radices(p, cs, &ra, &rb);
  else
    two_stage_radices(p, cs, &ra, &rb);
  return ra > 0;
}

template <typename T>
int autotune_plan(psatd_plan* p, hipStream_t s) {
  const int em = emax<T>::v;
  const size_t cs = sizeof(cx<T>);
  const size_t lds_small = std::min<size_t>(64 * 1024, lds_limit());
  const int nth = kLineThreads;
  const int lens[3] = {p->NX, p->NY, p->NZ};
  Axis* axes[3] = {&p->ax, &p->ay, &p->az};
  for (int a = 0; a < 3; ++a) {
    Axis& A = *axes[a];
    char key[160];
    std::snprintf(key, sizeof key, "%s|%c|n=%d|m=%d|other=%dx%d", p->fp64 ? "fp64" : "fp32", "xyz"[a], A.n,
                  A.sch.n, lens[(a + 1) % 3], lens[(a + 2) % 3]);
    // Tile sizes this build allows for a schedule of axis a (largest first, at most two),
    // and whether a given tile is one of the allowed ones.
    auto tile_limit = [&](const LineSchedule& sch) {
      if (a == 0)
        return fit_lines(sch, nth, em, cs, x_line_cap(p->NX), lds_small - (p->xtab ? x_table_bytes(p->NX) : 0));
      return fit_lines(sch, nth, em, cs, y_line_cap(p->NY), lds_small);
    };
    auto tiles_for = [&](const LineSchedule& sch) {
      std::vector<int> tl;
      if (a == 2) {
        for (int zt : kZThreads)
          if (z_fits(sch, zt, em, cs, p->zcols) && tl.size() < 2) tl.push_back(zt);
      } else {
        for (int t = tile_limit(sch); t >= 1 && tl.size() < 2; t = t / 2) tl.push_back(a == 0 ? 2 * t : t);
      }
      return tl;
    };
    auto tile_fits = [&](const LineSchedule& sch, int t) {
      if (a == 2) return (t == kZThreads[0] || t == kZThreads[1]) && z_fits(sch, t, em, cs, p->zcols);
      const int hi = tile_limit(sch);
      return a == 0 ? (t >= 2 && t % 2 == 0 && t / 2 <= hi) : (t >= 1 && t <= hi);
    };
    // A cached entry is used only if it still describes a valid schedule of this
    // plan under the current limits; otherwise it is dropped and the axis re-tuned.
    auto hit = tune_cache().find(key);
    if (hit != tune_cache().end()) {
      bool ok = valid_radices(hit->second.radix, A.sch.n);
      if (ok) {
        LineSchedule probe = A.sch;
        set_radices(&probe, hit->second.radix);
        ok = tile_fits(probe, hit->second.tile);
      }
      if (!ok) {
        tune_cache().erase(hit);
        hit = tune_cache().end();
      }
    }
    std::vector<std::vector<int>> cands;
    if (hit != tune_cache().end()) {
      cands.push_back(hit->second.radix);
    } else {
      cands = radix_candidates(A.sch.n, em, 6);
    }
    const LineSchedule saved = A.sch;
    const int saved_tile = a == 0 ? p->ty1 : (a == 1 ? p->nl_y : p->zthreads);
    float best = 1e30f;
    TuneEntry best_e{std::vector<int>(saved.radix, saved.radix + saved.nstages), saved_tile};
    for (auto& r : cands) {
      set_radices(&A.sch, r);
      launch_twiddles(A.tw, A.sch, p->fp64, s);
      std::vector<int> tl = hit != tune_cache().end() ? std::vector<int>{hit->second.tile} : tiles_for(A.sch);
      for (int t : tl) {
        if (t <= 0) continue;
        if (a == 0) {
          p->ty1 = t;
          p->ty5 = x_inv_tile(p, A.sch, em, cs, t, lds_small);
        } else if (a == 1) {
          p->nl_y = t;
        } else {
          p->zthreads = t;
        }
        const float ms = time_axis<T>(p, a, 3, s);
        if (hipGetLastError() != hipSuccess) continue;
        if (ms < best) {
          best = ms;
          best_e = TuneEntry{r, t};
        }
      }
    }
    set_radices(&A.sch, best_e.radix);
    launch_twiddles(A.tw, A.sch, p->fp64, s);
    if (a == 0) {
      p->ty1 = best_e.tile;
      p->ty5 = x_inv_tile(p, A.sch, em, cs, best_e.tile, lds_small);
    } else if (a == 1) {
      p->nl_y = best_e.tile;
    } else {
      p->zthreads = best_e.tile;
    }
    // Per pass of this axis, the two-stage kernel or the run-time-schedule one,
    // whichever is faster on the chosen schedule (a cached choice is reused).
    {
      const int passes_of_axis[3][2] = {{0, 4}, {1, 3}, {2, -1}};
      for (int pass : passes_of_axis[a]) {
        if (pass < 0) continue;
        const int bit = 1 << pass;
        if (!has_two_stage<T>(p, pass)) continue;
        if (hit != tune_cache().end() && hit->second.kern >= 0) {
          p->two_stage_mask = (p->two_stage_mask & ~bit) | (hit->second.kern & bit);
          continue;
        }
        // alternate the two kernels and keep each one's best time; leave the default
        // kernel of the pass only for a gain above 2 % (run-to-run noise is about 1 %)
        float t2 = 1e30f, t1 = 1e30f;
        for (int rep = 0; rep < 2; ++rep) {
          p->two_stage_mask |= bit;
          t2 = std::min(t2, time_pass<T>(p, pass, 3, s));
          p->two_stage_mask &= ~bit;
          t1 = std::min(t1, time_pass<T>(p, pass, 3, s));
        }
        if (hipGetLastError() != hipSuccess) continue;
        const bool two_stage_default = (kTwoStageDefault & bit) != 0;
        if (two_stage_default ? !(t1 < 0.98f * t2) : (t2 < 0.98f * t1)) p->two_stage_mask |= bit;
      }
      best_e.kern = p->two_stage_mask & ((a == 0) ? (1 | 16) : (a == 1) ? (2 | 8) : 4);
    }
    tune_cache()[key] = best_e;
  }
  return check_hip("autotune");
}

bool distinct(const void* const* a, int n) {
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j)
      if (a[i] == a[j]) return false;
  return true;
}

int check_geometry(const psatd_plan* p, const int origin[3], const int gdims[3]) {
  if (!origin || !gdims) return fail(PSATD_EINVAL, "origin / gdims is NULL");
  const int n[3] = {p->d.nx, p->d.ny, p->d.nz};
  for (int a = 0; a < 3; ++a) {
    if (gdims[a] <= 0) return fail(PSATD_EINVAL, "global sizes must be positive");
    if (origin[a] < 0 || origin[a] >= gdims[a]) return fail(PSATD_EINVAL, "origin must lie in [0, gdims)");
    if (n[a] > gdims[a]) return fail(PSATD_EINVAL, "interior larger than the global grid");
  }
  return PSATD_OK;
}

// Argument checks shared by the fused steps on G1.
int check_g1_call(const psatd_plan* p, void* const* g1, const int origin[3], const int gdims[3]) {
  if (!p || !g1) return fail(PSATD_EINVAL, "NULL argument");
  int rc = check_geometry(p, origin, gdims);
  if (rc) return rc;
  for (int f = 0; f < 11; ++f)
    if (!g1[f]) return fail(PSATD_EINVAL, "field pointer %d is NULL", f);
  if (!distinct(g1, 11)) return fail(PSATD_EINVAL, "field arrays must be distinct");
  if ((double)gdims[0] * gdims[1] * gdims[2] * p->rsize >= 4294967296.0)
    return fail(PSATD_EUNSUPPORTED, "global arrays of 4 GiB or more are not supported");
  return PSATD_OK;
}

// Inputs / outputs of a fused step on G1: gather with wrap, scatter of the interior.
StepIO g1_io(const psatd_plan* p, void* const* g1, const int origin[3], const int gdims[3]) {
  StepIO io{};
  io.wsA = p->wsA;
  io.wsB = p->wsB;
  for (int f = 0; f < 11; ++f) io.src[f] = g1[f];
  for (int f = 0; f < 6; ++f) io.dst[f] = g1[f];
  io.gather = 1;
  io.scatter = 1;
  io.GX = gdims[0];
  io.GY = gdims[1];
  io.GZ = gdims[2];
  const int g[3] = {p->d.ngx, p->d.ngy, p->d.ngz};
  int st[3];
  for (int a = 0; a < 3; ++a) st[a] = (int)((((long long)origin[a] - g[a]) % gdims[a] + gdims[a]) % gdims[a]);
  io.x0 = st[0];
  io.y0 = st[1];
  io.z0 = st[2];
  io.ox = origin[0];
  io.oy = origin[1];
  io.oz = origin[2];
  io.src_elems = (long long)gdims[0] * gdims[1] * gdims[2];
  io.dst_elems = io.src_elems;
  io.y_lo = p->d.ngy;
  io.y_hi = p->d.ngy + p->d.ny;
  io.z_lo = p->d.ngz;
  io.z_hi = p->d.ngz + p->d.nz;
  return io;
}

}  // namespace

// ---------------------------------------------------------------- batches
// A batch keeps one plan per box.  Binding it to a set of G1 arrays builds the
// kernel parameters of every box for every pass and uploads them, with the
// tile offsets, to device memory; each pass of a step is then one persistent
// launch per class of boxes with the same block size and a similar LDS size
// (kernels in passes.hip).  Steps can be replayed from a captured hipGraph.
struct psatd_batch {
  int nsub = 0;
  int fp64 = 0;
  int gd[3] = {0, 0, 0};
  std::vector<psatd_plan*> plans;
  std::vector<std::array<int, 3>> origins;
  void* descs[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};  // per-pass parameter arrays
  size_t desc_bytes[5] = {0, 0, 0, 0, 0};
  int* starts = nullptr;                                           // tile offsets of every launch class
  size_t starts_bytes = 0;
  // Launch classes of each pass: boxes whose blocks need the same thread count and
  // a similar LDS size run in one persistent launch sized for them (a box with
  // long chirp-z lines no longer sets the block shape of every other box).
  struct Class {
    int first = 0, nbox = 0;  // boxes [first, first + nbox) of the pass's descriptor array
    int soff = 0;             // their tile offsets at starts[soff .. soff + nbox]
    int total = 0;            // tiles
    int threads = 0;
    size_t lds = 0;
  };
  std::vector<Class> cls[5];
  hipEvent_t done = nullptr;  // completion of the last step / replay (see psatd_plan::done)
  hipStream_t last_stream = nullptr;
  bool in_flight_known = false;
  int totals[5] = {0, 0, 0, 0, 0};
  const void* bound[11] = {};
  bool is_bound = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;  // side stream for capture (the null stream cannot be captured)
  int graph_steps = 0;
  long long box_cells = 0, interior_cells = 0;
};

namespace {

void free_batch(psatd_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  for (int k = 0; k < 5; ++k) budget_free(b->descs[k], b->desc_bytes[k]);
  budget_free(b->starts, b->starts_bytes);
  if (b->done) (void)hipEventDestroy(b->done);
  for (psatd_plan* p : b->plans) free_plan(p);
  delete b;
}

template <typename P>
int upload(const std::vector<P>& v, void** dst, size_t* dst_bytes) {
  budget_free(*dst, *dst_bytes);
  *dst = nullptr;
  *dst_bytes = 0;
  if (budget_malloc(dst, v.size() * sizeof(P)) != hipSuccess) {
    (void)hipGetLastError();
    *dst = nullptr;
    return fail(PSATD_ENOMEM, "batch descriptor allocation failed");
  }
  *dst_bytes = v.size() * sizeof(P);
  if (hipMemcpy(*dst, v.data(), v.size() * sizeof(P), hipMemcpyHostToDevice) != hipSuccess)
    return check_hip("batch descriptor upload");
  return PSATD_OK;
}

// LDS a class of batched blocks is sized for: the next of a few fixed sizes.
size_t lds_bucket(size_t bytes) {
  static const size_t kb[] = {16, 24, 32, 40, 48, 64, 80, 96, 128, 160};
  for (size_t v : kb)
    if (bytes <= v * 1024) return v * 1024;
  return bytes;
}

template <typename P>
void order_pass(const std::vector<P>& in, const std::vector<int>& nt, const std::vector<int>& thr,
                const std::vector<size_t>& lds, std::vector<P>& out, std::vector<int>& starts,
                std::vector<psatd_batch::Class>& cls) {
  const int n = (int)in.size();
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int c) {
    return thr[a] != thr[c] ? thr[a] < thr[c] : lds_bucket(lds[a]) < lds_bucket(lds[c]);
  });
  out.clear();
  cls.clear();
  for (int j = 0; j < n; ++j) {
    const int i = idx[j];
    if (cls.empty() || cls.back().threads != thr[i] || lds_bucket(cls.back().lds) != lds_bucket(lds[i])) {
      psatd_batch::Class c;
      c.first = j;
      c.soff = (int)starts.size();
      c.threads = thr[i];
      starts.push_back(0);
      cls.push_back(c);
    }
    psatd_batch::Class& c = cls.back();
    c.nbox += 1;
    c.total += nt[i];
    c.lds = std::max(c.lds, lds[i]);
    starts.push_back(starts.back() + nt[i]);
    out.push_back(in[i]);
  }
}

template <typename T>
int bind_batch(psatd_batch* b, void* const* g1) {
  const int n = b->nsub;
  std::vector<XFwdParams<T>> x1(n), x1o;
  std::vector<YPassParams<T>> y2(n), y4(n), y2o, y4o;
  std::vector<ZPushParams<T>> z3(n), z3o;
  std::vector<XInvParams<T>> x5(n), x5o;
  std::vector<int> nt[5], thr[5];
  std::vector<size_t> ls[5];
  for (int k = 0; k < 5; ++k) {
    nt[k].resize(n);
    thr[k].resize(n);
    ls[k].resize(n);
  }
  for (int i = 0; i < n; ++i) {
    psatd_plan* p = b->plans[i];
    const StepIO io = g1_io(p, g1, b->origins[i].data(), b->gd);
    StepParams<T> sp;
    build_step<T>(p, io, sp, true);
    x1[i] = sp.x1;
    y2[i] = sp.y2;
    z3[i] = sp.z3;
    y4[i] = sp.y4;
    x5[i] = sp.x5;
    const int tiles[5] = {sp.x1.ntiles, sp.y2.ntiles, sp.z3.ntiles, sp.y4.ntiles, sp.x5.ntiles};
    const int threads[5] = {kLineThreads, kLineThreads, p->zthreads, kLineThreads, p->x5threads};
    const size_t bytes[5] = {xfwd_lds(sp.x1), ypass_lds(sp.y2), zpush_lds(sp.z3), ypass_lds(sp.y4), xinv_lds(sp.x5)};
    for (int k = 0; k < 5; ++k) {
      nt[k][i] = tiles[k];
      thr[k][i] = threads[k];
      ls[k][i] = bytes[k];
    }
  }
  std::vector<int> starts;
  order_pass(x1, nt[0], thr[0], ls[0], x1o, starts, b->cls[0]);
  order_pass(y2, nt[1], thr[1], ls[1], y2o, starts, b->cls[1]);
  order_pass(z3, nt[2], thr[2], ls[2], z3o, starts, b->cls[2]);
  order_pass(y4, nt[3], thr[3], ls[3], y4o, starts, b->cls[3]);
  order_pass(x5, nt[4], thr[4], ls[4], x5o, starts, b->cls[4]);
  for (int k = 0; k < 5; ++k) {
    b->totals[k] = 0;
    for (const auto& c : b->cls[k]) b->totals[k] += c.total;
  }
  int rc;
  if ((rc = upload(x1o, &b->descs[0], &b->desc_bytes[0])) || (rc = upload(y2o, &b->descs[1], &b->desc_bytes[1])) ||
      (rc = upload(z3o, &b->descs[2], &b->desc_bytes[2])) || (rc = upload(y4o, &b->descs[3], &b->desc_bytes[3])) ||
      (rc = upload(x5o, &b->descs[4], &b->desc_bytes[4])))
    return rc;
  void* st = b->starts;
  rc = upload(starts, &st, &b->starts_bytes);
  b->starts = (int*)st;
  if (rc) return rc;
  for (int f = 0; f < 11; ++f) b->bound[f] = g1[f];
  b->is_bound = true;
  return PSATD_OK;
}

template <typename P>
BatchArgs<P> class_args(const psatd_batch* b, int k, const psatd_batch::Class& c) {
  return BatchArgs<P>{(const P*)b->descs[k] + c.first, b->starts + c.soff, c.nbox, c.total};
}

// One persistent launch per class of every pass; the passes run in order (Jacobi
// order between the fills and the merges of a step is kept by the pass order).
template <typename T>
void enqueue_batch_step(const psatd_batch* b, hipStream_t s) {
  for (const auto& c : b->cls[0]) launch_xfwd_batch<T>(class_args<XFwdParams<T>>(b, 0, c), c.lds, s);
  for (const auto& c : b->cls[1]) launch_ypass_batch<T>(class_args<YPassParams<T>>(b, 1, c), 0, c.lds, s);
  for (const auto& c : b->cls[2]) launch_zpush_batch<T>(class_args<ZPushParams<T>>(b, 2, c), c.threads, c.lds, s);
  for (const auto& c : b->cls[3]) launch_ypass_batch<T>(class_args<YPassParams<T>>(b, 3, c), 1, c.lds, s);
  for (const auto& c : b->cls[4]) launch_xinv_batch<T>(class_args<XInvParams<T>>(b, 4, c), c.threads, c.lds, s);
}

int ensure_bound(psatd_batch* b, void* const* g1) {
  if (!g1) return fail(PSATD_EINVAL, "NULL argument");
  for (int f = 0; f < 11; ++f)
    if (!g1[f]) return fail(PSATD_EINVAL, "field pointer %d is NULL", f);
  if (!distinct(g1, 11)) return fail(PSATD_EINVAL, "field arrays must be distinct");
  bool same = b->is_bound;
  for (int f = 0; f < 11 && same; ++f) same = (b->bound[f] == g1[f]);
  if (same) return PSATD_OK;
  if (b->exec) {
    (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  if (b->graph) {
    (void)hipGraphDestroy(b->graph);
    b->graph = nullptr;
  }
  b->graph_steps = 0;
  return b->fp64 ? bind_batch<double>(b, g1) : bind_batch<float>(b, g1);
}

}  // namespace

// ================================================================ C ABI
// Error reporting for the other translation units of the library.
int psatd::report_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

extern "C" {

const char* psatd_last_error(void) { return g_err.c_str(); }

int psatd_plan_create_ex(const psatd_plan_desc* desc, psatd_plan** out) {
  g_err.clear();
  if (!out) return fail(PSATD_EINVAL, "out is NULL");
  *out = nullptr;
  return build_plan(desc, out);
}

psatd_plan* psatd_plan_create(int nx, int ny, int nz, int nguard, int order, double dx, double dt) {
  psatd_plan_desc d{};
  d.nx = nx;
  d.ny = ny;
  d.nz = nz;
  d.ngx = d.ngy = d.ngz = nguard;
  d.order = order;
  d.dx = d.dy = d.dz = dx;
  d.dt = dt;
  d.c = 1.0;
  d.eps0 = 1.0;
  d.precision = PSATD_FP32;
  d.flags = 0;
  psatd_plan* p = nullptr;
  return psatd_plan_create_ex(&d, &p) == PSATD_OK ? p : nullptr;
}

void psatd_plan_destroy(psatd_plan* plan) { free_plan(plan); }

int psatd_pml_set(psatd_plan* p, const int width[3], double sigma_max, double power) {
  if (!p || !width) return fail(PSATD_EINVAL, "NULL argument");
  if (p->d.flags & PSATD_FLAG_STAGGERED) return fail(PSATD_EUNSUPPORTED, "psatd_pml_set: collocated plans only");
  if (!p->wsA) return fail(PSATD_ESTATE, "psatd_pml_set: the plan was created without a workspace");
  const int n[3] = {p->NX, p->NY, p->NZ};
  for (int a = 0; a < 3; ++a)
    if (width[a] < 0 || 2 * width[a] > n[a])
      return fail(PSATD_EINVAL, "psatd_pml_set: layer width %d on axis %d must be in [0, %d]", width[a], a,
                  n[a] / 2);
  if (!(sigma_max >= 0) || !(power >= 0) || !std::isfinite(sigma_max) || !std::isfinite(power))
    return fail(PSATD_EINVAL, "psatd_pml_set: sigma_max and power must be finite and >= 0");
  const size_t rs = p->rsize;
  if ((size_t)12 * lds_line(p->az.sch.n) * 2 * rs > lds_limit())
    return fail(PSATD_EUNSUPPORTED, "psatd_pml_set: twelve z lines of %d points do not fit the LDS", p->az.sch.n);
  if (!p->pml_ready) {
    if (int rc = dalloc(p, &p->pml_wsB, (size_t)12 * p->npts * 2 * rs)) return rc;
    for (int a = 0; a < 3; ++a)
      if (int rc = dalloc(p, &p->pml_damp[a], (size_t)n[a] * rs)) return rc;
    for (int f = 0; f < 6; ++f) {
      if (int rc = dalloc(p, &p->pml_full[f], (size_t)p->ncell * rs)) return rc;
      if (int rc = dalloc(p, &p->pml_inc[f], (size_t)p->ncell * rs)) return rc;
    }
  }
  for (int a = 0; a < 3; ++a) {
    // sigma rises as sigma_max (depth / width)^power over `width` cells at each end
    std::vector<double> dd(n[a], 1.0);
    const int w = width[a];
    for (int i = 0; i < n[a]; ++i) {
      double depth = 0;
      if (i < w) depth = (double)(w - i) / w;
      else if (i >= n[a] - w) depth = (double)(i - (n[a] - w) + 1) / w;
      dd[i] = depth > 0 ? std::exp(-sigma_max * std::pow(depth, power) * std::fabs(p->d.dt)) : 1.0;
    }
    hipError_t e;
    if (p->fp64) {
      e = hipMemcpy(p->pml_damp[a], dd.data(), (size_t)n[a] * 8, hipMemcpyHostToDevice);
    } else {
      std::vector<float> df(dd.begin(), dd.end());
      e = hipMemcpy(p->pml_damp[a], df.data(), (size_t)n[a] * 4, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) return check_hip("psatd_pml_set");
  }
  p->pml_ready = true;
  return PSATD_OK;
}

int psatd_pml_step(psatd_plan* p, void* const* parts, const void* const* src, void* stream) {
  if (!p || !parts || !src) return fail(PSATD_EINVAL, "NULL argument");
  if (!p->pml_ready) return fail(PSATD_ESTATE, "psatd_pml_step: call psatd_pml_set first");
  const void* all[17];
  for (int f = 0; f < 12; ++f) all[f] = parts[f];
  for (int f = 0; f < 5; ++f) all[12 + f] = src[f];
  for (int f = 0; f < 17; ++f)
    if (!all[f]) return fail(PSATD_EINVAL, "psatd_pml_step: array %d is NULL", f);
  if (!distinct(all, 17)) return fail(PSATD_EINVAL, "psatd_pml_step: arrays must be distinct");
  const hipStream_t s = (hipStream_t)stream;
  int rc = guard_of(p).check(s, "psatd_pml_step");
  if (rc) return rc;
  launch_pml_sum(parts, p->pml_full, p->ncell, p->fp64, s);
  StepIO io{};
  io.wsA = p->wsA;
  io.wsB = p->pml_wsB;
  for (int f = 0; f < 6; ++f) io.src[f] = p->pml_full[f];
  for (int f = 0; f < 5; ++f) io.src[6 + f] = src[f];
  for (int f = 0; f < 6; ++f) io.dst[f] = p->pml_inc[f];
  io.gather = 0;
  io.src_elems = p->ncell;
  io.scatter = 0;
  io.dst_elems = p->ncell;
  io.y_lo = 0;
  io.y_hi = p->NY;
  io.z_lo = 0;
  io.z_hi = p->NZ;
  io.pml = 1;
  rc = p->fp64 ? run_pml<double>(p, io, parts, s) : run_pml<float>(p, io, parts, s);
  if (rc) return rc;
  return guard_of(p).mark(s, "psatd_pml_step");
}

int psatd_default_schedule(int n, int* radices, int max_radices, int* transform_len) {
  if (n < 1 || n > (1 << 24) || !radices || !transform_len || max_radices < 1)
    return fail(PSATD_EINVAL, "psatd_default_schedule: n = %d, max_radices = %d", n, max_radices);
  Axis a;
  if (!make_axis(n, emax<float>::v, &a)) return fail(PSATD_EUNSUPPORTED, "no schedule for n = %d", n);
  if (a.sch.nstages > max_radices) return fail(PSATD_EINVAL, "%d stages do not fit max_radices", a.sch.nstages);
  for (int i = 0; i < a.sch.nstages; ++i) radices[i] = a.sch.radix[i];
  *transform_len = a.sch.n;
  return a.sch.nstages;
}

int psatd_plan_query(const psatd_plan* p, int what, long long* value) {
  if (!p || !value) return fail(PSATD_EINVAL, "NULL argument");
  switch (what) {
    case PSATD_Q_BOX_X: *value = p->NX; break;
    case PSATD_Q_BOX_Y: *value = p->NY; break;
    case PSATD_Q_BOX_Z: *value = p->NZ; break;
    case PSATD_Q_PRECISION: *value = p->d.precision; break;
    case PSATD_Q_WORKSPACE_BYTES: *value = (long long)p->bytes; break;
    case PSATD_Q_SPECTRUM_POINTS: *value = p->npts; break;
    case PSATD_Q_Z_COLUMNS: *value = p->zcols; break;
    case PSATD_Q_TWO_STAGE: {
      long long m = 0;
      for (int pass = 0; pass < 5; ++pass)
        if ((p->two_stage_mask >> pass) & 1) {
          const bool ok = p->fp64 ? has_two_stage<double>(const_cast<psatd_plan*>(p), pass)
                                  : has_two_stage<float>(const_cast<psatd_plan*>(p), pass);
          if (ok) m |= 1LL << pass;
        }
      *value = m;
      break;
    }
    default: return fail(PSATD_EINVAL, "unknown query %d", what);
  }
  return PSATD_OK;
}

int psatd_plan_tables(const psatd_plan* p, void* dst, void* stream) {
  if (!p || !dst) return fail(PSATD_EINVAL, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  const size_t nc = 5 * (size_t)p->npts * p->rsize;
  const size_t nk = (size_t)(p->NXH + p->NY + p->NZ) * p->rsize;
  if (hipMemcpyAsync(dst, p->coef, nc, hipMemcpyDeviceToDevice, s) != hipSuccess ||
      hipMemcpyAsync((char*)dst + nc, p->kw, nk, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return check_hip("psatd_plan_tables");
  return PSATD_OK;
}

int psatd_set_device_budget(long long bytes) {
  g_budget.store(bytes < 0 ? -1 : bytes);
  return PSATD_OK;
}

long long psatd_device_bytes_in_use(void) { return g_live_bytes.load(); }

int psatd_tune_cache_load(const char* path, int* accepted, int* rejected) {
  if (!path) return fail(PSATD_EINVAL, "NULL path");
  load_tune_file(path, accepted, rejected);
  return PSATD_OK;
}

int psatd_plan_autotune(psatd_plan* p, const char* cache_path, void* stream) {
  if (!p) return fail(PSATD_EINVAL, "NULL plan");
  if (!p->wsA) return fail(PSATD_ESTATE, "psatd_plan_autotune: the plan was created without a workspace");
  const int grc = guard_of(p).check((hipStream_t)stream, "psatd_plan_autotune");
  if (grc) return grc;
  load_tune_file(cache_path);
  const int rc = p->fp64 ? autotune_plan<double>(p, (hipStream_t)stream) : autotune_plan<float>(p, (hipStream_t)stream);
  if (rc == PSATD_OK) save_tune_file(cache_path);
  return rc;
}

int psatd_plan_schedule(const psatd_plan* p, int axis, int* radices, int max_radices, int* tile) {
  if (!p || !radices || !tile || axis < 0 || axis > 2) return fail(PSATD_EINVAL, "bad argument");
  const Axis& A = axis == 0 ? p->ax : (axis == 1 ? p->ay : p->az);
  if (A.sch.nstages > max_radices) return fail(PSATD_EINVAL, "radix buffer too small");
  for (int i = 0; i < A.sch.nstages; ++i) radices[i] = A.sch.radix[i];
  *tile = axis == 0 ? p->ty1 : (axis == 1 ? p->nl_y : p->zthreads);
  return A.sch.nstages;
}

int psatd_plan_set_timing(psatd_plan* p, int enable) {
  if (!p) return fail(PSATD_EINVAL, "NULL plan");
  p->timing = enable ? 1 : 0;
  return PSATD_OK;
}

int psatd_plan_pass_times(psatd_plan* p, double ms[5], long long* nsteps) {
  if (!p || !ms || !nsteps) return fail(PSATD_EINVAL, "NULL argument");
  for (int i = 0; i < 5; ++i) ms[i] = 0.0;
  *nsteps = (long long)p->events.size();
  if (p->events.empty()) return PSATD_OK;
  if (hipEventSynchronize(p->events.back()[5]) != hipSuccess) {
    release_events(p);
    return check_hip("hipEventSynchronize");
  }
  for (auto& set : p->events)
    for (int i = 0; i < 5; ++i) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, set[i], set[i + 1]) == hipSuccess) ms[i] += t;
    }
  for (int i = 0; i < 5; ++i) ms[i] /= (double)p->events.size();
  release_events(p);
  return check_hip("psatd_plan_pass_times");
}

int psatd_push(psatd_plan* p, void* const E[3], void* const B[3], const void* const J[3], const void* rho_old,
               const void* rho_new, void* stream) {
  if (!p || !E || !B || !J) return fail(PSATD_EINVAL, "NULL argument");
  if (!p->wsA) return fail(PSATD_ESTATE, "psatd_push: the plan was created without a workspace");
  StepIO io{};
  io.wsA = p->wsA;
  io.wsB = p->wsB;
  const void* all[11] = {E[0], E[1], E[2], B[0], B[1], B[2], J[0], J[1], J[2], rho_old, rho_new};
  for (int f = 0; f < 11; ++f) {
    if (!all[f]) return fail(PSATD_EINVAL, "field pointer %d is NULL", f);
    io.src[f] = all[f];
  }
  if (!distinct(all, 11)) return fail(PSATD_EINVAL, "field arrays must be distinct");
  for (int f = 0; f < 3; ++f) {
    io.dst[f] = E[f];
    io.dst[3 + f] = B[f];
  }
  io.gather = 0;
  io.src_elems = p->ncell;
  io.scatter = 0;
  io.dst_elems = p->ncell;
  io.y_lo = 0;
  io.y_hi = p->NY;
  io.z_lo = 0;
  io.z_hi = p->NZ;
  return dispatch_step(p, io, (hipStream_t)stream);
}

int psatd_step_g1(psatd_plan* p, void* const* g1, const int origin[3], const int gdims[3], void* stream) {
  int rc = check_g1_call(p, g1, origin, gdims);
  if (rc) return rc;
  if (!p->wsA) return fail(PSATD_ESTATE, "psatd_step_g1: the plan was created without a workspace");
  return dispatch_step(p, g1_io(p, g1, origin, gdims), (hipStream_t)stream);
}

int psatd_step_g1_noalloc(psatd_plan* p, void* const* g1, const int origin[3], const int gdims[3], void* stream) {
  int rc = check_g1_call(p, g1, origin, gdims);
  if (rc) return rc;
  const size_t need = scratch_need(p);
  if (need > kScratchBytes)
    return fail(PSATD_EINVAL,
                "psatd_step_g1_noalloc: the box needs %zu bytes of workspace, above the %zu-byte static scratch "
                "(box %dx%dx%d)", need, kScratchBytes, p->NX, p->NY, p->NZ);
  ScratchSlot* slot = nullptr;
  if ((rc = scratch_slot(&slot))) return rc;
  hipStream_t s = (hipStream_t)stream;
  const StreamGuard g{&slot->done, &slot->last_stream, &slot->known};
  if ((rc = g.check(s, "psatd_step_g1_noalloc"))) return rc;
  StepIO io = g1_io(p, g1, origin, gdims);
  io.wsA = slot->base;
  io.wsB = (char*)slot->base + scratch_half(p);
  rc = p->fp64 ? run_step<double>(p, io, s, false) : run_step<float>(p, io, s, false);
  if (rc) return rc;
  return g.mark(s, "psatd_step_g1_noalloc");
}

int guard_fill(psatd_plan* p, const void* const* g1, void* const* box, int nfields, const int origin[3],
               const int gdims[3], void* stream) {
  if (!p || !g1 || !box) return fail(PSATD_EINVAL, "NULL argument");
  if (nfields < 1 || nfields > 16) return fail(PSATD_EINVAL, "nfields must be in [1, 16]");
  int rc = check_geometry(p, origin, gdims);
  if (rc) return rc;
  for (int f = 0; f < nfields; ++f)
    if (!g1[f] || !box[f]) return fail(PSATD_EINVAL, "field pointer %d is NULL", f);
  const int bd[3] = {p->NX, p->NY, p->NZ};
  const int g[3] = {p->d.ngx, p->d.ngy, p->d.ngz};
  int st[3];
  for (int a = 0; a < 3; ++a) st[a] = (int)((((long long)origin[a] - g[a]) % gdims[a] + gdims[a]) % gdims[a]);
  launch_guard_fill(g1, box, nfields, (int)p->rsize, bd, st, gdims, (hipStream_t)stream);
  return check_hip("guard_fill");
}

int guard_merge(psatd_plan* p, const void* const* box, void* const* g1, int nfields, const int origin[3],
                const int gdims[3], int mode, void* stream) {
  if (!p || !g1 || !box) return fail(PSATD_EINVAL, "NULL argument");
  if (nfields < 1 || nfields > 16) return fail(PSATD_EINVAL, "nfields must be in [1, 16]");
  if (mode != 0 && mode != 1) return fail(PSATD_EINVAL, "mode must be 0 (copy) or 1 (add)");
  int rc = check_geometry(p, origin, gdims);
  if (rc) return rc;
  for (int f = 0; f < nfields; ++f)
    if (!g1[f] || !box[f]) return fail(PSATD_EINVAL, "field pointer %d is NULL", f);
  const int bd[3] = {p->NX, p->NY, p->NZ};
  const int g[3] = {p->d.ngx, p->d.ngy, p->d.ngz};
  const int n[3] = {p->d.nx, p->d.ny, p->d.nz};
  launch_guard_merge(box, g1, nfields, (int)p->rsize, bd, g, n, origin, gdims, mode, (hipStream_t)stream);
  return check_hip("guard_merge");
}

int psatd_batch_create(int nsub, const psatd_plan_desc* subs, const int* origins, const int gdims[3],
                       psatd_batch** out) {
  g_err.clear();
  if (!out) return fail(PSATD_EINVAL, "out is NULL");
  *out = nullptr;
  if (nsub < 1 || !subs || !origins || !gdims) return fail(PSATD_EINVAL, "bad batch arguments");
  if ((double)gdims[0] * gdims[1] * gdims[2] * (subs[0].precision == PSATD_FP64 ? 8 : 4) >= 4294967296.0)
    return fail(PSATD_EUNSUPPORTED, "global arrays of 4 GiB or more are not supported");
  for (int i = 1; i < nsub; ++i) {
    const psatd_plan_desc &a = subs[0], &c = subs[i];
    if (a.precision != c.precision || a.dx != c.dx || a.dy != c.dy || a.dz != c.dz || a.dt != c.dt || a.c != c.c ||
        a.eps0 != c.eps0)
      return fail(PSATD_EINVAL, "box %d: precision, cell size, dt, c and eps0 must agree across the batch", i);
  }
  for (int i = 0; i < nsub; ++i)
    if (subs[i].flags & PSATD_FLAG_NO_WORKSPACE)
      return fail(PSATD_EINVAL, "box %d: batch boxes keep their own workspace (PSATD_FLAG_NO_WORKSPACE not allowed)", i);
  // Every box writes its interior back to G1 in the last pass of a step, while other
  // boxes of the same launch still run: two interiors sharing a G1 cell would race.
  for (int i = 0; i < nsub; ++i) {
    const int ni[3] = {subs[i].nx, subs[i].ny, subs[i].nz};
    for (int a = 0; a < 3; ++a)
      if (gdims[a] <= 0 || origins[3 * i + a] < 0 || origins[3 * i + a] >= gdims[a] || ni[a] <= 0 || ni[a] > gdims[a])
        return fail(PSATD_EINVAL, "box %d: interior must be non-empty, no larger than the grid, origin in [0, gdims)",
                    i);
  }
  for (int i = 0; i < nsub; ++i)
    for (int j = i + 1; j < nsub; ++j) {
      const int ni[3] = {subs[i].nx, subs[i].ny, subs[i].nz}, nj[3] = {subs[j].nx, subs[j].ny, subs[j].nz};
      bool all = true;
      for (int a = 0; a < 3 && all; ++a) {
        // periodic intervals [oi, oi + ni) and [oj, oj + nj) modulo G intersect
        const int G = gdims[a];
        const int dij = ((origins[3 * j + a] - origins[3 * i + a]) % G + G) % G;
        const int dji = ((origins[3 * i + a] - origins[3 * j + a]) % G + G) % G;
        all = dij < ni[a] || dji < nj[a];
      }
      if (all) return fail(PSATD_EINVAL, "boxes %d and %d: interiors overlap on the global grid", i, j);
    }
  psatd_batch* b = new psatd_batch;
  b->nsub = nsub;
  b->fp64 = subs[0].precision == PSATD_FP64;
  for (int a = 0; a < 3; ++a) b->gd[a] = gdims[a];
  for (int i = 0; i < nsub; ++i) {
    psatd_plan* p = nullptr;
    int rc = build_plan(&subs[i], &p);
    if (rc == PSATD_OK) rc = check_geometry(p, origins + 3 * i, gdims);
    if (rc != PSATD_OK) {
      std::string msg = g_err;
      if (p) free_plan(p);
      free_batch(b);
      return fail(rc, "box %d: %s", i, msg.c_str());
    }
    b->plans.push_back(p);
    b->origins.push_back({origins[3 * i], origins[3 * i + 1], origins[3 * i + 2]});
    b->box_cells += p->ncell;
    b->interior_cells += (long long)p->d.nx * p->d.ny * p->d.nz;
  }
  *out = b;
  return PSATD_OK;
}

int psatd_batch_step(psatd_batch* b, void* const* g1, void* stream) {
  if (!b) return fail(PSATD_EINVAL, "NULL batch");
  hipStream_t s = (hipStream_t)stream;
  const StreamGuard g{&b->done, &b->last_stream, &b->in_flight_known};
  int rc = g.check(s, "psatd_batch_step");
  if (rc) return rc;
  rc = ensure_bound(b, g1);
  if (rc) return rc;
  if (b->fp64)
    enqueue_batch_step<double>(b, s);
  else
    enqueue_batch_step<float>(b, s);
  rc = check_hip("psatd_batch_step");
  if (rc) return rc;
  return g.mark(s, "psatd_batch_step");
}

int psatd_batch_run(psatd_batch* b, void* const* g1, int nsteps, void* stream) {
  if (!b) return fail(PSATD_EINVAL, "NULL batch");
  if (nsteps < 1) return fail(PSATD_EINVAL, "nsteps must be >= 1");
  hipStream_t s = (hipStream_t)stream;
  const StreamGuard g{&b->done, &b->last_stream, &b->in_flight_known};
  int rc = g.check(s, "psatd_batch_run");
  if (rc) return rc;
  rc = ensure_bound(b, g1);
  if (rc) return rc;
  if (!b->exec || b->graph_steps != nsteps) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    if (!b->cap && hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
      b->cap = nullptr;
      return check_hip("capture stream");
    }
    if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return check_hip("begin capture");
    for (int i = 0; i < nsteps; ++i) {
      if (b->fp64)
        enqueue_batch_step<double>(b, b->cap);
      else
        enqueue_batch_step<float>(b, b->cap);
    }
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(b->cap, &g) != hipSuccess || !g) return check_hip("end capture");
    b->graph = g;
    if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
      b->exec = nullptr;
      return check_hip("graph instantiate");
    }
    b->graph_steps = nsteps;
  }
  if (hipGraphLaunch(b->exec, s) != hipSuccess) return check_hip("graph launch");
  return g.mark(s, "psatd_batch_run");
}

void psatd_batch_destroy(psatd_batch* b) { free_batch(b); }

int psatd_batch_autotune(psatd_batch* b, const char* cache_path, void* stream) {
  if (!b) return fail(PSATD_EINVAL, "NULL batch");
  load_tune_file(cache_path);
  for (psatd_plan* p : b->plans) {
    const int rc =
        p->fp64 ? autotune_plan<double>(p, (hipStream_t)stream) : autotune_plan<float>(p, (hipStream_t)stream);
    if (rc) return rc;
  }
  save_tune_file(cache_path);
  // descriptors and graphs hold the old schedules: rebuild them on the next step
  b->is_bound = false;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->graph_steps = 0;
  return PSATD_OK;
}

int psatd_batch_query(const psatd_batch* b, int what, long long* value) {
  if (!b || !value) return fail(PSATD_EINVAL, "NULL argument");
  switch (what) {
    case PSATD_QB_BOXES: *value = b->nsub; break;
    case PSATD_QB_TILES: {
      long long t = 0;
      for (int k = 0; k < 5; ++k) t += b->totals[k];
      *value = t;
      break;
    }
    case PSATD_QB_BOX_CELLS: *value = b->box_cells; break;
    case PSATD_QB_INTERIOR_CELLS: *value = b->interior_cells; break;
    case PSATD_QB_WORKSPACE_BYTES: {
      long long t = 0;
      for (const psatd_plan* p : b->plans) t += (long long)p->bytes;
      *value = t;
      break;
    }
    default: return fail(PSATD_EINVAL, "unknown query %d", what);
  }
  return PSATD_OK;
}

}  // extern "C"
