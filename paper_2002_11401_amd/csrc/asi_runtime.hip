// Host runtime behind the C ABI of include/asi.h: argument validation, the
// cell sort that seeds the device neighbour build, device-memory bridge,
// per-step launch sequence, batching with captured graphs, and the serving
// loop.  Every step of the model itself runs in the kernels of
// asi_kernels.hip.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <string>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/asi.h"
#include "asi_internal.h"

#include <rocprofiler-sdk-roctx/roctx.h>

using namespace asi;

namespace {

thread_local std::string g_err;

asi_status fail(asi_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// Device memory of one owner (handle or server), through the caller's
// allocator callbacks or hipMalloc.
struct DevMem {
  asi_device dev{};
  hipStream_t st = nullptr;
  std::vector<std::pair<void*, size_t>> blocks;
  size_t total = 0;
  bool fail_next = false;  // allocation fault injection (ASI_FAIL_ALLOC)

  void* alloc(size_t bytes) {
    if (bytes == 0) bytes = 16;
    bytes = (bytes + 255) & ~(size_t)255;
    void* p = nullptr;
    if (fail_next) return nullptr;
    if (dev.alloc) {
      p = dev.alloc(bytes, (void*)st, dev.ctx);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
    }
    if (p) {
      blocks.emplace_back(p, bytes);
      total += bytes;
    }
    return p;
  }
  void release(void* p) {
    if (!p) return;
    for (size_t k = 0; k < blocks.size(); ++k)
      if (blocks[k].first == p) {
        total -= blocks[k].second;
        if (dev.free)
          dev.free(p, (void*)st, dev.ctx);
        else
          (void)hipFree(p);
        blocks.erase(blocks.begin() + k);
        return;
      }
  }
  void release_all() {
    for (auto& b : blocks) {
      if (dev.free)
        dev.free(b.first, (void*)st, dev.ctx);
      else
        (void)hipFree(b.first);
    }
    blocks.clear();
    total = 0;
  }
};

struct TimerPair {
  hipEvent_t a, b;
  int kind;  // 0 field, 1 relax
};

}  // namespace

struct asi_sim {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;              // current device at create: the handle's GPU
  DevMem mem;
  int64_t n = 0, E = 0;
  int32_t D = 0, l1s = 6, relax_waves = 1;
  int32_t field_rows = 0;       // rows per workgroup of the high-degree pass (0: by size)
  size_t lds = 0;
  InstDev hI{};
  InstDev* dI = nullptr;
  RunDev* dR = nullptr;
  int32_t* blk_inst = nullptr;
  int32_t* blk_row0 = nullptr;
  int64_t nblocks = 0;
  double* dH = nullptr;
  double* dHloc = nullptr;
  double* dSig = nullptr;
  double* dWave = nullptr;
  double alpha = 0.0;
  double* dMpart = nullptr;   // [kMagPartials + 2] block sums, then the last result
  double* dMlog = nullptr;    // [K][2] magnetisation after each step's relax
  bool mag_log = false;
  int64_t K = 0;
  int64_t cur_step = -1;
  bool poisoned = false;
  bool timing = false;
  std::vector<TimerPair> timers;
  std::vector<hipEvent_t> spare_events;
  asi_timing tm{};
};

namespace {

#define HIPCHK(expr, sim)                                                              \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) {                                                            \
      if (sim) (sim)->poisoned = true;                                                 \
      return fail(ASI_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));     \
    }                                                                                  \
  } while (0)

// A named range on the profiler's timeline (roctx) for the duration of a
// library call: create, run/relax, tune, batch and server bursts.
struct Range {
  explicit Range(const char* name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

hipEvent_t take_event(asi_sim* s) {
  if (!s->spare_events.empty()) {
    hipEvent_t e = s->spare_events.back();
    s->spare_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Launch one field pass of the handle's (single) instance.
void field_pass(asi_sim* s) {
  TimerPair tp{};
  if (s->timing) {
    tp.a = take_event(s);
    tp.b = take_event(s);
    tp.kind = 0;
    (void)hipEventRecord(tp.a, s->stream);
  }
  if (s->hI.field_mode == kFieldFull && s->D >= kHdMinD)
    launch_field_hd(s->dI, s->dR, s->n, s->field_rows, s->hI.nch, s->stream);
  else
    launch_field(s->dI, s->dR, s->blk_inst, s->blk_row0, s->nblocks, s->stream);
  if (s->timing) {
    (void)hipEventRecord(tp.b, s->stream);
    s->timers.push_back(tp);
  }
}

void relax_pass(asi_sim* s) {
  TimerPair tp{};
  if (s->timing) {
    tp.a = take_event(s);
    tp.b = take_event(s);
    tp.kind = 1;
    (void)hipEventRecord(tp.a, s->stream);
  }
  launch_relax(s->dI, s->dR, 1, s->relax_waves, s->lds, !relax_may_speculate(s->D, s->relax_waves),
               s->stream);
  if (s->timing) {
    (void)hipEventRecord(tp.b, s->stream);
    s->timers.push_back(tp);
  }
}

void harvest_timers(asi_sim* s) {
  for (auto& tp : s->timers) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, tp.a, tp.b) == hipSuccess) {
      if (tp.kind == 0) {
        s->tm.field_launches++;
        s->tm.field_ms += ms;
      } else {
        s->tm.relax_launches++;
        s->tm.relax_ms += ms;
      }
    }
    s->spare_events.push_back(tp.a);
    s->spare_events.push_back(tp.b);
  }
  s->timers.clear();
}

asi_status check_handle(asi_sim* s) {
  if (!s) return fail(ASI_EINVAL, "null handle");
  if (s->poisoned) return fail(ASI_ESTATE, "handle poisoned by an earlier device error");
  return ASI_OK;
}

asi_status sync_and_check(asi_sim* s) {
  hipError_t e = hipStreamSynchronize(s->stream);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) {
    s->poisoned = true;
    return fail(ASI_EDEVICE, std::string("device error: ") + hipGetErrorString(e));
  }
  if (s->timing) harvest_timers(s);
  return ASI_OK;
}

asi_status validate(const asi_params* p) {
  if (!p) return fail(ASI_EINVAL, "params is NULL");
  if (p->struct_size != sizeof(asi_params))
    return fail(ASI_EINVAL, "asi_params.struct_size mismatch");
  if (p->n < 1 || p->n >= (int64_t)0x7fffffff) return fail(ASI_EINVAL, "n out of range");
  if (!p->xy || !p->theta) return fail(ASI_EINVAL, "xy and theta are required");
  if (!p->hk && (!(p->hk_mean > 0.0) || !std::isfinite(p->hk_mean) || !(p->k_disorder >= 0.0) ||
                 !std::isfinite(p->k_disorder)))
    return fail(ASI_EINVAL, "hk is NULL: hk_mean must be finite and > 0, k_disorder finite and >= 0");
  if (!(std::isfinite(p->alpha))) return fail(ASI_EINVAL, "alpha must be finite");
  if (!(p->neighbor_distance >= 0.0) || !std::isfinite(p->neighbor_distance))
    return fail(ASI_EINVAL, "neighbor_distance must be finite and >= 0");
  if (!(p->b > 0) || !(p->c > 0) || !(p->beta > 0) || !(p->gamma > 0) || !std::isfinite(p->b) ||
      std::isnan(p->c) || !std::isfinite(p->beta) || !std::isfinite(p->gamma))
    return fail(ASI_EINVAL, "astroid parameters b, beta, gamma must be finite and > 0, c > 0");
  if (!(p->thermal_std >= 0.0) || !std::isfinite(p->thermal_std))
    return fail(ASI_EINVAL, "thermal_std must be finite and >= 0");
  if (p->max_flips_per_step < 0 || p->flip_log_capacity < 0)
    return fail(ASI_EINVAL, "negative cap");
  if (p->field_mode < 0 || p->field_mode > 2)
    return fail(ASI_EINVAL, "field_mode must be 0, 1 or 2");
  for (int64_t i = 0; i < p->n; ++i) {
    if (!std::isfinite(p->xy[2 * i]) || !std::isfinite(p->xy[2 * i + 1]) ||
        !std::isfinite(p->theta[i]))
      return fail(ASI_EINVAL, "non-finite position or angle at magnet " + std::to_string(i));
    if (p->hk && (!(p->hk[i] > 0.0) || !std::isfinite(p->hk[i])))
      return fail(ASI_EINVAL, "hk must be finite and > 0 (magnet " + std::to_string(i) + ")");
    if (p->spin0 && p->spin0[i] != 1 && p->spin0[i] != -1)
      return fail(ASI_EINVAL, "spin0 values must be +1 or -1");
  }
  return ASI_OK;
}

template <class T>
T* dalloc(asi_sim* s, size_t count) {
  return static_cast<T*>(s->mem.alloc(sizeof(T) * count));
}

// Bytes a handle will hold on the device (used for admission control).
size_t footprint_estimate(int64_t n, int64_t D, int64_t K, int64_t log_cap) {
  const int64_t nsl = (n + kSlice - 1) / kSlice;
  size_t slots = (size_t)nsl * kSlice * (size_t)D;
  size_t b = slots * (4 + 8 + 8) + (size_t)n * (size_t)std::max<int64_t>(D, 1) * (4 + 8 + 8);
  b += (size_t)n * (4 + 8 + 8 + 8 + 1 + 1 + 8 * 7 + 4) + (size_t)(n + 8192) * 32;
  b += (size_t)nsl * 12 + (size_t)log_cap * 8 + (size_t)K * 20;
  if (D >= kHdMinD && nsl < kHdSplitSlices) b += (size_t)n * (size_t)((D + 63) / 64) * 16;
  b += 1 << 16;
  return b;
}

asi_status create_impl(const asi_params* p, const asi_device* dev, asi_sim* s) {
  asi_status st = validate(p);
  if (st != ASI_OK) return st;
  if (const char* f = std::getenv("ASI_FAIL_ALLOC")) s->mem.fail_next = (f[0] == '1');
  {
    static hipError_t cfg = configure_kernels();
    if (cfg != hipSuccess)
      return fail(ASI_EDEVICE, std::string("kernel configuration: ") + hipGetErrorString(cfg));
  }
  if (dev) s->mem.dev = *dev;
  HIPCHK(hipGetDevice(&s->device), s);
  if (dev && dev->stream) {
    s->stream = (hipStream_t)dev->stream;
  } else {
    HIPCHK(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking), s);
    s->own_stream = true;
  }
  s->mem.st = s->stream;
  const int64_t n = p->n;
  s->n = n;
  s->alpha = p->alpha;

  // host: unit vectors (libm), cell grid and the cell sort
  std::vector<double> x(n), y(n), mx(n), my(n);
  double xmin = p->xy[0], xmax = p->xy[0], ymin = p->xy[1], ymax = p->xy[1];
  for (int64_t i = 0; i < n; ++i) {
    x[i] = p->xy[2 * i];
    y[i] = p->xy[2 * i + 1];
    mx[i] = std::cos(p->theta[i]);
    my[i] = std::sin(p->theta[i]);
    xmin = std::min(xmin, x[i]);
    xmax = std::max(xmax, x[i]);
    ymin = std::min(ymin, y[i]);
    ymax = std::max(ymax, y[i]);
  }
  const double cut = p->neighbor_distance + 1e-9;
  const double cut2 = cut * cut;
  double cs = std::max(cut * (1.0 + 1e-6), 1e-6);
  const double cells_cap = 4.0 * (double)n + 1024.0;
  while (((xmax - xmin) / cs + 1.0) * ((ymax - ymin) / cs + 1.0) > cells_cap) cs *= 2.0;
  const int64_t gx = (int64_t)std::floor((xmax - xmin) / cs) + 1;
  const int64_t gy = (int64_t)std::floor((ymax - ymin) / cs) + 1;
  std::vector<int32_t> cx(n), cy(n), cstart(gx * gy + 1, 0), cmem(n);
  for (int64_t i = 0; i < n; ++i) {
    int64_t a = (int64_t)std::floor((x[i] - xmin) / cs);
    int64_t b = (int64_t)std::floor((y[i] - ymin) / cs);
    cx[i] = (int32_t)std::min(std::max(a, (int64_t)0), gx - 1);
    cy[i] = (int32_t)std::min(std::max(b, (int64_t)0), gy - 1);
    cstart[(int64_t)cy[i] * gx + cx[i] + 1]++;
  }
  for (int64_t c = 0; c < gx * gy; ++c) cstart[c + 1] += cstart[c];
  {
    std::vector<int32_t> fill(cstart.begin(), cstart.end() - 1);
    for (int64_t i = 0; i < n; ++i) cmem[fill[(int64_t)cy[i] * gx + cx[i]]++] = (int32_t)i;
  }

  // device: inputs
  double* dx = dalloc<double>(s, n);
  double* dy = dalloc<double>(s, n);
  double* dmx = dalloc<double>(s, n);
  double* dmy = dalloc<double>(s, n);
  double* dhk = dalloc<double>(s, n);
  int8_t* ds = dalloc<int8_t>(s, n);
  int32_t* dcx = dalloc<int32_t>(s, n);
  int32_t* dcy = dalloc<int32_t>(s, n);
  int32_t* dcs = dalloc<int32_t>(s, gx * gy + 1);
  int32_t* dcm = dalloc<int32_t>(s, n);
  int32_t* dlen = dalloc<int32_t>(s, n);
  int32_t* ddup = dalloc<int32_t>(s, 1);
  if (!dx || !dy || !dmx || !dmy || !dhk || !ds || !dcx || !dcy || !dcs || !dcm || !dlen || !ddup)
    return fail(ASI_ENOMEM, "device allocation failed (inputs)");
  std::vector<int8_t> s0(n, 1);
  if (p->spin0) std::memcpy(s0.data(), p->spin0, n);
  HIPCHK(hipMemcpyAsync(dx, x.data(), 8 * n, hipMemcpyHostToDevice, s->stream), s);
  HIPCHK(hipMemcpyAsync(dy, y.data(), 8 * n, hipMemcpyHostToDevice, s->stream), s);
  HIPCHK(hipMemcpyAsync(dmx, mx.data(), 8 * n, hipMemcpyHostToDevice, s->stream), s);
  HIPCHK(hipMemcpyAsync(dmy, my.data(), 8 * n, hipMemcpyHostToDevice, s->stream), s);
  if (p->hk) {
    HIPCHK(hipMemcpyAsync(dhk, p->hk, 8 * n, hipMemcpyHostToDevice, s->stream), s);
  } else {
    launch_draw_hk(dhk, n, p->hk_mean, p->k_disorder, p->disorder_seed, s->stream);
    HIPCHK(hipGetLastError(), s);
  }
  HIPCHK(hipMemcpyAsync(ds, s0.data(), n, hipMemcpyHostToDevice, s->stream), s);
  HIPCHK(hipMemcpyAsync(dcx, cx.data(), 4 * n, hipMemcpyHostToDevice, s->stream), s);
  HIPCHK(hipMemcpyAsync(dcy, cy.data(), 4 * n, hipMemcpyHostToDevice, s->stream), s);
  HIPCHK(hipMemcpyAsync(dcs, cstart.data(), 4 * (gx * gy + 1), hipMemcpyHostToDevice, s->stream),
         s);
  HIPCHK(hipMemcpyAsync(dcm, cmem.data(), 4 * n, hipMemcpyHostToDevice, s->stream), s);
  HIPCHK(hipMemsetAsync(ddup, 0, 4, s->stream), s);

  // device: neighbour counts -> padded row length
  launch_neighbour_count(dx, dy, dcx, dcy, dcs, dcm, n, gx, gy, cut2, dlen, ddup, s->stream);
  std::vector<int32_t> len(n);
  int32_t dup = 0;
  HIPCHK(hipMemcpyAsync(len.data(), dlen, 4 * n, hipMemcpyDeviceToHost, s->stream), s);
  HIPCHK(hipMemcpyAsync(&dup, ddup, 4, hipMemcpyDeviceToHost, s->stream), s);
  HIPCHK(hipStreamSynchronize(s->stream), s);
  if (dup) return fail(ASI_EINVAL, "coincident magnets (zero separation)");
  int64_t E = 0;
  int32_t D = 0;
  for (int64_t i = 0; i < n; ++i) {
    E += len[i];
    D = std::max(D, len[i]);
  }
  s->E = E;
  s->D = D;
  const int64_t nsl = (n + kSlice - 1) / kSlice;
  const size_t slots = (size_t)nsl * kSlice * (size_t)std::max(D, 1);
  int32_t* dcol = dalloc<int32_t>(s, slots);
  double* dA = dalloc<double>(s, slots);
  double* dB = dalloc<double>(s, slots);
  // row-major copy for the relax (every slot written by the fill)
  const size_t rslots = (size_t)n * (size_t)std::max(D, 1);
  int32_t* drcol = dalloc<int32_t>(s, rslots);
  double* drA = dalloc<double>(s, rslots);
  double* drBr = dalloc<double>(s, rslots);
  if (!dcol || !dA || !dB || !drcol || !drA || !drBr)
    return fail(ASI_ENOMEM, "device allocation failed (neighbour tables)");
  // rows of a partial last slice stay padded
  HIPCHK(hipMemsetAsync(dcol, 0xff, 4 * slots, s->stream), s);
  HIPCHK(hipMemsetAsync(dA, 0, 8 * slots, s->stream), s);
  HIPCHK(hipMemsetAsync(dB, 0, 8 * slots, s->stream), s);
  if (D == 0) {
    HIPCHK(hipMemsetAsync(drcol, 0xff, 4 * rslots, s->stream), s);
    HIPCHK(hipMemsetAsync(drA, 0, 8 * rslots, s->stream), s);
    HIPCHK(hipMemsetAsync(drBr, 0, 8 * rslots, s->stream), s);
  }
  if (D > 0)
    launch_neighbour_fill(dx, dy, dmx, dmy, dcx, dcy, dcs, dcm, n, gx, gy, cut2, p->alpha, D, dcol,
                          dA, dB, drcol, drA, drBr, s->stream);
  HIPCHK(hipStreamSynchronize(s->stream), s);
  s->mem.release(dcx);
  s->mem.release(dcy);
  s->mem.release(dcs);
  s->mem.release(dcm);
  s->mem.release(ddup);
  s->mem.release(dx);
  s->mem.release(dy);

  // device: state
  const int64_t log_cap = p->flip_log_capacity > 0 ? p->flip_log_capacity : 4 * n + 65536;
  InstDev& I = s->hI;
  I.n = n;
  I.D = D;
  s->l1s = relax_l1_shift(n);
  if (const char* e = std::getenv("ASI_L1_SHIFT")) {
    const int v = std::atoi(e);
    if (v > s->l1s && v <= 20) s->l1s = v;
  }
  I.l1_shift = s->l1s;
  I.len = dlen;
  I.col = dcol;
  I.A = dA;
  I.B = dB;
  I.rcol = drcol;
  I.rA = drA;
  I.rBr = drBr;
  I.mx = dmx;
  I.my = dmy;
  I.hk = dhk;
  I.b = p->b;
  I.c = p->c;
  I.e_par = 2.0 / p->gamma;
  I.e_perp = 2.0 / p->beta;
  I.sigma = p->thermal_std;
  I.seed = p->thermal_seed;
  I.H = nullptr;
  I.K = 0;
  I.s = ds;
  I.field_mode = p->field_mode;
  I.dirty = dalloc<uint8_t>(s, n);
  I.hd = dalloc<double2>(s, n);
  I.h = dalloc<double2>(s, n);
  I.key = dalloc<double>(s, n);
  I.t1key = dalloc<double>(s, nsl);
  I.t1idx = dalloc<uint32_t>(s, nsl);
  // per-chunk sums of the high-degree pass, where it may be split over its
  // chunks (a full-field instance of high degree and few slices)
  I.part = nullptr;
  I.nch = 0;
  if (I.field_mode == kFieldFull && D >= kHdMinD && nsl < kHdSplitSlices) {
    I.nch = (D + 63) / 64;
    I.part = dalloc<double2>(s, (size_t)I.nch * (size_t)n);
    if (!I.part) return fail(ASI_ENOMEM, "device allocation failed (chunk sums)");
  }
  I.log_t = dalloc<int32_t>(s, log_cap);
  I.log_j = dalloc<int32_t>(s, log_cap);
  I.log_cap = log_cap;
  I.step_flips = nullptr;
  I.max_flips = p->max_flips_per_step > 0 ? p->max_flips_per_step : 64 * n;
  I.ccap = n + 8192;
  I.ver = dalloc<uint32_t>(s, n);
  for (int b = 0; b < 2; ++b) {
    I.cpay[b] = dalloc<uint32_t>(s, I.ccap);
    I.ckey[b] = dalloc<double>(s, I.ccap);
    I.cver[b] = dalloc<uint32_t>(s, I.ccap);
    if (!I.cpay[b] || !I.ckey[b] || !I.cver[b])
      return fail(ASI_ENOMEM, "device allocation failed (candidate pool)");
  }
  I.ccount = dalloc<int32_t>(s, 1);
  if (!I.ver || !I.ccount) return fail(ASI_ENOMEM, "device allocation failed (candidate pool)");
  HIPCHK(hipMemsetAsync(I.ver, 0, 4 * n, s->stream), s);
  HIPCHK(hipMemsetAsync(I.ccount, 0, 4, s->stream), s);
  I.spec_min = 32;
  if (const char* e = std::getenv("ASI_SPEC_MIN")) I.spec_min = std::atoll(e);
  I.spec_switch = 2.5;
  if (const char* e = std::getenv("ASI_SPEC_SWITCH")) I.spec_switch = std::atof(e);
  s->dI = dalloc<InstDev>(s, 1);
  s->dR = dalloc<RunDev>(s, 1);
  s->nblocks = (n + kFieldBlock - 1) / kFieldBlock;
  s->blk_inst = dalloc<int32_t>(s, s->nblocks);
  s->blk_row0 = dalloc<int32_t>(s, s->nblocks);
  if (!I.dirty || !I.hd || !I.h || !I.key || !I.t1key || !I.t1idx ||
      !I.log_t || !I.log_j || !s->dI || !s->dR || !s->blk_inst || !s->blk_row0)
    return fail(ASI_ENOMEM, "device allocation failed (state)");
  HIPCHK(hipMemsetAsync(I.h, 0, 16 * n, s->stream), s);
  HIPCHK(hipMemsetAsync(I.hd, 0, 16 * n, s->stream), s);
  HIPCHK(hipMemsetAsync(I.dirty, 1, n, s->stream), s);
  std::vector<int32_t> bi(s->nblocks, 0), br(s->nblocks);
  for (int64_t b = 0; b < s->nblocks; ++b) br[b] = (int32_t)(b * kFieldBlock);
  HIPCHK(hipMemcpyAsync(s->blk_inst, bi.data(), 4 * s->nblocks, hipMemcpyHostToDevice, s->stream),
         s);
  HIPCHK(hipMemcpyAsync(s->blk_row0, br.data(), 4 * s->nblocks, hipMemcpyHostToDevice, s->stream),
         s);
  HIPCHK(hipMemcpyAsync(s->dI, &s->hI, sizeof(InstDev), hipMemcpyHostToDevice, s->stream), s);
  launch_set_run(s->dR, I.ccount, -1, -1, 0, 1, -1, s->stream);
  // 16 wavefronts: the speculative relax spreads up to 2048 member and
  // neighbour slots over 1024 lanes; touched tiles are rescanned in parallel
  s->relax_waves = kMaxRelaxWaves;
  if (const char* w = std::getenv("ASI_RELAX_WAVES")) {
    int v = std::atoi(w);
    if (v >= 1 && v <= kMaxRelaxWaves) s->relax_waves = v;
  }
  s->lds = relax_lds_bytes(n, s->l1s);
  return sync_and_check(s);
}

asi_status upload_desc(asi_sim* s) {
  HIPCHK(hipMemcpyAsync(s->dI, &s->hI, sizeof(InstDev), hipMemcpyHostToDevice, s->stream), s);
  return ASI_OK;
}

asi_status read_run(asi_sim* s, RunDev* r) {
  HIPCHK(hipMemcpyAsync(r, s->dR, sizeof(RunDev), hipMemcpyDeviceToHost, s->stream), s);
  return sync_and_check(s);
}

// steps [t0, t1) of the protocol (t0 may be -1 for the zero-field step)
asi_status ensure_mag_partials(asi_sim* s) {
  if (s->dMpart) return ASI_OK;
  s->dMpart = dalloc<double>(s, kMagPartials + 2);
  if (!s->dMpart) return fail(ASI_ENOMEM, "device allocation failed (magnetisation)");
  return ASI_OK;
}

// Per-step magnetisation log of the current protocol length, rows NaN until
// their step runs.
asi_status alloc_mag_log(asi_sim* s) {
  const int64_t cnt = 2 * std::max<int64_t>(1, s->K);
  s->dMlog = dalloc<double>(s, cnt);
  if (!s->dMlog) return fail(ASI_ENOMEM, "device allocation failed (magnetisation log)");
  std::vector<double> nan(cnt, std::nan(""));
  HIPCHK(hipMemcpyAsync(s->dMlog, nan.data(), 8 * cnt, hipMemcpyHostToDevice, s->stream), s);
  HIPCHK(hipStreamSynchronize(s->stream), s);
  return ASI_OK;
}

asi_status run_steps(asi_sim* s, int64_t t0, int64_t t1, int64_t* flips_out) {
  launch_set_run(s->dR, s->hI.ccount, t0, t1, t0 < t1 ? 1 : 0, 0, 0, s->stream);
  for (int64_t t = t0; t < t1; ++t) {
    field_pass(s);
    relax_pass(s);
    if (s->mag_log && t >= 0)
      launch_magnetization(s->hI.s, s->hI.mx, s->hI.my, s->n, s->dMpart, s->dMlog + 2 * t,
                           s->stream);
  }
  RunDev r{};
  asi_status st = read_run(s, &r);
  if (st != ASI_OK) return st;
  s->cur_step = r.cur_step;
  if (flips_out) *flips_out = r.flips_call;
  if (r.status == kPoolOverflow) {
    s->poisoned = true;
    return fail(ASI_EDEVICE, "candidate pool overflow at step " + std::to_string(r.cur_step));
  }
  if (r.status == ASI_ELOOP)
    return fail(ASI_ELOOP, "a relax exceeded max_flips_per_step at step " +
                               std::to_string(r.cur_step));
  return ASI_OK;
}

}  // namespace

// ======================================================================== ABI
extern "C" {

const char* asi_last_error(void) { return g_err.c_str(); }

asi_status asi_create(const asi_params* params, const asi_device* dev, asi_handle* out) {
  Range range("asi_create");
  if (!out) return fail(ASI_EINVAL, "out is NULL");
  *out = nullptr;
  auto* s = new (std::nothrow) asi_sim();
  if (!s) return fail(ASI_ENOMEM, "host allocation failed");
  asi_status st = create_impl(params, dev, s);
  if (st != ASI_OK) {
    std::string keep = g_err;
    (void)hipStreamSynchronize(s->stream);
    s->mem.release_all();
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
    g_err = keep;
    return st;
  }
  *out = s;
  return ASI_OK;
}

asi_status asi_set_field_protocol(asi_handle h, int64_t n_steps, const double* h_xy) {
  asi_status st = check_handle(h);
  if (st != ASI_OK) return st;
  if (n_steps < 0 || n_steps >= (int64_t)0x7fffffff || (n_steps > 0 && !h_xy))
    return fail(ASI_EINVAL, "bad protocol");
  if (h->hI.hloc_k > 1 && n_steps != h->hI.hloc_k)
    return fail(ASI_EINVAL, "protocol length differs from the local field series");
  if (h->hI.sigma_t && n_steps != h->K)
    return fail(ASI_EINVAL, "protocol length differs from the thermal schedule");
  for (int64_t k = 0; k < 2 * n_steps; ++k)
    if (!std::isfinite(h_xy[k])) return fail(ASI_EINVAL, "non-finite protocol value");
  HIPCHK(hipStreamSynchronize(h->stream), h);
  if (h->dH) h->mem.release(h->dH);
  if (h->hI.step_flips) h->mem.release(h->hI.step_flips);
  h->dH = dalloc<double>(h, std::max<int64_t>(1, 2 * n_steps));
  h->hI.step_flips = dalloc<int32_t>(h, std::max<int64_t>(1, n_steps));
  if (!h->dH || !h->hI.step_flips) return fail(ASI_ENOMEM, "device allocation failed (protocol)");
  if (n_steps > 0)
    HIPCHK(hipMemcpyAsync(h->dH, h_xy, 16 * n_steps, hipMemcpyHostToDevice, h->stream), h);
  HIPCHK(hipMemsetAsync(h->hI.step_flips, 0, 4 * std::max<int64_t>(1, n_steps), h->stream), h);
  h->K = n_steps;
  h->hI.H = h->dH;
  h->hI.K = n_steps;
  if (h->mag_log) {
    if (h->dMlog) h->mem.release(h->dMlog);
    h->dMlog = nullptr;
    st = alloc_mag_log(h);
    if (st != ASI_OK) {
      h->mag_log = false;
      return st;
    }
  }
  if (h->cur_step >= n_steps) h->cur_step = -1;
  st = upload_desc(h);
  if (st != ASI_OK) return st;
  return sync_and_check(h);
}

asi_status asi_set_local_field(asi_handle h, int64_t n_slabs, const double* h_loc) {
  asi_status st = check_handle(h);
  if (st != ASI_OK) return st;
  if (n_slabs < 0 || (n_slabs > 1 && n_slabs != h->K) || (n_slabs > 0 && !h_loc))
    return fail(ASI_EINVAL, "bad local field: n_slabs must be 0, 1 or the protocol length");
  const int64_t cnt = 2 * n_slabs * h->n;
  for (int64_t k = 0; k < cnt; ++k)
    if (!std::isfinite(h_loc[k])) return fail(ASI_EINVAL, "non-finite local field value");
  HIPCHK(hipStreamSynchronize(h->stream), h);
  if (h->dHloc) h->mem.release(h->dHloc);
  h->dHloc = nullptr;
  if (n_slabs > 0) {
    h->dHloc = dalloc<double>(h, cnt);
    if (!h->dHloc) return fail(ASI_ENOMEM, "device allocation failed (local field)");
    HIPCHK(hipMemcpyAsync(h->dHloc, h_loc, 8 * cnt, hipMemcpyHostToDevice, h->stream), h);
  }
  h->hI.hloc = reinterpret_cast<const double2*>(h->dHloc);
  h->hI.hloc_k = n_slabs;
  st = upload_desc(h);
  if (st != ASI_OK) return st;
  return sync_and_check(h);
}

asi_status asi_set_local_wave(asi_handle h, const double* xy, double amp, double kx, double ky,
                              double period_steps, double phase0, double angle) {
  asi_status st = check_handle(h);
  if (st != ASI_OK) return st;
  if (!std::isfinite(amp) || !std::isfinite(kx) || !std::isfinite(ky) ||
      !std::isfinite(period_steps) || period_steps == 0.0 || !std::isfinite(phase0) ||
      !std::isfinite(angle))
    return fail(ASI_EINVAL, "wave parameters must be finite, period_steps != 0");
  if (amp != 0.0 && !xy) return fail(ASI_EINVAL, "xy is NULL");
  std::vector<double> ph;
  if (amp != 0.0) {
    ph.resize(h->n);
    const double two_pi = 6.283185307179586;
    for (int64_t i = 0; i < h->n; ++i) {
      if (!std::isfinite(xy[2 * i]) || !std::isfinite(xy[2 * i + 1]))
        return fail(ASI_EINVAL, "non-finite position");
      ph[i] = two_pi * (kx * xy[2 * i] + ky * xy[2 * i + 1]) + phase0;
    }
  }
  HIPCHK(hipStreamSynchronize(h->stream), h);
  if (h->dWave) h->mem.release(h->dWave);
  h->dWave = nullptr;
  if (amp != 0.0) {
    h->dWave = dalloc<double>(h, h->n);
    if (!h->dWave) return fail(ASI_ENOMEM, "device allocation failed (wave)");
    HIPCHK(hipMemcpyAsync(h->dWave, ph.data(), 8 * h->n, hipMemcpyHostToDevice, h->stream), h);
    HIPCHK(hipStreamSynchronize(h->stream), h);
  }
  h->hI.wave_ph = h->dWave;
  h->hI.wave_amp = amp;
  h->hI.wave_w = 6.283185307179586 / period_steps;
  h->hI.wave_ex = std::cos(angle);
  h->hI.wave_ey = std::sin(angle);
  st = upload_desc(h);
  if (st != ASI_OK) return st;
  return sync_and_check(h);
}

asi_status asi_set_thermal_schedule(asi_handle h, int64_t n_steps, const double* sigma) {
  asi_status st = check_handle(h);
  if (st != ASI_OK) return st;
  if (n_steps < 0 || (n_steps > 0 && (n_steps != h->K || !sigma)))
    return fail(ASI_EINVAL, "bad thermal schedule: n_steps must be 0 or the protocol length");
  for (int64_t k = 0; k < n_steps; ++k)
    if (!(sigma[k] >= 0.0) || !std::isfinite(sigma[k]))
      return fail(ASI_EINVAL, "thermal schedule values must be finite and >= 0");
  HIPCHK(hipStreamSynchronize(h->stream), h);
  if (h->dSig) h->mem.release(h->dSig);
  h->dSig = nullptr;
  if (n_steps > 0) {
    h->dSig = dalloc<double>(h, n_steps);
    if (!h->dSig) return fail(ASI_ENOMEM, "device allocation failed (thermal schedule)");
    HIPCHK(hipMemcpyAsync(h->dSig, sigma, 8 * n_steps, hipMemcpyHostToDevice, h->stream), h);
  }
  h->hI.sigma_t = h->dSig;
  st = upload_desc(h);
  if (st != ASI_OK) return st;
  return sync_and_check(h);
}

asi_status asi_magnetization(asi_handle h, double* m_out) {
  asi_status st = check_handle(h);
  if (st != ASI_OK) return st;
  if (!m_out) return fail(ASI_EINVAL, "m_out is NULL");
  st = ensure_mag_partials(h);
  if (st != ASI_OK) return st;
  launch_magnetization(h->hI.s, h->hI.mx, h->hI.my, h->n, h->dMpart, h->dMpart + kMagPartials,
                       h->stream);
  HIPCHK(hipMemcpyAsync(m_out, h->dMpart + kMagPartials, 16, hipMemcpyDeviceToHost, h->stream), h);
  return sync_and_check(h);
}

asi_status asi_spin_correlation(asi_handle h, const double* xy, double bin_width,
                                int32_t n_bins, int64_t* sum_out, int64_t* count_out) {
  asi_status st = check_handle(h);
  if (st != ASI_OK) return st;
  if (!xy || !sum_out || !count_out) return fail(ASI_EINVAL, "NULL argument");
  if (!(bin_width > 0.0) || !std::isfinite(bin_width))
    return fail(ASI_EINVAL, "bin_width must be finite and > 0");
  if (n_bins < 1 || n_bins > kCorrMaxBins) return fail(ASI_EINVAL, "n_bins out of range");
  for (int64_t k = 0; k < 2 * h->n; ++k)
    if (!std::isfinite(xy[k])) return fail(ASI_EINVAL, "non-finite position");
  HIPCHK(hipStreamSynchronize(h->stream), h);
  double* dxy = dalloc<double>(h, 2 * h->n);
  uint64_t* dsc = dalloc<uint64_t>(h, 2 * (int64_t)n_bins);
  if (!dxy || !dsc) {
    if (dxy) h->mem.release(dxy);
    if (dsc) h->mem.release(dsc);
    return fail(ASI_ENOMEM, "device allocation failed (correlation)");
  }
  asi_status rs = ASI_OK;
  hipError_t e = hipMemcpyAsync(dxy, xy, 16 * h->n, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(dsc, 0, 16 * (size_t)n_bins, h->stream);
  if (e == hipSuccess) {
    launch_correlation(h->dI, h->n, dxy, bin_width, n_bins, std::fabs(h->alpha), dsc,
                       dsc + n_bins, h->stream);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(sum_out, dsc, 8 * (size_t)n_bins, hipMemcpyDeviceToHost,
                                          h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(count_out, dsc + n_bins, 8 * (size_t)n_bins,
                                          hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    h->poisoned = true;
    rs = fail(ASI_EDEVICE, std::string("correlation: ") + hipGetErrorString(e));
  }
  h->mem.release(dxy);
  h->mem.release(dsc);
  return rs;
}

asi_status asi_group_magnetization(asi_handle h, int64_t n_groups, const int64_t* ptr,
                                   const int32_t* idx, double* out) {
  asi_status st = check_handle(h);
  if (st != ASI_OK) return st;
  if (n_groups < 1 || n_groups >= ((int64_t)1 << 31) || !ptr || !idx || !out)
    return fail(ASI_EINVAL, "bad groups");
  if (ptr[0] != 0) return fail(ASI_EINVAL, "ptr[0] must be 0");
  for (int64_t g = 0; g < n_groups; ++g)
    if (ptr[g + 1] < ptr[g]) return fail(ASI_EINVAL, "ptr must not decrease");
  const int64_t ne = ptr[n_groups];
  for (int64_t e = 0; e < ne; ++e)
    if (idx[e] < 0 || idx[e] >= h->n) return fail(ASI_EINVAL, "magnet index out of range");
  HIPCHK(hipStreamSynchronize(h->stream), h);
  int64_t* dptr = dalloc<int64_t>(h, n_groups + 1);
  int32_t* didx = dalloc<int32_t>(h, std::max<int64_t>(1, ne));
  double* dout = dalloc<double>(h, 2 * n_groups);
  asi_status rs = ASI_OK;
  hipError_t e = (dptr && didx && dout) ? hipSuccess : hipErrorOutOfMemory;
  if (e == hipSuccess)
    e = hipMemcpyAsync(dptr, ptr, 8 * (n_groups + 1), hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess && ne > 0)
    e = hipMemcpyAsync(didx, idx, 4 * ne, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) {
    launch_group_magnetization(h->hI.s, h->hI.mx, h->hI.my, dptr, didx, n_groups, dout,
                               h->stream);
    e = hipGetLastError();
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(out, dout, 16 * n_groups, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e == hipErrorOutOfMemory && !(dptr && didx && dout)) {
    rs = fail(ASI_ENOMEM, "device allocation failed (groups)");
  } else if (e != hipSuccess) {
    h->poisoned = true;
    rs = fail(ASI_EDEVICE, std::string("group magnetisation: ") + hipGetErrorString(e));
  }
  h->mem.release(dptr);
  h->mem.release(didx);
  h->mem.release(dout);
  return rs;
}

}  // extern "C"

namespace {

// Device allocations of one call, released on every return path.
struct Scratch {
  DevMem* mem;
  std::vector<void*> ptrs;
  explicit Scratch(DevMem* m) : mem(m) {}
  template <class T>
  T* get(size_t count) {
    void* p = mem->alloc(sizeof(T) * std::max<size_t>(count, 1));
    if (p) ptrs.push_back(p);
    return static_cast<T*>(p);
  }
  ~Scratch() {
    for (void* p : ptrs) mem->release(p);
  }
};

// First-switch positions and twice-average ranks of the handle's flip log
// (Sec. IV.D), on the handle's stream, into pos and r2 (device, n each).
asi_status switching_ranks(asi_sim* h, Scratch& sc, unsigned long long*& pos, int64_t*& r2) {
  RunDev r{};
  asi_status st = read_run(h, &r);
  if (st != ASI_OK) return st;
  if (r.flips > h->hI.log_cap)
    return fail(ASI_ESTATE, "the flip log holds " + std::to_string(h->hI.log_cap) + " of " +
                                std::to_string(r.flips) +
                                " flips: raise flip_log_capacity to compare switching orders");
  const int64_t L = r.flips;
  pos = sc.get<unsigned long long>(h->n);
  r2 = sc.get<int64_t>(h->n);
  int64_t* tmp = sc.get<int64_t>(switching_scratch_count(L));
  if (!pos || !r2 || !tmp) return fail(ASI_ENOMEM, "device allocation failed (switching order)");
  launch_switching_ranks(h->hI.log_j, L, h->n, pos, r2, tmp, h->stream);
  HIPCHK(hipGetLastError(), h);
  return ASI_OK;
}

}  // namespace

extern "C" {

asi_status asi_switching_order(asi_handle h, int64_t* pos_out) {
  asi_status st = check_handle(h);
  if (st != ASI_OK) return st;
  if (!pos_out) return fail(ASI_EINVAL, "pos_out is NULL");
  Scratch sc(&h->mem);
  unsigned long long* pos = nullptr;
  int64_t* r2 = nullptr;
  st = switching_ranks(h, sc, pos, r2);
  if (st != ASI_OK) return st;
  HIPCHK(hipMemcpyAsync(pos_out, pos, 8 * h->n, hipMemcpyDeviceToHost, h->stream), h);
  return sync_and_check(h);
}

asi_status asi_switching_rho(asi_handle a, asi_handle b, double* rho_out, int64_t* sums_out) {
  asi_status st = check_handle(a);
  if (st == ASI_OK) st = check_handle(b);
  if (st != ASI_OK) return st;
  if (!rho_out) return fail(ASI_EINVAL, "rho_out is NULL");
  if (a->n != b->n) return fail(ASI_EINVAL, "the two instances differ in size");
  if (a->n < 2 || a->n > kRankCorrMaxN) return fail(ASI_EINVAL, "n must be in 2 .. 2^27");
  const int64_t n = a->n;
  Scratch sa(&a->mem), sb(&b->mem);
  unsigned long long *pa = nullptr, *pb = nullptr;
  int64_t *ra = nullptr, *rb = nullptr;
  st = switching_ranks(a, sa, pa, ra);
  if (st == ASI_OK && b != a) st = switching_ranks(b, sb, pb, rb);
  if (st != ASI_OK) return st;
  if (b == a) rb = ra;
  // b's ranks are read on a's stream
  st = sync_and_check(b);
  if (st != ASI_OK) return st;
  const int64_t nb = rank_corr_blocks(n);
  long long* part = sa.get<long long>(3 * nb);
  if (!part) return fail(ASI_ENOMEM, "device allocation failed (rank correlation)");
  launch_rank_correlation(ra, rb, n, part, a->stream);
  HIPCHK(hipGetLastError(), a);
  std::vector<long long> hp(3 * nb);
  HIPCHK(hipMemcpyAsync(hp.data(), part, 8 * 3 * nb, hipMemcpyDeviceToHost, a->stream), a);
  st = sync_and_check(a);
  if (st != ASI_OK) return st;
  // exact totals (|sum| < n^3 < 2^81), then rho in FP64 from the rounded totals
  __int128 sum[3] = {0, 0, 0};
  for (int64_t k = 0; k < nb; ++k)
    for (int c = 0; c < 3; ++c) sum[c] += (__int128)hp[3 * k + c];
  const double sab = (double)sum[0], saa = (double)sum[1], sbb = (double)sum[2];
  const double den = std::sqrt(saa * sbb);
  *rho_out = den > 0.0 ? sab / den : std::nan("");
  if (sums_out)
    for (int c = 0; c < 3; ++c) {
      sums_out[2 * c] = (int64_t)(uint64_t)sum[c];                  // low 64 bits
      sums_out[2 * c + 1] = (int64_t)(uint64_t)(sum[c] >> 64);      // high 64 bits (signed)
    }
  return ASI_OK;
}

asi_status asi_switching_rho_noalloc(asi_handle a, asi_handle b, double* rho_out,
                                     int64_t* sums_out) {
  asi_status st = check_handle(a);
  if (st == ASI_OK) st = check_handle(b);
  if (st != ASI_OK) return st;
  if (!rho_out) return fail(ASI_EINVAL, "rho_out is NULL");
  if (a->n != b->n) return fail(ASI_EINVAL, "the two instances differ in size");
  if (a->device != b->device) return fail(ASI_EINVAL, "the two instances are on different GPUs");
  if (a->n < 2 || a->n > kStaticRhoMaxN)
    return fail(ASI_EINVAL, "n must be in 2 .. 2^20 for the allocation-free comparison (n = " +
                                std::to_string(a->n) + "); asi_switching_rho takes up to 2^27");
  const int64_t n = a->n;
  RunDev ra{}, rb{};
  st = read_run(a, &ra);
  if (st == ASI_OK) st = read_run(b, &rb);
  if (st != ASI_OK) return st;
  for (const auto& r : {std::make_pair(a, ra.flips), std::make_pair(b, rb.flips)}) {
    if (r.second > r.first->hI.log_cap)
      return fail(ASI_ESTATE, "the flip log holds " + std::to_string(r.first->hI.log_cap) +
                                  " of " + std::to_string(r.second) +
                                  " flips: raise flip_log_capacity to compare switching orders");
    if (r.second > kStaticRhoMaxLog)
      return fail(ASI_EINVAL, "a flip log of " + std::to_string(r.second) +
                                  " flips exceeds the allocation-free limit of 2^24");
  }
  // the handles' GPU current while its scratch is looked up and used
  int prev = 0;
  HIPCHK(hipGetDevice(&prev), a);
  if (prev != a->device) HIPCHK(hipSetDevice(a->device), a);
  struct Restore {
    int dev, prev;
    ~Restore() {
      if (dev != prev) (void)hipSetDevice(prev);
    }
  } restore{a->device, prev};
  unsigned char* base = nullptr;
  HIPCHK(static_scratch_address(&base), a);
  const StaticRhoScratch S = carve_static_rho(base);
  // one call at a time per process: every call on a GPU uses its one array
  static std::mutex mu;
  std::lock_guard<std::mutex> lock(mu);
  // every scratch word this call reads is written earlier in the call, so
  // nothing needs clearing between calls
  launch_switching_ranks(a->hI.log_j, ra.flips, n, S.pos[0], S.r2[0], S.tmp[0], a->stream);
  HIPCHK(hipGetLastError(), a);
  const int64_t* r2b = S.r2[0];
  if (b != a) {
    launch_switching_ranks(b->hI.log_j, rb.flips, n, S.pos[1], S.r2[1], S.tmp[1], b->stream);
    HIPCHK(hipGetLastError(), b);
    st = sync_and_check(b);  // b's ranks are read on a's stream
    if (st != ASI_OK) return st;
    r2b = S.r2[1];
  }
  const int64_t nb = rank_corr_blocks(n);
  launch_rank_correlation(S.r2[0], r2b, n, S.part, a->stream);
  launch_rank_corr_total(S.part, nb, S.tot, a->stream);
  HIPCHK(hipGetLastError(), a);
  int64_t tot[6];
  HIPCHK(hipMemcpyAsync(tot, S.tot, sizeof(tot), hipMemcpyDeviceToHost, a->stream), a);
  st = sync_and_check(a);
  if (st != ASI_OK) return st;
  __int128 sum[3];
  for (int c = 0; c < 3; ++c)
    sum[c] = (__int128)(((unsigned __int128)(uint64_t)tot[2 * c + 1] << 64) |
                        (unsigned __int128)(uint64_t)tot[2 * c]);
  const double sab = (double)sum[0], saa = (double)sum[1], sbb = (double)sum[2];
  const double den = std::sqrt(saa * sbb);
  *rho_out = den > 0.0 ? sab / den : std::nan("");
  if (sums_out)
    for (int c = 0; c < 6; ++c) sums_out[c] = tot[c];
  return ASI_OK;
}

asi_status asi_set_magnetization_log(asi_handle h, int32_t enable) {
  asi_status st = check_handle(h);
  if (st != ASI_OK) return st;
  HIPCHK(hipStreamSynchronize(h->stream), h);
  if (h->dMlog) h->mem.release(h->dMlog);
  h->dMlog = nullptr;
  h->mag_log = false;
  if (!enable) return ASI_OK;
  st = ensure_mag_partials(h);
  if (st != ASI_OK) return st;
  st = alloc_mag_log(h);
  if (st != ASI_OK) return st;
  h->mag_log = true;
  return sync_and_check(h);
}

asi_status asi_get_magnetization_log(asi_handle h, double* out) {
  asi_status st = check_handle(h);
  if (st != ASI_OK) return st;
  if (!out) return fail(ASI_EINVAL, "out is NULL");
  if (!h->mag_log) return fail(ASI_ESTATE, "the magnetisation log is off");
  if (h->K > 0)
    HIPCHK(hipMemcpyAsync(out, h->dMlog, 16 * h->K, hipMemcpyDeviceToHost, h->stream), h);
  return sync_and_check(h);
}

asi_status asi_relax(asi_handle h, int64_t* flips_out) {
  Range range("asi_relax");
  asi_status st = check_handle(h);
  if (st != ASI_OK) return st;
  return run_steps(h, h->cur_step, h->cur_step + 1, flips_out);
}

asi_status asi_run(asi_handle h, int64_t t_begin, int64_t t_end, int64_t* flips_out) {
  Range range("asi_run");
  asi_status st = check_handle(h);
  if (st != ASI_OK) return st;
  if (t_begin < 0 || t_begin > t_end || t_end > h->K)
    return fail(ASI_EINVAL, "step range outside the protocol");
  if (flips_out) *flips_out = 0;
  if (t_begin == t_end) return ASI_OK;
  return run_steps(h, t_begin, t_end, flips_out);
}

static bool tuning_valid(const asi_sim* h, const asi_tuning* t) {
  const int32_t r = t->field_rows;
  return t->relax_waves >= 1 && t->relax_waves <= kMaxRelaxWaves &&
         t->l1_shift >= relax_l1_shift(h->n) && t->l1_shift <= 20 && t->spec_min >= 1 &&
         (r == 0 || r == 8 || r == 16 || r == 32 || r == 64);
}

static asi_status apply_tuning(asi_sim* h, const asi_tuning* t) {
  h->field_rows = t->field_rows;
  h->relax_waves = t->relax_waves;
  h->l1s = t->l1_shift;
  h->hI.l1_shift = t->l1_shift;
  h->hI.spec_min = t->spec_min;
  h->lds = relax_lds_bytes(h->n, t->l1_shift);
  return upload_desc(h);
}

asi_status asi_get_tuning(asi_handle h, asi_tuning* out) {
  asi_status st = check_handle(h);
  if (st != ASI_OK) return st;
  if (!out) return fail(ASI_EINVAL, "out is NULL");
  *out = asi_tuning{};
  out->relax_waves = h->relax_waves;
  out->l1_shift = h->l1s;
  out->spec_min = h->hI.spec_min;
  out->field_rows = h->field_rows;
  return ASI_OK;
}

}  // extern "C"

// ---- tuning cache: shapes found by asi_tune, keyed by the device
// architecture and the instance's size class, reused by later asi_tune calls
// on similar instances (any shapes give the same results; only speed
// differs).  Optionally persisted in the text file named by ASI_TUNE_CACHE;
// ASI_TUNE_NOCACHE=1 disables lookups.
namespace {

struct TuneKey {
  std::string arch;
  int32_t n_bucket, d_bucket, mode;
  bool operator<(const TuneKey& o) const {
    return std::tie(arch, n_bucket, d_bucket, mode) <
           std::tie(o.arch, o.n_bucket, o.d_bucket, o.mode);
  }
};
struct TuneVal {
  int32_t relax_waves, l1_delta, field_rows;
  int64_t spec_min;
};

std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune_cache;
bool g_tune_loaded = false;

int32_t log2_bucket(int64_t v) {
  int32_t b = 0;
  while (v > 1) {
    v >>= 1;
    ++b;
  }
  return b;
}

TuneKey tune_key(const asi_sim* h) {
  TuneKey k{"", log2_bucket(h->n), log2_bucket(std::max<int32_t>(h->D, 1)), h->hI.field_mode};
  hipDeviceProp_t prop{};
  if (hipGetDeviceProperties(&prop, h->device) == hipSuccess) k.arch = prop.gcnArchName;
  const size_t c = k.arch.find(':');  // feature suffixes (e.g. ":sramecc+") do not matter
  if (c != std::string::npos) k.arch.resize(c);
  return k;
}

// Caller holds g_tune_mu.
void tune_cache_load() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = std::getenv("ASI_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char arch[64];
  int nb, db, mode, w, dl, fr;
  long long sm;
  while (std::fscanf(f, "%63s %d %d %d %d %d %lld %d", arch, &nb, &db, &mode, &w, &dl, &sm,
                     &fr) == 8)
    g_tune_cache[TuneKey{arch, nb, db, mode}] = TuneVal{w, dl, fr, (int64_t)sm};
  std::fclose(f);
}

bool tune_cache_get(const asi_sim* h, asi_tuning* t) {
  if (const char* e = std::getenv("ASI_TUNE_NOCACHE"))
    if (e[0] == '1') return false;
  const TuneKey k = tune_key(h);
  std::lock_guard<std::mutex> lock(g_tune_mu);
  tune_cache_load();
  auto it = g_tune_cache.find(k);
  if (it == g_tune_cache.end()) return false;
  *t = asi_tuning{};
  t->relax_waves = it->second.relax_waves;
  t->l1_shift = relax_l1_shift(h->n) + it->second.l1_delta;
  t->spec_min = it->second.spec_min;
  t->field_rows = it->second.field_rows;
  return tuning_valid(h, t);
}

void tune_cache_put(const asi_sim* h, const asi_tuning& t) {
  const TuneKey k = tune_key(h);
  const TuneVal v{t.relax_waves, t.l1_shift - relax_l1_shift(h->n), t.field_rows, t.spec_min};
  std::lock_guard<std::mutex> lock(g_tune_mu);
  tune_cache_load();
  g_tune_cache[k] = v;
  const char* path = std::getenv("ASI_TUNE_CACHE");
  if (!path || !*path) return;
  if (FILE* f = std::fopen(path, "a")) {
    std::fprintf(f, "%s %d %d %d %d %d %lld %d\n", k.arch.c_str(), k.n_bucket, k.d_bucket,
                 k.mode, v.relax_waves, v.l1_delta, (long long)v.spec_min, v.field_rows);
    std::fclose(f);
  }
}

}  // namespace

extern "C" {

asi_status asi_set_tuning(asi_handle h, const asi_tuning* t) {
  asi_status st = check_handle(h);
  if (st != ASI_OK) return st;
  if (!t) return fail(ASI_EINVAL, "tuning is NULL");
  if (!tuning_valid(h, t)) return fail(ASI_EINVAL, "tuning out of range");
  HIPCHK(hipStreamSynchronize(h->stream), h);
  st = apply_tuning(h, t);
  if (st != ASI_OK) return st;
  return sync_and_check(h);
}

asi_status asi_tune(asi_handle h, int64_t sample_steps, asi_tuning* out) {
  Range range("asi_tune");
  asi_status st = check_handle(h);
  if (st != ASI_OK) return st;
  if (h->K <= 0) return fail(ASI_ESTATE, "no field protocol set");
  const int64_t t0 = h->cur_step + 1;
  if (t0 >= h->K) return fail(ASI_EINVAL, "no protocol step left to sample");
  const int64_t t1 = std::min(h->K, t0 + std::max<int64_t>(sample_steps, 1));
  {
    asi_tuning cached{};
    if (tune_cache_get(h, &cached)) {  // a similar instance was tuned before
      HIPCHK(hipStreamSynchronize(h->stream), h);
      st = apply_tuning(h, &cached);
      if (st == ASI_OK) st = sync_and_check(h);
      if (st != ASI_OK) return st;
      if (out) *out = cached;  // trials == 0: taken from the cache
      return ASI_OK;
    }
  }
  const int64_t n = h->n, nsl = (n + kSlice - 1) / kSlice;
  InstDev& I = h->hI;
  // the mutable state a step reads or writes (the candidate pool is rebuilt
  // by every field pass; flip-log entries past the cursor are rewritten by
  // the real run)
  struct Arr {
    void* p;
    size_t bytes;
    void* snap;
  };
  std::vector<Arr> arrs = {{I.s, (size_t)n, nullptr},          {I.dirty, (size_t)n, nullptr},
                           {I.hd, 16 * (size_t)n, nullptr},     {I.h, 16 * (size_t)n, nullptr},
                           {I.key, 8 * (size_t)n, nullptr},     {I.ver, 4 * (size_t)n, nullptr},
                           {I.t1key, 8 * (size_t)nsl, nullptr}, {I.t1idx, 4 * (size_t)nsl, nullptr},
                           {I.step_flips + t0, 4 * (size_t)(t1 - t0), nullptr}};
  // trials are not charged to the handle's kernel timing
  st = sync_and_check(h);
  if (st != ASI_OK) return st;
  const bool timing0 = h->timing;
  h->timing = false;
  auto release = [&]() {
    for (auto& a : arrs)
      if (a.snap) h->mem.release(a.snap);
  };
  for (auto& a : arrs) {
    a.snap = h->mem.alloc(a.bytes);
    if (!a.snap) {
      release();
      h->timing = timing0;
      return fail(ASI_ENOMEM, "device allocation failed (tuning snapshot)");
    }
    HIPCHK(hipMemcpyAsync(a.snap, a.p, a.bytes, hipMemcpyDeviceToDevice, h->stream), h);
  }
  RunDev r0{};
  st = read_run(h, &r0);
  if (st != ASI_OK) {
    release();
    h->timing = timing0;
    return st;
  }
  const int64_t step0 = h->cur_step;
  auto restore = [&]() -> asi_status {
    for (auto& a : arrs)
      HIPCHK(hipMemcpyAsync(a.p, a.snap, a.bytes, hipMemcpyDeviceToDevice, h->stream), h);
    HIPCHK(hipMemcpyAsync(h->dR, &r0, sizeof(RunDev), hipMemcpyHostToDevice, h->stream), h);
    h->cur_step = step0;
    return sync_and_check(h);
  };
  asi_tuning cur{};
  (void)asi_get_tuning(h, &cur);
  const asi_tuning first = cur;
  bool have_ref = false;
  int64_t ref_flips = 0;
  uint64_t ref_hash = 0;
  int32_t trials = 0;
  // one timed sample under shapes c; every sample must match the first
  auto trial = [&](const asi_tuning& c, double& ms) -> asi_status {
    asi_status e = restore();
    if (e == ASI_OK) e = apply_tuning(h, &c);
    if (e == ASI_OK) e = sync_and_check(h);
    if (e != ASI_OK) return e;
    const double ta = now_s();
    int64_t f = 0;
    e = run_steps(h, t0, t1, &f);
    ms = (now_s() - ta) * 1e3;
    if (e != ASI_OK) return e;
    RunDev r{};
    e = read_run(h, &r);
    if (e != ASI_OK) return e;
    ++trials;
    if (!have_ref) {
      have_ref = true;
      ref_flips = r.flips;
      ref_hash = r.hash;
    } else if (r.flips != ref_flips || r.hash != ref_hash) {
      return fail(ASI_ESTATE, "launch shapes changed the flips (tuning aborted)");
    }
    return ASI_OK;
  };
  double best_ms = 0.0;
  st = trial(cur, best_ms);
  const double default_ms = best_ms;
  asi_tuning best = cur;
  auto consider = [&](asi_tuning c) -> asi_status {
    if (!tuning_valid(h, &c)) return ASI_OK;
    double ms = 0.0;
    asi_status e = trial(c, ms);
    if (e != ASI_OK) return e;
    if (ms < 0.97 * best_ms) {  // a clear win only
      best_ms = ms;
      best = c;
    }
    return ASI_OK;
  };
  // 0. rows per workgroup of the high-degree full-field pass
  if (st == ASI_OK && I.field_mode == kFieldFull && h->D >= kHdMinD) {
    const int32_t rows[] = {8, 16, 32, 64};
    for (int32_t r : rows) {
      if (st != ASI_OK) break;
      asi_tuning c = best;
      c.field_rows = r;
      st = consider(c);
    }
  }
  // 1. speculation threshold (only where the degree allows speculation)
  if (st == ASI_OK && h->D <= kSpecMaxD && cur.relax_waves == kMaxRelaxWaves) {
    const int64_t mins[] = {8, 256, INT64_MAX};
    for (int64_t m : mins) {
      if (st != ASI_OK || m == cur.spec_min) continue;
      asi_tuning c = best;
      c.spec_min = m;
      st = consider(c);
    }
  }
  // 2. first-level tile of the max tree
  for (int dl = 1; st == ASI_OK && dl <= 2; ++dl) {
    asi_tuning c = best;
    c.l1_shift = cur.l1_shift + dl;
    st = consider(c);
  }
  // 3. workgroup size, where the relax does not speculate
  if (st == ASI_OK && (h->D > kSpecMaxD || best.spec_min == INT64_MAX)) {
    const int32_t ws[] = {8, 4};
    for (int32_t w : ws) {
      if (st != ASI_OK) break;
      asi_tuning c = best;
      c.relax_waves = w;
      st = consider(c);
    }
  }
  asi_status st2 = restore();
  if (st2 == ASI_OK) st2 = apply_tuning(h, st == ASI_OK ? &best : &first);
  if (st2 == ASI_OK) st2 = sync_and_check(h);
  release();
  h->timing = timing0;
  if (st != ASI_OK) return st;
  if (st2 != ASI_OK) return st2;
  tune_cache_put(h, best);
  if (out) {
    *out = best;
    out->default_ms = default_ms;
    out->tuned_ms = best_ms;
    out->trials = trials;
  }
  return ASI_OK;
}

asi_status asi_compute_fields(asi_handle h, int64_t t) {
  Range range("asi_compute_fields");
  asi_status st = check_handle(h);
  if (st != ASI_OK) return st;
  if (t < -1 || t >= h->K) return fail(ASI_EINVAL, "step outside the protocol");
  launch_set_run(h->dR, h->hI.ccount, t, t + 1, 1, 0, 0, h->stream);
  field_pass(h);
  // the pass appended every flippable magnet to the candidate pool: empty
  // it, so that a later relax sees only its own step's entries
  launch_set_run(h->dR, h->hI.ccount, t, t, 0, 0, 0, h->stream);
  return sync_and_check(h);
}

asi_status asi_get_state(asi_handle h, int8_t* spins, double* h_par, double* h_perp,
                         int64_t* step_out) {
  asi_status st = check_handle(h);
  if (st != ASI_OK) return st;
  if (spins) HIPCHK(hipMemcpyAsync(spins, h->hI.s, h->n, hipMemcpyDeviceToHost, h->stream), h);
  std::vector<double2> f;
  if (h_par || h_perp) {
    f.resize(h->n);
    HIPCHK(hipMemcpyAsync(f.data(), h->hI.h, 16 * h->n, hipMemcpyDeviceToHost, h->stream), h);
  }
  st = sync_and_check(h);
  if (st != ASI_OK) return st;
  for (int64_t i = 0; i < (int64_t)f.size(); ++i) {
    if (h_par) h_par[i] = f[i].x;
    if (h_perp) h_perp[i] = f[i].y;
  }
  if (step_out) *step_out = h->cur_step;
  return ASI_OK;
}

asi_status asi_set_state(asi_handle h, const int8_t* spins, int64_t step) {
  asi_status st = check_handle(h);
  if (st != ASI_OK) return st;
  if (!spins) return fail(ASI_EINVAL, "spins is NULL");
  if (step < -1 || step >= std::max<int64_t>(h->K, 0)) {
    if (!(step == -1)) return fail(ASI_EINVAL, "step outside the protocol");
  }
  for (int64_t i = 0; i < h->n; ++i)
    if (spins[i] != 1 && spins[i] != -1) return fail(ASI_EINVAL, "spins must be +1 or -1");
  HIPCHK(hipStreamSynchronize(h->stream), h);
  HIPCHK(hipMemcpyAsync(h->hI.s, spins, h->n, hipMemcpyHostToDevice, h->stream), h);
  HIPCHK(hipMemsetAsync(h->hI.dirty, 1, h->n, h->stream), h);
  launch_set_run(h->dR, h->hI.ccount, step, step, 0, 1, step, h->stream);
  h->cur_step = step;
  return sync_and_check(h);
}

asi_status asi_get_flip_log(asi_handle h, int64_t cap, int32_t* step, int32_t* idx,
                            int64_t* count_out, uint64_t* hash_out) {
  asi_status st = check_handle(h);
  if (st != ASI_OK) return st;
  if (cap < 0 || (cap > 0 && (!step || !idx))) return fail(ASI_EINVAL, "bad log buffers");
  RunDev r{};
  st = read_run(h, &r);
  if (st != ASI_OK) return st;
  const int64_t m = std::min(std::min(cap, r.flips), h->hI.log_cap);
  if (m > 0) {
    HIPCHK(hipMemcpyAsync(step, h->hI.log_t, 4 * m, hipMemcpyDeviceToHost, h->stream), h);
    HIPCHK(hipMemcpyAsync(idx, h->hI.log_j, 4 * m, hipMemcpyDeviceToHost, h->stream), h);
    st = sync_and_check(h);
    if (st != ASI_OK) return st;
  }
  if (count_out) *count_out = r.flips;
  if (hash_out) *hash_out = r.hash;
  return ASI_OK;
}

asi_status asi_get_step_flips(asi_handle h, int32_t* out) {
  asi_status st = check_handle(h);
  if (st != ASI_OK) return st;
  if (!out) return fail(ASI_EINVAL, "out is NULL");
  if (h->K > 0)
    HIPCHK(hipMemcpyAsync(out, h->hI.step_flips, 4 * h->K, hipMemcpyDeviceToHost, h->stream), h);
  return sync_and_check(h);
}

asi_status asi_get_info(asi_handle h, asi_info* out) {
  if (!h || !out) return fail(ASI_EINVAL, "null argument");
  out->n = h->n;
  out->n_edges = h->E;
  out->max_degree = h->D;
  out->relax_waves = h->relax_waves;
  out->device_bytes = (int64_t)h->mem.total;
  out->field_pass_bytes = 20.0 * (double)h->E + 53.0 * (double)h->n +
                          (h->hI.hloc ? 16.0 * (double)h->n : 0.0) +
                          (h->hI.wave_ph ? 8.0 * (double)h->n : 0.0);
  out->flip_log_capacity = h->hI.log_cap;
  return ASI_OK;
}

asi_status asi_set_timing(asi_handle h, int32_t enable) {
  asi_status st = check_handle(h);
  if (st != ASI_OK) return st;
  st = sync_and_check(h);
  if (st != ASI_OK) return st;
  h->timing = enable != 0;
  h->tm = asi_timing{};
  return ASI_OK;
}

asi_status asi_get_timing(asi_handle h, asi_timing* out) {
  asi_status st = check_handle(h);
  if (st != ASI_OK) return st;
  if (!out) return fail(ASI_EINVAL, "out is NULL");
  st = sync_and_check(h);
  if (st != ASI_OK) return st;
  *out = h->tm;
  return ASI_OK;
}

asi_status asi_destroy(asi_handle h) {
  if (!h) return ASI_OK;
  (void)hipStreamSynchronize(h->stream);
  for (auto& tp : h->timers) {
    (void)hipEventDestroy(tp.a);
    (void)hipEventDestroy(tp.b);
  }
  for (auto e : h->spare_events) (void)hipEventDestroy(e);
  h->mem.release_all();
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
  return ASI_OK;
}

}  // extern "C"

// ======================================================================== batch
namespace {

// A device-resident table of instances driven by one field launch and one
// relax launch per step.  Used by asi_batch_run and by the server.
struct Table {
  DevMem mem;
  int32_t count = 0;
  InstDev* dI = nullptr;
  RunDev* dR = nullptr;
  int32_t* blk_inst = nullptr;
  int32_t* blk_row0 = nullptr;
  int64_t nblocks = 0;
  int32_t waves = 1;
  size_t lds = 0;
  bool tree_only = false;  // no instance of the table may speculate
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;

  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
  ~Table() {
    drop_graph();
    mem.release_all();
  }
};

// (Re)build the launch tables for the given instance descriptors.
asi_status table_build(Table& T, const std::vector<InstDev>& insts,
                       const std::vector<int32_t>& waves, const std::vector<size_t>& lds,
                       hipStream_t st) {
  T.drop_graph();
  T.mem.st = st;
  T.mem.release_all();
  T.count = (int32_t)insts.size();
  std::vector<int32_t> bi, br;
  T.waves = 1;
  T.lds = 0;
  for (int32_t k = 0; k < T.count; ++k) {
    const int64_t nb = (insts[k].n + kFieldBlock - 1) / kFieldBlock;
    for (int64_t b = 0; b < nb; ++b) {
      bi.push_back(k);
      br.push_back((int32_t)(b * kFieldBlock));
    }
    T.waves = std::max(T.waves, waves[k]);
    T.lds = std::max(T.lds, lds[k]);
  }
  if (const char* w = std::getenv("ASI_BATCH_RELAX_WAVES")) {
    int v = std::atoi(w);
    if (v >= 1 && v <= kMaxRelaxWaves) T.waves = v;
  }
  T.tree_only = true;
  for (int32_t k = 0; k < T.count; ++k)
    if (insts[k].n > 0 && relax_may_speculate(insts[k].D, T.waves)) T.tree_only = false;
  T.nblocks = (int64_t)bi.size();
  T.dI = static_cast<InstDev*>(T.mem.alloc(sizeof(InstDev) * std::max(1, T.count)));
  T.dR = static_cast<RunDev*>(T.mem.alloc(sizeof(RunDev) * std::max(1, T.count)));
  T.blk_inst = static_cast<int32_t*>(T.mem.alloc(4 * std::max<int64_t>(1, T.nblocks)));
  T.blk_row0 = static_cast<int32_t*>(T.mem.alloc(4 * std::max<int64_t>(1, T.nblocks)));
  if (!T.dI || !T.dR || !T.blk_inst || !T.blk_row0)
    return fail(ASI_ENOMEM, "device allocation failed (batch tables)");
  if (T.count > 0) {
    HIPCHK(hipMemcpyAsync(T.dI, insts.data(), sizeof(InstDev) * T.count, hipMemcpyHostToDevice, st),
           (asi_sim*)nullptr);
  }
  if (T.nblocks > 0) {
    HIPCHK(hipMemcpyAsync(T.blk_inst, bi.data(), 4 * T.nblocks, hipMemcpyHostToDevice, st),
           (asi_sim*)nullptr);
    HIPCHK(hipMemcpyAsync(T.blk_row0, br.data(), 4 * T.nblocks, hipMemcpyHostToDevice, st),
           (asi_sim*)nullptr);
  }
  HIPCHK(hipStreamSynchronize(st), (asi_sim*)nullptr);
  return ASI_OK;
}

void table_step(Table& T, hipStream_t st) {
  launch_field(T.dI, T.dR, T.blk_inst, T.blk_row0, T.nblocks, st);
  launch_relax(T.dI, T.dR, T.count, T.waves, T.lds, T.tree_only, st);
}

asi_status table_capture(Table& T, hipStream_t st) {
  T.drop_graph();
  HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), (asi_sim*)nullptr);
  table_step(T, st);
  HIPCHK(hipStreamEndCapture(st, &T.graph), (asi_sim*)nullptr);
  HIPCHK(hipGraphInstantiate(&T.exec, T.graph, nullptr, nullptr, 0), (asi_sim*)nullptr);
  return ASI_OK;
}

}  // namespace

extern "C" asi_status asi_batch_run(asi_handle* hs, int32_t count, int32_t mode,
                                    int64_t* flips_out) {
  Range range("asi_batch_run");
  if (!hs || count < 1) return fail(ASI_EINVAL, "no handles");
  if (mode < 0 || mode > 2) return fail(ASI_EINVAL, "batch mode must be 0, 1 or 2");
  for (int32_t k = 0; k < count; ++k) {
    asi_status st = check_handle(hs[k]);
    if (st != ASI_OK) return st;
    for (int32_t m = 0; m < k; ++m)
      if (hs[m] == hs[k]) return fail(ASI_EINVAL, "a handle appears twice in the batch");
  }
  std::vector<InstDev> insts(count);
  std::vector<RunDev> runs(count);
  std::vector<int32_t> waves(count);
  std::vector<size_t> lds(count);
  int64_t max_steps = 0;
  for (int32_t k = 0; k < count; ++k) {
    asi_sim* h = hs[k];
    asi_status st = read_run(h, &runs[k]);
    if (st != ASI_OK) return st;
    insts[k] = h->hI;
    waves[k] = h->relax_waves;
    lds[k] = h->lds;
    RunDev& r = runs[k];
    r.t = h->cur_step + 1;
    r.t_end = h->K;
    r.active = r.t < r.t_end ? 1 : 0;
    r.status = 0;
    r.flips_call = 0;
    max_steps = std::max(max_steps, r.t_end - r.t);
  }
  hipStream_t st = nullptr;
  HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), (asi_sim*)nullptr);
  asi_status res = ASI_OK;
  {
    Table T;
    T.mem.dev = hs[0]->mem.dev;
    res = table_build(T, insts, waves, lds, st);
    if (res == ASI_OK) {
      hipError_t e = hipMemcpyAsync(T.dR, runs.data(), sizeof(RunDev) * count,
                                    hipMemcpyHostToDevice, st);
      if (e != hipSuccess) res = fail(ASI_EDEVICE, hipGetErrorString(e));
    }
    if (res == ASI_OK && max_steps > 0) {
      if (mode == 2) {
        launch_field(T.dI, T.dR, T.blk_inst, T.blk_row0, T.nblocks, st);
        launch_fused(T.dI, T.dR, T.count, T.waves, T.lds, max_steps, 0, 1, st);
      } else {
        if (mode == 1) res = table_capture(T, st);
        for (int64_t s = 0; res == ASI_OK && s < max_steps; ++s) {
          if (T.exec) {
            hipError_t e = hipGraphLaunch(T.exec, st);
            if (e != hipSuccess) res = fail(ASI_EDEVICE, hipGetErrorString(e));
          } else {
            table_step(T, st);
          }
        }
      }
    }
    if (res == ASI_OK) {
      hipError_t e = hipMemcpyAsync(runs.data(), T.dR, sizeof(RunDev) * count,
                                    hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e == hipSuccess) e = hipGetLastError();
      if (e != hipSuccess) res = fail(ASI_EDEVICE, hipGetErrorString(e));
    }
    (void)hipStreamSynchronize(st);
  }
  (void)hipStreamDestroy(st);
  if (res != ASI_OK) {
    if (res == ASI_EDEVICE)
      for (int32_t k = 0; k < count; ++k) hs[k]->poisoned = true;
    return res;
  }
  bool loop = false, overflow = false;
  for (int32_t k = 0; k < count; ++k) {
    asi_sim* h = hs[k];
    HIPCHK(hipMemcpyAsync(h->dR, &runs[k], sizeof(RunDev), hipMemcpyHostToDevice, h->stream), h);
    HIPCHK(hipStreamSynchronize(h->stream), h);
    h->cur_step = runs[k].cur_step;
    if (flips_out) flips_out[k] = runs[k].flips_call;
    if (runs[k].status == ASI_ELOOP) loop = true;
    if (runs[k].status == kPoolOverflow) {
      h->poisoned = true;
      overflow = true;
    }
  }
  if (overflow) return fail(ASI_EDEVICE, "candidate pool overflow");
  if (loop) return fail(ASI_ELOOP, "an instance exceeded max_flips_per_step");
  return ASI_OK;
}

// ======================================================================== server
namespace {

struct Job {
  int64_t id = 0;
  asi_params p{};
  std::vector<double> xy, theta, hk, H;
  std::vector<double> loc, sig;   // local field [loc_k][n][2], thermal schedule [K] (optional)
  int64_t loc_k = 0;
  std::vector<int8_t> spin0;
  int64_t K = 0;
  size_t foot = 0;
  asi_sim* h = nullptr;  // while resident
  int32_t slot = -1;
  int state = 0;         // 0 queued, 1 resident, 2 done, 3 failed
  int32_t passed = 0;    // later jobs admitted while this one waited at the head
  asi_status err = ASI_OK;
  std::vector<int8_t> spins_out;
  int64_t flips = 0;
  uint64_t hash = 0;
  double t_admit = 0, t_done = 0;
};

// Upper bound of any magnet's neighbour count from cell occupancies: with
// cells of side cs = cutoff / 4, the neighbours of a magnet lie in the cells
// whose nearest point to the magnet's cell is within the cutoff (a disc of
// about 69 cells), so the bound is the largest population of such a block
// (about 1.4 times the disc's expected count, instead of 2.9 times for a
// 3 x 3 block of cutoff-sized cells).  The grid is coarsened while it would
// exceed 4n + 1024 cells.
int64_t degree_bound(const asi_params* p) {
  const int64_t n = p->n;
  double xmin = p->xy[0], xmax = p->xy[0], ymin = p->xy[1], ymax = p->xy[1];
  for (int64_t i = 0; i < n; ++i) {
    xmin = std::min(xmin, p->xy[2 * i]);
    xmax = std::max(xmax, p->xy[2 * i]);
    ymin = std::min(ymin, p->xy[2 * i + 1]);
    ymax = std::max(ymax, p->xy[2 * i + 1]);
  }
  const double cut = (p->neighbor_distance + 1e-9) * (1.0 + 1e-6);
  double cs = std::max(cut / 4.0, 1e-6);
  const double cap = 4.0 * (double)n + 1024.0;
  while (((xmax - xmin) / cs + 1.0) * ((ymax - ymin) / cs + 1.0) > cap) cs *= 2.0;
  const int64_t gx = (int64_t)std::floor((xmax - xmin) / cs) + 1;
  const int64_t gy = (int64_t)std::floor((ymax - ymin) / cs) + 1;
  std::vector<int32_t> cnt(gx * gy, 0);
  for (int64_t i = 0; i < n; ++i) {
    int64_t a = std::min(std::max((int64_t)std::floor((p->xy[2 * i] - xmin) / cs), (int64_t)0), gx - 1);
    int64_t b = std::min(std::max((int64_t)std::floor((p->xy[2 * i + 1] - ymin) / cs), (int64_t)0), gy - 1);
    cnt[b * gx + a]++;
  }
  // cell offsets whose nearest points are within the cutoff
  const int64_t r = (int64_t)std::ceil(cut / cs);
  std::vector<std::pair<int64_t, int64_t>> offs;
  for (int64_t dy = -r; dy <= r; ++dy)
    for (int64_t dx = -r; dx <= r; ++dx) {
      const double ex = (double)std::max<int64_t>(std::llabs(dx) - 1, 0) * cs;
      const double ey = (double)std::max<int64_t>(std::llabs(dy) - 1, 0) * cs;
      if (ex * ex + ey * ey <= cut * cut) offs.emplace_back(dx, dy);
    }
  int64_t best = 0;
  for (int64_t y = 0; y < gy; ++y)
    for (int64_t x = 0; x < gx; ++x) {
      if (!cnt[y * gx + x]) continue;
      int64_t s = 0;
      for (const auto& o : offs) {
        const int64_t xx = x + o.first, yy = y + o.second;
        if (xx >= 0 && xx < gx && yy >= 0 && yy < gy) s += cnt[yy * gx + xx];
      }
      best = std::max(best, s - 1);
    }
  return std::min<int64_t>(best, n - 1);
}

}  // namespace

struct asi_server {
  asi_device dev{};   // bursts run on dev.stream
  asi_device cdev{};  // admission (job creation) runs on cdev.stream
  hipStream_t stream = nullptr, cstream = nullptr;
  size_t budget = 0, used = 0;
  int32_t max_slots = 0;
  int64_t next_id = 0;
  std::map<int64_t, std::unique_ptr<Job>> jobs;
  std::deque<int64_t> queue;
  std::vector<int64_t> slots;  // job id per slot, -1 free
  Table T;
  bool dirty = true;
  std::vector<RunDev> runs;     // host copy of every slot's run cursor
  RunDev* rb = nullptr;         // pinned read-back of the burst's cursors
  std::vector<char> in_burst;   // slot took part in the running burst
  int64_t clock_hz = 100000000;  // device constant-rate clock
  int64_t big_magnets = 0;       // see kBigMagnets
  int32_t tail_jobs = 0;         // see kTailJobs
  double quiet_scale = 1.0;      // see kQuietBurstScale
  asi_server_stats stats{};
};

namespace {

// Inside the fused kernel a job's field phase streams through a single
// compute unit.  When at most kTailJobs jobs are resident and one has at
// least kBigMagnets magnets, the device is mostly idle and that phase would
// dominate: such a burst is a sequence of rounds, each a grid-wide field pass
// and one relax step of every job, until the budget is spent.
constexpr int64_t kBigMagnets = 1 << 17;
constexpr int32_t kTailJobs = 8;
// In the tail regime with nothing queued, a burst runs kQuietBurstScale
// times the asked budget, and each round relaxes every job's step to its end
// with the relax kernel (no deadline: no pause, whose resume would rebuild
// the candidate structures, and the relax kernel's lighter register use):
// bursts exist to bound how long an arriving job waits for admission, and
// none is waiting.  A round can then outlast the budget by one step's relax.
constexpr double kQuietBurstScale = 8.0;

asi_status server_rebuild(asi_server* S) {
  std::vector<InstDev> insts(S->max_slots);
  std::vector<int32_t> waves(S->max_slots, 1);
  std::vector<size_t> lds(S->max_slots, 0);
  for (int32_t k = 0; k < S->max_slots; ++k) {
    if (S->slots[k] < 0) {
      insts[k] = InstDev{};
      insts[k].n = 0;
      continue;
    }
    Job& J = *S->jobs[S->slots[k]];
    insts[k] = J.h->hI;
    waves[k] = J.h->relax_waves;
    lds[k] = J.h->lds;
  }
  asi_status st = table_build(S->T, insts, waves, lds, S->stream);
  if (st != ASI_OK) return st;
  HIPCHK(hipMemcpyAsync(S->T.dR, S->runs.data(), sizeof(RunDev) * S->max_slots,
                        hipMemcpyHostToDevice, S->stream),
         (asi_sim*)nullptr);
  S->dirty = false;
  return ASI_OK;
}

// Admit queued jobs in arrival order while a slot is free.  A job whose
// footprint does not fit the remaining budget is passed by later jobs that
// fit, until max_slots jobs have passed it at the head of the queue; then
// admission waits for memory to free up for it.  Creation runs on the
// admission stream, alongside a running burst.
asi_status server_admit(asi_server* S) {
  size_t qi = 0;
  int32_t slot = 0;
  while (qi < S->queue.size()) {
    while (slot < S->max_slots && S->slots[slot] >= 0) ++slot;
    if (slot >= S->max_slots) break;
    Job& J = *S->jobs[S->queue[qi]];
    if (S->used + J.foot > S->budget) {
      if (qi == 0 && J.passed >= S->max_slots) break;
      ++qi;
      continue;
    }
    S->queue.erase(S->queue.begin() + (std::ptrdiff_t)qi);
    if (qi > 0) S->jobs[S->queue.front()]->passed++;
    asi_params p = J.p;
    p.xy = J.xy.data();
    p.theta = J.theta.data();
    p.hk = J.hk.empty() ? nullptr : J.hk.data();
    p.spin0 = J.spin0.empty() ? nullptr : J.spin0.data();
    asi_handle h = nullptr;
    asi_status st = asi_create(&p, &S->cdev, &h);
    if (st == ASI_OK) st = asi_set_field_protocol(h, J.K, J.H.data());
    if (st == ASI_OK && J.loc_k > 0) st = asi_set_local_field(h, J.loc_k, J.loc.data());
    if (st == ASI_OK && !J.sig.empty()) st = asi_set_thermal_schedule(h, J.K, J.sig.data());
    if (st != ASI_OK) {
      if (h) asi_destroy(h);
      J.state = 3;
      J.err = st;
      J.t_done = now_s();
      continue;
    }
    J.h = h;
    J.slot = slot;
    J.state = 1;
    J.t_admit = now_s();
    S->used += J.foot;
    S->slots[slot] = J.id;
    RunDev r{};
    r.t = 0;
    r.t_end = J.K;
    r.active = 1;
    r.hash = 0xcbf29ce484222325ull;
    r.cur_step = -1;
    S->runs[slot] = r;
    S->dirty = true;
    S->stats.admitted++;
  }
  HIPCHK(hipStreamSynchronize(S->cstream), (asi_sim*)nullptr);
  return ASI_OK;
}

}  // namespace

extern "C" {

asi_status asi_server_create(const asi_device* dev, size_t hbm_budget_bytes, int32_t max_slots,
                             asi_server_t* out) {
  if (!out || max_slots < 1 || hbm_budget_bytes == 0) return fail(ASI_EINVAL, "bad server args");
  auto* S = new (std::nothrow) asi_server();
  if (!S) return fail(ASI_ENOMEM, "host allocation failed");
  if (dev) S->dev = *dev;
  if (hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess) {
    delete S;
    return fail(ASI_EDEVICE, "stream creation failed");
  }
  if (hipStreamCreateWithFlags(&S->cstream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipStreamDestroy(S->stream);
    delete S;
    return fail(ASI_EDEVICE, "stream creation failed");
  }
  if (hipHostMalloc((void**)&S->rb, sizeof(RunDev) * max_slots, hipHostMallocDefault) !=
      hipSuccess) {
    (void)hipStreamDestroy(S->cstream);
    (void)hipStreamDestroy(S->stream);
    delete S;
    return fail(ASI_ENOMEM, "pinned host allocation failed");
  }
  S->dev.stream = S->stream;
  S->cdev = S->dev;
  S->cdev.stream = S->cstream;
  S->budget = hbm_budget_bytes;
  S->max_slots = max_slots;
  S->slots.assign(max_slots, -1);
  S->runs.assign(max_slots, RunDev{});
  S->in_burst.assign(max_slots, 0);
  S->T.mem.dev = S->dev;
  S->big_magnets = kBigMagnets;
  S->tail_jobs = kTailJobs;
  S->quiet_scale = kQuietBurstScale;
  if (const char* v = std::getenv("ASI_SERVER_QUIET_SCALE")) {
    const double q = std::atof(v);
    if (q >= 1.0 && q <= 1000.0) S->quiet_scale = q;
  }
  if (const char* v = std::getenv("ASI_SERVER_BIG")) {  // threshold overrides
    const long long b = std::atoll(v);
    if (b >= 1) S->big_magnets = b;
  }
  if (const char* v = std::getenv("ASI_SERVER_TAIL")) {
    const int b = std::atoi(v);
    if (b >= 0) S->tail_jobs = b;
  }
  {
    int dev_id = 0, khz = 0;
    if (hipGetDevice(&dev_id) == hipSuccess &&
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev_id) == hipSuccess &&
        khz > 0)
      S->clock_hz = (int64_t)khz * 1000;
  }
  *out = S;
  return ASI_OK;
}

asi_status asi_server_submit(asi_server_t S, const asi_params* p, int64_t n_steps,
                             const double* h_xy, int64_t* job_id_out) {
  return asi_server_submit_fields(S, p, n_steps, h_xy, 0, nullptr, nullptr, job_id_out);
}

asi_status asi_server_submit_fields(asi_server_t S, const asi_params* p, int64_t n_steps,
                                    const double* h_xy, int64_t loc_slabs, const double* h_loc,
                                    const double* sigma, int64_t* job_id_out) {
  if (!S || !job_id_out) return fail(ASI_EINVAL, "null argument");
  asi_status st = validate(p);
  if (st != ASI_OK) return st;
  if (n_steps < 1 || !h_xy) return fail(ASI_EINVAL, "a job needs a protocol of >= 1 step");
  if (loc_slabs < 0 || (loc_slabs > 1 && loc_slabs != n_steps) || (loc_slabs > 0 && !h_loc))
    return fail(ASI_EINVAL, "bad local field: loc_slabs must be 0, 1 or n_steps");
  for (int64_t k = 0; k < 2 * loc_slabs * p->n; ++k)
    if (!std::isfinite(h_loc[k])) return fail(ASI_EINVAL, "non-finite local field value");
  if (sigma)
    for (int64_t k = 0; k < n_steps; ++k)
      if (!(sigma[k] >= 0.0) || !std::isfinite(sigma[k]))
        return fail(ASI_EINVAL, "thermal schedule values must be finite and >= 0");
  auto J = std::make_unique<Job>();
  if (loc_slabs > 0) J->loc.assign(h_loc, h_loc + 2 * loc_slabs * p->n);
  J->loc_k = loc_slabs;
  if (sigma) J->sig.assign(sigma, sigma + n_steps);
  J->p = *p;
  J->xy.assign(p->xy, p->xy + 2 * p->n);
  J->theta.assign(p->theta, p->theta + p->n);
  if (p->hk) J->hk.assign(p->hk, p->hk + p->n);
  if (p->spin0) J->spin0.assign(p->spin0, p->spin0 + p->n);
  J->H.assign(h_xy, h_xy + 2 * n_steps);
  J->K = n_steps;
  const int64_t log_cap = p->flip_log_capacity > 0 ? p->flip_log_capacity : 4 * p->n + 65536;
  J->foot = footprint_estimate(p->n, degree_bound(p), n_steps, log_cap) +
            (size_t)(16 * loc_slabs * p->n) + (sigma ? (size_t)(8 * n_steps) : 0);
  if (J->foot > S->budget) return fail(ASI_ENOMEM, "job footprint exceeds the server budget");
  J->id = S->next_id++;
  *job_id_out = J->id;
  S->queue.push_back(J->id);
  S->jobs[J->id] = std::move(J);
  return ASI_OK;
}

asi_status asi_server_step(asi_server_t S, double budget_ms, int32_t* active_out) {
  Range range("asi_server_step");
  if (!S) return fail(ASI_EINVAL, "null server");
  if (!(budget_ms > 0.0)) return fail(ASI_EINVAL, "budget_ms must be > 0");
  int32_t resident = 0;
  int64_t max_n = 0;
  bool tail = false, quiet = false;
  double t_end = 0.0;
  for (int32_t k = 0; k < S->max_slots; ++k) {
    S->in_burst[k] = S->slots[k] >= 0;
    if (S->slots[k] >= 0) {
      ++resident;
      max_n = std::max(max_n, S->jobs[S->slots[k]]->p.n);
    }
  }
  // 1. launch a burst over the jobs resident now
  if (resident > 0) {
    if (S->dirty) {
      const double t = now_s();
      asi_status st = server_rebuild(S);
      if (st != ASI_OK) return st;
      S->stats.rebuild_s += now_s() - t;
    }
    // The field launch covers every active job (new jobs' neighbour gathers
    // run grid-wide here) and rebuilds paused relaxes; then each job's
    // workgroup relaxes and goes on through its later steps until the
    // deadline.  In the tail regime the first round is launched here, the
    // others after admission.
    const double t_burst = now_s();
    tail = resident <= S->tail_jobs && max_n >= S->big_magnets;
    quiet = tail && S->queue.empty();
    if (quiet) budget_ms *= S->quiet_scale;
    const int64_t ticks = std::max<int64_t>(1, (int64_t)(budget_ms * 1e-3 * (double)S->clock_hz));
    launch_field(S->T.dI, S->T.dR, S->T.blk_inst, S->T.blk_row0, S->T.nblocks, S->stream);
    if (quiet)
      launch_relax(S->T.dI, S->T.dR, S->T.count, S->T.waves, S->T.lds, S->T.tree_only,
                   S->stream);
    else
      launch_fused(S->T.dI, S->T.dR, S->T.count, S->T.waves, S->T.lds, tail ? 1 : INT64_MAX,
                   ticks, 1, S->stream);
    HIPCHK(hipMemcpyAsync(S->rb, S->T.dR, sizeof(RunDev) * S->max_slots, hipMemcpyDeviceToHost,
                          S->stream),
           (asi_sim*)nullptr);
    t_end = t_burst + budget_ms * 1e-3;
    S->stats.bursts++;
  }
  // 2. admission, while the burst runs
  {
    const double t = now_s();
    asi_status st = server_admit(S);
    S->stats.admit_s += now_s() - t;
    if (st != ASI_OK) return st;
  }
  // 3. burst results: retire finished jobs
  if (resident > 0) {
    double t = now_s();
    HIPCHK(hipStreamSynchronize(S->stream), (asi_sim*)nullptr);
    HIPCHK(hipGetLastError(), (asi_sim*)nullptr);
    // tail regime: one more step of every job per round, each relax allowed
    // to run to the end of the burst's budget
    while (tail) {
      bool more = false;
      for (int32_t k = 0; k < S->max_slots; ++k)
        if (S->in_burst[k] && S->rb[k].active) more = true;
      const double left = t_end - now_s();
      if (!more || left <= 0.0) break;
      const int64_t ticks = std::max<int64_t>(1, (int64_t)(left * (double)S->clock_hz));
      launch_field(S->T.dI, S->T.dR, S->T.blk_inst, S->T.blk_row0, S->T.nblocks, S->stream);
      if (quiet)
        launch_relax(S->T.dI, S->T.dR, S->T.count, S->T.waves, S->T.lds, S->T.tree_only,
                   S->stream);
      else
        launch_fused(S->T.dI, S->T.dR, S->T.count, S->T.waves, S->T.lds, 1, ticks, 1, S->stream);
      HIPCHK(hipMemcpyAsync(S->rb, S->T.dR, sizeof(RunDev) * S->max_slots,
                            hipMemcpyDeviceToHost, S->stream),
             (asi_sim*)nullptr);
      HIPCHK(hipStreamSynchronize(S->stream), (asi_sim*)nullptr);
      HIPCHK(hipGetLastError(), (asi_sim*)nullptr);
    }
    S->stats.wait_s += now_s() - t;
    t = now_s();
    for (int32_t k = 0; k < S->max_slots; ++k) {
      if (!S->in_burst[k]) continue;
      RunDev& r = S->runs[k];
      r = S->rb[k];
      if (r.paused) S->stats.pauses++;
      if (r.active || r.paused) continue;
      Job& J = *S->jobs[S->slots[k]];
      J.flips = r.flips;
      J.hash = r.hash;
      J.spins_out.resize(J.p.n);
      HIPCHK(hipMemcpyAsync(J.spins_out.data(), J.h->hI.s, J.p.n, hipMemcpyDeviceToHost, S->stream),
             (asi_sim*)nullptr);
      HIPCHK(hipStreamSynchronize(S->stream), (asi_sim*)nullptr);
      J.state = r.status == 0 ? 2 : 3;
      J.err = r.status == 0 ? ASI_OK : (r.status == kPoolOverflow ? ASI_EDEVICE : ASI_ELOOP);
      J.t_done = now_s();
      asi_destroy(J.h);
      J.h = nullptr;
      S->used -= J.foot;
      S->slots[k] = -1;
      S->runs[k] = RunDev{};
      S->dirty = true;
      S->stats.retired++;
    }
    S->stats.retire_s += now_s() - t;
  }
  if (active_out) {
    int32_t a = (int32_t)S->queue.size();
    for (int32_t k = 0; k < S->max_slots; ++k) a += S->slots[k] >= 0;
    *active_out = a;
  }
  return ASI_OK;
}

asi_status asi_measure_load_latency(const asi_device* dev, int64_t bytes, int64_t hops,
                                    int32_t lanes, uint64_t seed, double* ns_out) {
  if (!ns_out || hops < 1 || lanes < 1 || lanes > 64 || bytes < 128 * 64 ||
      bytes > ((int64_t)1 << 36))
    return fail(ASI_EINVAL, "need ns_out, hops >= 1, 1 <= lanes <= 64 and 8 KiB <= bytes <= 2^36");
  // one element per 128-byte line, the lines visited in a random cycle
  const int64_t lines = bytes / 128;
  if (lines * 32 > (int64_t)0x7fffffff) return fail(ASI_EINVAL, "buffer too large");
  std::vector<int32_t> order(lines);
  for (int64_t k = 0; k < lines; ++k) order[k] = (int32_t)k;
  uint64_t x = seed * 0x9E3779B97F4A7C15ull + 1;
  for (int64_t k = lines - 1; k > 0; --k) {  // Fisher-Yates with a 64-bit LCG
    x = x * 6364136223846793005ull + 1442695040888963407ull;
    const int64_t r = (int64_t)((x >> 11) % (uint64_t)(k + 1));
    std::swap(order[k], order[r]);
  }
  // start at line 0: rotate the cycle so that it begins there
  const int64_t z = std::find(order.begin(), order.end(), 0) - order.begin();
  std::rotate(order.begin(), order.begin() + z, order.end());
  std::vector<int32_t> chain((size_t)lines * 32, 0);
  for (int64_t k = 0; k < lines; ++k)
    chain[(size_t)order[k] * 32] = order[(k + 1) % lines] * 32;
  // check: one cycle through every line, every target in bounds
  {
    std::vector<char> seen(lines, 0);
    int64_t p = 0;
    for (int64_t k = 0; k < lines; ++k) {
      if (p < 0 || p >= lines * 32 || (p % 32) != 0 || seen[p / 32])
        return fail(ASI_EDEVICE, "pointer chain is not one cycle");
      seen[p / 32] = 1;
      p = chain[(size_t)p];
    }
    if (p != 0) return fail(ASI_EDEVICE, "pointer chain is not one cycle");
  }
  // lane l starts l/64 of the way round the cycle
  std::vector<int32_t> starts(64);
  for (int l = 0; l < 64; ++l) starts[l] = order[(size_t)(l * lines / 64)] * 32;
  DevMem mem;
  if (dev) mem.dev = *dev;
  hipStream_t st = nullptr;
  bool own = false;
  if (dev && dev->stream) {
    st = (hipStream_t)dev->stream;
  } else {
    HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), (asi_sim*)nullptr);
    own = true;
  }
  mem.st = st;
  asi_status rs = ASI_OK;
  int32_t* dchain = static_cast<int32_t*>(mem.alloc(4 * chain.size()));
  int32_t* dstarts = static_cast<int32_t*>(mem.alloc(4 * 64));
  unsigned long long* dout = static_cast<unsigned long long*>(mem.alloc(8 * 65));
  unsigned long long out[65] = {0};
  hipError_t e = (dchain && dstarts && dout) ? hipSuccess : hipErrorOutOfMemory;
  if (e == hipSuccess)
    e = hipMemcpyAsync(dchain, chain.data(), 4 * chain.size(), hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dstarts, starts.data(), 4 * 64, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) {
    // A first pass warms the address translations: the whole cycle for a
    // buffer of at most 64 MiB (which then sits in the caches), else `hops`
    // steps per lane.  The timed pass continues from where each lane's first
    // pass stopped, so in a large buffer every timed load is to a line not
    // touched before (far beyond the last-level cache: an HBM access).
    const int64_t warm = bytes <= ((int64_t)64 << 20) ? lines : std::min<int64_t>(hops, lines);
    launch_chase(dchain, dstarts, lanes, warm, dout, st);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(out, dout, 8 * 65, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess) {
    for (int l = 0; l < lanes; ++l) {
      const unsigned long long q = out[1 + l];
      if (q >= (unsigned long long)(lines * 32) || (q % 32) != 0) {
        e = hipErrorUnknown;  // cannot happen: every index in the cycle is in bounds
        break;
      }
      starts[l] = (int32_t)q;
    }
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(dstarts, starts.data(), 4 * 64, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) {
    launch_chase(dchain, dstarts, lanes, hops, dout, st);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(out, dout, 8 * 65, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  int dev_id = 0, khz = 0;
  if (e == hipSuccess) e = hipGetDevice(&dev_id);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev_id);
  if (e == hipErrorOutOfMemory && !(dchain && dstarts && dout))
    rs = fail(ASI_ENOMEM, "device allocation failed (pointer chase)");
  else if (e != hipSuccess)
    rs = fail(ASI_EDEVICE, std::string("pointer chase: ") + hipGetErrorString(e));
  else if (khz <= 0)
    rs = fail(ASI_EDEVICE, "device clock rate unknown");
  else
    *ns_out = (double)out[0] / ((double)khz * 1e3) * 1e9 / (double)hops;
  (void)hipStreamSynchronize(st);
  mem.release_all();
  if (own) (void)hipStreamDestroy(st);
  return rs;
}

asi_status asi_server_get_stats(asi_server_t S, asi_server_stats* out) {
  if (!S || !out) return fail(ASI_EINVAL, "null argument");
  *out = S->stats;
  return ASI_OK;
}

asi_status asi_server_poll(asi_server_t S, int64_t job_id, int32_t* done_out) {
  if (!S || !done_out) return fail(ASI_EINVAL, "null argument");
  auto it = S->jobs.find(job_id);
  if (it == S->jobs.end()) return fail(ASI_EINVAL, "unknown job");
  *done_out = it->second->state >= 2 ? 1 : 0;
  return ASI_OK;
}

asi_status asi_server_take(asi_server_t S, int64_t job_id, int8_t* spins, int64_t* flips,
                           uint64_t* flip_hash, double* t_admit, double* t_done) {
  if (!S) return fail(ASI_EINVAL, "null server");
  auto it = S->jobs.find(job_id);
  if (it == S->jobs.end()) return fail(ASI_EINVAL, "unknown job");
  Job& J = *it->second;
  if (J.state < 2) return fail(ASI_EBUSY, "job not finished");
  asi_status err = J.err;
  if (spins && !J.spins_out.empty()) std::memcpy(spins, J.spins_out.data(), J.p.n);
  if (flips) *flips = J.flips;
  if (flip_hash) *flip_hash = J.hash;
  if (t_admit) *t_admit = J.t_admit;
  if (t_done) *t_done = J.t_done;
  S->jobs.erase(it);
  if (err != ASI_OK) return fail(err, "job failed");
  return ASI_OK;
}

asi_status asi_server_destroy(asi_server_t S) {
  if (!S) return ASI_OK;
  (void)hipStreamSynchronize(S->stream);
  for (auto& kv : S->jobs)
    if (kv.second->h) asi_destroy(kv.second->h);
  S->jobs.clear();
  S->T.drop_graph();
  S->T.mem.release_all();
  if (S->rb) (void)hipHostFree(S->rb);
  (void)hipStreamDestroy(S->cstream);
  (void)hipStreamDestroy(S->stream);
  delete S;
  return ASI_OK;
}

}  // extern "C"
