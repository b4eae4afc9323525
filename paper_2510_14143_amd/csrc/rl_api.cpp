// C-ABI layer of the Richardson-Lucy library: argument validation, plan
// (workspace, transfer function, radix schedules, launch shapes) and the pass
// sequences of rl_iterate and conv3d_fft.  The declarations and their
// contracts are in include/rl.h.
#include <rocprofiler-sdk-roctx/roctx.h>
#include "../../include/rl.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <new>
#include <string>
#include <unordered_set>
#include <vector>

#include "rl_internal.h"

using rlmi::PencilArgs;
using rlmi::Sched;
using rlmi::XArgs;

namespace {

constexpr uint64_t kMagic = 0x31504c4d494c52ull;  // live plan
constexpr uint64_t kDead = 0xdeadbeefdeadbeefull;
constexpr int64_t kMaxNx = 4096;
constexpr int64_t kMaxNyz = 4096;
constexpr size_t kMaxLds = 65536;        // X pass work-group LDS budget
constexpr size_t kMaxPencilLds = 163840;  // gfx950: 160 KB per work-group
constexpr int kStatBlocks = 256;

thread_local std::string g_err;

// Live plans.  Handles are checked against this set, never dereferenced
// first, so a destroyed or foreign handle is reported instead of touched.
std::mutex g_plans_mu;
std::unordered_set<const void*>& live_plans() {
  static std::unordered_set<const void*> s;
  return s;
}
bool plan_is_live(const void* p) {
  std::lock_guard<std::mutex> g(g_plans_mu);
  return live_plans().count(p) != 0;
}
void plan_register(const void* p) {
  std::lock_guard<std::mutex> g(g_plans_mu);
  live_plans().insert(p);
}
bool plan_unregister(const void* p) {
  std::lock_guard<std::mutex> g(g_plans_mu);
  return live_plans().erase(p) != 0;
}

rl_status fail(rl_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

rl_status hip_fail(hipError_t e, const char* what) {
  const char* name = hipGetErrorString(e);
  (void)hipGetLastError();  // clear sticky launch error state where possible
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
    return fail(RL_E_NOMEM, std::string(what) + ": " + (name ? name : "?"));
  return fail(RL_E_DEVICE, std::string(what) + ": " + (name ? name : "?"));
}

bool sync_debug_on();

// Result of a kernel launch on `stream`; with RLMI_SYNC_DEBUG=1 (and the stream
// not under graph capture) the stream is synchronised and an execution fault is
// reported against this launch.
rl_status launched(hipError_t e, hipStream_t stream, const char* what) {
  if (e != hipSuccess) return hip_fail(e, (std::string(what) + " launch").c_str());
  if (!sync_debug_on()) return RL_OK;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
    return RL_OK;
  if ((e = hipStreamSynchronize(stream)) != hipSuccess)
    return hip_fail(e, (std::string("execution of ") + what + " (RLMI_SYNC_DEBUG)").c_str());
  return RL_OK;
}

// Environment switches, read once per process: RLMI_SYNC_DEBUG=1 synchronises the
// plan's stream after every kernel launch outside graph capture and reports an
// execution fault against the launch that caused it; RLMI_AUTOTUNE=1 / 0 turns
// the autotuner on / off for every plan, whatever its options ask.
int env_flag(const char* name) {
  const char* v = std::getenv(name);
  if (!v || !*v) return -1;
  return std::strcmp(v, "0") == 0 ? 0 : 1;
}

bool sync_debug_on() {
  static const bool on = env_flag("RLMI_SYNC_DEBUG") == 1;
  return on;
}

int autotune_override() {
  static const int v = env_flag("RLMI_AUTOTUNE");
  return v;
}

bool is_pow2(int64_t v) { return v >= 1 && (v & (v - 1)) == 0; }

// A thread holds E elements of its transform, E carrying every odd factor of the
// length, so the odd part of a length is limited to what fits in E <= 30:
// lengths o * 2^a with o in {1, 3, 5, 7, 9, 15} (radices 16, 8, 4, 2, 3, 5, 7).
int64_t odd_part(int64_t v) {
  while (v > 0 && v % 2 == 0) v /= 2;
  return v;
}

int64_t pow2_part(int64_t v) { return v & -v; }

bool length_ok(int64_t L) {
  if (L < 1) return false;
  const int64_t o = odd_part(L);
  return o == 1 || o == 3 || o == 5 || o == 7 || o == 9 || o == 15;
}

// Elements-per-thread values the kernels are built for (ascending).
constexpr int kE[] = {1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 12, 14, 15, 16, 18, 20, 24, 30};

// Radices of the schedule for length L with E elements per thread: the largest
// power-of-two radix dividing E first, then the power-of-two remainder, then the
// odd radices 7, 5, 3 (3 last).
std::vector<int> radices(int64_t L, int E) {
  int64_t n = L;
  std::vector<int> odd;
  for (int r : {7, 5, 3})
    while (n % r == 0) {
      n /= r;
      odd.push_back(r);
    }
  int big = 1;
  for (int r : {16, 8, 4, 2})
    if (E % r == 0) {
      big = r;
      break;
    }
  std::vector<int> rads;
  while (n > 1) {
    int r = big;
    while (r > 1 && n % r) r /= 2;
    if (r == 1) break;  // E without a factor 2 for an even length: rejected by e_ok
    rads.push_back(r);
    n /= r;
  }
  for (int r : odd) rads.push_back(r);
  return rads;
}

// A caller-chosen E for length L: divides L into a power-of-two thread count
// <= max_p, carries every odd factor of L, and leaves radices the schedule can use.
bool e_ok(int64_t L, int E, int64_t max_p) {
  bool known = false;
  for (int k : kE) known = known || (k == E);
  if (!known || L % E != 0) return false;
  const int64_t P = L / E;
  if (!is_pow2(P) || P > max_p) return false;
  if (odd_part(E) != odd_part(L)) return false;
  const int64_t l2 = pow2_part(L);
  if (l2 != 1 && pow2_part(E) < 2) return false;
  return radices(L, E).size() <= (size_t)rlmi::kMaxStages;
}

// Largest E = odd part * 2^j of L with E <= cap (and at least one factor 2 when L
// is even); 0 if none.
int e_with_cap(int64_t L, int cap) {
  const int64_t o = odd_part(L);
  int best = 0;
  for (int E : kE)
    if (E <= cap && E > best && odd_part(E) == o && L % E == 0 &&
        (pow2_part(L) == 1 || pow2_part(E) >= 2) &&
        radices(L, E).size() <= (size_t)rlmi::kMaxStages)
      best = E;
  return best;
}

// Y and Z pencils (a work-group per group of pencils, any thread count): where no
// E carries the whole odd part of L (odd parts 27, 45, 135, ...; e.g. 2160 =
// 16 * 135), E only needs every odd prime of L, so that each radix-3/5/7 stage
// still takes its R inputs from one thread's registers; the thread count P = L/E
// then carries the remaining odd factor.
bool strict_e_exists(int64_t L, int64_t max_p) {
  for (int E : kE)
    if (e_ok(L, E, max_p)) return true;
  return false;
}

bool e_ok_relaxed(int64_t L, int E, int64_t max_p) {
  bool known = false;
  for (int k : kE) known = known || (k == E);
  if (!known || L < 1 || L % E != 0 || L / E > max_p) return false;
  int64_t o = odd_part(L);
  for (int r : {3, 5, 7}) {
    if (o % r == 0 && E % r != 0) return false;
    while (o % r == 0) o /= r;
  }
  if (o != 1) return false;  // a prime the radix stages do not have
  if (pow2_part(L) != 1 && pow2_part(E) < 2) return false;
  return radices(L, E).size() <= (size_t)rlmi::kMaxStages;
}

bool e_ok_yz(int64_t L, int E, int64_t max_p) {
  return strict_e_exists(L, max_p) ? e_ok(L, E, max_p) : e_ok_relaxed(L, E, max_p);
}

int pick_e(int64_t L) {
  if (L == 1) return 1;
  if (is_pow2(L)) return (int)(L < 16 ? L : 16);
  int e = e_with_cap(L, 24);
  if (e == 0) e = e_with_cap(L, 30);
  if (e == 0)  // relaxed pencil rule: the largest E that applies
    for (int E : kE)
      if (e_ok_relaxed(L, E, 1 << 20) && E > e) e = E;
  return e;
}

// X pass: few elements per thread so that one row fills (up to) a wavefront;
// the many short-lived waves hide the latency of the fused two-transform pass.
int pick_e_x(int64_t M) {
  if (is_pow2(M)) {
    if (M <= 4) return (int)M;
    return (int)(M / 4 <= 64 ? 4 : M / 64);
  }
  // the smallest valid E >= 2 * odd part with at most 64 threads per row, else
  // the largest valid E
  const int64_t o = odd_part(M);
  int best_ge = 0, best_any = 0;
  for (int E : kE)
    if (e_ok(M, E, 64)) {
      if (E >= 2 * o && best_ge == 0) best_ge = E;
      best_any = E;
    }
  return best_ge > 0 ? best_ge : best_any > 0 ? best_any : pick_e(M);
}

// Split precision: 16 elements per thread (radix-16 stages) when the length is a
// power of two >= 16 with at most max_p threads per transform; else 0 (default).
int split_e(int64_t L, int64_t max_p) {
  return (is_pow2(L) && L >= 16 && L / 16 <= max_p) ? 16 : 0;
}

// Y pass: 8 elements per thread for power-of-two lengths up to 512.
int pick_e_y(int64_t L) {
  if (is_pow2(L) && L >= 8 && L <= 512) return 8;
  return pick_e(L);
}

// Radix schedule of radices(L, E); ns = 0 if it has more than kMaxStages stages
// (callers validate E with e_ok first).
Sched make_sched(int64_t L, int E, int table_stride) {
  Sched sc;
  std::memset(&sc, 0, sizeof(sc));
  const std::vector<int> rads = radices(L, E);
  if (rads.size() > (size_t)rlmi::kMaxStages) return sc;
  int64_t p = 1;
  sc.ns = (int)rads.size();
  for (int s = 0; s < sc.ns; ++s) {
    sc.r[s] = rads[s];
    sc.p[s] = (int)p;
    sc.tm[s] = (int)(table_stride * (L / (p * rads[s])));
    p *= rads[s];
  }
  return sc;
}

struct Axis {
  int64_t L = 1;
  int E = 1;
  int P = 1;
  Sched sc{};
};

struct Pencil {
  Axis ax;
  size_t lds = 0;
  dim3 grid, block;
  PencilArgs args{};
};

struct TimedLaunch {
  int kind;
  hipEvent_t a, b;
};

}  // namespace

struct rl_plan_s {
  uint64_t magic = kMagic;
  int device = 0;
  hipStream_t stream = nullptr;
  int64_t nz = 0, ny = 0, nx = 0;
  int64_t M = 0, ncols = 0, xt = 0, nvox = 0, nrows = 0;  // transform grid
  // the caller's volumes (vz, vy, vx) at the grid's low corner, and the PSF shape
  int64_t vz = 0, vy = 0, vx = 0, vnvox = 0;
  int64_t psf_z = 0, psf_y = 0, psf_x = 0;
  int boundary = RL_BOUNDARY_PERIODIC;
  size_t spec_elems = 0;
  float2* spec = nullptr;
  float2* otf = nullptr;
  float2* tw_x = nullptr;
  float2* tw_y = nullptr;
  float2* tw_z = nullptr;
  double* partials = nullptr;
  size_t n_partials = 0;
  unsigned* counter = nullptr;
  double* stats = nullptr;
  double* flux = nullptr;
  int flux_cap = 0;
  int flux_count = 0;
  // X pass
  Axis axx;
  int x_rpw = 1, x_rs = 0;
  size_t x_lds = 0;
  dim3 x_grid, x_block;
  // Y and Z passes
  Pencil py, pz;
  int precision = RL_PRECISION_FP32;
  // extrapolated iteration (single-volume plans)
  int accel = RL_ACCEL_NONE;
  float* hstep = nullptr;         // last step x_k - x_{k-1}
  float* gchg = nullptr;          // last change x_k - y_{k-1}
  float* alpha32 = nullptr;       // alpha per iteration (flux_cap + 1 entries)
  double* alpha64 = nullptr;
  double* acc_partials = nullptr; // [2][X work-groups]
  // metric-guided stopping (single-volume plans)
  int* stop = nullptr;            // [0] stopped, [1] iterations carried out, [2] metric entries
  double* met_partials = nullptr; // [kMetRows][X work-groups]
  double* mhist = nullptr;        // metric per check (flux_cap + 1 entries)
  bool stop_call = false;         // the last iterate call used a stop rule
  int stop_max = 0;               // its max_iter
  const int* active_stop = nullptr;  // passed to every launch while a stop call is enqueued
  // Fourier shell correlation (allocated on first use)
  float2* spec2 = nullptr;        // second spectrum
  double* fsc_part = nullptr;     // shell partials, fsc_cap shells
  double* fsc_out = nullptr;
  int fsc_cap = 0;
  // FSC-guided stopping (allocated on first use): transform-only plan of the half
  // shape, which owns the two half-size sub-volumes and the FSC buffers
  rl_plan fsc_sub = nullptr;
  float* fsc_a = nullptr;
  float* fsc_b = nullptr;
  // structural similarity (allocated on first use)
  double* ssim_a = nullptr;       // X window sums, 5 channels
  double* ssim_b = nullptr;       // X and Y window sums
  double* ssim_part = nullptr;    // per-work-group sums of window SSIMs
  double* ssim_range = nullptr;   // [0] range of the reference, then range partials
  // batched volumes of this shape (a class of a batch plan); 1 for a single plan
  int count = 1;
  const float** d_tab = nullptr;  // device tables of per-volume pointers (count each)
  float** u_tab = nullptr;
  int* iter_dev = nullptr;        // device iteration index for graph replays
  // batch container (is_batch): classes of equal shape, input-order mapping
  bool is_batch = false;
  std::vector<rl_plan> classes;
  std::vector<int> vol_class, vol_index;
  std::vector<hipStream_t> cls_streams;
  std::vector<hipEvent_t> cls_events;
  hipEvent_t fork_event = nullptr;
  hipStream_t cap_stream = nullptr;  // private stream the iteration graphs are captured on
  hipGraphExec_t graph_full = nullptr, graph_last = nullptr;
  int batch_n = 0;                // iterations of the last rl_iterate_batch call
  // persistent batched iteration (batch container): one k_persist launch per
  // iteration; [0] = every pass, [1] = the last iteration (no forward chain)
  bool persist = false;
  bool persist_shapes = false;    // class plan: launch shapes of the persistent kernel's work-groups
  rlmi::PersistClass* p_cls = nullptr;
  std::vector<rlmi::PersistClass> p_host;  // host copy of p_cls
  std::vector<int> p_qtotal[2];            // tickets per queue and launch
  rlmi::PersistSeg* p_segs[2] = {nullptr, nullptr};
  int* p_qseg[2] = {nullptr, nullptr};
  int p_nq = 0, p_grid = 0, p_nvrow = 0, p_cap = 0;
  size_t p_lds = 0;
  int* p_tickets = nullptr;       // [iteration][queue]
  int* p_done = nullptr;          // [iteration][volume][pass]
  int* p_error = nullptr;
  // applied launch choice (elements per thread and work-group widths)
  int ch_x_e = 0, ch_y_e = 0, ch_y_txb = 0, ch_z_e = 0, ch_z_txb = 0, ch_z_swap = 0;
  bool tuned = false;
  // timing
  bool timing = false;
  std::vector<TimedLaunch> events;
  size_t n_events = 0;
};

namespace {

rl_status check_plan(rl_plan p) {
  if (!p) return fail(RL_E_INVALID, "plan is NULL");
  if (!plan_is_live(p) || p->magic != kMagic)
    return fail(RL_E_INVALID, "plan handle is not a live plan");
  return RL_OK;
}

rl_status check_shape(const int64_t* shape) {
  if (!shape) return fail(RL_E_INVALID, "shape is NULL");
  for (int i = 0; i < 3; ++i)
    if (shape[i] < 1) return fail(RL_E_INVALID, "every dimension must be >= 1");
  const int64_t nz = shape[0], ny = shape[1], nx = shape[2];
  if (nx % 2 != 0 || nx < 4)
    return fail(RL_E_UNSUPPORTED, "nx must be even and >= 4");
  auto has_e = [](int64_t L, int64_t max_p) {
    for (int E : kE)
      if (e_ok(L, E, max_p)) return true;
    return false;
  };
  static const char* kLens = "o * 2^a with o in {1, 3, 5, 7, 9, 15}";
  if (!length_ok(nx / 2) || nx > kMaxNx || !has_e(nx / 2, 64))
    return fail(RL_E_UNSUPPORTED, std::string("nx/2 must be ") + kLens +
                                      ", nx <= 4096, split over at most 64 threads");
  auto has_e_yz = [](int64_t L) {
    for (int E : kE)
      if (e_ok_yz(L, E, 1024)) return true;
    return false;
  };
  static const char* kLensYz =
      " must be 2^a 3^b 5^c 7^d <= 4096 with an elements-per-thread count that every odd "
      "prime divides (at most 8 radix stages)";
  if (ny > kMaxNyz || !has_e_yz(ny)) return fail(RL_E_UNSUPPORTED, std::string("ny") + kLensYz);
  if (nz > kMaxNyz || !has_e_yz(nz)) return fail(RL_E_UNSUPPORTED, std::string("nz") + kLensYz);
  return RL_OK;
}

// A data pointer must be a 16-byte aligned device allocation on `device`
// (or on any device if *device < 0) that covers `bytes` from `ptr`.
rl_status check_dev_ptr(const void* ptr, size_t bytes, int* device, const char* name) {
  if (!ptr) return fail(RL_E_INVALID, std::string(name) + " is NULL");
  if (reinterpret_cast<uintptr_t>(ptr) % 16 != 0)
    return fail(RL_E_INVALID, std::string(name) + " is not 16-byte aligned");
  hipPointerAttribute_t attr;
  std::memset(&attr, 0, sizeof(attr));
  hipError_t e = hipPointerGetAttributes(&attr, ptr);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(RL_E_INVALID, std::string(name) + " is not a device pointer");
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
    return fail(RL_E_INVALID, std::string(name) + " is not device memory");
  if (*device >= 0 && attr.device != *device)
    return fail(RL_E_INVALID, std::string(name) + " lives on another device than the plan");
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  e = hipMemGetAddressRange(&base, &size, const_cast<void*>(ptr));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(RL_E_INVALID, std::string(name) + ": cannot query its allocation");
  }
  const char* b = reinterpret_cast<const char*>(base);
  const char* q = reinterpret_cast<const char*>(ptr);
  if (q < b || (size_t)(q - b) + bytes > size)
    return fail(RL_E_INVALID, std::string(name) + " is smaller than the volume");
  *device = attr.device;
  return RL_OK;
}

void release(rl_plan p) {
  if (!p) return;
  (void)hipSetDevice(p->device);
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  else (void)hipDeviceSynchronize();
  for (auto& t : p->events) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  (void)hipFree(p->spec);
  (void)hipFree(p->otf);
  (void)hipFree(p->tw_x);
  (void)hipFree(p->tw_y);
  (void)hipFree(p->tw_z);
  (void)hipFree(p->partials);
  (void)hipFree(p->counter);
  (void)hipFree(p->stats);
  (void)hipFree(p->flux);
  (void)hipFree(p->iter_dev);
  (void)hipFree(p->d_tab);
  (void)hipFree(p->u_tab);
  (void)hipFree(p->hstep);
  (void)hipFree(p->gchg);
  (void)hipFree(p->alpha32);
  (void)hipFree(p->alpha64);
  (void)hipFree(p->acc_partials);
  (void)hipFree(p->stop);
  (void)hipFree(p->met_partials);
  (void)hipFree(p->mhist);
  (void)hipFree(p->spec2);
  (void)hipFree(p->fsc_part);
  (void)hipFree(p->fsc_out);
  (void)hipFree(p->ssim_a);
  (void)hipFree(p->ssim_b);
  (void)hipFree(p->ssim_part);
  (void)hipFree(p->ssim_range);
  (void)hipFree(p->fsc_a);
  (void)hipFree(p->fsc_b);
  if (p->fsc_sub) release(p->fsc_sub);
  (void)hipFree(p->p_cls);
  for (int k = 0; k < 2; ++k) {
    (void)hipFree(p->p_segs[k]);
    (void)hipFree(p->p_qseg[k]);
  }
  (void)hipFree(p->p_tickets);
  (void)hipFree(p->p_done);
  (void)hipFree(p->p_error);
  for (rl_plan c : p->classes) release(c);
  if (p->graph_full) (void)hipGraphExecDestroy(p->graph_full);
  if (p->graph_last) (void)hipGraphExecDestroy(p->graph_last);
  for (hipEvent_t ev : p->cls_events) (void)hipEventDestroy(ev);
  if (p->fork_event) (void)hipEventDestroy(p->fork_event);
  for (hipStream_t cs : p->cls_streams) (void)hipStreamDestroy(cs);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  p->magic = kDead;
  delete p;
}

// Work-group thread bound of the pencil kernels of E elements per thread (and, for
// the compile-time pencil kernels, length L).
int max_threads_for(int E, int64_t L = 0) {
  if (E == 8 || E == 16) return 1024;
  const int ct = rlmi::pencil_ct_max_threads(E, (int)L);
  return rlmi::pencil_compiled_len(E, (int)L, ct) > 0 ? ct : rlmi::kPencilMaxThreads;
}

Axis make_axis(int64_t L, int e = 0) {
  Axis ax;
  ax.L = L;
  ax.E = e > 0 ? e : pick_e(L);
  ax.P = (int)(L / ax.E);
  ax.sc = make_sched(L, ax.E, 1);
  return ax;
}

void finish_pencil(Pencil& pc, int txb) {
  pc.args.L = (int)pc.ax.L;
  pc.args.P = pc.ax.P;
  pc.args.TXB = txb;
  pc.args.TXP = txb;
  pc.args.lin = pc.args.lout = (int)pc.ax.L;
  // exchange buffer (L x TXP) followed by the twiddle table (L); the kernel
  // places the table at offset L * TXP whether or not the exchange is used
  pc.lds = (size_t)pc.ax.L * (txb + 1) * sizeof(float2);
  pc.block = dim3((unsigned)(txb * pc.ax.P));
}

int pow2_floor(int v) {
  int r = 1;
  while (r * 2 <= v) r *= 2;
  return r;
}

bool pencil_fits(const Pencil& pc) {
  return (int)pc.block.x <= max_threads_for(pc.ax.E, pc.ax.L) && pc.lds <= kMaxPencilLds;
}

// Y pass: one work-group per (tile column, z); lanes = `req` (a power of two
// <= 16; 0 = 16) columns of the tile, halved until the work-group fits.
Pencil make_pencil_y(int64_t ny, int64_t nz, int64_t xt, int64_t ncols, int req, int e,
                     int maxt_cap = 1024) {
  Pencil pc;
  pc.ax = make_axis(ny, e);
  const int maxt = std::min(max_threads_for(pc.ax.E, pc.ax.L), maxt_cap);
  int txb = req > 0 ? pow2_floor(req < rlmi::kTile ? req : rlmi::kTile) : rlmi::kTile;
  while (txb > 1 && ((int64_t)txb * pc.ax.P > maxt ||
                     (size_t)ny * (txb + 1) * sizeof(float2) > kMaxPencilLds))
    txb >>= 1;
  finish_pencil(pc, txb);
  pc.args.xsplit = rlmi::kTile / txb;
  pc.args.ncols = (int)ncols;
  pc.args.xstride = ny * rlmi::kTile;
  pc.args.ostride = xt * ny * rlmi::kTile;
  pc.args.estride = rlmi::kTile;
  pc.grid = dim3((unsigned)(xt * pc.args.xsplit), (unsigned)nz);
  return pc;
}

// Z pass: one work-group per (tile column, group of ty rows); lanes = 16 * ty
// consecutive elements (ty whole tile rows), so each z step reads 128 * ty
// bytes.  `req` = requested lanes (a power of two <= 64; 0 = 32); ty must divide
// ny; the width is halved until the work-group fits.
Pencil make_pencil_z(int64_t nz, int64_t ny, int64_t xt, int64_t ncols, int req, int e,
                     int maxt_cap = 1024) {
  Pencil pc;
  pc.ax = make_axis(nz, e);
  const int maxt = std::min(max_threads_for(pc.ax.E, pc.ax.L), maxt_cap);
  auto fits = [&](int txb) {
    if (txb >= rlmi::kTile && ny % (txb / rlmi::kTile) != 0) return false;
    return (int64_t)txb * pc.ax.P <= maxt &&
           (size_t)nz * (txb + 1) * sizeof(float2) <= kMaxPencilLds;
  };
  int txb = req > 0 ? pow2_floor(req < 4 * rlmi::kTile ? req : 4 * rlmi::kTile) : 2 * rlmi::kTile;
  while (txb > 1 && !fits(txb)) txb >>= 1;
  finish_pencil(pc, txb);
  pc.args.ncols = (int)ncols;
  pc.args.xstride = ny * rlmi::kTile;
  pc.args.estride = xt * ny * rlmi::kTile;
  if (txb >= rlmi::kTile) {
    const int ty = txb / rlmi::kTile;
    pc.args.xsplit = 1;
    pc.args.ostride = (int64_t)ty * rlmi::kTile;
    pc.grid = dim3((unsigned)xt, (unsigned)(ny / ty));
  } else {
    pc.args.xsplit = rlmi::kTile / txb;
    pc.args.ostride = rlmi::kTile;
    pc.grid = dim3((unsigned)(xt * pc.args.xsplit), (unsigned)ny);
  }
  return pc;
}

// --- launches (optionally bracketed by timing events) -----------------------

// With timing enabled, hands out the event pair the next launch passes to its
// dispatch (start and end stamped by the kernel itself); else both are null.
rl_status timed_begin(rl_plan p, int kind, size_t* slot, hipEvent_t* ev0, hipEvent_t* ev1) {
  *ev0 = *ev1 = nullptr;
  if (!p->timing) return RL_OK;
  if (p->n_events == p->events.size()) {
    TimedLaunch t{kind, nullptr, nullptr};
    if (hipEventCreate(&t.a) != hipSuccess || hipEventCreate(&t.b) != hipSuccess)
      return hip_fail(hipGetLastError(), "hipEventCreate");
    p->events.push_back(t);
  }
  *slot = p->n_events++;
  p->events[*slot].kind = kind;
  *ev0 = p->events[*slot].a;
  *ev1 = p->events[*slot].b;
  return RL_OK;
}

// One pencil pass over `nvol` consecutive volumes starting at `data` (and at
// the plan's OTF for the filtered modes); nvol = 0 means all of the plan's.
// lin / lout > 0: only pencil elements below them are read / written; outer > 0:
// only that many outer blocks (Y pass: z planes) are launched.
rl_status run_pencil(rl_plan p, const Pencil& pc, int mode, float2* data, const float2* tw,
                     int kind, int nvol = 0, int lin = 0, int lout = 0, int outer = 0) {
  if (pc.ax.L == 1 && (mode == rlmi::PM_FWD || mode == rlmi::PM_INV)) return RL_OK;  // identity
  size_t slot = 0;
  hipEvent_t ev0, ev1;
  rl_status st = timed_begin(p, kind, &slot, &ev0, &ev1);
  if (st != RL_OK) return st;
  dim3 grid = pc.grid;
  grid.z = (unsigned)(nvol > 0 ? nvol : p->count);
  PencilArgs args = pc.args;
  if (lin > 0) args.lin = lin;
  if (lout > 0) args.lout = lout;
  if (outer > 0) (args.swap ? grid.x : grid.y) = (unsigned)outer;
  args.vstride = (long long)p->spec_elems;
  args.stop = p->active_stop;
  hipError_t e = rlmi::launch_pencil(mode, pc.ax.E, p->precision, grid, pc.block, pc.lds,
                                     p->stream, data, p->otf, tw, args, pc.ax.sc, ev0, ev1);
  return launched(e, p->stream, "pencil pass");
}

// Grid rows the X passes cover: the planes of the caller's volume.
int64_t x_rows(rl_plan p) { return p->vz * p->ny; }

XArgs base_xargs(rl_plan p, float2* spec) {
  XArgs a;
  std::memset(&a, 0, sizeof(a));
  a.spec = spec;
  a.zstride = p->xt * p->ny * rlmi::kTile;
  a.tstride = p->ny * rlmi::kTile;
  a.ny = (int)p->ny;
  a.vx = (int)p->vx;
  a.vy = (int)p->vy;
  a.vz = (int)p->vz;
  a.rin_stride = p->vx;
  a.rout_stride = p->vx;
  a.M = (int)p->M;
  a.P = p->axx.P;
  a.RPW = p->x_rpw;
  a.RS = p->x_rs;
  a.nrows = (int)x_rows(p);
  a.nvol = p->count;
  a.stop = p->active_stop;
  a.vstride = (long long)p->spec_elems;
  return a;
}

// rows > 0: cover that many grid rows instead of the volume's.
rl_status run_x(rl_plan p, int mode, const XArgs& a, int kind, int64_t rows = 0) {
  size_t slot = 0;
  hipEvent_t ev0, ev1;
  rl_status st = timed_begin(p, kind, &slot, &ev0, &ev1);
  if (st != RL_OK) return st;
  dim3 grid = p->x_grid;
  if (rows > 0) grid.x = (unsigned)((rows + p->x_rpw - 1) / p->x_rpw);
  grid.y = (unsigned)a.nvol;
  hipError_t e = rlmi::launch_xrow(mode, p->axx.E, p->precision, grid, p->x_block, p->x_lds,
                                   p->stream, a, p->axx.sc, p->tw_x, ev0, ev1);
  return launched(e, p->stream, "X pass");
}

// spectrum (X-transformed) -> spectrum (X-transformed) of H x or H^T x:
// Y forward, Z forward * (conj) OTF * Z inverse, Y inverse.
// With the zero boundary only the caller's volume (vz planes, vy rows) of the
// grid holds data between passes: the forward Y pass reads vy rows of vz planes,
// the Z pass reads and writes vz planes, the inverse Y pass writes vy rows; the
// rest of the grid is read as zero and never written.
rl_status run_y_fwd(rl_plan p) {
  return run_pencil(p, p->py, rlmi::PM_FWD, p->spec, p->tw_y, RL_KERNEL_Y, 0, (int)p->vy, 0,
                    (int)p->vz);
}

rl_status run_yz_filter(rl_plan p, bool adjoint) {
  rl_status st;
  if ((st = run_y_fwd(p)) != RL_OK) return st;
  if ((st = run_pencil(p, p->pz, adjoint ? rlmi::PM_FCKI : rlmi::PM_FKI, p->spec, p->tw_z,
                       RL_KERNEL_Z_OTF, 0, (int)p->vz, (int)p->vz)) != RL_OK)
    return st;
  return run_pencil(p, p->py, rlmi::PM_INV, p->spec, p->tw_y, RL_KERNEL_Y, 0, 0, (int)p->vy,
                    (int)p->vz);
}

// Launch choice: elements per thread and lane widths per pass (0 = default).
struct Choice {
  int x_e = 0, y_e = 0, y_txb = 0, z_e = 0, z_txb = 0, z_swap = 0;
};

// X pass shape for E = x_e: each wavefront owns 64 / P whole rows, up to
// kXMaxThreads / 64 waves per work-group.
bool configure_x(rl_plan p, int x_e) {
  Axis ax = make_axis(p->M, x_e > 0 ? x_e : pick_e_x(p->M));
  ax.sc = make_sched(p->M, ax.E, 2);
  if (ax.P > 64 || 64 % ax.P != 0) return false;
  const int rows_per_wave = 64 / ax.P;
  const int rs = (int)(p->M + 1 + ((p->M + 1) >> rlmi::kXPad) + 1);  // padded row
  // split-precision stages (E = 16) stage 16-byte granules in each wave's rows:
  // keep them aligned; they add the static MFMA operand table to the LDS
  const bool mfma = p->precision != RL_PRECISION_FP32 && ax.E == 16;
  if (mfma && (rows_per_wave * rs) % 2 != 0) return false;
  const size_t fixed = mfma ? rlmi::kSplitTabBytes : 0;
  auto lds_for = [&](int w) {
    return (size_t)(2 * p->M + (int64_t)w * rows_per_wave * rs) * sizeof(float2) + fixed;
  };
  // persistent batch classes: work-groups of the persistent kernel's size
  int waves = p->persist_shapes ? rlmi::kPersistThreads / 64 : rlmi::kXMaxThreads / 64;
  while (waves > 1 && lds_for(waves) > kMaxLds) waves >>= 1;
  if (lds_for(waves) > kMaxLds) return false;
  p->axx = ax;
  p->x_rs = rs;
  p->x_rpw = waves * rows_per_wave;
  p->x_lds = lds_for(waves) - fixed;  // dynamic part
  p->x_block = dim3((unsigned)(64 * waves));
  p->x_grid = dim3((unsigned)((x_rows(p) + p->x_rpw - 1) / p->x_rpw));
  p->ch_x_e = ax.E;
  return true;
}

// Split-precision work-groups stay at <= 512 threads (their register budget).
int pencil_thread_cap(rl_plan p) { return p->precision == RL_PRECISION_FP32 ? 1024 : 512; }

// Work-groups above 64 KB of LDS need the kernel attribute set once; done here
// (host side, outside any graph capture) for every mode the pass may launch.
bool prepare_pencil(rl_plan p, const Pencil& pc) {
  for (int mode : {rlmi::PM_FWD, rlmi::PM_INV, rlmi::PM_FKI, rlmi::PM_FCKI})
    if (rlmi::prepare_pencil(mode, pc.ax.E, pc.args.L, p->precision, pc.block, pc.lds) !=
        hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
  return true;
}

// The pencil's LDS with the split-precision operand table where it applies.
bool pencil_fits_plan(rl_plan p, const Pencil& pc) {
  const size_t extra =
      (p->precision != RL_PRECISION_FP32 && pc.ax.E == 16) ? rlmi::kSplitTabBytes : 0;
  return pencil_fits(pc) && pc.lds + extra <= kMaxPencilLds;
}

bool configure_y(rl_plan p, int y_e, int y_txb) {
  Pencil pc = make_pencil_y(p->ny, p->nz, p->xt, p->ncols, y_txb,
                            y_e > 0 ? y_e : pick_e_y(p->ny), pencil_thread_cap(p));
  if (!pencil_fits_plan(p, pc) || (int)pc.block.x > pencil_thread_cap(p) ||
      !prepare_pencil(p, pc))
    return false;
  p->py = pc;
  p->ch_y_e = pc.ax.E;
  p->ch_y_txb = pc.args.TXB;
  return true;
}

bool configure_z(rl_plan p, int z_e, int z_txb, int z_swap) {
  Pencil pc = make_pencil_z(p->nz, p->ny, p->xt, p->ncols, z_txb, z_e, pencil_thread_cap(p));
  if (!pencil_fits_plan(p, pc) || (int)pc.block.x > pencil_thread_cap(p) ||
      !prepare_pencil(p, pc))
    return false;
  if (z_swap) {  // outer (y group) index fastest: resident work-groups share tile columns
    if (pc.grid.x > 65535) return false;
    pc.args.swap = 1;
    pc.grid = dim3(pc.grid.y, pc.grid.x);
  }
  p->ch_z_swap = z_swap ? 1 : 0;
  p->pz = pc;
  p->ch_z_e = pc.ax.E;
  p->ch_z_txb = pc.args.TXB;
  return true;
}

bool configure(rl_plan p, const Choice& c) {
  if (!configure_x(p, c.x_e) || !configure_y(p, c.y_e, c.y_txb) ||
      !configure_z(p, c.z_e, c.z_txb, c.z_swap))
    return false;
  // every transform needs an element count the kernels and the schedule support
  return e_ok(p->M, p->axx.E, 64) && e_ok_yz(p->ny, p->py.ax.E, 1 << 20) &&
         e_ok_yz(p->nz, p->pz.ax.E, 1 << 20);
}

// --- launch shapes of the persistent batched kernel ----------------------------
// Every pass of a class must split into work-groups of exactly kPersistThreads
// threads with element counts the kernel is built for: X rows of 2 waves, Y and Z
// pencils of lanes x threads-per-pencil = kPersistThreads.  persist_choice finds such a
// choice for a shape (default-first candidate order); false if there is none.
constexpr int kPersistXWaves = rlmi::kPersistThreads / 64;

bool persist_x_ok(int64_t M, int E) {
  if (!rlmi::persist_x_e(E) || !e_ok(M, E, 64)) return false;
  const int64_t P = M / E;
  const int64_t rs = M + 1 + ((M + 1) >> rlmi::kXPad) + 1;
  return (size_t)(2 * M + kPersistXWaves * (64 / P) * rs) * sizeof(float2) <= kMaxLds;
}

bool persist_y_ok(int64_t ny, int E, int txb) {
  const int64_t P = rlmi::kPersistThreads / txb;
  return txb <= rlmi::kTile && ny % P == 0 && ny / P == E && rlmi::persist_yz_e(E) &&
         e_ok_yz(ny, E, 1024) && (size_t)ny * (txb + 1) * sizeof(float2) <= kMaxPencilLds;
}

bool persist_z_ok(int64_t nz, int64_t ny, int E, int txb) {
  const int64_t P = rlmi::kPersistThreads / txb;
  if (txb >= rlmi::kTile && ny % (txb / rlmi::kTile) != 0) return false;
  return nz % P == 0 && nz / P == E && rlmi::persist_yz_e(E) && e_ok_yz(nz, E, 1024) &&
         (size_t)nz * (txb + 1) * sizeof(float2) <= kMaxPencilLds;
}

constexpr int kPersistYLanes[] = {16, 8, 4};
constexpr int kPersistZLanes[] = {32, 16, 64, 8};

bool persist_choice(int64_t nz, int64_t ny, int64_t nx, Choice* c) {
  const int64_t M = nx / 2;
  int xe = 0;
  for (int e : {pick_e_x(M), 4, 8, 2, 6})
    if (persist_x_ok(M, e)) {
      xe = e;
      break;
    }
  int ye = 0, yt = 0, ze = 0, zt = 0;
  for (int t : kPersistYLanes) {
    const int64_t P = rlmi::kPersistThreads / t;
    if (ny % P == 0 && persist_y_ok(ny, (int)(ny / P), t)) {
      ye = (int)(ny / P);
      yt = t;
      break;
    }
  }
  for (int t : kPersistZLanes) {
    const int64_t P = rlmi::kPersistThreads / t;
    if (nz % P == 0 && persist_z_ok(nz, ny, (int)(nz / P), t)) {
      ze = (int)(nz / P);
      zt = t;
      break;
    }
  }
  if (!xe || !ye || !ze) return false;
  c->x_e = xe;
  c->y_e = ye;
  c->y_txb = yt;
  c->z_e = ze;
  c->z_txb = zt;
  c->z_swap = 0;
  return true;
}

// The configured shapes of a class plan run in the persistent kernel.
bool persist_fits(rl_plan c) {
  return c->precision == RL_PRECISION_FP32 && c->x_block.x == (unsigned)rlmi::kPersistThreads &&
         rlmi::persist_x_e(c->axx.E) && c->py.block.x == (unsigned)rlmi::kPersistThreads &&
         rlmi::persist_yz_e(c->py.ax.E) && c->pz.block.x == (unsigned)rlmi::kPersistThreads &&
         rlmi::persist_yz_e(c->pz.ax.E);
}

// --- autotuner ---------------------------------------------------------------
// Times candidate elements-per-thread and lane widths for each pass on the
// plan's own buffers (HIP events, median of a few launches) and keeps the
// fastest per pass; ties keep the earlier (default-first) candidate.  Results
// can be cached in the text file named by RLMI_TUNE_CACHE, keyed by GPU
// architecture, runtime version and shape.

std::string tune_key(rl_plan p) {
  hipDeviceProp_t prop;
  std::memset(&prop, 0, sizeof(prop));
  (void)hipGetDeviceProperties(&prop, p->device);
  int rt = 0;
  (void)hipRuntimeGetVersion(&rt);
  std::ostringstream k;
  k << prop.gcnArchName << "/hip" << rt << "/" << p->nz << "x" << p->ny << "x" << p->nx;
  if (p->precision != RL_PRECISION_FP32) k << "/split" << p->precision;  // its own choice
  if (p->persist_shapes) k << "/persist";
  std::string s = k.str();
  for (char& ch : s)
    if (ch == ' ') ch = '_';
  return s;
}

// The last line with this key wins, so a line appended after re-tuning
// supersedes an earlier one.
bool cache_lookup(const std::string& key, Choice* c) {
  const char* path = std::getenv("RLMI_TUNE_CACHE");
  if (!path || !*path) return false;
  std::ifstream f(path);
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    std::istringstream ls(line);
    std::string k;
    Choice t;
    if ((ls >> k >> t.x_e >> t.y_e >> t.y_txb >> t.z_e >> t.z_txb >> t.z_swap) && k == key) {
      *c = t;
      found = true;
    }
  }
  return found;
}

void cache_store(const std::string& key, const Choice& c) {
  const char* path = std::getenv("RLMI_TUNE_CACHE");
  if (!path || !*path) return;
  std::ofstream f(path, std::ios::app);
  f << key << " " << c.x_e << " " << c.y_e << " " << c.y_txb << " " << c.z_e << " " << c.z_txb
    << " " << c.z_swap << "\n";
}


// Median time (ms) of `reps` runs of `fn` on the plan's stream.
template <typename F>
rl_status time_ms(rl_plan p, F fn, float* ms) {
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return hip_fail(hipGetLastError(), "hipEventCreate");
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return hip_fail(hipGetLastError(), "hipEventCreate");
  }
  // bursts of back-to-back launches: an event pair around a single short launch
  // mostly measures the events themselves
  constexpr int kBurst = 8;
  rl_status st = fn();  // warm-up
  float t[3] = {0, 0, 0};
  for (int r = 0; r < 3 && st == RL_OK; ++r) {
    (void)hipEventRecord(a, p->stream);
    for (int k = 0; k < kBurst && st == RL_OK; ++k) st = fn();
    (void)hipEventRecord(b, p->stream);
    if (hipEventSynchronize(b) != hipSuccess) st = hip_fail(hipGetLastError(), "tuning run");
    else (void)hipEventElapsedTime(&t[r], a, b);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  std::sort(t, t + 3);
  *ms = t[1];
  return st;
}

// pencil: the Y / Z rule (e_ok_yz), else the X rule (e_ok)
std::vector<int> e_candidates(int64_t L, int64_t max_p, int precision, bool pencil) {
  std::vector<int> out;
  if (precision != RL_PRECISION_FP32 && split_e(L, max_p) == 16) return {16};
  for (int e : {4, 8, 16, 2, 6, 12, 24, 3, 20, 10, 5, 14, 7, 18, 9, 30, 15})
    if (pencil ? e_ok_yz(L, e, max_p) : e_ok(L, e, max_p)) out.push_back(e);
  return out;
}

rl_status autotune(rl_plan p, Choice* best) {
  float* dbuf = nullptr;
  float* ubuf = nullptr;
  const size_t bytes = (size_t)p->vnvox * sizeof(float);
  hipError_t e;
  if ((e = hipMalloc(&dbuf, bytes)) != hipSuccess) return hip_fail(e, "hipMalloc(tuning)");
  if ((e = hipMalloc(&ubuf, bytes)) != hipSuccess) {
    (void)hipFree(dbuf);
    return hip_fail(e, "hipMalloc(tuning)");
  }
  rl_status st = RL_OK;
  // benign contents: d = u = 1.0, spectrum = 0
  if ((e = hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(dbuf), 0x3f800000u, p->vnvox,
                             p->stream)) != hipSuccess ||
      (e = hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(ubuf), 0x3f800000u, p->vnvox,
                             p->stream)) != hipSuccess ||
      (e = hipMemsetAsync(p->spec, 0, p->spec_elems * sizeof(float2), p->stream)) != hipSuccess)
    st = hip_fail(e, "tuning buffers");
  Choice c = *best;
  // A candidate replaces the plan's configured (default) shape only when its burst
  // is faster by more than kTuneMargin: bursts of one pass kind run without the
  // other passes in between, so differences of a few percent between close
  // candidates do not carry over to the iteration sequence reliably.
  constexpr float kTuneMargin = 0.03f;
  const int def_xe = p->axx.E, def_ye = p->py.ax.E, def_ytxb = p->py.args.TXB;
  const int def_ze = p->pz.ax.E, def_ztxb = p->pz.args.TXB, def_zsw = p->pz.args.swap;
  float def_ms = 1e30f;
  // X: fused ratio + update
  float bt = 1e30f;
  for (int xe : e_candidates(p->M, 64, RL_PRECISION_FP32, false)) {  // X stays FP32
    if (st != RL_OK) break;
    if (p->persist_shapes && !persist_x_ok(p->M, xe)) continue;
    if (!configure_x(p, xe)) continue;
    float ms = 0.f;
    st = time_ms(p, [&]() {
      XArgs r = base_xargs(p, p->spec);
      r.d = dbuf;
      rl_status s2 = run_x(p, rlmi::XM_RATIO, r, RL_KERNEL_OTHER);
      if (s2 != RL_OK) return s2;
      XArgs u = base_xargs(p, p->spec);
      u.u = ubuf;
      u.partials = p->partials;
      u.iter = 0;
      u.do_fwd = 1;
      return run_x(p, rlmi::XM_UPDATE, u, RL_KERNEL_OTHER);
    }, &ms);
    if (st == RL_OK && xe == def_xe) def_ms = ms;
    if (st == RL_OK && ms < bt) {
      bt = ms;
      c.x_e = xe;
    }
  }
  if (def_ms <= bt * (1.f + kTuneMargin)) c.x_e = def_xe;
  // Y: forward + inverse
  bt = 1e30f;
  def_ms = 1e30f;
  if (p->ny > 1) {
    for (int ye : e_candidates(p->ny, 1024, p->precision, true))
      for (int w : {16, 8, 4}) {
        if (p->persist_shapes ? !persist_y_ok(p->ny, ye, w) : w == 4) continue;
        if (st != RL_OK || !configure_y(p, ye, w) || p->py.args.TXB != w) continue;
        float ms = 0.f;
        st = time_ms(p, [&]() {
          rl_status s2 = run_pencil(p, p->py, rlmi::PM_FWD, p->spec, p->tw_y, RL_KERNEL_OTHER);
          return s2 != RL_OK ? s2 : run_pencil(p, p->py, rlmi::PM_INV, p->spec, p->tw_y,
                                               RL_KERNEL_OTHER);
        }, &ms);
        if (st == RL_OK && ye == def_ye && w == def_ytxb) def_ms = ms;
        if (st == RL_OK && ms < bt) {
          bt = ms;
          c.y_e = ye;
          c.y_txb = w;
        }
      }
    if (def_ms <= bt * (1.f + kTuneMargin)) {
      c.y_e = def_ye;
      c.y_txb = def_ytxb;
    }
  }
  // Z: forward * K * inverse
  bt = 1e30f;
  def_ms = 1e30f;
  for (int ze : e_candidates(p->nz, 1024, p->precision, true))
    for (int w : {32, 16, 64, 8})
    for (int sw : {0, 1}) {
      if (p->persist_shapes ? (sw || !persist_z_ok(p->nz, p->ny, ze, w)) : w == 8) continue;
      if (st != RL_OK || !configure_z(p, ze, w, sw) || p->pz.args.TXB != w) continue;
      float ms = 0.f;
      st = time_ms(p, [&]() {
        return run_pencil(p, p->pz, rlmi::PM_FKI, p->spec, p->tw_z, RL_KERNEL_OTHER);
      }, &ms);
      if (st == RL_OK && ze == def_ze && w == def_ztxb && sw == def_zsw) def_ms = ms;
      if (st == RL_OK && ms < bt) {
        bt = ms;
        c.z_e = ze;
        c.z_txb = w;
        c.z_swap = sw;
      }
    }
  if (def_ms <= bt * (1.f + kTuneMargin)) {
    c.z_e = def_ze;
    c.z_txb = def_ztxb;
    c.z_swap = def_zsw;
  }
  (void)hipStreamSynchronize(p->stream);
  (void)hipFree(dbuf);
  (void)hipFree(ubuf);
  if (st != RL_OK) return st;
  *best = c;
  return RL_OK;
}

rl_status check_options(const int64_t shape[3], const rl_options* opt) {
  if (!opt) return RL_OK;
  if (opt->precision != RL_PRECISION_FP32 && opt->precision != RL_PRECISION_SPLIT_BF16 &&
      opt->precision != RL_PRECISION_SPLIT_FP16)
    return fail(RL_E_INVALID, "unknown precision");
  if (opt->tile_x < 0 || opt->tile_x > 64) return fail(RL_E_INVALID, "tile_x must be in [0, 64]");
  if (opt->x_elems != 0 && !e_ok(shape[2] / 2, opt->x_elems, 64))
    return fail(RL_E_INVALID, "x_elems does not fit nx/2");
  if (opt->yz_elems != 0 &&
      (!e_ok_yz(shape[1], opt->yz_elems, 1024) || !e_ok_yz(shape[0], opt->yz_elems, 1024)))
    return fail(RL_E_INVALID, "yz_elems does not fit ny and nz");
  if (opt->autotune != 0 && opt->autotune != 1) return fail(RL_E_INVALID, "autotune must be 0 or 1");
  if (opt->accel != RL_ACCEL_NONE && opt->accel != RL_ACCEL_BIGGS_ANDREWS)
    return fail(RL_E_INVALID, "unknown accel");
  return RL_OK;
}

rl_status check_boundary(int boundary) {
  if (boundary != RL_BOUNDARY_PERIODIC && boundary != RL_BOUNDARY_ZERO)
    return fail(RL_E_INVALID, "unknown boundary");
  return RL_OK;
}

// Where a plan's volumes, PSF and transform grid sit: the caller's volume
// (vol) at the low corner of the grid, the PSF (psf <= vol per axis) centred
// on grid voxel 0.  Periodic: grid = vol.  Zero: grid >= vol + psf/2 per axis,
// so that no wrapped term of the circular convolution on the grid reaches the
// volume (the offsets of the PSF entries lie in [-psf/2, psf - 1 - psf/2]).
struct Geometry {
  int64_t grid[3], vol[3], psf[3];
  int boundary;
};

// Transform length >= need that `fits` accepts (a supported length o * 2^a with
// an element count for it) of least estimated cost L * w(o); -1 if none below
// 2^31.  w is the time per element of a pass relative to power-of-two lengths,
// measured on MI355X: odd parts 3 and 5 cost little more, 9 and 15 (whose
// element counts leave only radix-2 stages or long registers) about twice.
template <typename F>
int64_t next_len(int64_t need, F fits) {
  static const struct {
    int64_t o;
    double w;
  } kCost[] = {{1, 1.0}, {3, 1.05}, {5, 1.2}, {7, 1.6}, {9, 2.0}, {15, 2.2}};
  int64_t best = -1;
  double best_cost = 0.0;
  for (const auto& c : kCost)
    for (int64_t L = c.o; L < ((int64_t)1 << 31); L *= 2)
      if (L >= need && fits(L)) {
        const double cost = (double)L * c.w;
        if (best < 0 || cost < best_cost) {
          best = L;
          best_cost = cost;
        }
        break;
      }
  return best;
}

rl_status make_geometry(const int64_t shape[3], const rl_options* opt, int boundary,
                        Geometry* g) {
  if (!shape) return fail(RL_E_INVALID, "shape is NULL");
  g->boundary = boundary;
  for (int i = 0; i < 3; ++i) {
    if (shape[i] < 1) return fail(RL_E_INVALID, "every dimension must be >= 1");
    if (shape[i] > (int64_t)1 << 30) return fail(RL_E_UNSUPPORTED, "dimension too large");
    g->vol[i] = shape[i];
    const int64_t ps = opt ? opt->psf_shape[i] : 0;
    if (ps < 0 || ps > shape[i])
      return fail(RL_E_INVALID, "psf_shape must be 0 (the volume's) or in [1, volume dimension]");
    g->psf[i] = ps > 0 ? ps : shape[i];
  }
  if (boundary == RL_BOUNDARY_PERIODIC) {
    rl_status st = check_shape(shape);
    if (st != RL_OK) return st;
    for (int i = 0; i < 3; ++i) g->grid[i] = shape[i];
    return RL_OK;
  }
  auto has_e = [](int64_t L, int64_t max_p) {
    for (int E : kE)
      if (e_ok(L, E, max_p)) return true;
    return false;
  };
  for (int i = 0; i < 2; ++i)
    g->grid[i] = next_len(g->vol[i] + g->psf[i] / 2,
                          [&](int64_t L) { return L <= kMaxNyz && has_e(L, 1024); });  // strict lengths
  const int64_t need_x = g->vol[2] + g->psf[2] / 2;
  const int64_t half = next_len((need_x + 1) / 2 < 2 ? 2 : (need_x + 1) / 2,
                                [&](int64_t m) { return 2 * m <= kMaxNx && has_e(m, 64); });
  g->grid[2] = half > 0 ? 2 * half : -1;
  for (int i = 0; i < 3; ++i)
    if (g->grid[i] < 1)
      return fail(RL_E_UNSUPPORTED, "zero boundary: no supported padded transform length for "
                                    "dimension " + std::to_string(i) + " (needs " +
                                        std::to_string(g->vol[i] + g->psf[i] / 2) + ")");
  rl_status st = check_shape(g->grid);
  if (st != RL_OK)
    return fail(st, "zero boundary: the padded transform grid " + std::to_string(g->grid[0]) +
                        "x" + std::to_string(g->grid[1]) + "x" + std::to_string(g->grid[2]) +
                        " is not supported (" + g_err + ")");
  return RL_OK;
}

rl_status check_device_present() {
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev < 1) {
    (void)hipGetLastError();
    return fail(RL_E_DEVICE, "no HIP device available");
  }
  return RL_OK;
}

// Build the plan of `count` volumes of one (validated) shape on `device`;
// psfs[i] is volume i's PSF (validated device pointers).  psfs == nullptr builds
// a transform-only plan (no transfer function; used for the half-size transforms
// of the single-image FSC).  Synchronous.
rl_status build_class(const Geometry& geo, int count, const float* const* psfs, int device,
                      const rl_options* opt, hipStream_t stream, rl_plan* out,
                      bool persist_shapes = false) {
  rl_status st;
  hipError_t e;
  const int64_t nz = geo.grid[0], ny = geo.grid[1], nx = geo.grid[2];
  const int64_t nvox = nz * ny * nx;
  rl_plan p = new (std::nothrow) rl_plan_s();
  if (!p) return fail(RL_E_NOMEM, "host allocation failed");
  p->device = device;
  p->stream = stream;
  p->count = count;
  p->nz = nz;
  p->ny = ny;
  p->nx = nx;
  p->M = nx / 2;
  p->ncols = p->M + 1;
  p->xt = (p->ncols + rlmi::kTile - 1) / rlmi::kTile;  // 16-column tiles per row
  p->nvox = nvox;
  p->nrows = nz * ny;
  p->vz = geo.vol[0];
  p->vy = geo.vol[1];
  p->vx = geo.vol[2];
  p->vnvox = p->vz * p->vy * p->vx;
  p->psf_z = geo.psf[0];
  p->psf_y = geo.psf[1];
  p->psf_x = geo.psf[2];
  p->boundary = geo.boundary;
  p->spec_elems = (size_t)nz * p->xt * ny * rlmi::kTile;

  // launch choice: options first, defaults for the rest
  p->precision = opt ? opt->precision : RL_PRECISION_FP32;
  p->accel = opt ? opt->accel : RL_ACCEL_NONE;
  Choice choice;
  if (p->precision != RL_PRECISION_FP32) {
    // split precision runs the radix-16 stages of the Y and Z transforms on MFMA:
    // 16 elements per thread wherever the length has radix-16 stages (other
    // lengths stay FP32).  The fused X passes keep their FP32 radix-8/4 schedule
    // unless x_elems = 16 is requested: with 16 elements per thread they hold the
    // row, the real operand and the MFMA operands at once, over 200 registers and
    // one wavefront per SIMD.
    choice.y_e = split_e(ny, 1024);
    choice.z_e = split_e(nz, 1024);
  }
  if (opt) {
    const int tx = opt->tile_x > 0 ? pow2_floor(opt->tile_x) : 0;
    if (opt->x_elems) choice.x_e = opt->x_elems;
    if (opt->yz_elems) choice.y_e = choice.z_e = opt->yz_elems;
    choice.y_txb = tx > rlmi::kTile ? rlmi::kTile : tx;
    choice.z_txb = tx;
  }
  if (persist_shapes) {  // launch shapes the persistent batched kernel runs
    p->persist_shapes = true;
    if (!persist_choice(nz, ny, nx, &choice)) {
      delete p;
      return fail(RL_E_UNSUPPORTED, "shape has no launch shapes for the persistent kernel");
    }
  }
  const bool want_tune =
      autotune_override() >= 0 ? autotune_override() == 1 : (opt && opt->autotune);
  if (!configure(p, choice)) {
    delete p;
    return fail(RL_E_UNSUPPORTED, "shape needs more LDS or threads than a work-group may use");
  }
  if ((e = hipSetDevice(device)) != hipSuccess) {
    delete p;
    return hip_fail(e, "hipSetDevice");
  }
  p->flux_cap = psfs ? 128 : 1;
  // >= any X grid times the iteration capacity times the volumes
  p->n_partials = (size_t)p->nrows * p->flux_cap * count;
  if (p->n_partials < 3 * (size_t)kStatBlocks) p->n_partials = 3 * kStatBlocks;
  const size_t spec_bytes = p->spec_elems * sizeof(float2) * (size_t)count;
  if ((e = hipMalloc(&p->spec, spec_bytes)) != hipSuccess ||
      (psfs && (e = hipMalloc(&p->otf, spec_bytes)) != hipSuccess) ||
      (e = hipMalloc(&p->tw_x, (size_t)nx * sizeof(float2))) != hipSuccess ||
      (e = hipMalloc(&p->tw_y, (size_t)ny * sizeof(float2))) != hipSuccess ||
      (e = hipMalloc(&p->tw_z, (size_t)nz * sizeof(float2))) != hipSuccess ||
      (e = hipMalloc(&p->partials, p->n_partials * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&p->counter, 4 * sizeof(unsigned))) != hipSuccess ||
      (e = hipMalloc(&p->stats, 4 * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&p->flux, (size_t)p->flux_cap * count * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&p->iter_dev, sizeof(int))) != hipSuccess ||
      (e = hipMalloc(&p->d_tab, (size_t)count * sizeof(float*))) != hipSuccess ||
      (e = hipMalloc(&p->u_tab, (size_t)count * sizeof(float*))) != hipSuccess) {
    st = hip_fail(e, "hipMalloc");
    release(p);
    return st;
  }
  if (count == 1 &&
      ((e = hipMalloc(&p->stop, 4 * sizeof(int))) != hipSuccess ||
       (e = hipMalloc(&p->met_partials, rlmi::kMetRows * (size_t)p->nrows * sizeof(double))) !=
           hipSuccess ||
       (e = hipMalloc(&p->mhist, (size_t)(p->flux_cap + 1) * sizeof(double))) != hipSuccess)) {
    st = hip_fail(e, "hipMalloc(stopping state)");
    release(p);
    return st;
  }
  if (p->accel != RL_ACCEL_NONE) {
    const size_t vb = (size_t)p->vnvox * sizeof(float);
    if ((e = hipMalloc(&p->hstep, vb)) != hipSuccess ||
        (e = hipMalloc(&p->gchg, vb)) != hipSuccess ||
        (e = hipMalloc(&p->alpha32, (size_t)(p->flux_cap + 1) * sizeof(float))) != hipSuccess ||
        (e = hipMalloc(&p->alpha64, (size_t)(p->flux_cap + 1) * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&p->acc_partials, 2 * (size_t)p->nrows * sizeof(double))) != hipSuccess) {
      st = hip_fail(e, "hipMalloc(extrapolation state)");
      release(p);
      return st;
    }
  }
#define RL_TRY(expr)                    \
  do {                                  \
    hipError_t e_ = (expr);             \
    if (e_ != hipSuccess) {             \
      st = hip_fail(e_, #expr);         \
      release(p);                       \
      return st;                        \
    }                                   \
  } while (0)
  RL_TRY(hipMemsetAsync(p->counter, 0, 4 * sizeof(unsigned), p->stream));
  RL_TRY(rlmi::launch_twiddles(p->tw_x, (int)nx, p->stream));
  RL_TRY(rlmi::launch_twiddles(p->tw_y, (int)ny, p->stream));
  RL_TRY(rlmi::launch_twiddles(p->tw_z, (int)nz, p->stream));
  for (int v = 0; psfs && v < count; ++v) {
    const float* psf = psfs[v];
    RL_TRY(rlmi::launch_psf_stats(psf, p->psf_z * p->psf_y * p->psf_x, p->partials,
                                  kStatBlocks, p->counter, p->stats, p->stream));
    double stats[3] = {0, 0, 0};
    RL_TRY(hipMemcpyAsync(stats, p->stats, 3 * sizeof(double), hipMemcpyDeviceToHost, p->stream));
    RL_TRY(hipStreamSynchronize(p->stream));
    const std::string which = count > 1 ? " (volume " + std::to_string(v) + " of its shape)" : "";
    if (stats[2] != 0.0) {
      release(p);
      return fail(RL_E_INVALID, "psf has non-finite entries" + which);
    }
    if (stats[1] < 0.0) {
      release(p);
      return fail(RL_E_INVALID, "psf has negative entries" + which);
    }
    if (!(stats[0] > 0.0) || !std::isfinite(stats[0])) {
      release(p);
      return fail(RL_E_INVALID, "psf must have a positive finite sum" + which);
    }
    // OTF / N: scaled, centred PSF written as dense real rows into the spectrum
    // workspace, transformed along X into the volume's OTF slot, then along Y and Z.
    float2* otf_v = p->otf + (size_t)v * p->spec_elems;
    const double scale = 1.0 / (stats[0] * (double)nvox);
    RL_TRY(rlmi::launch_psf_prep(psf, (int)p->psf_z, (int)p->psf_y, (int)p->psf_x,
                                 reinterpret_cast<float*>(p->spec), (int)nz, (int)ny, (int)nx, nx,
                                 scale, p->stream));
    // the prepared kernel covers the whole grid
    XArgs a = base_xargs(p, otf_v);
    a.rin = reinterpret_cast<const float*>(p->spec);
    a.rin_stride = nx;
    a.vx = (int)nx;
    a.vy = (int)ny;
    a.vz = (int)nz;
    a.nrows = (int)p->nrows;
    a.nvol = 1;
    if ((st = run_x(p, rlmi::XM_R2C, a, RL_KERNEL_OTHER, p->nrows)) != RL_OK ||
        (st = run_pencil(p, p->py, rlmi::PM_FWD, otf_v, p->tw_y, RL_KERNEL_OTHER, 1)) != RL_OK ||
        (st = run_pencil(p, p->pz, rlmi::PM_FWD, otf_v, p->tw_z, RL_KERNEL_OTHER, 1)) != RL_OK) {
      release(p);
      return st;
    }
  }
  // into the order the Z pass reads it (through the spectrum workspace)
  if (psfs) {
    RL_TRY(rlmi::launch_otf_zmajor(p->otf, p->spec, count, (int)nz, (int)ny, (int)p->xt,
                                   (int)p->ncols, p->stream));
    RL_TRY(hipMemcpyAsync(p->otf, p->spec, spec_bytes, hipMemcpyDeviceToDevice, p->stream));
  }
  RL_TRY(hipStreamSynchronize(p->stream));
#undef RL_TRY
  if (want_tune) {
    const std::string key = tune_key(p);
    Choice tuned = choice;
    bool cached = cache_lookup(key, &tuned);
    if (cached && (!configure(p, tuned) || (p->persist_shapes && !persist_fits(p)))) {
      // a stale or edited line: tune afresh
      cached = false;
      tuned = choice;
    }
    if (!cached) {
      if ((st = autotune(p, &tuned)) != RL_OK) {
        release(p);
        return st;
      }
      cache_store(key, tuned);
      if (!configure(p, tuned) || (p->persist_shapes && !persist_fits(p))) {
        release(p);
        return fail(RL_E_INTERNAL, "tuned configuration does not apply");
      }
    }
    p->tuned = true;
  }
  *out = p;
  return RL_OK;
}

rl_status create_impl(const int64_t shape[3], const float* psf, int boundary,
                      const rl_options* opt, rl_plan* out) {
  if (!out) return fail(RL_E_INVALID, "out is NULL");
  *out = nullptr;
  rl_status st = check_boundary(boundary);
  if (st != RL_OK) return st;
  Geometry geo;
  if ((st = make_geometry(shape, opt, boundary, &geo)) != RL_OK) return st;
  if ((st = check_options(geo.grid, opt)) != RL_OK) return st;
  if (!psf) return fail(RL_E_INVALID, "psf is NULL");
  if (reinterpret_cast<uintptr_t>(psf) % 16 != 0)
    return fail(RL_E_INVALID, "psf is not 16-byte aligned");
  if ((st = check_device_present()) != RL_OK) return st;
  const int64_t pnvox = geo.psf[0] * geo.psf[1] * geo.psf[2];
  int device = -1;
  if ((st = check_dev_ptr(psf, (size_t)pnvox * sizeof(float), &device, "psf")) != RL_OK) return st;
  rl_plan p = nullptr;
  const float* psfs[1] = {psf};
  hipStream_t stream = opt ? reinterpret_cast<hipStream_t>(opt->stream) : nullptr;
  if ((st = build_class(geo, 1, psfs, device, opt, stream, &p)) != RL_OK) return st;
  plan_register(p);
  *out = p;
  return RL_OK;
}

// Grow the per-iteration flux array and the [iteration][volume][work-group]
// partial table of a (class) plan to hold n_iter iterations.
rl_status ensure_flux_capacity(rl_plan p, int n_iter, bool* grew) {
  if (grew) *grew = false;
  if (n_iter <= p->flux_cap) return RL_OK;
  double* nf = nullptr;
  double* np = nullptr;
  float* na32 = nullptr;
  double* na64 = nullptr;
  const size_t nparts = (size_t)n_iter * p->nrows * p->count;
  hipError_t e;
  if ((e = hipMalloc(&nf, (size_t)n_iter * p->count * sizeof(double))) != hipSuccess)
    return hip_fail(e, "hipMalloc(flux)");
  if ((e = hipMalloc(&np, nparts * sizeof(double))) != hipSuccess) {
    (void)hipFree(nf);
    return hip_fail(e, "hipMalloc(flux partials)");
  }
  if (p->accel != RL_ACCEL_NONE &&
      ((e = hipMalloc(&na32, (size_t)(n_iter + 1) * sizeof(float))) != hipSuccess ||
       (e = hipMalloc(&na64, (size_t)(n_iter + 1) * sizeof(double))) != hipSuccess)) {
    (void)hipFree(nf);
    (void)hipFree(np);
    (void)hipFree(na32);
    return hip_fail(e, "hipMalloc(alpha)");
  }
  double* nh = nullptr;
  if (p->mhist && (e = hipMalloc(&nh, (size_t)(n_iter + 1) * sizeof(double))) != hipSuccess) {
    (void)hipFree(nf);
    (void)hipFree(np);
    (void)hipFree(na32);
    (void)hipFree(na64);
    return hip_fail(e, "hipMalloc(metric history)");
  }
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  else (void)hipDeviceSynchronize();
  (void)hipFree(p->flux);
  (void)hipFree(p->partials);
  p->flux = nf;
  p->partials = np;
  if (p->accel != RL_ACCEL_NONE) {
    (void)hipFree(p->alpha32);
    (void)hipFree(p->alpha64);
    p->alpha32 = na32;
    p->alpha64 = na64;
  }
  if (nh) {
    (void)hipFree(p->mhist);
    p->mhist = nh;
  }
  p->n_partials = nparts;
  p->flux_cap = n_iter;
  if (grew) *grew = true;
  return RL_OK;
}

// Spectrum of H u (transformed back along Z and Y) for every volume of the plan.
// u == nullptr: per-volume estimates from the plan's device table.
rl_status enqueue_prologue(rl_plan p, const float* u) {
  XArgs a = base_xargs(p, p->spec);
  a.rin = u;
  a.rin_tab = u ? nullptr : p->u_tab;
  rl_status st = run_x(p, rlmi::XM_R2C, a, RL_KERNEL_X_R2C);
  return st != RL_OK ? st : run_yz_filter(p, false);
}

// One RL iteration for every volume of the plan (d/u == nullptr: device tables).
// The iteration index for the flux partials is `it`, or *iter_ptr if non-null.
// partials: the flux partial table (nullptr = the plan's own).
rl_status enqueue_iteration(rl_plan p, const float* d, float* u, int it, const int* iter_ptr,
                            bool do_fwd, double* partials = nullptr) {
  rl_status st;
  XArgs r = base_xargs(p, p->spec);
  r.d = d;
  r.d_tab = d ? nullptr : p->d_tab;
  if ((st = run_x(p, rlmi::XM_RATIO, r, RL_KERNEL_X_RATIO)) != RL_OK) return st;
  if ((st = run_yz_filter(p, true)) != RL_OK) return st;
  XArgs w = base_xargs(p, p->spec);
  w.u = u;
  w.u_tab = u ? nullptr : p->u_tab;
  w.partials = partials ? partials : p->partials;
  w.iter = it;
  w.iter_ptr = iter_ptr;
  w.do_fwd = do_fwd ? 1 : 0;
  if ((st = run_x(p, rlmi::XM_UPDATE, w, RL_KERNEL_X_UPDATE)) != RL_OK) return st;
  if (do_fwd && (st = run_yz_filter(p, false)) != RL_OK) return st;
  return RL_OK;
}

// flux[it * count + v] for it < n_iter, on `stream`.
rl_status enqueue_flux_reduce(rl_plan p, int n_iter, hipStream_t stream,
                              const double* partials = nullptr) {
  hipStream_t keep = p->stream;
  p->stream = stream;
  size_t slot = 0;
  hipEvent_t ev0, ev1;
  rl_status st = timed_begin(p, RL_KERNEL_OTHER, &slot, &ev0, &ev1);
  if (st == RL_OK) {
    hipError_t e = rlmi::launch_flux_reduce(partials ? partials : p->partials, (int)p->x_grid.x,
                                            n_iter * p->count, p->flux, stream, ev0, ev1);
    st = launched(e, stream, "flux reduction");
  }
  p->stream = keep;
  return st;
}

// Extrapolated (Biggs-Andrews) iteration: x_k lives in `u`, the step h_k and
// change g_{k-1} in plan buffers, alpha_k on the device.
XArgs accel_xargs(rl_plan p, float* u, int it) {
  XArgs a = base_xargs(p, p->spec);
  a.u = u;
  a.hstep = p->hstep;
  a.gchg = p->gchg;
  a.alpha = p->alpha32;
  a.acc_partials = p->acc_partials;
  a.partials = p->partials;
  a.iter = it;
  return a;
}

// Spectrum of H y_it, y_it = max(x_it + alpha_it h_it, 0).
rl_status enqueue_accel_predict(rl_plan p, float* u, int it) {
  rl_status st = run_x(p, rlmi::XM_PREDICT, accel_xargs(p, u, it), RL_KERNEL_X_R2C);
  return st != RL_OK ? st : run_yz_filter(p, false);
}

rl_status enqueue_accel_iteration(rl_plan p, const float* d, float* u, int it, bool last) {
  rl_status st;
  XArgs r = base_xargs(p, p->spec);
  r.d = d;
  if ((st = run_x(p, rlmi::XM_RATIO, r, RL_KERNEL_X_RATIO)) != RL_OK) return st;
  if ((st = run_yz_filter(p, true)) != RL_OK) return st;
  if ((st = run_x(p, rlmi::XM_UPDATE_ACC, accel_xargs(p, u, it), RL_KERNEL_X_UPDATE)) != RL_OK)
    return st;
  size_t slot = 0;
  hipEvent_t ev0, ev1;
  if ((st = timed_begin(p, RL_KERNEL_OTHER, &slot, &ev0, &ev1)) != RL_OK) return st;
  hipError_t e = rlmi::launch_accel_alpha(p->acc_partials, (int)p->x_grid.x, it, p->alpha32,
                                          p->alpha64, p->stream, ev0, ev1);
  if ((st = launched(e, p->stream, "alpha reduction")) != RL_OK) return st;
  return last ? RL_OK : enqueue_accel_predict(p, u, it + 1);
}

rl_status iterate_impl(rl_plan p, const float* observed, float* estimate, int n_iter) {
  rl_status st = check_plan(p);
  if (st != RL_OK) return st;
  if (p->is_batch) return fail(RL_E_INVALID, "batch plans iterate with rl_iterate_batch");
  if (n_iter < 0) return fail(RL_E_INVALID, "n_iter must be >= 0");
  const size_t bytes = (size_t)p->vnvox * sizeof(float);
  int dev = p->device;
  if ((st = check_dev_ptr(observed, bytes, &dev, "observed")) != RL_OK) return st;
  if ((st = check_dev_ptr(estimate, bytes, &dev, "estimate")) != RL_OK) return st;
  if (n_iter == 0) return RL_OK;
  hipError_t e = hipSetDevice(p->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  if ((st = ensure_flux_capacity(p, n_iter, nullptr)) != RL_OK) return st;
  p->flux_count = n_iter;
  p->stop_call = false;
  if (p->accel != RL_ACCEL_NONE) {
    if ((st = enqueue_accel_predict(p, estimate, 0)) != RL_OK) return st;
    for (int it = 0; it < n_iter; ++it)
      if ((st = enqueue_accel_iteration(p, observed, estimate, it, it + 1 == n_iter)) != RL_OK)
        return st;
    return enqueue_flux_reduce(p, n_iter, p->stream);
  }
  if ((st = enqueue_prologue(p, estimate)) != RL_OK) return st;
  for (int it = 0; it < n_iter; ++it)
    if ((st = enqueue_iteration(p, observed, estimate, it, nullptr, it + 1 < n_iter)) != RL_OK)
      return st;
  return enqueue_flux_reduce(p, n_iter, p->stream);
}

// --- the iteration without allocation ------------------------------------------
// Device scratch of rl_iterate_noalloc: the FP64 flux partials [iteration][X
// work-group] live in this fixed array instead of plan memory that may have to
// grow.  Host code must not pass the array's name to a kernel (it is a host-side
// stand-in there); it uses the device address looked up once per device.
constexpr size_t kScratchDoubles = (size_t)1 << 20;  // 8 MiB per device
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (current), looked up on the first call.
rl_status scratch_on(int device, double** out) {
  if (device < 0 || device >= kMaxDevices) return fail(RL_E_UNSUPPORTED, "device index too large");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[device] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[device];
  return RL_OK;
}

rl_status iterate_noalloc_impl(rl_plan p, const float* observed, float* estimate, int n_iter) {
  rl_status st = check_plan(p);
  if (st != RL_OK) return st;
  if (p->is_batch) return fail(RL_E_INVALID, "batch plans iterate with rl_iterate_batch");
  if (p->accel != RL_ACCEL_NONE)
    return fail(RL_E_UNSUPPORTED, "rl_iterate_noalloc runs the plain iteration (no extrapolation)");
  if (p->timing)
    return fail(RL_E_UNSUPPORTED, "rl_iterate_noalloc does not run with per-launch timing");
  if (n_iter < 0) return fail(RL_E_INVALID, "n_iter must be >= 0");
  const size_t need = (size_t)n_iter * p->x_grid.x;
  if (need > kScratchDoubles)
    return fail(RL_E_INVALID, "rl_iterate_noalloc: n_iter * X work-groups = " +
                                  std::to_string(need) + " exceeds the scratch of " +
                                  std::to_string(kScratchDoubles) + " values");
  if (n_iter > p->flux_cap)
    return fail(RL_E_INVALID, "rl_iterate_noalloc: n_iter exceeds the plan's flux capacity (" +
                                  std::to_string(p->flux_cap) + ")");
  const size_t bytes = (size_t)p->vnvox * sizeof(float);
  int dev = p->device;
  if ((st = check_dev_ptr(observed, bytes, &dev, "observed")) != RL_OK) return st;
  if ((st = check_dev_ptr(estimate, bytes, &dev, "estimate")) != RL_OK) return st;
  if (n_iter == 0) return RL_OK;
  hipError_t e = hipSetDevice(p->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  double* part = nullptr;
  if ((st = scratch_on(p->device, &part)) != RL_OK) return st;
  p->flux_count = n_iter;
  p->stop_call = false;
  // every [iteration][work-group] slot read by the reduction is written by that
  // iteration's update pass first, so the scratch needs no clearing
  if ((st = enqueue_prologue(p, estimate)) != RL_OK) return st;
  for (int it = 0; it < n_iter; ++it)
    if ((st = enqueue_iteration(p, observed, estimate, it, nullptr, it + 1 < n_iter, part)) !=
        RL_OK)
      return st;
  return enqueue_flux_reduce(p, n_iter, p->stream, part);
}

constexpr int kSsimRangeBlocks = 512;

struct SsimGeom {
  int64_t nxo, nyo, nzo, blocks;  // valid window positions; work-groups of the last pass
};

SsimGeom ssim_geom(rl_plan p) {
  SsimGeom g;
  g.nxo = p->vx - 6;
  g.nyo = p->vy - 6;
  g.nzo = p->vz - 6;
  g.blocks = ((g.nxo + 255) / 256) * g.nyo * ((g.nzo + 31) / 32);
  return g;
}

rl_status ssim_buffers(rl_plan p) {
  if (p->vz < 7 || p->vy < 7 || p->vx < 7)
    return fail(RL_E_UNSUPPORTED, "SSIM needs every dimension >= 7 (7x7x7 windows)");
  if (p->vy > 65535 + 6 || p->vz > 65535 + 6)
    return fail(RL_E_UNSUPPORTED, "SSIM needs ny, nz <= 65541");
  if (p->ssim_a) return RL_OK;
  const SsimGeom g = ssim_geom(p);
  hipError_t e;
  if ((e = hipMalloc(&p->ssim_a, 5 * (size_t)p->vz * p->vy * g.nxo * sizeof(double))) !=
          hipSuccess ||
      (e = hipMalloc(&p->ssim_b, 5 * (size_t)p->vz * g.nyo * g.nxo * sizeof(double))) !=
          hipSuccess ||
      (e = hipMalloc(&p->ssim_part, (size_t)g.blocks * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&p->ssim_range, (1 + 2 * (size_t)kSsimRangeBlocks) * sizeof(double))) !=
          hipSuccess) {
    (void)hipFree(p->ssim_a);
    (void)hipFree(p->ssim_b);
    (void)hipFree(p->ssim_part);
    p->ssim_a = p->ssim_b = p->ssim_part = nullptr;
    return hip_fail(e, "hipMalloc(SSIM buffers)");
  }
  return RL_OK;
}

rl_status enqueue_ssim(rl_plan p, const float* u, const float* ref, bool want_range) {
  hipError_t e = rlmi::launch_ssim(u, ref, (int)p->vz, (int)p->vy, (int)p->vx, p->ssim_a, p->ssim_b,
                                   p->ssim_range + 1, kSsimRangeBlocks, p->ssim_range,
                                   p->ssim_part, want_range, p->active_stop, p->stream);
  return launched(e, p->stream, "SSIM");
}

rl_status ssim_impl(rl_plan p, const float* u, const float* ref, double* value) {
  rl_status st = check_plan(p);
  if (st != RL_OK) return st;
  if (p->is_batch) return fail(RL_E_UNSUPPORTED, "rl_ssim takes a single-volume plan");
  if (!value) return fail(RL_E_INVALID, "value is NULL");
  const size_t bytes = (size_t)p->vnvox * sizeof(float);
  int dev = p->device;
  if ((st = check_dev_ptr(u, bytes, &dev, "u")) != RL_OK) return st;
  if ((st = check_dev_ptr(ref, bytes, &dev, "reference")) != RL_OK) return st;
  hipError_t e = hipSetDevice(p->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  if ((st = ssim_buffers(p)) != RL_OK) return st;
  if ((st = enqueue_ssim(p, u, ref, true)) != RL_OK) return st;
  const SsimGeom g = ssim_geom(p);
  std::vector<double> h((size_t)g.blocks);
  if ((e = hipStreamSynchronize(p->stream)) != hipSuccess) return hip_fail(e, "execution");
  if ((e = hipMemcpy(h.data(), p->ssim_part, h.size() * sizeof(double), hipMemcpyDeviceToHost)) !=
      hipSuccess)
    return hip_fail(e, "hipMemcpy(SSIM)");
  double t = 0.0;
  for (double v : h) t += v;  // fixed order
  *value = t / (double)(g.nxo * g.nyo * g.nzo);
  return RL_OK;
}

rl_status fsc_lcm(rl_plan p, int64_t* lcm);
rl_status fsc_buffers(rl_plan p, int nbins);
rl_status enqueue_fsc(rl_plan p, const float* a, const float* b, int nbins, double threshold,
                      int64_t lcm);

// Shape rules of FSC-guided stopping (no device work): a periodic plan with even
// dimensions whose halves are transform lengths.
rl_status fsc_stop_check(rl_plan p, const rl_stop_rule* rule, int* nbins, double* fthr) {
  if (p->boundary != RL_BOUNDARY_PERIODIC)
    return fail(RL_E_UNSUPPORTED, "FSC-guided stopping needs a periodic plan");
  *nbins = rule->fsc_bins == 0 ? 64 : rule->fsc_bins;
  if (*nbins < 2 || *nbins > 1024) return fail(RL_E_INVALID, "fsc_bins must be 0 or in [2, 1024]");
  if (!std::isfinite(rule->fsc_threshold)) return fail(RL_E_INVALID, "fsc_threshold must be finite");
  *fthr = rule->fsc_threshold == 0.0 ? 1.0 / 7.0 : rule->fsc_threshold;
  const int64_t half[3] = {p->nz / 2, p->ny / 2, p->nx / 2};
  if (p->nz % 2 || p->ny % 2 || p->nx % 2 || half[0] < 1 || half[1] < 1)
    return fail(RL_E_UNSUPPORTED, "FSC-guided stopping needs even dimensions");
  rl_status st = check_shape(half);
  if (st != RL_OK)
    return fail(RL_E_UNSUPPORTED, "FSC-guided stopping: the half-size transforms are not "
                                  "supported (" + g_err + ")");
  return RL_OK;
}

// Transform-only plan of the half shape with its FSC buffers, and the two half-size
// sub-volumes (first use; kept with the plan).
rl_status fsc_stop_setup(rl_plan p, int nbins, int64_t* lcm) {
  if (!p->fsc_sub) {
    Geometry geo;
    geo.boundary = RL_BOUNDARY_PERIODIC;
    const int64_t half[3] = {p->nz / 2, p->ny / 2, p->nx / 2};
    for (int i = 0; i < 3; ++i) geo.grid[i] = geo.vol[i] = geo.psf[i] = half[i];
    rl_plan sub = nullptr;
    rl_status st = build_class(geo, 1, nullptr, p->device, nullptr, p->stream, &sub);
    if (st != RL_OK) return st;
    p->fsc_sub = sub;
  }
  rl_plan sub = p->fsc_sub;
  sub->stream = p->stream;
  hipError_t e;
  const size_t hb = (size_t)sub->nvox * sizeof(float);
  if (!p->fsc_a && (e = hipMalloc(&p->fsc_a, hb)) != hipSuccess)
    return hip_fail(e, "hipMalloc(FSC half volume)");
  if (!p->fsc_b && (e = hipMalloc(&p->fsc_b, hb)) != hipSuccess)
    return hip_fail(e, "hipMalloc(FSC half volume)");
  rl_status st = fsc_lcm(sub, lcm);
  if (st != RL_OK) return st;
  return fsc_buffers(sub, nbins);
}

// Single-image FSC resolution of u into the half-size plan's fsc_out, guarded by
// the plan's stop flag: diagonal split, two forward transforms, shell sums.
rl_status enqueue_fsc_stop(rl_plan p, const float* u, int nbins, double fthr, int64_t lcm) {
  rl_plan sub = p->fsc_sub;
  hipError_t e = rlmi::launch_split_diag(u, (int)p->nz, (int)p->ny, (int)p->nx, p->fsc_a,
                                         p->fsc_b, p->stream, p->active_stop);
  if (rl_status ls = launched(e, p->stream, "split"); ls != RL_OK) return ls;
  sub->stream = p->stream;
  sub->active_stop = p->active_stop;
  rl_status st = enqueue_fsc(sub, p->fsc_a, p->fsc_b, nbins, fthr, lcm);
  sub->active_stop = nullptr;
  return st;
}

// Metric-guided stopping: every launch of the call reads the plan's stop flag
// and does nothing once the metric kernel has set it, so the whole call is
// enqueued at once and ends early on the device without a host round trip.
rl_status iterate_stop_impl(rl_plan p, const float* observed, float* estimate, int max_iter,
                            const rl_stop_rule* rule) {
  rl_status st = check_plan(p);
  if (st != RL_OK) return st;
  if (p->is_batch || !p->stop) return fail(RL_E_UNSUPPORTED, "stop rules need a single-volume plan");
  if (p->accel != RL_ACCEL_NONE)
    return fail(RL_E_UNSUPPORTED, "stop rules are not available with extrapolation");
  if (!rule) return fail(RL_E_INVALID, "rule is NULL");
  if (rule->metric != RL_STOP_LOGLIK && rule->metric != RL_STOP_CHANGE &&
      rule->metric != RL_STOP_PSNR && rule->metric != RL_STOP_SSIM &&
      rule->metric != RL_STOP_FSC)
    return fail(RL_E_INVALID, "unknown stop metric");
  if (!std::isfinite(rule->threshold)) return fail(RL_E_INVALID, "threshold must be finite");
  if (rule->min_iter < 0) return fail(RL_E_INVALID, "min_iter must be >= 0");
  if (max_iter < 0) return fail(RL_E_INVALID, "max_iter must be >= 0");
  const size_t bytes = (size_t)p->vnvox * sizeof(float);
  int dev = p->device;
  if ((st = check_dev_ptr(observed, bytes, &dev, "observed")) != RL_OK) return st;
  if ((st = check_dev_ptr(estimate, bytes, &dev, "estimate")) != RL_OK) return st;
  if ((rule->metric == RL_STOP_PSNR || rule->metric == RL_STOP_SSIM) &&
      (st = check_dev_ptr(rule->reference, bytes, &dev, "reference")) != RL_OK)
    return st;
  int fsc_bins = 0;
  double fsc_thr = 0.0;
  int64_t fsc_l = 0;
  if (rule->metric == RL_STOP_FSC && (st = fsc_stop_check(p, rule, &fsc_bins, &fsc_thr)) != RL_OK)
    return st;
  hipError_t e = hipSetDevice(p->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  if (rule->metric == RL_STOP_SSIM && (st = ssim_buffers(p)) != RL_OK) return st;
  if (rule->metric == RL_STOP_FSC && (st = fsc_stop_setup(p, fsc_bins, &fsc_l)) != RL_OK)
    return st;
  if ((st = ensure_flux_capacity(p, max_iter > 0 ? max_iter : 1, nullptr)) != RL_OK) return st;
  if ((e = hipMemsetAsync(p->stop, 0, 4 * sizeof(int), p->stream)) != hipSuccess)
    return hip_fail(e, "hipMemsetAsync(stop)");
  p->flux_count = max_iter;
  p->stop_call = true;
  p->stop_max = max_iter;
  if (max_iter == 0) return RL_OK;
  const int metric = rule->metric;
  const int groups = (int)p->x_grid.x;
  const SsimGeom sg = ssim_geom(p);
  auto decide = [&](int it) -> rl_status {
    const bool ssim = metric == RL_STOP_SSIM, fsc = metric == RL_STOP_FSC;
    const double* mp = ssim  ? p->ssim_part
                       : fsc ? p->fsc_sub->fsc_out + 4 * (size_t)(fsc_bins + 1)  // resolution
                             : p->met_partials;
    hipError_t me = rlmi::launch_metric(
        mp, ssim ? (int)sg.blocks : fsc ? 1 : groups, metric, it, rule->threshold,
        rule->min_iter, ssim ? (long long)(sg.nxo * sg.nyo * sg.nzo) : (long long)p->vnvox,
        p->mhist, p->stop, p->stream);
    return me == hipSuccess ? RL_OK : hip_fail(me, "metric launch");
  };
  p->active_stop = p->stop;
  st = enqueue_prologue(p, estimate);
  for (int it = 0; it < max_iter && st == RL_OK; ++it) {
    XArgs r = base_xargs(p, p->spec);
    r.d = observed;
    if (metric == RL_STOP_LOGLIK) {
      r.metric = rlmi::MET_LOGLIK;
      r.met_partials = p->met_partials;
    }
    if ((st = run_x(p, metric == RL_STOP_LOGLIK ? rlmi::XM_RATIO_LL : rlmi::XM_RATIO, r,
                    RL_KERNEL_X_RATIO)) != RL_OK)
      break;
    if (metric == RL_STOP_LOGLIK && (st = decide(it)) != RL_OK) break;
    if ((st = run_yz_filter(p, true)) != RL_OK) break;
    XArgs w = base_xargs(p, p->spec);
    w.u = estimate;
    w.partials = p->partials;
    w.iter = it;
    w.do_fwd = it + 1 < max_iter ? 1 : 0;
    const bool fused = metric == RL_STOP_CHANGE || metric == RL_STOP_PSNR;
    if (fused) {
      w.metric = metric == RL_STOP_CHANGE ? rlmi::MET_CHANGE : rlmi::MET_PSNR;
      w.met_partials = p->met_partials;
      w.ref = rule->reference;
    }
    const int umode = !fused                    ? rlmi::XM_UPDATE
                      : metric == RL_STOP_CHANGE ? rlmi::XM_UPDATE_CHG
                                                 : rlmi::XM_UPDATE_PSNR;
    if ((st = run_x(p, umode, w, RL_KERNEL_X_UPDATE)) != RL_OK)
      break;
    if (metric == RL_STOP_SSIM &&
        (st = enqueue_ssim(p, estimate, rule->reference, it == 0)) != RL_OK)
      break;
    if (metric == RL_STOP_FSC &&
        (st = enqueue_fsc_stop(p, estimate, fsc_bins, fsc_thr, fsc_l)) != RL_OK)
      break;
    if (metric != RL_STOP_LOGLIK && (st = decide(it)) != RL_OK) break;
    if (w.do_fwd && (st = run_yz_filter(p, false)) != RL_OK) break;
  }
  p->active_stop = nullptr;
  if (st != RL_OK) return st;
  return enqueue_flux_reduce(p, max_iter, p->stream);
}

// Iterations carried out by the last call with a stop rule (synchronises).
rl_status stop_state(rl_plan p, int* n_done, int* n_hist) {
  int h[4] = {0, 0, 0, 0};
  hipError_t e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return hip_fail(e, "execution");
  if ((e = hipMemcpy(h, p->stop, sizeof(h), hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(e, "hipMemcpy(stop)");
  *n_done = h[0] ? h[1] : p->stop_max;
  *n_hist = h[2];
  return RL_OK;
}

// Half spectrum of a real volume of the plan's shape into `spec` (forward along X,
// Y and Z; no filter).
rl_status forward3(rl_plan p, const float* x, float2* spec) {
  XArgs a = base_xargs(p, spec);
  a.rin = x;
  rl_status st = run_x(p, rlmi::XM_R2C, a, RL_KERNEL_OTHER);
  if (st == RL_OK) st = run_pencil(p, p->py, rlmi::PM_FWD, spec, p->tw_y, RL_KERNEL_OTHER);
  if (st == RL_OK) st = run_pencil(p, p->pz, rlmi::PM_FWD, spec, p->tw_z, RL_KERNEL_OTHER);
  return st;
}

// lcm of the grid dimensions, the common denominator of the exact shell index
// (below 2^21 keeps its integer arithmetic inside 64 bits).
rl_status fsc_lcm(rl_plan p, int64_t* lcm) {
  auto gcd = [](int64_t x, int64_t y) {
    while (y) {
      const int64_t t = x % y;
      x = y;
      y = t;
    }
    return x;
  };
  int64_t l = p->nz;
  l = l / gcd(l, p->ny) * p->ny;
  l = l / gcd(l, p->nx) * p->nx;
  if (l >= ((int64_t)1 << 21))
    return fail(RL_E_UNSUPPORTED, "FSC: lcm of the dimensions must be below 2^21");
  *lcm = l;
  return RL_OK;
}

// Second spectrum and shell-sum buffers of a plan for nbins shells (first use or
// more shells than before).
rl_status fsc_buffers(rl_plan p, int nbins) {
  hipError_t e;
  if (!p->spec2 &&
      (e = hipMalloc(&p->spec2, p->spec_elems * sizeof(float2))) != hipSuccess)
    return hip_fail(e, "hipMalloc(second spectrum)");
  if (nbins + 1 > p->fsc_cap) {
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    else (void)hipDeviceSynchronize();
    (void)hipFree(p->fsc_part);
    (void)hipFree(p->fsc_out);
    p->fsc_part = nullptr;
    p->fsc_out = nullptr;
    p->fsc_cap = 0;
    const size_t groups = (size_t)p->nz * p->xt;
    if ((e = hipMalloc(&p->fsc_part, groups * (nbins + 1) * 3 * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&p->fsc_out, (4 * (size_t)(nbins + 1) + 1) * sizeof(double))) !=
            hipSuccess)
      return hip_fail(e, "hipMalloc(shell sums)");
    p->fsc_cap = nbins + 1;
  }
  return RL_OK;
}

// FSC of volumes a and b of the plan's shape into p->fsc_out (curve, sums,
// resolution); every launch honours the plan's active stop flag.
rl_status enqueue_fsc(rl_plan p, const float* a, const float* b, int nbins, double threshold,
                      int64_t lcm) {
  rl_status st;
  if ((st = forward3(p, a, p->spec)) != RL_OK) return st;
  if ((st = forward3(p, b, p->spec2)) != RL_OK) return st;
  hipError_t e = rlmi::launch_fsc(p->spec, p->spec2, (int)p->nz, (int)p->ny, (int)p->nx,
                                  (int)p->xt, nbins, (long long)lcm, threshold, p->fsc_part,
                                  p->fsc_out, p->stream, p->active_stop);
  return launched(e, p->stream, "shell correlation");
}

rl_status fsc_impl(rl_plan p, const float* a, const float* b, int nbins, double threshold,
                   double* curve, double* resolution) {
  rl_status st = check_plan(p);
  if (st != RL_OK) return st;
  if (p->is_batch) return fail(RL_E_UNSUPPORTED, "rl_fsc takes a single-volume plan");
  if (p->boundary != RL_BOUNDARY_PERIODIC)
    return fail(RL_E_UNSUPPORTED, "rl_fsc needs a periodic plan (its grid is the volume)");
  if (nbins < 2 || nbins > 1024) return fail(RL_E_INVALID, "nbins must be in [2, 1024]");
  if (!std::isfinite(threshold)) return fail(RL_E_INVALID, "threshold must be finite");
  if (!curve) return fail(RL_E_INVALID, "curve is NULL");
  const size_t bytes = (size_t)p->vnvox * sizeof(float);
  int dev = p->device;
  if ((st = check_dev_ptr(a, bytes, &dev, "a")) != RL_OK) return st;
  if ((st = check_dev_ptr(b, bytes, &dev, "b")) != RL_OK) return st;
  hipError_t e = hipSetDevice(p->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  int64_t lcm = 0;
  if ((st = fsc_lcm(p, &lcm)) != RL_OK) return st;
  if ((st = fsc_buffers(p, nbins)) != RL_OK) return st;
  if ((st = enqueue_fsc(p, a, b, nbins, threshold, lcm)) != RL_OK) return st;
  std::vector<double> h(4 * (size_t)(nbins + 1) + 1);
  if ((e = hipStreamSynchronize(p->stream)) != hipSuccess) return hip_fail(e, "execution");
  if ((e = hipMemcpy(h.data(), p->fsc_out, h.size() * sizeof(double), hipMemcpyDeviceToHost)) !=
      hipSuccess)
    return hip_fail(e, "hipMemcpy(shell correlation)");
  for (int i = 0; i <= nbins; ++i) curve[i] = h[(size_t)i];
  if (resolution) *resolution = h[4 * (size_t)(nbins + 1)];
  return RL_OK;
}

// --- batched volumes -----------------------------------------------------------

// Tables of the persistent batched kernel: one PersistClass per shape class, and
// per XCD queue the pass-major run of tiles of its volumes (volumes assigned to
// queues by decreasing voxel count, each to the least loaded queue).
// The persistent batched kernel is switched off: with it, a batch of small volumes
// did not finish within two minutes.  Its completion polls had been compiled into
// plain device-scope loads (the compiler folds an atomic add of zero into a load);
// they now poll with a compare-and-swap that never changes the counter, which has
// not yet run on the GPU.  Plans refuse RL_BATCH_PERSISTENT until it has.
constexpr bool kPersistentBatchEnabled = false;

rl_status setup_persist(rl_plan b) {
  for (rl_plan c : b->classes)
    if (!persist_fits(c))
      return fail(RL_E_INTERNAL, "a shape class is not configured for the persistent kernel");
  hipDeviceProp_t prop;
  std::memset(&prop, 0, sizeof(prop));
  hipError_t e = hipGetDeviceProperties(&prop, b->device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  // gfx950: 32 compute units per XCD
  const int nq = std::max(1, std::min(rlmi::kPersistMaxQueues, prop.multiProcessorCount / 32));
  std::vector<rlmi::PersistClass> pcs(b->classes.size());
  size_t lds = 0;
  for (size_t ci = 0; ci < b->classes.size(); ++ci) {
    rl_plan c = b->classes[ci];
    rlmi::PersistClass& pc = pcs[ci];
    std::memset(&pc, 0, sizeof(pc));
    pc.xr = base_xargs(c, c->spec);
    pc.xr.d_tab = c->d_tab;
    pc.xu = base_xargs(c, c->spec);
    pc.xu.u_tab = c->u_tab;
    pc.xu.partials = c->partials;
    pc.xu.iter_ptr = b->iter_dev;
    pc.xu.do_fwd = 1;
    pc.py = c->py.args;
    pc.pz = c->pz.args;
    pc.py.vstride = pc.pz.vstride = (long long)c->spec_elems;
    pc.py.stop = pc.pz.stop = nullptr;
    pc.sx = c->axx.sc;
    pc.sy = c->py.ax.sc;
    pc.sz = c->pz.ax.sc;
    pc.twx = c->tw_x;
    pc.twy = c->tw_y;
    pc.twz = c->tw_z;
    pc.spec = c->spec;
    pc.otf = c->otf;
    pc.ex = c->axx.E;
    pc.ey = c->py.ax.E;
    pc.ez = c->pz.ax.E;
    pc.xtiles = (int)c->x_grid.x;
    pc.ygx = (int)c->py.grid.x;
    pc.ytiles = (int)(c->py.grid.x * c->py.grid.y);
    pc.zgx = (int)c->pz.grid.x;
    pc.ztiles = (int)(c->pz.grid.x * c->pz.grid.y);
    lds = std::max({lds, c->x_lds, c->py.lds, c->pz.lds});
  }
  // volumes to queues: decreasing voxel count, least loaded queue first
  std::vector<int> order(b->count);
  for (int v = 0; v < b->count; ++v) order[v] = v;
  auto vox = [&](int v) { return b->classes[b->vol_class[v]]->nvox; };
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return vox(a) > vox(c); });
  std::vector<std::vector<int>> qv(nq);
  std::vector<int64_t> load(nq, 0);
  for (int v : order) {
    const int q = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    qv[q].push_back(v);
    load[q] += vox(v);
  }
  hipError_t e2;
  for (int k = 0; k < 2; ++k) {
    const int npass = k == 0 ? rlmi::kPersistPasses : 5;
    std::vector<rlmi::PersistSeg> segs;
    std::vector<int> qseg(nq + 1, 0);
    for (int q = 0; q < nq; ++q) {
      qseg[q] = (int)segs.size();
      int first = 0;
      for (int pass = 0; pass < npass; ++pass)
        for (int v : qv[q]) {
          const int ci = b->vol_class[v];
          const rlmi::PersistClass& pc = pcs[ci];
          const int kind = pass & 3;
          const int tiles = kind == 0 ? pc.xtiles : kind == 2 ? pc.ztiles : pc.ytiles;
          segs.push_back(rlmi::PersistSeg{pass, ci, b->vol_index[v], v, tiles, first});
          first += tiles;
        }
    }
    qseg[nq] = (int)segs.size();
    b->p_qtotal[k].assign(nq, 0);
    for (int q = 0; q < nq; ++q)
      if (qseg[q + 1] > qseg[q])
        b->p_qtotal[k][q] = segs[qseg[q + 1] - 1].first + segs[qseg[q + 1] - 1].tiles;
    if ((e2 = hipMalloc(&b->p_segs[k], segs.size() * sizeof(rlmi::PersistSeg))) != hipSuccess ||
        (e2 = hipMalloc(&b->p_qseg[k], qseg.size() * sizeof(int))) != hipSuccess ||
        (e2 = hipMemcpy(b->p_segs[k], segs.data(), segs.size() * sizeof(rlmi::PersistSeg),
                        hipMemcpyHostToDevice)) != hipSuccess ||
        (e2 = hipMemcpy(b->p_qseg[k], qseg.data(), qseg.size() * sizeof(int),
                        hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(e2, "persistent kernel tables");
  }
  if ((e2 = hipMalloc(&b->p_cls, pcs.size() * sizeof(rlmi::PersistClass))) != hipSuccess ||
      (e2 = hipMemcpy(b->p_cls, pcs.data(), pcs.size() * sizeof(rlmi::PersistClass),
                      hipMemcpyHostToDevice)) != hipSuccess ||
      (e2 = hipMalloc(&b->p_error, rlmi::kPersistMaxQueues * sizeof(int))) != hipSuccess)
    return hip_fail(e2, "persistent kernel tables");
  int per_cu = 0;
  if ((e2 = rlmi::persist_occupancy(lds, &per_cu)) != hipSuccess || per_cu < 1)
    return hip_fail(e2 != hipSuccess ? e2 : hipErrorInvalidConfiguration,
                    "persistent kernel occupancy");
  b->p_host = pcs;
  b->p_nq = nq;
  b->p_lds = lds;
  b->p_grid = per_cu * prop.multiProcessorCount;
  b->p_nvrow = b->count;
  b->persist = true;
  return RL_OK;
}

// Per-iteration tickets and completion counters for n_iter iterations.
rl_status ensure_persist_capacity(rl_plan b, int n_iter, bool* grew) {
  *grew = false;
  if (n_iter <= b->p_cap) return RL_OK;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  else (void)hipDeviceSynchronize();
  (void)hipFree(b->p_tickets);
  (void)hipFree(b->p_done);
  b->p_tickets = b->p_done = nullptr;
  b->p_cap = 0;
  hipError_t e;
  if ((e = hipMalloc(&b->p_tickets, (size_t)n_iter * b->p_nq * sizeof(int))) != hipSuccess ||
      (e = hipMalloc(&b->p_done, (size_t)n_iter * b->p_nvrow * rlmi::kPersistPasses *
                                     sizeof(int))) != hipSuccess)
    return hip_fail(e, "hipMalloc(persistent counters)");
  b->p_cap = n_iter;
  *grew = true;
  return RL_OK;
}

rlmi::PersistArgs persist_args(rl_plan b, int k) {
  rlmi::PersistArgs a;
  std::memset(&a, 0, sizeof(a));
  a.cls = b->p_cls;
  a.segs = b->p_segs[k];
  a.qseg = b->p_qseg[k];
  a.nq = b->p_nq;
  a.npass = k == 0 ? rlmi::kPersistPasses : 5;
  a.nvrow = b->p_nvrow;
  a.iter_ptr = b->iter_dev;
  a.tickets = b->p_tickets;
  a.done = b->p_done;
  a.error = b->p_error;
  a.spin_limit = 1 << 16;  // a small fraction of a second of polling
  return a;
}

rl_status create_batch_impl(int count, const int64_t* shapes, const float* const* psfs,
                            int boundary, const rl_options* opt, rl_plan* out) {
  if (!out) return fail(RL_E_INVALID, "out is NULL");
  *out = nullptr;
  if (count < 1 || count > 65535) return fail(RL_E_INVALID, "count must be in [1, 65535]");
  if (!shapes || !psfs) return fail(RL_E_INVALID, "shapes or psfs is NULL");
  rl_status st;
  for (int v = 0; v < count; ++v) {
    if ((st = check_shape(shapes + 3 * v)) != RL_OK)
      return fail(st, "volume " + std::to_string(v) + ": " + g_err);
    if ((st = check_options(shapes + 3 * v, opt)) != RL_OK)
      return fail(st, "volume " + std::to_string(v) + ": " + g_err);
    if (!psfs[v]) return fail(RL_E_INVALID, "psf of volume " + std::to_string(v) + " is NULL");
    if (opt && opt->accel != RL_ACCEL_NONE)
      return fail(RL_E_UNSUPPORTED, "extrapolation is available for single-volume plans only");
    if (reinterpret_cast<uintptr_t>(psfs[v]) % 16 != 0)
      return fail(RL_E_INVALID, "psf of volume " + std::to_string(v) + " is not 16-byte aligned");
  }
  if ((st = check_boundary(boundary)) != RL_OK) return st;
  if (boundary != RL_BOUNDARY_PERIODIC)
    return fail(RL_E_UNSUPPORTED, "batch plans use the periodic boundary");
  if (opt && (opt->psf_shape[0] || opt->psf_shape[1] || opt->psf_shape[2]))
    return fail(RL_E_UNSUPPORTED, "batch plans take PSFs of their volumes' shapes");
  if (opt && opt->tile_x != 0)
    return fail(RL_E_INVALID, "batch plans choose work-group widths per shape (tile_x must be 0)");
  const int mode = opt ? opt->batch_mode : RL_BATCH_AUTO;
  if (mode != RL_BATCH_AUTO && mode != RL_BATCH_PERSISTENT && mode != RL_BATCH_GRAPH)
    return fail(RL_E_INVALID, "unknown batch_mode");
  if (mode == RL_BATCH_PERSISTENT && !kPersistentBatchEnabled)
    return fail(RL_E_UNSUPPORTED, "the persistent batched kernel is switched off: its completion "
                                  "waits did not finish on the GPU (batch_mode AUTO or GRAPH "
                                  "runs the per-pass graph)");
  // the persistent kernel needs 128-thread launch shapes for every shape class
  bool all_fit = kPersistentBatchEnabled && (!opt || opt->precision == RL_PRECISION_FP32);
  for (int v = 0; v < count && all_fit; ++v) {
    Choice c;
    all_fit = persist_choice(shapes[3 * v], shapes[3 * v + 1], shapes[3 * v + 2], &c);
  }
  if (mode == RL_BATCH_PERSISTENT && !all_fit)
    return fail(RL_E_UNSUPPORTED, "a volume shape has no launch shapes for the persistent kernel "
                                  "(every pass must split into 128-thread work-groups, FP32)");
  const bool use_persist = all_fit && mode != RL_BATCH_GRAPH;
  if ((st = check_device_present()) != RL_OK) return st;
  int device = -1;
  for (int v = 0; v < count; ++v) {
    const int64_t nvox = shapes[3 * v] * shapes[3 * v + 1] * shapes[3 * v + 2];
    if ((st = check_dev_ptr(psfs[v], (size_t)nvox * sizeof(float), &device,
                            "psf of a volume")) != RL_OK)
      return st;
  }
  rl_plan b = new (std::nothrow) rl_plan_s();
  if (!b) return fail(RL_E_NOMEM, "host allocation failed");
  b->is_batch = true;
  b->device = device;
  b->stream = opt ? reinterpret_cast<hipStream_t>(opt->stream) : nullptr;
  b->count = count;
  b->nz = shapes[0];
  b->ny = shapes[1];
  b->nx = shapes[2];
  b->vol_class.assign(count, -1);
  b->vol_index.assign(count, -1);
  hipError_t e;
  if ((e = hipSetDevice(device)) != hipSuccess) {
    delete b;
    return hip_fail(e, "hipSetDevice");
  }
  if ((e = hipMalloc(&b->iter_dev, sizeof(int))) != hipSuccess ||
      (e = hipEventCreateWithFlags(&b->fork_event, hipEventDisableTiming)) != hipSuccess ||
      (e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking)) != hipSuccess) {
    st = hip_fail(e, "batch setup");
    release(b);
    return st;
  }
  // classes: volumes of equal shape, in order of first appearance
  for (int v = 0; v < count; ++v) {
    if (b->vol_class[v] >= 0) continue;
    const int64_t* sh = shapes + 3 * v;
    std::vector<int> members;
    for (int w = v; w < count; ++w)
      if (shapes[3 * w] == sh[0] && shapes[3 * w + 1] == sh[1] && shapes[3 * w + 2] == sh[2])
        members.push_back(w);
    hipStream_t cs = nullptr;
    hipEvent_t ce = nullptr;
    if ((e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess) {
      st = hip_fail(e, "hipStreamCreate");
      release(b);
      return st;
    }
    b->cls_streams.push_back(cs);
    if ((e = hipEventCreateWithFlags(&ce, hipEventDisableTiming)) != hipSuccess) {
      st = hip_fail(e, "hipEventCreate");
      release(b);
      return st;
    }
    b->cls_events.push_back(ce);
    std::vector<const float*> cpsf;
    for (int w : members) cpsf.push_back(psfs[w]);
    rl_plan c = nullptr;
    Geometry geo;
    geo.boundary = RL_BOUNDARY_PERIODIC;
    for (int i = 0; i < 3; ++i) geo.grid[i] = geo.vol[i] = geo.psf[i] = sh[i];
    if ((st = build_class(geo, (int)members.size(), cpsf.data(), device, opt, cs, &c,
                          use_persist)) != RL_OK) {
      const std::string msg = g_err;
      release(b);
      return fail(st, msg);
    }
    const int ci = (int)b->classes.size();
    b->classes.push_back(c);
    for (size_t k = 0; k < members.size(); ++k) {
      b->vol_class[members[k]] = ci;
      b->vol_index[members[k]] = (int)k;
    }
  }
  if (use_persist && (st = setup_persist(b)) != RL_OK) {
    const std::string msg = g_err;
    release(b);
    return fail(st, msg);
  }
  plan_register(b);
  *out = b;
  return RL_OK;
}

// One iteration of one shape class, advancing the class's own iteration counter,
// captured on the class's private stream and launched there: the classes of a
// batch run their iterations independently of each other and meet once per
// call, not once per iteration.
rl_status capture_class_graph(rl_plan c, bool do_fwd, hipGraphExec_t* exec) {
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
  rl_status st = enqueue_iteration(c, nullptr, nullptr, 0, c->iter_dev, do_fwd);
  if (st == RL_OK && (e = rlmi::launch_advance(c->iter_dev, c->stream)) != hipSuccess)
    st = hip_fail(e, "iteration counter launch");
  const hipError_t ee = hipStreamEndCapture(c->stream, &g);
  if (st != RL_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (ee != hipSuccess) return hip_fail(ee, "hipStreamEndCapture");
  e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  return e == hipSuccess ? RL_OK : hip_fail(e, "hipGraphInstantiate");
}

// One persistent launch (k = 0: every pass, 1: the last iteration) and the
// iteration counter's advance, captured on the plan's private stream.
rl_status capture_persist_graph(rl_plan b, int k, hipGraphExec_t* exec) {
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
  hipError_t le = rlmi::launch_persist(persist_args(b, k), b->p_grid, b->p_lds, b->cap_stream);
  if (le == hipSuccess) le = rlmi::launch_advance(b->iter_dev, b->cap_stream);
  e = hipStreamEndCapture(b->cap_stream, &g);
  if (le != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return hip_fail(le, "persistent kernel launch");
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  return e == hipSuccess ? RL_OK : hip_fail(e, "hipGraphInstantiate");
}

rl_status iterate_batch_impl(rl_plan b, const float* const* observed, float* const* estimate,
                             int n_iter) {
  rl_status st = check_plan(b);
  if (st != RL_OK) return st;
  if (!b->is_batch) return fail(RL_E_INVALID, "not a batch plan (use rl_iterate)");
  if (n_iter < 0) return fail(RL_E_INVALID, "n_iter must be >= 0");
  if (!observed || !estimate) return fail(RL_E_INVALID, "observed or estimate is NULL");
  for (int v = 0; v < b->count; ++v) {
    const rl_plan c = b->classes[b->vol_class[v]];
    const size_t bytes = (size_t)c->vnvox * sizeof(float);
    int dev = b->device;
    if ((st = check_dev_ptr(observed[v], bytes, &dev, "observed volume")) != RL_OK ||
        (st = check_dev_ptr(estimate[v], bytes, &dev, "estimate volume")) != RL_OK)
      return fail(st, "volume " + std::to_string(v) + ": " + g_err);
  }
  if (n_iter == 0) return RL_OK;
  hipError_t e = hipSetDevice(b->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  bool rebuild = false;
  for (rl_plan c : b->classes) {
    bool grew = false;
    if ((st = ensure_flux_capacity(c, n_iter, &grew)) != RL_OK) return st;
    rebuild = rebuild || grew;
    c->flux_count = n_iter;
  }
  if (b->persist) {
    bool grew = false;
    if ((st = ensure_persist_capacity(b, n_iter, &grew)) != RL_OK) return st;
    rebuild = rebuild || grew;
  }
  if (rebuild && b->persist) {  // the classes' flux partial tables may have moved
    for (size_t ci = 0; ci < b->classes.size(); ++ci)
      b->p_host[ci].xu.partials = b->classes[ci]->partials;
    if ((e = hipMemcpy(b->p_cls, b->p_host.data(),
                       b->p_host.size() * sizeof(rlmi::PersistClass), hipMemcpyHostToDevice)) !=
        hipSuccess)
      return hip_fail(e, "persistent kernel tables");
  }
  if (rebuild) {  // partial tables moved: captured kernel arguments are stale
    if (b->graph_full) (void)hipGraphExecDestroy(b->graph_full);
    if (b->graph_last) (void)hipGraphExecDestroy(b->graph_last);
    b->graph_full = b->graph_last = nullptr;
    for (rl_plan c : b->classes) {
      if (c->graph_full) (void)hipGraphExecDestroy(c->graph_full);
      if (c->graph_last) (void)hipGraphExecDestroy(c->graph_last);
      c->graph_full = c->graph_last = nullptr;
    }
  }
  if (b->persist) {
    if (!b->graph_full && (st = capture_persist_graph(b, 0, &b->graph_full)) != RL_OK) return st;
    if (!b->graph_last && (st = capture_persist_graph(b, 1, &b->graph_last)) != RL_OK) return st;
  } else {
    for (rl_plan c : b->classes) {
      if (!c->graph_full && (st = capture_class_graph(c, true, &c->graph_full)) != RL_OK) return st;
      if (!c->graph_last && (st = capture_class_graph(c, false, &c->graph_last)) != RL_OK)
        return st;
    }
  }
  // per-volume pointer tables (ordered after earlier work on b->stream)
  for (size_t ci = 0; ci < b->classes.size(); ++ci) {
    rl_plan c = b->classes[ci];
    std::vector<const float*> dt(c->count);
    std::vector<float*> ut(c->count);
    for (int v = 0; v < b->count; ++v)
      if (b->vol_class[v] == (int)ci) {
        dt[b->vol_index[v]] = observed[v];
        ut[b->vol_index[v]] = estimate[v];
      }
    if ((e = hipMemcpyAsync(c->d_tab, dt.data(), dt.size() * sizeof(float*),
                            hipMemcpyHostToDevice, b->stream)) != hipSuccess ||
        (e = hipMemcpyAsync(c->u_tab, ut.data(), ut.size() * sizeof(float*),
                            hipMemcpyHostToDevice, b->stream)) != hipSuccess)
      return hip_fail(e, "pointer tables");
  }
  if ((e = rlmi::launch_set_counter(b->iter_dev, 0, b->stream)) != hipSuccess)
    return hip_fail(e, "iteration counter launch");
  if (b->persist &&
      ((e = rlmi::launch_zero_ints(b->p_tickets, (long long)n_iter * b->p_nq, b->stream)) !=
           hipSuccess ||
       (e = rlmi::launch_zero_ints(b->p_done,
                                   (long long)n_iter * b->p_nvrow * rlmi::kPersistPasses,
                                   b->stream)) != hipSuccess ||
       (e = rlmi::launch_zero_ints(b->p_error, rlmi::kPersistMaxQueues, b->stream)) !=
           hipSuccess))
    return hip_fail(e, "persistent counters");
  // prologue per class, forked from b->stream; with the persistent kernel the
  // classes join again before its iterations, otherwise each class runs its
  // iterations on its own stream (its counter from 0) and they join at the end
  if ((e = hipEventRecord(b->fork_event, b->stream)) != hipSuccess)
    return hip_fail(e, "hipEventRecord");
  for (size_t ci = 0; ci < b->classes.size(); ++ci) {
    rl_plan c = b->classes[ci];
    if ((e = hipStreamWaitEvent(c->stream, b->fork_event, 0)) != hipSuccess)
      return hip_fail(e, "hipStreamWaitEvent");
    if ((st = enqueue_prologue(c, nullptr)) != RL_OK) return st;
    if (!b->persist && (e = rlmi::launch_set_counter(c->iter_dev, 0, c->stream)) != hipSuccess)
      return hip_fail(e, "iteration counter launch");
    if (b->persist && ((e = hipEventRecord(b->cls_events[ci], c->stream)) != hipSuccess ||
                       (e = hipStreamWaitEvent(b->stream, b->cls_events[ci], 0)) != hipSuccess))
      return hip_fail(e, "prologue join");
  }
  if (b->persist) {
    for (int it = 0; it < n_iter; ++it)
      if ((st = launched(hipGraphLaunch(it + 1 < n_iter ? b->graph_full : b->graph_last,
                                        b->stream),
                         b->stream, "batch iteration graph")) != RL_OK)
        return st;
  } else {
    for (int it = 0; it < n_iter; ++it)
      for (rl_plan c : b->classes)
        if ((st = launched(hipGraphLaunch(it + 1 < n_iter ? c->graph_full : c->graph_last,
                                          c->stream),
                           c->stream, "class iteration graph")) != RL_OK)
          return st;
    for (size_t ci = 0; ci < b->classes.size(); ++ci)
      if ((e = hipEventRecord(b->cls_events[ci], b->classes[ci]->stream)) != hipSuccess ||
          (e = hipStreamWaitEvent(b->stream, b->cls_events[ci], 0)) != hipSuccess)
        return hip_fail(e, "class join");
  }
  for (rl_plan c : b->classes)
    if ((st = enqueue_flux_reduce(c, n_iter, b->stream)) != RL_OK) return st;
  b->batch_n = n_iter;
  return RL_OK;
}

rl_status conv_impl(rl_plan p, const float* x, float* out) {
  rl_status st = check_plan(p);
  if (st != RL_OK) return st;
  if (p->is_batch) return fail(RL_E_UNSUPPORTED, "conv3d_fft takes a single-volume plan");
  const size_t bytes = (size_t)p->vnvox * sizeof(float);
  int dev = p->device;
  if ((st = check_dev_ptr(x, bytes, &dev, "x")) != RL_OK) return st;
  if ((st = check_dev_ptr(out, bytes, &dev, "out")) != RL_OK) return st;
  hipError_t e = hipSetDevice(p->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  XArgs a = base_xargs(p, p->spec);
  a.rin = x;
  if ((st = run_x(p, rlmi::XM_R2C, a, RL_KERNEL_X_R2C)) != RL_OK) return st;
  if ((st = run_yz_filter(p, false)) != RL_OK) return st;
  XArgs c = base_xargs(p, p->spec);
  c.rout = out;
  return run_x(p, rlmi::XM_C2R, c, RL_KERNEL_X_C2R);
}

}  // namespace

namespace {
// A roctx range over one entry point, so that the calls appear by name in a
// rocprofv3 marker trace beside their kernels; without an attached tool the two
// calls return at once.
struct ApiRange {
  explicit ApiRange(const char* name) { roctxRangePushA(name); }
  ~ApiRange() { roctxRangePop(); }
  ApiRange(const ApiRange&) = delete;
  ApiRange& operator=(const ApiRange&) = delete;
};
}  // namespace

extern "C" {

rl_status rl_plan_create(const int64_t shape[3], const float* psf, int boundary, rl_plan* out) {
  ApiRange range("rl_plan_create");
  try {
    return create_impl(shape, psf, boundary, nullptr, out);
  } catch (const std::bad_alloc&) {
    return fail(RL_E_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(RL_E_INTERNAL, "unexpected exception in rl_plan_create");
  }
}

rl_status rl_plan_create_ex(const int64_t shape[3], const float* psf, int boundary,
                            const rl_options* opt, rl_plan* out) {
  ApiRange range("rl_plan_create_ex");
  try {
    return create_impl(shape, psf, boundary, opt, out);
  } catch (const std::bad_alloc&) {
    return fail(RL_E_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(RL_E_INTERNAL, "unexpected exception in rl_plan_create_ex");
  }
}

rl_status rl_plan_create_batch(int count, const int64_t* shapes, const float* const* psfs,
                               int boundary, const rl_options* opt, rl_plan* out) {
  ApiRange range("rl_plan_create_batch");
  try {
    return create_batch_impl(count, shapes, psfs, boundary, opt, out);
  } catch (const std::bad_alloc&) {
    return fail(RL_E_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(RL_E_INTERNAL, "unexpected exception in rl_plan_create_batch");
  }
}

rl_status rl_iterate_batch(rl_plan p, const float* const* observed, float* const* estimate,
                           int n_iter) {
  ApiRange range("rl_iterate_batch");
  try {
    return iterate_batch_impl(p, observed, estimate, n_iter);
  } catch (...) {
    return fail(RL_E_INTERNAL, "unexpected exception in rl_iterate_batch");
  }
}

rl_status rl_iterate(rl_plan p, const float* observed, float* estimate, int n_iter) {
  ApiRange range("rl_iterate");
  try {
    return iterate_impl(p, observed, estimate, n_iter);
  } catch (...) {
    return fail(RL_E_INTERNAL, "unexpected exception in rl_iterate");
  }
}

rl_status rl_iterate_noalloc(rl_plan p, const float* observed, float* estimate, int n_iter) {
  ApiRange range("rl_iterate_noalloc");
  try {
    return iterate_noalloc_impl(p, observed, estimate, n_iter);
  } catch (...) {
    return fail(RL_E_INTERNAL, "unexpected exception in rl_iterate_noalloc");
  }
}

rl_status conv3d_fft(rl_plan p, const float* x, float* out) {
  ApiRange range("conv3d_fft");
  try {
    return conv_impl(p, x, out);
  } catch (...) {
    return fail(RL_E_INTERNAL, "unexpected exception in conv3d_fft");
  }
}

void rl_plan_destroy(rl_plan p) {
  if (!p || !plan_unregister(p)) return;
  try {
    release(p);
  } catch (...) {
  }
}

rl_status rl_plan_set_stream(rl_plan p, void* hip_stream) {
  rl_status st = check_plan(p);
  if (st != RL_OK) return st;
  p->stream = reinterpret_cast<hipStream_t>(hip_stream);
  return RL_OK;
}

rl_status rl_plan_get_flux(rl_plan p, double* flux, int cap, int* n_written) {
  rl_status st = check_plan(p);
  if (st != RL_OK) return st;
  if (!n_written) return fail(RL_E_INVALID, "n_written is NULL");
  if (cap < 0 || (cap > 0 && !flux)) return fail(RL_E_INVALID, "flux buffer is NULL");
  hipError_t e = hipSetDevice(p->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  if ((e = hipStreamSynchronize(p->stream)) != hipSuccess) return hip_fail(e, "execution");
  std::vector<double> h;
  if (!p->is_batch) {
    int n = p->flux_count;
    if (p->stop_call) {
      int done = 0, nh = 0;
      if ((st = stop_state(p, &done, &nh)) != RL_OK) return st;
      n = done < n ? done : n;
    }
    h.resize((size_t)n);
    if (n > 0 && (e = hipMemcpy(h.data(), p->flux, (size_t)n * sizeof(double),
                                hipMemcpyDeviceToHost)) != hipSuccess)
      return hip_fail(e, "hipMemcpy(flux)");
  } else {
    if (p->persist) {
      int errs[rlmi::kPersistMaxQueues] = {};
      if ((e = hipMemcpy(errs, p->p_error, sizeof(errs), hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "hipMemcpy(persistent kernel state)");
      int err = 0;
      for (int q = 0; q < rlmi::kPersistMaxQueues; ++q) err |= errs[q];
      if (err)
        return fail(RL_E_INTERNAL, "persistent kernel: a wait for a completion counter ran "
                                   "past its bound; the estimates of that call are not valid");
      // every queue handed out all of its tiles in every launch (a queue whose XCD
      // ran no work-group would leave its volumes untouched)
      const int n = p->batch_n;
      std::vector<int> tk((size_t)n * p->p_nq);
      if (n > 0 && (e = hipMemcpy(tk.data(), p->p_tickets, tk.size() * sizeof(int),
                                  hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "hipMemcpy(persistent kernel state)");
      for (int it = 0; it < n; ++it)
        for (int q = 0; q < p->p_nq; ++q)
          if (tk[(size_t)it * p->p_nq + q] < p->p_qtotal[it + 1 < n ? 0 : 1][q])
            return fail(RL_E_INTERNAL, "persistent kernel: queue " + std::to_string(q) +
                                           " was not drained in iteration " + std::to_string(it));
    }
    // volume-major: flux[v * n + it]
    const int n = p->batch_n;
    h.assign((size_t)n * p->count, 0.0);
    for (size_t ci = 0; ci < p->classes.size() && n > 0; ++ci) {
      rl_plan c = p->classes[ci];
      std::vector<double> cf((size_t)n * c->count);
      if ((e = hipMemcpy(cf.data(), c->flux, cf.size() * sizeof(double),
                         hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "hipMemcpy(flux)");
      for (int v = 0; v < p->count; ++v)
        if (p->vol_class[v] == (int)ci)
          for (int it = 0; it < n; ++it)
            h[(size_t)v * n + it] = cf[(size_t)it * c->count + p->vol_index[v]];
    }
  }
  const int n = (int)h.size();
  *n_written = n;
  for (int i = 0; i < n && i < cap; ++i) flux[i] = h[(size_t)i];
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(h[(size_t)i]))
      return fail(RL_E_NUMERIC, "non-finite flux at entry " + std::to_string(i));
  return RL_OK;
}

rl_status rl_ssim(rl_plan p, const float* u, const float* reference, double* value) {
  ApiRange range("rl_ssim");
  try {
    return ssim_impl(p, u, reference, value);
  } catch (...) {
    return fail(RL_E_INTERNAL, "unexpected exception in rl_ssim");
  }
}

rl_status rl_fsc(rl_plan p, const float* a, const float* b, int nbins, double threshold,
                 double* curve, double* resolution) {
  ApiRange range("rl_fsc");
  try {
    return fsc_impl(p, a, b, nbins, threshold, curve, resolution);
  } catch (...) {
    return fail(RL_E_INTERNAL, "unexpected exception in rl_fsc");
  }
}

rl_status rl_split_diagonal(const float* u, const int64_t shape[3], float* a, float* b,
                            void* hip_stream) {
  try {
    if (!shape) return fail(RL_E_INVALID, "shape is NULL");
    for (int i = 0; i < 3; ++i)
      if (shape[i] < 2 || shape[i] % 2 != 0 || shape[i] > ((int64_t)1 << 30))
        return fail(RL_E_INVALID, "every dimension must be even and >= 2");
    if (shape[1] / 2 > 65535 || shape[0] / 2 > 65535)
      return fail(RL_E_UNSUPPORTED, "ny/2 and nz/2 must be <= 65535");
    const int64_t n = shape[0] * shape[1] * shape[2];
    int dev = -1;
    rl_status st = check_dev_ptr(u, (size_t)n * sizeof(float), &dev, "u");
    if (st != RL_OK) return st;
    if ((st = check_dev_ptr(a, (size_t)(n / 8) * sizeof(float), &dev, "a")) != RL_OK) return st;
    if ((st = check_dev_ptr(b, (size_t)(n / 8) * sizeof(float), &dev, "b")) != RL_OK) return st;
    hipError_t e = hipSetDevice(dev);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    e = rlmi::launch_split_diag(u, (int)shape[0], (int)shape[1], (int)shape[2], a, b,
                                reinterpret_cast<hipStream_t>(hip_stream));
    return e == hipSuccess ? RL_OK : hip_fail(e, "split launch");
  } catch (...) {
    return fail(RL_E_INTERNAL, "unexpected exception in rl_split_diagonal");
  }
}

rl_status rl_iterate_stop(rl_plan p, const float* observed, float* estimate, int max_iter,
                          const rl_stop_rule* rule) {
  ApiRange range("rl_iterate_stop");
  try {
    return iterate_stop_impl(p, observed, estimate, max_iter, rule);
  } catch (...) {
    return fail(RL_E_INTERNAL, "unexpected exception in rl_iterate_stop");
  }
}

rl_status rl_plan_get_stop(rl_plan p, int* n_done, double* history, int cap, int* n_history) {
  rl_status st = check_plan(p);
  if (st != RL_OK) return st;
  if (!n_done || !n_history) return fail(RL_E_INVALID, "n_done or n_history is NULL");
  if (cap < 0 || (cap > 0 && !history)) return fail(RL_E_INVALID, "history buffer is NULL");
  if (p->is_batch || !p->stop_call)
    return fail(RL_E_INVALID, "the plan's last call was not rl_iterate_stop");
  hipError_t e = hipSetDevice(p->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  int done = 0, nh = 0;
  if ((st = stop_state(p, &done, &nh)) != RL_OK) return st;
  std::vector<double> h((size_t)nh);
  if (nh > 0 && (e = hipMemcpy(h.data(), p->mhist, (size_t)nh * sizeof(double),
                               hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(e, "hipMemcpy(metric history)");
  *n_done = done;
  *n_history = nh;
  for (int i = 0; i < nh && i < cap; ++i) history[i] = h[(size_t)i];
  return RL_OK;
}

rl_status rl_plan_get_alpha(rl_plan p, double* alpha, int cap, int* n_written) {
  rl_status st = check_plan(p);
  if (st != RL_OK) return st;
  if (!n_written) return fail(RL_E_INVALID, "n_written is NULL");
  if (cap < 0 || (cap > 0 && !alpha)) return fail(RL_E_INVALID, "alpha buffer is NULL");
  if (p->is_batch || p->accel == RL_ACCEL_NONE)
    return fail(RL_E_INVALID, "the plan was not created with extrapolation");
  hipError_t e = hipSetDevice(p->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  if ((e = hipStreamSynchronize(p->stream)) != hipSuccess) return hip_fail(e, "execution");
  const int n = p->flux_count;
  std::vector<double> h((size_t)n);
  if (n > 0 && (e = hipMemcpy(h.data(), p->alpha64, (size_t)n * sizeof(double),
                              hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(e, "hipMemcpy(alpha)");
  *n_written = n;
  for (int i = 0; i < n && i < cap; ++i) alpha[i] = h[(size_t)i];
  return RL_OK;
}

rl_status rl_plan_get_grid(rl_plan p, int64_t grid[3]) {
  rl_status st = check_plan(p);
  if (st != RL_OK) return st;
  if (!grid) return fail(RL_E_INVALID, "grid is NULL");
  if (p->is_batch) p = p->classes[0];
  grid[0] = p->nz;
  grid[1] = p->ny;
  grid[2] = p->nx;
  return RL_OK;
}

rl_status rl_plan_get_info(rl_plan p, int64_t shape[3], int64_t* spectrum_pitch) {
  rl_status st = check_plan(p);
  if (st != RL_OK) return st;
  if (shape) {
    shape[0] = p->is_batch ? p->nz : p->vz;
    shape[1] = p->is_batch ? p->ny : p->vy;
    shape[2] = p->is_batch ? p->nx : p->vx;
  }
  if (spectrum_pitch) *spectrum_pitch = p->xt * rlmi::kTile;
  return RL_OK;
}

rl_status rl_plan_get_launch(rl_plan p, int out[8]) {
  rl_status st = check_plan(p);
  if (st != RL_OK) return st;
  if (!out) return fail(RL_E_INVALID, "out is NULL");
  out[7] = p->persist ? 1 : 0;
  if (p->is_batch) p = p->classes[0];  // configuration of the first volume's shape
  out[0] = p->ch_x_e;
  out[1] = p->ch_y_e;
  out[2] = p->ch_y_txb;
  out[3] = p->ch_z_e;
  out[4] = p->ch_z_txb;
  out[5] = p->tuned ? 1 : 0;
  out[6] = p->ch_z_swap;
  return RL_OK;
}

rl_status rl_plan_time_pass(rl_plan p, int kind, const float* observed, float* estimate,
                            int reps, double* ms_per_launch) {
  ApiRange range("rl_plan_time_pass");
  rl_status st = check_plan(p);
  if (st != RL_OK) return st;
  if (p->is_batch) return fail(RL_E_UNSUPPORTED, "time passes on a single-volume plan");
  if (!ms_per_launch) return fail(RL_E_INVALID, "ms_per_launch is NULL");
  if (reps < 1 || reps > 100000) return fail(RL_E_INVALID, "reps must be in [1, 100000]");
  if (kind != RL_KERNEL_X_RATIO && kind != RL_KERNEL_X_UPDATE && kind != RL_KERNEL_Y &&
      kind != RL_KERNEL_Z_OTF)
    return fail(RL_E_INVALID, "kind must be X_RATIO, X_UPDATE, Y or Z_OTF");
  const size_t bytes = (size_t)p->vnvox * sizeof(float);
  int dev = p->device;
  if ((st = check_dev_ptr(observed, bytes, &dev, "observed")) != RL_OK) return st;
  if ((st = check_dev_ptr(estimate, bytes, &dev, "estimate")) != RL_OK) return st;
  hipError_t e = hipSetDevice(p->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  const bool timing = p->timing;
  p->timing = false;
  auto one = [&]() -> rl_status {
    switch (kind) {
      case RL_KERNEL_X_RATIO: {
        XArgs r = base_xargs(p, p->spec);
        r.d = observed;
        return run_x(p, rlmi::XM_RATIO, r, kind);
      }
      case RL_KERNEL_X_UPDATE: {
        XArgs w = base_xargs(p, p->spec);
        w.u = estimate;
        w.partials = p->partials;
        w.do_fwd = 1;
        return run_x(p, rlmi::XM_UPDATE, w, kind);
      }
      case RL_KERNEL_Y:
        return run_y_fwd(p);
      default:
        return run_pencil(p, p->pz, rlmi::PM_FKI, p->spec, p->tw_z, kind, 0, (int)p->vz,
                          (int)p->vz);
    }
  };
  hipEvent_t a = nullptr, b = nullptr;
  if ((e = hipEventCreate(&a)) != hipSuccess || (e = hipEventCreate(&b)) != hipSuccess) {
    if (a) (void)hipEventDestroy(a);
    p->timing = timing;
    return hip_fail(e, "hipEventCreate");
  }
  st = one();  // warm-up
  if (st == RL_OK && (e = hipEventRecord(a, p->stream)) != hipSuccess) st = hip_fail(e, "record");
  for (int r = 0; r < reps && st == RL_OK; ++r) st = one();
  if (st == RL_OK && (e = hipEventRecord(b, p->stream)) != hipSuccess) st = hip_fail(e, "record");
  if (st == RL_OK && (e = hipEventSynchronize(b)) != hipSuccess) st = hip_fail(e, "execution");
  float ms = 0.f;
  if (st == RL_OK && (e = hipEventElapsedTime(&ms, a, b)) != hipSuccess) st = hip_fail(e, "elapsed");
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  p->timing = timing;
  if (st == RL_OK) *ms_per_launch = (double)ms / reps;
  return st;
}

rl_status rl_plan_get_pass_kernel(rl_plan p, int kind, char* name, size_t cap, int64_t* threads) {
  rl_status st = check_plan(p);
  if (st != RL_OK) return st;
  if (p->is_batch) return fail(RL_E_UNSUPPORTED, "pass kernels of a single-volume plan");
  if (!name || !threads) return fail(RL_E_INVALID, "name or threads is NULL");
  std::string s;
  int64_t n = 0;
  auto pencil = [&](const Pencil& pc, int m0, int m1) {
    // the instantiation launch_pencil picks for this shape and precision
    const int maxt = (int)pc.block.x > rlmi::kPencilMaxThreads ? 1024 : rlmi::kPencilMaxThreads;
    const int prec = (pc.ax.E == 16 && pc.block.x % 64 == 0) ? p->precision : 0;
    const int cl = rlmi::pencil_compiled_len(pc.ax.E, pc.args.L, (int)pc.block.x);
    for (int m : {m0, m1}) {
      if (!s.empty()) s += "|";
      if (cl > 0)
        s += "k_pencil_ct<" + std::to_string(pc.ax.E) + ", " + std::to_string(m) + ", " +
             std::to_string(prec) + ", " + std::to_string(cl) + ">";
      else
        s += "k_pencil<" + std::to_string(pc.ax.E) + ", " + std::to_string(m) + ", " +
             std::to_string(maxt) + ", " + std::to_string(prec) + ">";
    }
    n = (int64_t)pc.grid.x * pc.grid.y * pc.block.x;
  };
  switch (kind) {
    case RL_KERNEL_X_RATIO:
    case RL_KERNEL_X_UPDATE:
    {
      const int mode = kind == RL_KERNEL_X_RATIO ? (int)rlmi::XM_RATIO : (int)rlmi::XM_UPDATE;
      const int prec = p->axx.E == 16 ? p->precision : 0;
      s = "k_xrow<" + std::to_string(p->axx.E) + ", " + std::to_string(mode) + ", " +
          std::to_string(prec) + ", " +
          std::to_string(rlmi::xrow_compiled_len(mode, p->axx.E, (int)p->M, prec)) + ">";
    }
      n = (int64_t)p->x_grid.x * p->x_block.x;
      break;
    case RL_KERNEL_Y: pencil(p->py, rlmi::PM_FWD, rlmi::PM_INV); break;
    case RL_KERNEL_Z_OTF: pencil(p->pz, rlmi::PM_FKI, rlmi::PM_FCKI); break;
    default: return fail(RL_E_INVALID, "kind must be X_RATIO, X_UPDATE, Y or Z_OTF");
  }
  if (s.size() + 1 > cap) return fail(RL_E_INVALID, "name buffer too small");
  std::memcpy(name, s.c_str(), s.size() + 1);
  *threads = n;
  return RL_OK;
}

rl_status rl_plan_set_timing(rl_plan p, int enable) {
  rl_status st = check_plan(p);
  if (st != RL_OK) return st;
  if (p->is_batch) return fail(RL_E_UNSUPPORTED, "batch plans replay graphs; time them whole");
  p->timing = enable != 0;
  p->n_events = 0;
  return RL_OK;
}

rl_status rl_plan_get_timing(rl_plan p, int count[RL_KERNEL_KINDS], double ms[RL_KERNEL_KINDS]) {
  rl_status st = check_plan(p);
  if (st != RL_OK) return st;
  if (!count || !ms) return fail(RL_E_INVALID, "output arrays are NULL");
  for (int k = 0; k < RL_KERNEL_KINDS; ++k) {
    count[k] = 0;
    ms[k] = 0.0;
  }
  hipError_t e = hipSetDevice(p->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  if ((e = hipStreamSynchronize(p->stream)) != hipSuccess) return hip_fail(e, "execution");
  for (size_t i = 0; i < p->n_events; ++i) {
    float t = 0.f;
    if ((e = hipEventElapsedTime(&t, p->events[i].a, p->events[i].b)) != hipSuccess)
      return hip_fail(e, "hipEventElapsedTime");
    count[p->events[i].kind] += 1;
    ms[p->events[i].kind] += (double)t;
  }
  p->n_events = 0;
  return RL_OK;
}

rl_status rl_probe_copy(const void* src, void* dst, size_t bytes, void* hip_stream) {
  try {
    if (bytes == 0) return RL_OK;
    if (bytes % 16 != 0) return fail(RL_E_INVALID, "bytes must be a multiple of 16");
    int dev = -1;
    rl_status st = check_dev_ptr(src, bytes, &dev, "src");
    if (st != RL_OK) return st;
    if ((st = check_dev_ptr(dst, bytes, &dev, "dst")) != RL_OK) return st;
    hipError_t e = hipSetDevice(dev);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    e = rlmi::launch_copy(src, dst, bytes, reinterpret_cast<hipStream_t>(hip_stream));
    return e == hipSuccess ? RL_OK : hip_fail(e, "copy launch");
  } catch (...) {
    return fail(RL_E_INTERNAL, "unexpected exception in rl_probe_copy");
  }
}

const char* rl_status_string(rl_status s) {
  // a caller may pass any int: read the bits, not the enum (whose C++ range is 0..7)
  static_assert(sizeof(rl_status) == sizeof(int), "rl_status is passed as an int");
  int v = 0;
  std::memcpy(&v, &s, sizeof(v));
  switch (v) {
    case RL_OK: return "RL_OK";
    case RL_E_INVALID: return "RL_E_INVALID";
    case RL_E_UNSUPPORTED: return "RL_E_UNSUPPORTED";
    case RL_E_NOMEM: return "RL_E_NOMEM";
    case RL_E_DEVICE: return "RL_E_DEVICE";
    case RL_E_NUMERIC: return "RL_E_NUMERIC";
    case RL_E_INTERNAL: return "RL_E_INTERNAL";
  }
  return "RL_E_UNKNOWN";
}

const char* rl_last_error(void) { return g_err.c_str(); }

}  // extern "C"
