// C-ABI layer of the Richardson-Lucy library: argument validation, plan
// (workspace, transfer function, radix schedules, launch shapes) and the pass
// sequences of rl_iterate and conv3d_fft.  The declarations and their
// contracts are in include/rl.h.
#include "../../include/rl.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
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
constexpr int64_t kMaxNx = 2048;
constexpr int64_t kMaxNyz = 1024;
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

bool is_pow2(int64_t v) { return v >= 1 && (v & (v - 1)) == 0; }

// Lengths handled by the radix set {16, 8, 4, 2} plus one final radix-3 stage.
bool length_ok(int64_t L) {
  if (L < 1) return false;
  if (L % 3 == 0) L /= 3;
  return is_pow2(L);
}

int64_t pow2_part(int64_t v) { return v & -v; }

// A caller-chosen E for length L: divides L into a power-of-two thread count
// <= max_p, carries every factor 3 of L, and leaves radices the schedule can use.
bool e_ok(int64_t L, int E, int64_t max_p) {
  static const int kE[] = {1, 2, 3, 4, 6, 8, 12, 16, 24};
  bool known = false;
  for (int k : kE) known = known || (k == E);
  if (!known || L % E != 0) return false;
  const int64_t P = L / E;
  if (!is_pow2(P) || P > max_p) return false;
  if (L % 3 == 0 && E % 3 != 0) return false;
  if (E % 3 == 0 && L % 3 != 0) return false;
  const int64_t l2 = pow2_part(L);
  return l2 == 1 || pow2_part(E) >= 2;
}

int pick_e(int64_t L) {
  if (L == 1) return 1;
  if (is_pow2(L)) return (int)(L < 16 ? L : 16);
  return (int)(L < 24 ? L : 24);  // 3 * 2^a
}

// X pass: few elements per thread so that one row fills (up to) a wavefront;
// the many short-lived waves hide the latency of the fused two-transform pass.
int pick_e_x(int64_t M) {
  if (is_pow2(M)) {
    if (M <= 4) return (int)M;
    return (int)(M / 4 <= 64 ? 4 : M / 64);
  }
  if (M <= 12) return (int)M;           // 3, 6, 12
  return (int)(M / 12 <= 64 ? 12 : 24);  // 3 * 2^a
}

// Y pass: 8 elements per thread for power-of-two lengths up to 512.
int pick_e_y(int64_t L) {
  if (is_pow2(L) && L >= 8 && L <= 512) return 8;
  return pick_e(L);
}

// Radix schedule: the largest power-of-two radix dividing E first, then the
// power-of-two remainder, then radix 3 last (its stage needs no index wrap).
Sched make_sched(int64_t L, int E, int table_stride) {
  Sched sc;
  std::memset(&sc, 0, sizeof(sc));
  int64_t n = L;
  int threes = 0;
  while (n % 3 == 0) {
    n /= 3;
    ++threes;
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
    rads.push_back(r);
    n /= r;
  }
  for (int t = 0; t < threes; ++t) rads.push_back(3);
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
  int64_t M = 0, ncols = 0, xt = 0, nvox = 0, nrows = 0;
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
  if (!length_ok(nx / 2) || nx > kMaxNx)
    return fail(RL_E_UNSUPPORTED, "nx must be 2^a or 3*2^a and <= 2048");
  if (!length_ok(ny) || ny > kMaxNyz)
    return fail(RL_E_UNSUPPORTED, "ny must be 1, 2^a or 3*2^a and <= 1024");
  if (!length_ok(nz) || nz > kMaxNyz)
    return fail(RL_E_UNSUPPORTED, "nz must be 1, 2^a or 3*2^a and <= 1024");
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
  p->magic = kDead;
  delete p;
}

int max_threads_for(int E) { return (E == 8 || E == 16) ? 1024 : rlmi::kPencilMaxThreads; }

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
  // exchange buffer (L x TXP) followed by the twiddle table (L); the kernel
  // places the table at offset L * TXP whether or not the exchange is used
  pc.lds = (size_t)pc.ax.L * (txb + 1) * sizeof(float2);
  pc.block = dim3((unsigned)(txb * pc.ax.P));
}

// Y pass: one work-group per (tile column, z); lanes = up to 16 columns of the tile.
Pencil make_pencil_y(int64_t ny, int64_t nz, int64_t xt, int64_t ncols, int tile_x, int e) {
  Pencil pc;
  pc.ax = make_axis(ny, e);
  int txb = rlmi::kTile;
  if (tile_x > 0 && tile_x < txb) {
    txb = 1;
    while (txb * 2 <= tile_x) txb *= 2;
  }
  while (txb > 1 && ((int64_t)txb * pc.ax.P > max_threads_for(pc.ax.E) ||
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
// consecutive elements (ty whole tile rows), so each z step reads 128 * ty bytes.
Pencil make_pencil_z(int64_t nz, int64_t ny, int64_t xt, int64_t ncols, int tile_x, int e) {
  Pencil pc;
  pc.ax = make_axis(nz, e);
  const int maxt = max_threads_for(pc.ax.E);
  auto fits = [&](int txb) {
    return (int64_t)txb * pc.ax.P <= maxt &&
           (size_t)nz * (txb + 1) * sizeof(float2) <= kMaxPencilLds;
  };
  int txb;
  if (tile_x > 0 && tile_x < rlmi::kTile) {
    txb = 1;
    while (txb * 2 <= tile_x) txb *= 2;
  } else {
    int ty = tile_x >= rlmi::kTile ? tile_x / rlmi::kTile : 2;
    while (ty > 1 && (ny % ty != 0 || !fits(ty * rlmi::kTile))) ty >>= 1;
    txb = ty * rlmi::kTile;
  }
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

rl_status timed_begin(rl_plan p, int kind, size_t* slot) {
  if (!p->timing) return RL_OK;
  if (p->n_events == p->events.size()) {
    TimedLaunch t{kind, nullptr, nullptr};
    if (hipEventCreate(&t.a) != hipSuccess || hipEventCreate(&t.b) != hipSuccess)
      return hip_fail(hipGetLastError(), "hipEventCreate");
    p->events.push_back(t);
  }
  *slot = p->n_events++;
  p->events[*slot].kind = kind;
  hipError_t e = hipEventRecord(p->events[*slot].a, p->stream);
  return e == hipSuccess ? RL_OK : hip_fail(e, "hipEventRecord");
}

rl_status timed_end(rl_plan p, size_t slot) {
  if (!p->timing) return RL_OK;
  hipError_t e = hipEventRecord(p->events[slot].b, p->stream);
  return e == hipSuccess ? RL_OK : hip_fail(e, "hipEventRecord");
}

rl_status run_pencil(rl_plan p, const Pencil& pc, int mode, float2* data, const float2* tw,
                     int kind) {
  if (pc.ax.L == 1 && (mode == rlmi::PM_FWD || mode == rlmi::PM_INV)) return RL_OK;  // identity
  size_t slot = 0;
  rl_status st = timed_begin(p, kind, &slot);
  if (st != RL_OK) return st;
  hipError_t e = rlmi::launch_pencil(mode, pc.ax.E, pc.grid, pc.block, pc.lds, p->stream, data,
                                     p->otf, tw, pc.args, pc.ax.sc);
  if (e != hipSuccess) return hip_fail(e, "pencil pass launch");
  return timed_end(p, slot);
}

XArgs base_xargs(rl_plan p, float2* spec) {
  XArgs a;
  std::memset(&a, 0, sizeof(a));
  a.spec = spec;
  a.zstride = p->xt * p->ny * rlmi::kTile;
  a.tstride = p->ny * rlmi::kTile;
  a.ny = (int)p->ny;
  a.M = (int)p->M;
  a.P = p->axx.P;
  a.RPW = p->x_rpw;
  a.RS = p->x_rs;
  a.nrows = (int)p->nrows;
  return a;
}

rl_status run_x(rl_plan p, int mode, const XArgs& a, int kind) {
  size_t slot = 0;
  rl_status st = timed_begin(p, kind, &slot);
  if (st != RL_OK) return st;
  hipError_t e = rlmi::launch_xrow(mode, p->axx.E, p->x_grid, p->x_block, p->x_lds, p->stream, a,
                                   p->axx.sc, p->tw_x);
  if (e != hipSuccess) return hip_fail(e, "X pass launch");
  return timed_end(p, slot);
}

// spectrum (X-transformed) -> spectrum (X-transformed) of H x or H^T x:
// Y forward, Z forward * (conj) OTF * Z inverse, Y inverse.
rl_status run_yz_filter(rl_plan p, bool adjoint) {
  rl_status st;
  if ((st = run_pencil(p, p->py, rlmi::PM_FWD, p->spec, p->tw_y, RL_KERNEL_Y)) != RL_OK) return st;
  if ((st = run_pencil(p, p->pz, adjoint ? rlmi::PM_FCKI : rlmi::PM_FKI, p->spec, p->tw_z,
                       RL_KERNEL_Z_OTF)) != RL_OK)
    return st;
  return run_pencil(p, p->py, rlmi::PM_INV, p->spec, p->tw_y, RL_KERNEL_Y);
}

rl_status create_impl(const int64_t shape[3], const float* psf, int boundary,
                      const rl_options* opt, rl_plan* out) {
  if (!out) return fail(RL_E_INVALID, "out is NULL");
  *out = nullptr;
  rl_status st = check_shape(shape);
  if (st != RL_OK) return st;
  if (boundary == RL_BOUNDARY_ZERO)
    return fail(RL_E_UNSUPPORTED, "only the periodic boundary is implemented");
  if (boundary != RL_BOUNDARY_PERIODIC) return fail(RL_E_INVALID, "unknown boundary");
  if (opt && opt->precision != RL_PRECISION_FP32)
    return fail(RL_E_UNSUPPORTED, "only FP32 precision is implemented");
  if (opt && (opt->tile_x < 0 || opt->tile_x > 64))
    return fail(RL_E_INVALID, "tile_x must be in [0, 64]");
  if (opt && opt->x_elems != 0 && !e_ok(shape[2] / 2, opt->x_elems, 64))
    return fail(RL_E_INVALID, "x_elems does not fit nx/2");
  if (opt && opt->yz_elems != 0 &&
      (!e_ok(shape[1], opt->yz_elems, 1024) || !e_ok(shape[0], opt->yz_elems, 1024)))
    return fail(RL_E_INVALID, "yz_elems does not fit ny and nz");
  if (!psf) return fail(RL_E_INVALID, "psf is NULL");
  if (reinterpret_cast<uintptr_t>(psf) % 16 != 0)
    return fail(RL_E_INVALID, "psf is not 16-byte aligned");
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev < 1) {
    (void)hipGetLastError();
    return fail(RL_E_DEVICE, "no HIP device available");
  }
  const int64_t nz = shape[0], ny = shape[1], nx = shape[2];
  const int64_t nvox = nz * ny * nx;
  int device = -1;
  if ((st = check_dev_ptr(psf, (size_t)nvox * sizeof(float), &device, "psf")) != RL_OK) return st;

  rl_plan p = new (std::nothrow) rl_plan_s();
  if (!p) return fail(RL_E_NOMEM, "host allocation failed");
  p->device = device;
  p->stream = opt ? reinterpret_cast<hipStream_t>(opt->stream) : nullptr;
  p->nz = nz;
  p->ny = ny;
  p->nx = nx;
  p->M = nx / 2;
  p->ncols = p->M + 1;
  p->xt = (p->ncols + rlmi::kTile - 1) / rlmi::kTile;  // 16-column tiles per row
  p->nvox = nvox;
  p->nrows = nz * ny;
  p->spec_elems = (size_t)nz * p->xt * ny * rlmi::kTile;

  // X pass shape
  p->axx.L = p->M;
  p->axx.E = (opt && opt->x_elems) ? opt->x_elems : pick_e_x(p->M);
  p->axx.P = (int)(p->M / p->axx.E);
  p->axx.sc = make_sched(p->M, p->axx.E, 2);
  // each wavefront owns 64 / P whole rows; up to kXMaxThreads / 64 waves per work-group
  const int rows_per_wave = 64 / p->axx.P;
  int waves = rlmi::kXMaxThreads / 64;
  p->x_rs = (int)(p->M + 1 + ((p->M + 1) >> rlmi::kXPad) + 1);  // padded row
  auto x_lds_for = [&](int w) {
    return (size_t)(2 * p->M + (int64_t)w * rows_per_wave * p->x_rs) * sizeof(float2);
  };
  while (waves > 1 && x_lds_for(waves) > kMaxLds) waves >>= 1;
  p->x_rpw = waves * rows_per_wave;
  p->x_lds = x_lds_for(waves);
  p->x_block = dim3((unsigned)(64 * waves));
  p->x_grid = dim3((unsigned)((p->nrows + p->x_rpw - 1) / p->x_rpw));
  // Y: pencils along Y, outer = z; Z: pencils along Z, outer = y
  const int tile_x = opt ? opt->tile_x : 0;
  const int yz_e = opt ? opt->yz_elems : 0;
  p->py = make_pencil_y(ny, nz, p->xt, p->ncols, tile_x, yz_e ? yz_e : pick_e_y(ny));
  p->pz = make_pencil_z(nz, ny, p->xt, p->ncols, tile_x, yz_e);
  if (p->x_lds > kMaxLds || p->py.lds > kMaxPencilLds || p->pz.lds > kMaxPencilLds ||
      (int)p->py.block.x > max_threads_for(p->py.ax.E) ||
      (int)p->pz.block.x > max_threads_for(p->pz.ax.E)) {
    delete p;
    return fail(RL_E_UNSUPPORTED, "shape needs more LDS than a work-group may use");
  }

  if ((e = hipSetDevice(device)) != hipSuccess) {
    delete p;
    return hip_fail(e, "hipSetDevice");
  }
  p->flux_cap = 128;
  p->n_partials = (size_t)p->x_grid.x * p->flux_cap;
  if (p->n_partials < 3 * (size_t)kStatBlocks) p->n_partials = 3 * kStatBlocks;
  const size_t spec_bytes = p->spec_elems * sizeof(float2);
  if ((e = hipMalloc(&p->spec, spec_bytes)) != hipSuccess ||
      (e = hipMalloc(&p->otf, spec_bytes)) != hipSuccess ||
      (e = hipMalloc(&p->tw_x, (size_t)nx * sizeof(float2))) != hipSuccess ||
      (e = hipMalloc(&p->tw_y, (size_t)ny * sizeof(float2))) != hipSuccess ||
      (e = hipMalloc(&p->tw_z, (size_t)nz * sizeof(float2))) != hipSuccess ||
      (e = hipMalloc(&p->partials, p->n_partials * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&p->counter, 4 * sizeof(unsigned))) != hipSuccess ||
      (e = hipMalloc(&p->stats, 4 * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&p->flux, (size_t)p->flux_cap * sizeof(double))) != hipSuccess) {
    st = hip_fail(e, "hipMalloc");
    release(p);
    return st;
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
  RL_TRY(rlmi::launch_psf_stats(psf, nvox, p->partials, kStatBlocks, p->counter, p->stats,
                                p->stream));
  double stats[3] = {0, 0, 0};
  RL_TRY(hipMemcpyAsync(stats, p->stats, 3 * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  RL_TRY(hipStreamSynchronize(p->stream));
  if (stats[2] != 0.0) {
    release(p);
    return fail(RL_E_INVALID, "psf has non-finite entries");
  }
  if (stats[1] < 0.0) {
    release(p);
    return fail(RL_E_INVALID, "psf has negative entries");
  }
  if (!(stats[0] > 0.0) || !std::isfinite(stats[0])) {
    release(p);
    return fail(RL_E_INVALID, "psf must have a positive finite sum");
  }
  // OTF / N: scaled, centred PSF written as dense real rows into the spectrum
  // workspace, transformed along X into the OTF buffer, then along Y and Z.
  const double scale = 1.0 / (stats[0] * (double)nvox);
  RL_TRY(rlmi::launch_psf_prep(psf, reinterpret_cast<float*>(p->spec), (int)nz, (int)ny, (int)nx,
                               nx, scale, p->stream));
  XArgs a = base_xargs(p, p->otf);
  a.rin = reinterpret_cast<const float*>(p->spec);
  a.rin_stride = nx;
  if ((st = run_x(p, rlmi::XM_R2C, a, RL_KERNEL_OTHER)) != RL_OK) {
    release(p);
    return st;
  }
  if ((st = run_pencil(p, p->py, rlmi::PM_FWD, p->otf, p->tw_y, RL_KERNEL_OTHER)) != RL_OK ||
      (st = run_pencil(p, p->pz, rlmi::PM_FWD, p->otf, p->tw_z, RL_KERNEL_OTHER)) != RL_OK) {
    release(p);
    return st;
  }
  RL_TRY(hipStreamSynchronize(p->stream));
#undef RL_TRY
  plan_register(p);
  *out = p;
  return RL_OK;
}

rl_status iterate_impl(rl_plan p, const float* observed, float* estimate, int n_iter) {
  rl_status st = check_plan(p);
  if (st != RL_OK) return st;
  if (n_iter < 0) return fail(RL_E_INVALID, "n_iter must be >= 0");
  const size_t bytes = (size_t)p->nvox * sizeof(float);
  int dev = p->device;
  if ((st = check_dev_ptr(observed, bytes, &dev, "observed")) != RL_OK) return st;
  if ((st = check_dev_ptr(estimate, bytes, &dev, "estimate")) != RL_OK) return st;
  if (n_iter == 0) return RL_OK;
  hipError_t e = hipSetDevice(p->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  if (n_iter > p->flux_cap) {
    // grow the flux array and the [iteration][work-group] partial table
    double* nf = nullptr;
    double* np = nullptr;
    const size_t nparts = (size_t)n_iter * p->x_grid.x;
    if ((e = hipMalloc(&nf, (size_t)n_iter * sizeof(double))) != hipSuccess)
      return hip_fail(e, "hipMalloc(flux)");
    if ((e = hipMalloc(&np, nparts * sizeof(double))) != hipSuccess) {
      (void)hipFree(nf);
      return hip_fail(e, "hipMalloc(flux partials)");
    }
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    else (void)hipDeviceSynchronize();
    (void)hipFree(p->flux);
    (void)hipFree(p->partials);
    p->flux = nf;
    p->partials = np;
    p->n_partials = nparts;
    p->flux_cap = n_iter;
  }
  p->flux_count = n_iter;

  // prologue: spectrum of H u0, transformed back along Z and Y
  XArgs a = base_xargs(p, p->spec);
  a.rin = estimate;
  a.rin_stride = p->nx;
  if ((st = run_x(p, rlmi::XM_R2C, a, RL_KERNEL_X_R2C)) != RL_OK) return st;
  if ((st = run_yz_filter(p, false)) != RL_OK) return st;
  for (int it = 0; it < n_iter; ++it) {
    XArgs r = base_xargs(p, p->spec);
    r.d = observed;
    if ((st = run_x(p, rlmi::XM_RATIO, r, RL_KERNEL_X_RATIO)) != RL_OK) return st;
    if ((st = run_yz_filter(p, true)) != RL_OK) return st;
    XArgs u = base_xargs(p, p->spec);
    u.u = estimate;
    u.partials = p->partials;
    u.iter = it;
    u.do_fwd = (it + 1 < n_iter) ? 1 : 0;
    if ((st = run_x(p, rlmi::XM_UPDATE, u, RL_KERNEL_X_UPDATE)) != RL_OK) return st;
    if (u.do_fwd && (st = run_yz_filter(p, false)) != RL_OK) return st;
  }
  size_t slot = 0;
  if ((st = timed_begin(p, RL_KERNEL_OTHER, &slot)) != RL_OK) return st;
  if ((e = rlmi::launch_flux_reduce(p->partials, (int)p->x_grid.x, n_iter, p->flux, p->stream)) !=
      hipSuccess)
    return hip_fail(e, "flux reduction launch");
  return timed_end(p, slot);
}

rl_status conv_impl(rl_plan p, const float* x, float* out) {
  rl_status st = check_plan(p);
  if (st != RL_OK) return st;
  const size_t bytes = (size_t)p->nvox * sizeof(float);
  int dev = p->device;
  if ((st = check_dev_ptr(x, bytes, &dev, "x")) != RL_OK) return st;
  if ((st = check_dev_ptr(out, bytes, &dev, "out")) != RL_OK) return st;
  hipError_t e = hipSetDevice(p->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  XArgs a = base_xargs(p, p->spec);
  a.rin = x;
  a.rin_stride = p->nx;
  if ((st = run_x(p, rlmi::XM_R2C, a, RL_KERNEL_X_R2C)) != RL_OK) return st;
  if ((st = run_yz_filter(p, false)) != RL_OK) return st;
  XArgs c = base_xargs(p, p->spec);
  c.rout = out;
  c.rout_stride = p->nx;
  return run_x(p, rlmi::XM_C2R, c, RL_KERNEL_X_C2R);
}

}  // namespace

extern "C" {

rl_status rl_plan_create(const int64_t shape[3], const float* psf, int boundary, rl_plan* out) {
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
  try {
    return create_impl(shape, psf, boundary, opt, out);
  } catch (const std::bad_alloc&) {
    return fail(RL_E_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(RL_E_INTERNAL, "unexpected exception in rl_plan_create_ex");
  }
}

rl_status rl_iterate(rl_plan p, const float* observed, float* estimate, int n_iter) {
  try {
    return iterate_impl(p, observed, estimate, n_iter);
  } catch (...) {
    return fail(RL_E_INTERNAL, "unexpected exception in rl_iterate");
  }
}

rl_status conv3d_fft(rl_plan p, const float* x, float* out) {
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
  const int n = p->flux_count;
  std::vector<double> h((size_t)n);
  if (n > 0 && (e = hipMemcpy(h.data(), p->flux, (size_t)n * sizeof(double),
                              hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(e, "hipMemcpy(flux)");
  *n_written = n;
  for (int i = 0; i < n && i < cap; ++i) flux[i] = h[(size_t)i];
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(h[(size_t)i]))
      return fail(RL_E_NUMERIC, "non-finite flux at iteration " + std::to_string(i));
  return RL_OK;
}

rl_status rl_plan_get_info(rl_plan p, int64_t shape[3], int64_t* spectrum_pitch) {
  rl_status st = check_plan(p);
  if (st != RL_OK) return st;
  if (shape) {
    shape[0] = p->nz;
    shape[1] = p->ny;
    shape[2] = p->nx;
  }
  if (spectrum_pitch) *spectrum_pitch = p->xt * rlmi::kTile;
  return RL_OK;
}

rl_status rl_plan_set_timing(rl_plan p, int enable) {
  rl_status st = check_plan(p);
  if (st != RL_OK) return st;
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
  switch (s) {
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
