// Internal interface between the C-ABI layer (rl_api.cpp) and the HIP kernels
// (rl_kernels.hip).  Not installed; not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rlmi {

constexpr int kMaxStages = 8;
// Work-group size limits the kernels are compiled for (register budget).
constexpr int kPencilMaxThreads = 512;
constexpr int kXMaxThreads = 256;
// X-pass LDS rows: one spare slot after every 4 elements (radix-4 stages).
constexpr int kXPad = 2;
// Static LDS of the split-precision kernels: the MFMA A-operand table (both
// signs, 64 lanes, four 16-byte operands), beside their dynamic LDS.
constexpr int kSplitTabBytes = 2 * 64 * 4 * 16;

// Radix schedule of one axis transform of length L, executed in this order.
// Stage s has radix r[s], input span p[s] (product of earlier radices) and
// twiddle-table multiplier tm[s] = table_stride * L / (p[s] * r[s]), so that
// the twiddle for input j of butterfly k is table[j * k * tm[s]].
struct Sched {
  int ns;
  int r[kMaxStages];
  int p[kMaxStages];
  int tm[kMaxStages];
};

// Half-spectrum layout ("x-tile major"): complex element (z, y, kx) of a volume
// with ny rows and XT = ceil((nx/2 + 1) / 16) column tiles lives at
//   ((z * XT + kx / 16) * ny + y) * 16 + kx % 16.
// A tile column (fixed z and kx / 16) is ny * 128 contiguous bytes.
// The transfer function (OTF) is stored "z major" instead, in the order the Z
// pass (the only one that reads it) consumes it: with t = kx / 16 and w the
// tile's width (16, or for the last tile the valid columns left, ncols - 16 t),
// element (z, y, kx) at
//   t * ny * nz * 16 + (y * nz + z) * w + kx % 16,
// so that a work-group's reads of one tile row over all z are nz * 8 w
// contiguous bytes, and the last tile's padding columns are not stored (for
// even nx it holds the Nyquist column alone).
constexpr int kTile = 16;

// Geometry of a strided pencil pass (Y or Z axis).  A work-group covers TXB
// consecutive complex elements ("lanes") of a tile row group and all L elements
// of each of those pencils:
//   lane c of block (bx, by): xb = bx / xsplit, c = (bx % xsplit) * TXB + lane,
//   element e at xb * xstride + by * ostride + c + e * estride,
//   valid when xb * 16 + (c % 16) < ncols.
struct PencilArgs {
  int L;       // transform length
  int P;       // threads per pencil (L / E)
  int TXB;     // lanes per work-group (power of two)
  int TXP;     // LDS stride per pencil element, in complex elements (>= TXB)
  int xsplit;  // work-groups per 16-column tile (16 / TXB when TXB < 16, else 1)
  int ncols;   // valid columns (nx/2 + 1)
  long long xstride;
  long long ostride;
  long long estride;
  long long vstride;  // complex elements between volumes (work-group z index = volume)
  int swap;           // 1: tile index from blockIdx.y and outer index from blockIdx.x
  int lin;            // elements e >= lin of a pencil read as zero (not loaded)
  int lout;           // elements e >= lout are not stored
  const int* stop;    // if non-null and *stop != 0 the launch does nothing
};

enum PencilMode { PM_FWD = 0, PM_INV = 1, PM_FKI = 2, PM_FCKI = 3 };
// Stopping metrics (values of rl_stop_metric).
enum Metric { MET_NONE = 0, MET_LOGLIK = 1, MET_CHANGE = 2, MET_PSNR = 3, MET_SSIM = 4,
              MET_FSC = 5 };
constexpr int kMetRows = 7;
// XM_PREDICT and XM_UPDATE_ACC are the two X passes of the extrapolated
// (Biggs-Andrews) iteration: the prediction y = max(x + alpha h, 0) transformed
// forward, and the update from y that also keeps the step h and the change g.
enum XMode {
  XM_R2C = 0,
  XM_C2R = 1,
  XM_RATIO = 2,
  XM_UPDATE = 3,
  XM_PREDICT = 4,
  XM_UPDATE_ACC = 5,
  XM_RATIO_LL = 6,    // XM_RATIO that also accumulates the log-likelihood (MET_LOGLIK)
  XM_UPDATE_CHG = 7,  // XM_UPDATE that also accumulates the MET_CHANGE sums
  XM_UPDATE_PSNR = 8  // XM_UPDATE that also accumulates the MET_PSNR sums
};

// Row length M the X-pass kernel of (mode, E, M, prec) is compiled for (0 = the
// runtime schedule): the per-iteration ratio and update passes of power-of-two
// rows M in {64, 128, 256, 512} with E in {4, 8} elements per thread and at most
// 64 threads per row, of the rows 3 * 2^a of the batched volumes (M in {24, 48,
// 96}, E = 6), and of the 2560-sample rows of the paper's stack (M = 1280 =
// 4^4 * 5, E = 20).
constexpr int xrow_compiled_len(int mode, int E, int M, int prec) {
  return ((mode == XM_RATIO || mode == XM_UPDATE) && prec == 0 &&
          (((E == 4 || E == 8) && (M == 64 || M == 128 || M == 256 || M == 512) && M / E <= 64) ||
           (E == 6 && (M == 24 || M == 48 || M == 96)) || (E == 20 && M == 1280)))
             ? M
             : 0;
}

// Thread bound of the compile-time pencil kernel of (E, L): the 2160-point pencils
// of the paper's stack (E = 30, 72 threads per pencil) run 8 lanes, 576 threads.
constexpr int pencil_ct_max_threads(int E, int L) {
  return (E == 30 && L == 2160) ? 576 : E == 8 ? 1024 : kPencilMaxThreads;
}

// Length L the pencil kernel of (E, L, work-group threads) is compiled for (0 =
// the runtime schedule): power-of-two pencils L in {128, 256, 512} with 16
// elements per thread, in every precision (the split-precision forms run their
// 16-point MFMA stages there), and L in {32, ..., 512} with 8 (work-groups up to
// 1024 threads); the pencils 3 * 2^a of the batched volumes (L in {24, 48, 96}
// with 6 elements, L in {48, 96, 192} with 12); and the 2160-point pencils with 30.
constexpr int pencil_compiled_len(int E, int L, int threads) {
  return ((E == 16 && (L == 128 || L == 256 || L == 512)) ||
          (E == 8 && (L == 32 || L == 64 || L == 128 || L == 256 || L == 512)) ||
          (E == 6 && (L == 24 || L == 48 || L == 96)) ||
          (E == 12 && (L == 48 || L == 96 || L == 192)) || (E == 30 && L == 2160)) &&
                 threads <= pencil_ct_max_threads(E, L)
             ? L
             : 0;
}

// Arguments of an X-row pass (contiguous axis, real <-> half spectrum).
struct XArgs {
  float2* spec;          // half spectrum, x-tile-major layout (see kTile)
  long long zstride;     // complex elements per z plane (XT * ny * 16)
  long long tstride;     // complex elements per tile column (ny * 16)
  int ny;
  const float* rin;      // XM_R2C: real input rows, `rin_stride` floats apart
  long long rin_stride;
  float* rout;           // XM_C2R: real output rows, `rout_stride` floats apart
  long long rout_stride;
  const float* d;        // XM_RATIO: observed rows (dense, nx floats apart)
  float* u;              // XM_UPDATE: estimate rows (dense), updated in place
  // Batched volumes (work-group y index = volume): when a table is non-null the
  // volume's pointer is taken from it instead of rin / rout / d / u above.
  const float* const* rin_tab;
  float* const* rout_tab;
  const float* const* d_tab;
  float* const* u_tab;
  long long vstride;     // complex elements between the volumes' spectra
  double* partials;      // XM_UPDATE: FP64 partial flux, [iter][volume][work-group]
  int iter;
  const int* iter_ptr;   // XM_UPDATE: if non-null, the iteration index is *iter_ptr
  int nvol;              // volumes in this launch (>= 1)
  int do_fwd;            // XM_UPDATE: also transform the new estimate forward
  // Extrapolated iteration (single volume; dense rows like u):
  float* hstep;          // h = x_k - x_{k-1}; XM_UPDATE_ACC replaces it by x_{k+1} - x_k
  float* gchg;           // XM_UPDATE_ACC: g_{k-1} = x_k - y_{k-1}, replaced by g_k
  const float* alpha;    // alpha[k] (FP32); not read (taken as 0) when iter == 0
  double* acc_partials;  // XM_UPDATE_ACC: [2][work-group] FP64 partials of
                         // <g_k, g_{k-1}> and <g_{k-1}, g_{k-1}>
  // Metric-guided stopping (single volume): if stop is non-null and *stop != 0
  // the launch does nothing.  XM_RATIO_LL, XM_UPDATE_CHG and XM_UPDATE_PSNR
  // accumulate their metric's work-group partials (FP64) into
  // met_partials[row * gridDim.x + work-group] (rows as for launch_metric).
  const int* stop;
  int metric;
  double* met_partials;
  const float* ref;      // MET_PSNR: reference volume (dense rows like u)
  // Real rows (rin, rout, d, u, hstep, gchg, ref) cover the caller's volume
  // vz x vy x vx at the low corner of the transform grid: grid row (z, y) is
  // real row z * vy + y when z < vz and y < vy, and holds vx floats (the rest of
  // the grid row reads as zero and is not written).  rin / rout rows are
  // rin_stride / rout_stride floats apart, the others vx.
  int vx, vy, vz;
  int M;                 // complex row length nx/2
  int P;                 // threads per row (M / E)
  int RPW;               // rows per work-group (a multiple of 64 / P)
  int RS;                // LDS row stride in complex elements (>= M + 1)
  int nrows;             // grid rows covered by the launch (row = z * ny + y)
};

// --- persistent batched iteration -------------------------------------------
// One launch runs every pass of one Richardson-Lucy iteration of every volume of
// a batch.  Work-groups of kPersistThreads (128) threads take tiles (one work-group's
// share of one pass of one volume, exactly as the per-pass kernels split it)
// from a work queue in pass-major order and wait, before a tile of pass s of
// volume v, until every tile of pass s - 1 of v has completed.  Each volume is
// assigned to one XCD and its tiles are taken only by work-groups running on that
// XCD, so producer and consumer of every dependency share an L2: completion is a
// store wait plus an atomic increment in that L2, and a wait ends with an L1
// invalidation (no L2 writeback).  Switched off on the host side: plans refuse
// the persistent mode (its waits did not finish on the GPU).
constexpr int kPersistThreads = 128;
constexpr int kPersistPasses = 8;  // X ratio, Y, Z conj K, Y^-1, X update, Y, Z K, Y^-1
constexpr int kPersistMaxQueues = 16;

// Per shape class: the arguments its per-pass launches would get.
struct PersistClass {
  XArgs xr, xu;           // ratio and update passes (per-volume pointer tables)
  PencilArgs py, pz;      // Y and Z passes (vstride set)
  Sched sx, sy, sz;
  const float2* twx;
  const float2* twy;
  const float2* twz;
  float2* spec;
  const float2* otf;
  int ex, ey, ez;         // elements per thread of the X, Y and Z transforms
  int xtiles;             // X work-groups per volume
  int ygx, ytiles;        // Y grid x extent and work-groups per volume
  int zgx, ztiles;        // Z grid x extent and work-groups per volume
};

// A run of tiles: pass `pass` of volume `vol` (index within its class `cls`),
// counter row `vrow`; tickets [first, first + tiles) of its queue.
struct PersistSeg {
  int pass, cls, vol, vrow, tiles, first;
};

struct PersistArgs {
  const PersistClass* cls;
  const PersistSeg* segs;   // queue q owns segs[qseg[q] .. qseg[q + 1])
  const int* qseg;
  int nq;                   // queues (XCDs); work-groups on XCD >= nq take no work
  int npass;                // passes this launch runs (8, or 5 on the last iteration)
  int nvrow;                // counter rows (volumes)
  const int* iter_ptr;      // iteration index within the call
  int* tickets;             // [iteration][queue], zero at the start of the call
  int* done;                // [iteration][volume][pass] completed tiles, zero at the start
  int* error;               // [queue]: set to 1 when a dependency wait runs past its bound
  int spin_limit;           // polls of a counter before giving up
};

// Element counts the persistent kernel is built for (other classes use the
// per-pass graph).
constexpr bool persist_x_e(int E) { return E == 2 || E == 4 || E == 6; }
constexpr bool persist_yz_e(int E) { return E == 4 || E == 6 || E == 8 || E == 12; }

hipError_t launch_persist(const PersistArgs& a, int grid, size_t lds, hipStream_t s);
// Resident work-groups of the persistent kernel per CU with `lds` bytes of LDS.
hipError_t persist_occupancy(size_t lds, int* blocks_per_cu);
// *counter = 0 for n ints (a fill kernel; graph-capture safe).
hipError_t launch_zero_ints(int* p, long long n, hipStream_t s);
// out <- in (nvol volumes of the x-tile-major layout) in the z-major OTF order,
// the last tile stored ncols - 16 (xt - 1) columns wide.
hipError_t launch_otf_zmajor(const float2* in, float2* out, int nvol, int nz, int ny, int xt,
                             int ncols, hipStream_t s);

// Pencil kernels exist for work-groups of up to 512 threads (all E) and up to
// 1024 threads (E = 8 and 16 only).
// prec: 0 = FP32 butterflies; 1 / 2 = radix-16 stages of E = 16 transforms on
// MFMA with BF16 / FP16 hi-lo split operands (other stages stay FP32).
// ev0 / ev1 (may be null): timing events stamped by the kernel's own dispatch.
hipError_t launch_pencil(int mode, int E, int prec, dim3 grid, dim3 block, size_t lds,
                         hipStream_t s, float2* data, const float2* otf, const float2* tw,
                         const PencilArgs& a, const Sched& sc, hipEvent_t ev0 = nullptr,
                         hipEvent_t ev1 = nullptr);
// Sets the kernel attributes a launch with this shape needs (no launch).
hipError_t prepare_pencil(int mode, int E, int L, int prec, dim3 block, size_t lds);
hipError_t launch_xrow(int mode, int E, int prec, dim3 grid, dim3 block, size_t lds,
                       hipStream_t s, const XArgs& a, const Sched& sc, const float2* tw,
                       hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
hipError_t launch_twiddles(float2* tab, int n, hipStream_t s);
// flux[r] = sum_g partials[r * groups + g] for r < rows (a row is one
// (iteration, volume) pair), summed in a fixed order.
hipError_t launch_flux_reduce(const double* partials, int groups, int rows, double* flux,
                              hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// Extrapolation weight of the next iteration from the XM_UPDATE_ACC partials of
// iteration `it` (summed in a fixed order): alpha[it + 1] = <g_it, g_it-1> /
// <g_it-1, g_it-1> clipped to [0, 1] (0 for it == 0 or a zero denominator),
// stored in FP32 (alpha32, read by the kernels) and FP64 (alpha64, reported).
// For it == 0 it also writes alpha[0] = 0.
hipError_t launch_accel_alpha(const double* acc_partials, int groups, int it, float* alpha32,
                              double* alpha64, hipStream_t s, hipEvent_t ev0 = nullptr,
                              hipEvent_t ev1 = nullptr);
// Metric of iteration `it` from the work-group partials (rows: LOGLIK: sum of
// d log q - q; CHANGE: sum (u' - u)^2, sum u^2; PSNR: sum u', u'^2, u' g, g, g^2,
// min g, max g; SSIM: sum of window SSIMs, nvox = number of windows; FSC: one row
// holding the resolution, groups = 1), stored in
// hist[it]; then the stop decision (see rl.h): stop[0] = 1 and stop[1] =
// iterations carried out.  stop[2] = entries of hist.
// Does nothing once stop[0] is set.
hipError_t launch_metric(const double* met_partials, int groups, int metric, int it,
                         double threshold, int min_iter, long long nvox, double* hist, int* stop,
                         hipStream_t s);
// Mean-SSIM partials of u against g (dense nz x ny x nx, every dimension >= 7):
// window sums along X into buf_a (5 * nz * ny * (nx-6) doubles), along Y into buf_b
// (5 * nz * (ny-6) * (nx-6)), then along Z with the SSIM of each window summed per
// work-group into part (ceil((nx-6)/256) * (ny-6) * ceil((nz-6)/32) doubles).  With
// want_range, *range = max(g) - min(g) first (range_part: 2 * range_blocks).
// If stop is non-null and *stop != 0 the kernels do nothing.
hipError_t launch_ssim(const float* u, const float* g, int nz, int ny, int nx, double* buf_a,
                       double* buf_b, double* range_part, int range_blocks, double* range,
                       double* part, bool want_range, const int* stop, hipStream_t s);
// a = u[0::2, 0::2, 0::2], b = u[1::2, 1::2, 1::2] of a dense nz x ny x nx volume
// (even dimensions; a and b hold (nz/2)(ny/2)(nx/2) floats each).
// If stop is non-null and *stop != 0 the kernel does nothing.
hipError_t launch_split_diag(const float* u, int nz, int ny, int nx, float* a, float* b,
                             hipStream_t s, const int* stop = nullptr);
// Fourier shell correlation of two half spectra (tiled layout of an nz x ny x nx
// grid with xt tiles; lcm = lcm(nz, ny, nx) < 2^21): part holds
// nz * xt * (nbins + 1) * 3 doubles, out 4 * (nbins + 1) + 1 (curve, the three
// sums per shell, resolution).  If stop is non-null and *stop != 0 the kernels
// do nothing.
hipError_t launch_fsc(const float2* F, const float2* G, int nz, int ny, int nx, int xt, int nbins,
                      long long lcm, double threshold, double* part, double* out,
                      hipStream_t s, const int* stop = nullptr);
// *counter += 1 (one thread); used to advance a device-side iteration index.
hipError_t launch_advance(int* counter, hipStream_t s);
// *counter = value (one thread).
hipError_t launch_set_counter(int* counter, int value, hipStream_t s);
// out[0] = sum(h), out[1] = min(h), out[2] = number of non-finite entries (FP64).
hipError_t launch_psf_stats(const float* h, long long n, double* partials, int nblk,
                            unsigned* counter, double* out, hipStream_t s);
// Writes the PSF h (shape pz x py x px, each <= the grid's) times `scale`,
// centred on voxel 0 of the periodic grid nz x ny x nx (zero elsewhere), as
// real rows `out_row_stride` floats apart.
hipError_t launch_psf_prep(const float* h, int pz, int py, int px, float* out, int nz, int ny,
                           int nx, long long out_row_stride, double scale, hipStream_t s);
hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s);

}  // namespace rlmi
