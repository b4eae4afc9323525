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

// Geometry of a strided pencil pass (Y or Z axis) over the half spectrum.
// Element e of the pencil for (outer o, column x) sits at
//   o * ostride + e * estride + x   (complex elements).
struct PencilArgs {
  int L;       // transform length
  int P;       // threads per pencil (L / E)
  int TX;      // columns per work-group (power of two)
  int TXP;     // LDS row stride in complex elements (>= TX)
  int ncols;   // valid columns (nx/2 + 1)
  long long estride;
  long long ostride;
};

enum PencilMode { PM_FWD = 0, PM_INV = 1, PM_FKI = 2, PM_FCKI = 3 };
enum XMode { XM_R2C = 0, XM_C2R = 1, XM_RATIO = 2, XM_UPDATE = 3 };

// Arguments of an X-row pass (contiguous axis, real <-> half spectrum).
struct XArgs {
  float2* spec;          // half-spectrum rows, `pitch` complex apart
  long long pitch;
  const float* rin;      // XM_R2C: real input rows, `rin_stride` floats apart
  long long rin_stride;
  float* rout;           // XM_C2R: real output rows, `rout_stride` floats apart
  long long rout_stride;
  const float* d;        // XM_RATIO: observed rows (dense, nx floats apart)
  float* u;              // XM_UPDATE: estimate rows (dense), updated in place
  double* partials;      // XM_UPDATE: FP64 partial flux, [iter][work-group]
  int iter;
  int do_fwd;            // XM_UPDATE: also transform the new estimate forward
  int M;                 // complex row length nx/2
  int P;                 // threads per row (M / E)
  int RPW;               // rows per work-group (a multiple of 64 / P)
  int RS;                // LDS row stride in complex elements (>= M + 1)
  int nrows;             // nz * ny
};

hipError_t launch_pencil(int mode, int E, dim3 grid, dim3 block, size_t lds, hipStream_t s,
                         float2* data, const float2* otf, const float2* tw,
                         const PencilArgs& a, const Sched& sc);
hipError_t launch_xrow(int mode, int E, dim3 grid, dim3 block, size_t lds, hipStream_t s,
                       const XArgs& a, const Sched& sc, const float2* tw);
hipError_t launch_twiddles(float2* tab, int n, hipStream_t s);
// flux[it] = sum_g partials[it * groups + g] for it < n_iter, summed in a fixed order.
hipError_t launch_flux_reduce(const double* partials, int groups, int n_iter, double* flux,
                              hipStream_t s);
// out[0] = sum(h), out[1] = min(h), out[2] = number of non-finite entries (FP64).
hipError_t launch_psf_stats(const float* h, long long n, double* partials, int nblk,
                            unsigned* counter, double* out, hipStream_t s);
hipError_t launch_psf_prep(const float* h, float* out, int nz, int ny, int nx,
                           long long out_row_stride, double scale, hipStream_t s);
hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s);

}  // namespace rlmi
