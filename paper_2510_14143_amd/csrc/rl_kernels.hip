// HIP kernels for gfx950: FFT passes of the periodic 3-D Richardson-Lucy
// iteration (paper §4.3), with the ratio and update steps fused into the
// passes along the contiguous X axis.
//
// Transform scheme.  Each 1-D transform of length L runs as a sequence of
// Stockham radix stages (radices 16, 8, 4, 2, and 3 as the last stage).  A
// thread owns E elements of its pencil, element i + P*m in register m
// (P = L/E threads per pencil).  Stage (p, R) processes butterflies
// b = i + q*P, q < E/R, whose inputs are elements b + j*L/R (registers
// q + j*E/R); it multiplies input j by w_{pR}^{j*k} with k = b mod p, applies
// an R-point DFT, and writes output jj to position (b - k)*R + k + jj*p.  All
// but the last stage exchange through LDS; the last stage's outputs land in
// natural order in the same registers, so global loads and stores of a pass
// are always "element i + P*m".
//
// The half spectrum (nx/2 + 1 complex columns per row) is stored x-tile major:
// [Z][column tile][Y][16], so a tile column is one contiguous run of ny * 128
// bytes.  The Y pass reads whole tile columns, the Z pass reads 128 * ty bytes
// per z step, and the X pass reads 128-byte row pieces of 16-row bands.  Real
// rows are transformed as complex rows of half length (even samples in the real
// part, odd in the imaginary part) followed by the split into even and odd
// spectra.
#include "rl_internal.h"

#include <hip/hip_ext.h>

namespace rlmi {

// ---------------------------------------------------------------------------
// complex helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 conjf2(float2 a) { return make_float2(a.x, -a.y); }
// multiply by S*i (S = +1 or -1)
template <int S>
__device__ __forceinline__ float2 mul_si(float2 a) {
  return S > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// Ordering point for LDS traffic that stays inside one wavefront: the lanes of
// a wave execute in lock step and a wave's LDS operations complete in issue
// order, so only the compiler must be kept from moving accesses across it.
// A copy of v that the compiler cannot see through: index arithmetic derived from
// it is not merged with that of an earlier transform of the same schedule (which
// would keep every such address in a register from one transform to the other).
__device__ __forceinline__ int opaque_int(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <bool WAVE>
__device__ __forceinline__ void exch_sync() {
  if constexpr (WAVE) wave_sync();
  else __syncthreads();
}

// cos(2 pi k / 16), k = 0..15
__device__ constexpr float kCos16[16] = {
    1.0f,  0.92387953251128674f,  0.70710678118654752f,  0.38268343236508977f,
    0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
   -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f,
    0.0f,  0.38268343236508977f,  0.70710678118654752f,  0.92387953251128674f};

// a * exp(S * 2 pi i K / R) for R in {2, 4, 8, 16}, with the trivial angles special-cased.
template <int R, int K, int S>
__device__ __forceinline__ float2 rot(float2 a) {
  constexpr int k = ((K % R) + R) % R;
  if constexpr (k == 0) {
    return a;
  } else if constexpr (2 * k == R) {
    return make_float2(-a.x, -a.y);
  } else if constexpr (4 * k == R) {
    return mul_si<S>(a);
  } else if constexpr (4 * k == 3 * R) {
    return mul_si<-S>(a);
  } else {
    constexpr int t = k * (16 / R);
    const float c = kCos16[t];
    const float s = S * kCos16[(t + 12) & 15];  // sin(2 pi t / 16)
    return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
  }
}

// In-register R-point DFT, y_k = sum_j x_j exp(S * 2 pi i j k / R), natural order.
template <int R, int S>
struct Dft;

template <int S>
struct Dft<2, S> {
  __device__ __forceinline__ static void run(float2* x) {
    float2 a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  }
};

template <int S>
struct Dft<3, S> {
  __device__ __forceinline__ static void run(float2* x) {
    constexpr float h = 0.86602540378443865f;  // sqrt(3)/2
    float2 a = x[0], b = x[1], c = x[2];
    float2 t1 = cadd(b, c);
    float2 t2 = make_float2(a.x - 0.5f * t1.x, a.y - 0.5f * t1.y);
    float2 d = csub(b, c);
    float2 t3 = make_float2(S * h * d.x, S * h * d.y);
    float2 it3 = make_float2(-t3.y, t3.x);  // i * t3
    x[0] = cadd(a, t1);
    x[1] = cadd(t2, it3);
    x[2] = csub(t2, it3);
  }
};

template <int S>
struct Dft<4, S> {
  __device__ __forceinline__ static void run(float2* x) {
    float2 s0 = cadd(x[0], x[2]), d0 = csub(x[0], x[2]);
    float2 s1 = cadd(x[1], x[3]), d1 = mul_si<S>(csub(x[1], x[3]));
    x[0] = cadd(s0, s1);
    x[2] = csub(s0, s1);
    x[1] = cadd(d0, d1);
    x[3] = csub(d0, d1);
  }
};

// cos and sin of 2 pi k / R (R = 5, 7), rounded from FP64 values.
template <int R>
__device__ __forceinline__ constexpr float cos_2pi(int k);
template <int R>
__device__ __forceinline__ constexpr float sin_2pi(int k);
template <>
__device__ __forceinline__ constexpr float cos_2pi<5>(int k) {
  return k == 0 ? 1.f : (k == 1 || k == 4) ? 0.30901699437494742f : -0.80901699437494742f;
}
template <>
__device__ __forceinline__ constexpr float sin_2pi<5>(int k) {
  return k == 0 ? 0.f
         : k == 1 ? 0.95105651629515357f
         : k == 2 ? 0.58778525229247313f
         : k == 3 ? -0.58778525229247313f
                  : -0.95105651629515357f;
}
template <>
__device__ __forceinline__ constexpr float cos_2pi<7>(int k) {
  return k == 0 ? 1.f
         : (k == 1 || k == 6) ? 0.62348980185873353f
         : (k == 2 || k == 5) ? -0.22252093395631440f
                              : -0.90096886790241913f;
}
template <>
__device__ __forceinline__ constexpr float sin_2pi<7>(int k) {
  return k == 0 ? 0.f
         : k == 1 ? 0.78183148246802981f
         : k == 2 ? 0.97492791218182361f
         : k == 3 ? 0.43388373911755812f
         : k == 4 ? -0.43388373911755812f
         : k == 5 ? -0.97492791218182361f
                  : -0.78183148246802981f;
}

// Odd prime radix R by the pair symmetry of the DFT: with t_k = x_k + x_{R-k} and
// d_k = x_k - x_{R-k} (k = 1 .. (R-1)/2), X_m = x_0 + sum_k cos(2 pi mk/R) t_k
// -/+ i sum_k sin(2 pi mk/R) d_k and X_{R-m} the same with the sign flipped
// (upper sign forward, S = -1).
template <int R, int S>
struct DftOdd {
  __device__ __forceinline__ static void run(float2* x) {
    constexpr int H = (R - 1) / 2;
    float2 t[H], d[H];
#pragma unroll
    for (int k = 1; k <= H; ++k) {
      t[k - 1] = cadd(x[k], x[R - k]);
      d[k - 1] = csub(x[k], x[R - k]);
    }
    const float2 x0 = x[0];
    float2 sum = x0;
#pragma unroll
    for (int k = 0; k < H; ++k) sum = cadd(sum, t[k]);
    x[0] = sum;
#pragma unroll
    for (int m = 1; m <= H; ++m) {
      float2 a = x0, b = make_float2(0.f, 0.f);
#pragma unroll
      for (int k = 1; k <= H; ++k) {
        const float c = cos_2pi<R>((m * k) % R), sn = sin_2pi<R>((m * k) % R);
        a = make_float2(a.x + c * t[k - 1].x, a.y + c * t[k - 1].y);
        b = make_float2(b.x + sn * d[k - 1].x, b.y + sn * d[k - 1].y);
      }
      const float2 ib = make_float2(-b.y, b.x);  // i * b
      x[m] = (S < 0) ? csub(a, ib) : cadd(a, ib);
      x[R - m] = (S < 0) ? cadd(a, ib) : csub(a, ib);
    }
  }
};

template <int S>
struct Dft<5, S> : DftOdd<5, S> {};
template <int S>
struct Dft<7, S> : DftOdd<7, S> {};

// Radix-2 decimation in time: split into even and odd halves.
template <int R, int S>
struct Dft {
  static_assert(R == 8 || R == 16, "unsupported radix");
  template <int K>
  __device__ __forceinline__ static void combine(float2* x, const float2* e, const float2* o) {
    if constexpr (K < R / 2) {
      float2 t = rot<R, K, S>(o[K]);
      x[K] = cadd(e[K], t);
      x[K + R / 2] = csub(e[K], t);
      combine<K + 1>(x, e, o);
    }
  }
  __device__ __forceinline__ static void run(float2* x) {
    float2 e[R / 2], o[R / 2];
#pragma unroll
    for (int j = 0; j < R / 2; ++j) {
      e[j] = x[2 * j];
      o[j] = x[2 * j + 1];
    }
    Dft<R / 2, S>::run(e);
    Dft<R / 2, S>::run(o);
    combine<0>(x, e, o);
  }
};

// ---------------------------------------------------------------------------
// Split-precision 16-point DFT on MFMA
// ---------------------------------------------------------------------------
// A 16-point complex DFT is the 32x32 real matrix [[Fr, -S Fi], [S Fi, Fr]]
// applied to (re_0..15, im_0..15).  A wavefront computes its 64 threads' DFTs
// as 4 groups of 16 columns with v_mfma_f32_16x16x32_{bf16,f16}: operands are
// split x = hi + lo (hi = RNE(x), lo = RNE(x - hi)) and the three products
// Fhi*Xhi + Fhi*Xlo + Flo*Xhi accumulate in FP32.  FP16 inputs are scaled per
// DFT by a power of two (largest magnitude below 2^14); the scale is undone on
// the FP32 result.  Operand lane layout (16x16x32): lane l holds A row l%16 and
// B column l%16 over K = 8*(l/16) .. +7; D rows 4*(l/16) .. +3 of column l%16.
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int PREC>
struct SplitT;

template <>
struct SplitT<1> {  // BF16 hi/lo
  typedef __bf16 T;
  typedef __bf16 V8 __attribute__((ext_vector_type(8)));
  static constexpr bool kScale = false;
  __device__ __forceinline__ static f32x4 mma(V8 a, V8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

template <>
struct SplitT<2> {  // FP16 hi/lo with a power-of-two scale per DFT
  typedef _Float16 T;
  typedef _Float16 V8 __attribute__((ext_vector_type(8)));
  static constexpr bool kScale = true;
  __device__ __forceinline__ static f32x4 mma(V8 a, V8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

// A operands of the 16-point DFT per lane: lane l holds row n = l % 16 of the
// real-output block [Fr, -S Fi] and of the imaginary-output block [S Fi, Fr] over
// K = 8g .. 8g+7 (g = l / 16), each split into hi and lo.  They depend only on the
// lane and the sign, so every work-group computes them once into this LDS table,
// [sign: forward, inverse][lane][re hi, re lo, im hi, im lo] (8 KB), which the
// host adds to the kernel's LDS budget (kSplitTabBytes).
template <int PREC>
__device__ __forceinline__ typename SplitT<PREC>::V8* split_atab() {
  __shared__ typename SplitT<PREC>::V8 tab[2 * 64 * 4];
  return tab;
}

// Every thread of the work-group calls this; a barrier must follow before use.
template <int PREC>
__device__ __forceinline__ void split_atab_fill() {
  typedef SplitT<PREC> ST;
  typedef typename ST::T T;
  typename ST::V8* tab = split_atab<PREC>();
  for (int e = threadIdx.x; e < 2 * 64 * 4; e += blockDim.x) {
    const int S = (e >> 8) ? 1 : -1;
    const int l = (e >> 2) & 63, w = e & 3;
    const int n = l & 15, g = l >> 4;
    typename ST::V8 v;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int kk = 8 * g + q, k = kk & 15, t = (n * k) & 15;
      const float c = kCos16[t], sn = kCos16[(t + 12) & 15];
      const float val = (w < 2) ? (kk < 16 ? c : -S * sn) : (kk < 16 ? S * sn : c);
      const T hi = (T)val;
      v[q] = (w & 1) ? (T)(val - (float)hi) : hi;
    }
    tab[e] = v;
  }
}

// Staging slot (in float4 units) of 16-byte granule G (0..7) of row t: rows of 32
// floats, granules XOR-swizzled by f(t) = (n ^ n >> 3) & 7 with n = t mod 16, which
// takes distinct values on every 8 consecutive rows of a 16-row group and on its
// even and on its odd rows.  A row's granules, and one granule across 8 or 16 rows
// of a group, thus fall into distinct LDS banks with 128-byte and with 256-byte
// bank spans.  f depends on t mod 16 only, so the slots of row 16 grp + n are those
// of row n plus 128 grp: one address register serves all four column groups.
// Granules 0..3 hold the real parts of a 16-point pencil, 4..7 the imaginary ones.
__device__ __forceinline__ int stg_q(int t, int G) {
  const int n = t & 15;
  return 8 * t + (G ^ ((n ^ (n >> 3)) & 7));
}

// y[0..15] of every thread of the wavefront <- its 16-point DFT (sign S).
// `stg` is a wave-private, 16-byte aligned LDS area of 64 * 32 floats; all 64
// lanes must call.  The 16 pencils of column group grp (rows 16 grp .. 16 grp + 15)
// are transformed and written back before the next group is read: a group's
// outputs overwrite only its own rows, whose inputs every lane of the wave has
// read before the MFMAs that consume them, so at most two accumulators are live.
template <int PREC, int S>
__device__ __forceinline__ void dft16_mfma(float2 (&y)[16], float* stg) {
  typedef SplitT<PREC> ST;
  typedef typename ST::T T;
  typedef typename ST::V8 V8;
  const int l = threadIdx.x & 63;
  const int n = l & 15, g = l >> 4;
  const V8* at = split_atab<PREC>() + ((S < 0 ? 0 : 1) * 64 + l) * 4;
  const V8 are_hi = at[0], are_lo = at[1], aim_hi = at[2], aim_lo = at[3];
  float4* s4 = reinterpret_cast<float4*>(stg);
  // stage the inputs: thread t's (re_0..15, im_0..15) in row t
#pragma unroll
  for (int G = 0; G < 4; ++G) {
    s4[stg_q(l, G)] = make_float4(y[4 * G].x, y[4 * G + 1].x, y[4 * G + 2].x, y[4 * G + 3].x);
    s4[stg_q(l, 4 + G)] = make_float4(y[4 * G].y, y[4 * G + 1].y, y[4 * G + 2].y, y[4 * G + 3].y);
  }
  wave_sync();
#pragma unroll
  for (int grp = 0; grp < 4; ++grp) {
    const int row = 16 * grp + n;
    // K = 8g .. 8g+7 of pencil `row`: granules 2g and 2g+1
    const float4 lo4 = s4[stg_q(row, 2 * g)], hi4 = s4[stg_q(row, 2 * g + 1)];
    const float x[8] = {lo4.x, lo4.y, lo4.z, lo4.w, hi4.x, hi4.y, hi4.z, hi4.w};
    float sc = 1.f, inv = 1.f;
    if constexpr (ST::kScale) {
      float mx = 0.f;
#pragma unroll
      for (int q = 0; q < 8; ++q) mx = fmaxf(mx, fabsf(x[q]));
      mx = fmaxf(mx, __shfl_xor(mx, 16, 64));
      mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
      if (mx > 0.f && isfinite(mx)) {
        int e;
        (void)frexpf(mx, &e);  // mx < 2^e
        // largest magnitude just below 2^14; the shift is capped so the scale stays
        // finite for tiny inputs (e.g. the far tail of a PSF), which then round to 0
        const int sh = min(14 - e, 64);
        sc = ldexpf(1.f, sh);
        inv = ldexpf(1.f, -sh);
      }
    }
    V8 bh, bl;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const float xs = x[q] * sc;
      const T h = (T)xs;
      bh[q] = h;
      bl[q] = (T)(xs - (float)h);
    }
    const f32x4 z = {0.f, 0.f, 0.f, 0.f};
    f32x4 r = ST::mma(are_hi, bh, z);
    r = ST::mma(are_hi, bl, r);
    r = ST::mma(are_lo, bh, r);
    f32x4 im = ST::mma(aim_hi, bh, z);
    im = ST::mma(aim_hi, bl, im);
    im = ST::mma(aim_lo, bh, im);
    // outputs 4g .. 4g+3 of pencil `row`: real parts in granule g, imaginary in 4 + g
    s4[stg_q(row, g)] = make_float4(r[0] * inv, r[1] * inv, r[2] * inv, r[3] * inv);
    s4[stg_q(row, 4 + g)] = make_float4(im[0] * inv, im[1] * inv, im[2] * inv, im[3] * inv);
  }
  wave_sync();
#pragma unroll
  for (int G = 0; G < 4; ++G) {
    const float4 re = s4[stg_q(l, G)], im = s4[stg_q(l, 4 + G)];
    y[4 * G] = make_float2(re.x, im.x);
    y[4 * G + 1] = make_float2(re.y, im.y);
    y[4 * G + 2] = make_float2(re.z, im.z);
    y[4 * G + 3] = make_float2(re.w, im.w);
  }
  wave_sync();
}

// ---------------------------------------------------------------------------
// Stockham stages
// ---------------------------------------------------------------------------
// tw: table of exp(-2 pi i m / T) (forward sign); inverse transforms conjugate it.
// lds element n of this thread's pencil lives at lds[n * ls + lo].
// LDS slot of pencil element n: with PAD > 0 one spare slot follows every 2^PAD
// elements, which spreads power-of-two strides over the banks.
template <int PAD>
__device__ __forceinline__ int lslot(int n) {
  if constexpr (PAD > 0) return n + (n >> PAD);
  else return n;
}

// PREC > 0 with R = E = 16: the butterfly runs on MFMA (dft16_mfma) using the
// wave's staging area `stg`; a barrier (WAVE: wavefront, else work-group)
// separates that from the stage's LDS output writes.
template <int E, int R, int S, int PAD, int PREC = 0, bool WAVE = false>
__device__ __forceinline__ void stage(float2 (&v)[E], int i, int P, int p, int tm, bool last,
                                      const float2* __restrict__ tw, float2* lds, int ls, int lo,
                                      float* stg = nullptr) {
  constexpr int V = E / R;
#pragma unroll
  for (int q = 0; q < V; ++q) {
    const int b = i + q * P;
    // position inside the current span p: the schedule puts every odd radix after
    // all power-of-two ones, so p is a power of two before any power-of-two stage
    int k;
    if constexpr ((R & (R - 1)) == 0)
      k = last ? b : (b & (p - 1));
    else
      k = last ? b : (b % p);
    float2 y[R];
#pragma unroll
    for (int j = 0; j < R; ++j) y[j] = v[q + j * V];
    if (p > 1) {
#pragma unroll
      for (int j = 1; j < R; ++j) {
        const float2 w = tw[j * k * tm];
        y[j] = (S < 0) ? cmul(y[j], w) : cmulc(y[j], w);
      }
    }
    if constexpr (PREC > 0 && R == 16 && E == 16) {
      dft16_mfma<PREC, S>(y, stg);
      exch_sync<WAVE>();  // all staging areas are free before outputs land in LDS
    } else {
      Dft<R, S>::run(y);
    }
    if (last) {
#pragma unroll
      for (int j = 0; j < R; ++j) v[q + j * V] = y[j];
    } else {
      const int base = (b - k) * R + k;
#pragma unroll
      for (int j = 0; j < R; ++j) lds[lslot<PAD>(base + j * p) * ls + lo] = y[j];
    }
  }
}

// Full 1-D transform of this thread's pencil; natural order in and out.
// WAVE = false: the pencil spans the work-group and every thread must call this
// (it contains barriers).  WAVE = true: the pencil lives inside one wavefront.
template <int E, int S, bool WAVE = false, int PAD = 0, int PREC = 0>
__device__ __forceinline__ void fft(float2 (&v)[E], const Sched& sc, int i, int P,
                                    const float2* __restrict__ tw, float2* lds, int ls, int lo,
                                    float* stg = nullptr) {
  for (int s = 0; s < sc.ns; ++s) {
    const bool last = (s == sc.ns - 1);
    const int r = sc.r[s], p = sc.p[s], tm = sc.tm[s];
    switch (r) {
      case 16:
        if constexpr (E % 16 == 0)
          stage<E, 16, S, PAD, PREC, WAVE>(v, i, P, p, tm, last, tw, lds, ls, lo, stg);
        break;
      case 8:
        if constexpr (E % 8 == 0) stage<E, 8, S, PAD>(v, i, P, p, tm, last, tw, lds, ls, lo);
        break;
      case 4:
        if constexpr (E % 4 == 0) stage<E, 4, S, PAD>(v, i, P, p, tm, last, tw, lds, ls, lo);
        break;
      case 2:
        if constexpr (E % 2 == 0) stage<E, 2, S, PAD>(v, i, P, p, tm, last, tw, lds, ls, lo);
        break;
      case 3:
        if constexpr (E % 3 == 0) stage<E, 3, S, PAD>(v, i, P, p, tm, last, tw, lds, ls, lo);
        break;
      case 5:
        if constexpr (E % 5 == 0) stage<E, 5, S, PAD>(v, i, P, p, tm, last, tw, lds, ls, lo);
        break;
      case 7:
        if constexpr (E % 7 == 0) stage<E, 7, S, PAD>(v, i, P, p, tm, last, tw, lds, ls, lo);
        break;
      default:
        break;
    }
    if (!last) {
      exch_sync<WAVE>();
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = lds[lslot<PAD>(i + P * m) * ls + lo];
      exch_sync<WAVE>();
    }
  }
}

// ---------------------------------------------------------------------------
// Compile-time schedules (power-of-two lengths of the X rows)
// ---------------------------------------------------------------------------
// The stages of fft() with the length, the elements per thread, and every
// stage's radix, span and twiddle stride known at compile time, for rows that
// one wavefront holds (LDS stride 1).  The index arithmetic of the runtime
// schedule (spans, butterfly positions, LDS slots, twiddle indices) then folds
// into constants and LDS immediate offsets: the fused X passes, whose vector
// instruction issue bounds them, run about half the instructions.
struct CtSched {
  int ns;
  int r[kMaxStages];
  int p[kMaxStages];
};

// The host's radix order for a length L: the largest power-of-two radix
// dividing E, repeated, the rest of the power of two by the next smaller ones,
// then the odd factors (every 7, every 5, every 3).
constexpr CtSched ct_sched(int L, int E) {
  CtSched s{0, {0, 0, 0, 0, 0, 0, 0, 0}, {0, 0, 0, 0, 0, 0, 0, 0}};
  int n = L, nodd = 0;
  int odd[kMaxStages] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int r : {7, 5, 3})
    while (n % r == 0 && nodd < kMaxStages) {
      n /= r;
      odd[nodd++] = r;
    }
  const int big = E % 16 == 0 ? 16 : E % 8 == 0 ? 8 : E % 4 == 0 ? 4 : E % 2 == 0 ? 2 : 1;
  int p = 1;
  while (n > 1 && big > 1 && s.ns < kMaxStages) {
    int r = big;
    while (r > 1 && n % r) r /= 2;
    if (r == 1) break;
    s.r[s.ns] = r;
    s.p[s.ns] = p;
    p *= r;
    n /= r;
    ++s.ns;
  }
  for (int q = 0; q < nodd && s.ns < kMaxStages; ++q) {
    s.r[s.ns] = odd[q];
    s.p[s.ns] = p;
    p *= odd[q];
    ++s.ns;
  }
  return s;
}

template <int E, int R, int S, int PAD, int P, int p, int TM, bool LAST>
__device__ __forceinline__ void stage_ct(float2 (&v)[E], int i, const float2* __restrict__ tw,
                                         float2* lds) {
  constexpr int V = E / R;
#pragma unroll
  for (int q = 0; q < V; ++q) {
    const int b = i + q * P;
    const int k = LAST ? b : (int)((unsigned)b % (unsigned)p);
    float2 y[R];
#pragma unroll
    for (int j = 0; j < R; ++j) y[j] = v[q + j * V];
    if constexpr (p > 1) {
#pragma unroll
      for (int j = 1; j < R; ++j) {
        const float2 w = tw[j * k * TM];
        y[j] = (S < 0) ? cmul(y[j], w) : cmulc(y[j], w);
      }
    }
    Dft<R, S>::run(y);
    if constexpr (LAST) {
#pragma unroll
      for (int j = 0; j < R; ++j) v[q + j * V] = y[j];
    } else {
      const int base = (b - k) * R + k;
#pragma unroll
      for (int j = 0; j < R; ++j) lds[lslot<PAD>(base + j * p)] = y[j];
    }
  }
}

// Full transform of a wave-held row of length L (twiddle table stride TS);
// natural order in and out, like fft<E, S, true, PAD>.
template <int E, int S, int PAD, int L, int TS, int ST = 0>
__device__ __forceinline__ void fft_ct(float2 (&v)[E], int i, const float2* __restrict__ tw,
                                       float2* lds) {
  constexpr CtSched cs = ct_sched(L, E);
  if constexpr (ST < cs.ns) {
    constexpr int P = L / E, R = cs.r[ST], p = cs.p[ST];
    constexpr bool last = ST == cs.ns - 1;
    stage_ct<E, R, S, PAD, P, p, TS * (L / (p * R)), last>(v, i, tw, lds);
    if constexpr (!last) {
      wave_sync();
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = lds[lslot<PAD>(i + P * m)];
      wave_sync();
      fft_ct<E, S, PAD, L, TS, ST + 1>(v, i, tw, lds);
    }
  }
}

// X-row transform: the compile-time schedule when CM (the row length) is
// non-zero, else the runtime one.
template <int E, int S, int PREC, int CM>
__device__ __forceinline__ void fft_row(float2 (&v)[E], const Sched& sc, int i, int P,
                                        const float2* __restrict__ tw, float2* row, float* stg) {
  if constexpr (CM > 0) fft_ct<E, S, kXPad, CM, 2>(v, i, tw, row);
  else fft<E, S, true, kXPad, PREC>(v, sc, i, P, tw, row, 1, 0, stg);
}

// Compile-time schedule of a work-group pencil (power-of-two length L, LDS
// element n of this thread's pencil at lds[n * ls + lo]): the stages of fft()
// with radix, span and twiddle stride folded into constants.  PREC > 0 runs
// the 16-point stages on MFMA (dft16_mfma); its staging areas lie inside the
// exchange buffer, so a work-group barrier separates them from the stage's
// output writes.
template <int E, int R, int S, int P, int p, int TM, bool LAST, int PREC>
__device__ __forceinline__ void stage_ctp(float2 (&v)[E], int i, const float2* __restrict__ tw,
                                          float2* lds, int ls, int lo, float* stg) {
  constexpr int V = E / R;
#pragma unroll
  for (int q = 0; q < V; ++q) {
    const int b = i + q * P;
    const int k = LAST ? b : (int)((unsigned)b % (unsigned)p);
    float2 y[R];
#pragma unroll
    for (int j = 0; j < R; ++j) y[j] = v[q + j * V];
    if constexpr (p > 1) {
#pragma unroll
      for (int j = 1; j < R; ++j) {
        const float2 w = tw[j * k * TM];
        y[j] = (S < 0) ? cmul(y[j], w) : cmulc(y[j], w);
      }
    }
    if constexpr (PREC > 0 && R == 16 && E == 16) {
      dft16_mfma<PREC, S>(y, stg);
      if constexpr (!LAST) __syncthreads();  // every staging area is free
    } else {
      Dft<R, S>::run(y);
    }
    if constexpr (LAST) {
#pragma unroll
      for (int j = 0; j < R; ++j) v[q + j * V] = y[j];
    } else {
      const int base = (b - k) * R + k;
#pragma unroll
      for (int j = 0; j < R; ++j) lds[(base + j * p) * ls + lo] = y[j];
    }
  }
}

template <int E, int S, int L, int PREC, int ST = 0>
__device__ __forceinline__ void fft_ctp(float2 (&v)[E], int i, const float2* __restrict__ tw,
                                        float2* lds, int ls, int lo, float* stg) {
  constexpr CtSched cs = ct_sched(L, E);
  if constexpr (ST < cs.ns) {
    constexpr int P = L / E, R = cs.r[ST], p = cs.p[ST];
    constexpr bool last = ST == cs.ns - 1;
    stage_ctp<E, R, S, P, p, L / (p * R), last, PREC>(v, i, tw, lds, ls, lo, stg);
    if constexpr (!last) {
      __syncthreads();
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = lds[(i + P * m) * ls + lo];
      __syncthreads();
      fft_ctp<E, S, L, PREC, ST + 1>(v, i, tw, lds, ls, lo, stg);
    }
  }
}

// ---------------------------------------------------------------------------
// Y / Z pencil pass
// ---------------------------------------------------------------------------
// Work-group = TXB lanes x P threads; lanes run along contiguous complex
// elements of the tiled layout, so a wavefront access covers TXB consecutive
// elements of 64/TXB pencil positions (for the Y pass the whole work-group
// reads one contiguous tile column).
// 1024-thread work-groups of the forward and inverse passes with E = 8 are held to
// 64 VGPRs (8 waves per SIMD), so that two of them share a CU; the filtered
// passes (which hold the transfer function too) are not, since at 64 VGPRs they
// would spill.
// One work-group tile of a pencil pass: (gx, gy) is the tile's position in the
// pass's launch grid, vz the volume (all threads of the work-group call it).
// CL > 0: the pencil length is CL (compile-time schedule).
template <int E, int MODE, int PREC = 0, int CL = 0>
__device__ __forceinline__ void pencil_tile(float2* __restrict__ data,
                                            const float2* __restrict__ otf,
                                            const float2* __restrict__ twg, const PencilArgs& a,
                                            const Sched& sc, int gx, int gy, int vz, float2* lds) {
  const int tid = threadIdx.x;
  const int P = CL > 0 ? CL / E : a.P;
  // twiddle table (L entries) after the exchange buffer
  float2* tw = lds + (size_t)a.L * a.TXP;
  const int lane = tid & (a.TXB - 1);
  const int i = tid / a.TXB;
  const int bx = a.swap ? gy : gx;  // tile (and split) index
  const int by = a.swap ? gx : gy;  // outer index
  const int xb = bx / a.xsplit;
  const int c = (bx - xb * a.xsplit) * a.TXB + lane;
  const bool ok = xb * kTile + (c & (kTile - 1)) < a.ncols;
  const long long base = (long long)vz * a.vstride + (long long)xb * a.xstride +
                         (long long)by * a.ostride + c;

  // Every element index lies inside the spectrum buffer (padding columns and rows
  // beyond lin included).  With few elements per thread, or short compiled
  // pencils, the loads issue unconditionally, back to back, and the zeros are
  // selected afterwards; otherwise the extra registers this takes (in the
  // filtered passes the compiler then also hoists the transfer function's loads
  // above the forward transform) cost more occupancy than the branches cost time
  // (measured on the 256- and 2160-point pencils).  The runtime-schedule
  // kernels keep the branches above 6 elements: held to 64 registers in
  // 1024-thread work-groups, they would spill.
  constexpr bool kUncond =
      E <= 6 || (CL > 0 && E <= 12 && (MODE == PM_FWD || MODE == PM_INV || CL <= 192));
  float2 v[E];
  if constexpr (kUncond) {
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = data[base + (long long)(i + P * m) * a.estride];
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = (ok && i + P * m < a.lin) ? v[m] : make_float2(0.f, 0.f);
  } else {
#pragma unroll
    for (int m = 0; m < E; ++m)
      v[m] = (ok && i + P * m < a.lin) ? data[base + (long long)(i + P * m) * a.estride]
                                          : make_float2(0.f, 0.f);
  }
  // the table is copied after the pencil loads are issued, so that they are not
  // held back behind its loads
  for (int t = tid; t < a.L; t += blockDim.x) tw[t] = twg[t];
  if constexpr (PREC > 0) split_atab_fill<PREC>();
  __syncthreads();  // twiddles in LDS

  // split-precision stages stage their operands in this wave's slice of the exchange buffer
  float* stg = reinterpret_cast<float*>(lds) + (tid >> 6) * (64 * 32);
  if constexpr (MODE != PM_INV) {
    if constexpr (CL > 0) fft_ctp<E, -1, CL, PREC>(v, i, tw, lds, a.TXP, lane, stg);
    else fft<E, -1, false, 0, PREC>(v, sc, i, P, tw, lds, a.TXP, lane, stg);
  }
  if constexpr (MODE == PM_FKI || MODE == PM_FCKI) {
    // the transfer function in its z-major order: the work-group's tile (a
    // uniform base; the last tile stored only as wide as its valid columns)
    // and this thread's row and column within it, element z at w z from there
    // (the in-tile offset is below ny * 16 * L <= 2^28)
    const float2* ot = otf + ((long long)vz * a.vstride + (long long)xb * a.xstride * a.L);
    const int w = min(kTile, a.ncols - xb * kTile);
    const int off = by * (int)a.ostride + c;  // within the tile's [y][16]
    const int oo = (off >> 4) * (w * a.L) + (ok ? (off & (kTile - 1)) : 0) + i * w;
#pragma unroll
    for (int m = 0; m < E; ++m) {
      float2 k;
      if constexpr (kUncond) {
        k = ot[oo + P * m * w];
        k = ok ? k : make_float2(0.f, 0.f);
      } else {
        k = ok ? ot[oo + P * m * w] : make_float2(0.f, 0.f);
      }
      v[m] = (MODE == PM_FKI) ? cmul(v[m], k) : cmulc(v[m], k);
    }
  }
  if constexpr (MODE != PM_FWD) {
    if constexpr (CL > 0) {
      // with both transforms in one kernel, fresh copies of the index operands keep
      // the inverse's LDS addresses from being merged with the forward's (which
      // would hold every one of them in a register through both transforms)
      int ls = a.TXP;
      if constexpr (MODE != PM_INV) asm volatile("" : "+s"(ls));
      fft_ctp<E, +1, CL, PREC>(v, MODE != PM_INV ? opaque_int(i) : i, tw, lds, ls,
                               MODE != PM_INV ? opaque_int(lane) : lane, stg);
    } else {
      fft<E, +1, false, 0, PREC>(v, sc, i, P, tw, lds, a.TXP, lane, stg);
    }
  }

  if (ok) {
#pragma unroll
    for (int m = 0; m < E; ++m)
      if (i + P * m < a.lout) data[base + (long long)(i + P * m) * a.estride] = v[m];
  }
}

template <int E, int MODE, int MAXT, int PREC = 0>
__global__ void __launch_bounds__(MAXT, (MAXT == 1024 && E == 8 && MODE <= PM_INV) ? 8 : 1)
    k_pencil(float2* __restrict__ data, const float2* __restrict__ otf,
             const float2* __restrict__ twg, PencilArgs a, Sched sc) {
  if (a.stop && *a.stop) return;  // stopped: the whole work-group leaves together
  extern __shared__ __attribute__((aligned(16))) float2 lds[];
  pencil_tile<E, MODE, PREC>(data, otf, twg, a, sc, blockIdx.x, blockIdx.y, blockIdx.z, lds);
}

// Pencils of compile-time length L (pencil_compiled_len).  The forward and inverse
// passes with 8 elements per thread are held to 64 registers, so that two
// 1024-thread work-groups share a CU (as for the runtime-schedule kernel).
template <int E, int MODE, int PREC, int L>
__global__ void __launch_bounds__(pencil_ct_max_threads(E, L), (E == 8 && MODE <= PM_INV) ? 8 : 1)
    k_pencil_ct(float2* __restrict__ data, const float2* __restrict__ otf,
                const float2* __restrict__ twg, PencilArgs a) {
  if (a.stop && *a.stop) return;  // stopped: the whole work-group leaves together
  extern __shared__ __attribute__((aligned(16))) float2 lds[];
  pencil_tile<E, MODE, PREC, L>(data, otf, twg, a, Sched{}, blockIdx.x, blockIdx.y, blockIdx.z,
                                lds);
}

// ---------------------------------------------------------------------------
// X row pass (contiguous axis)
// ---------------------------------------------------------------------------
// Each wavefront owns whole rows (P = M/E lanes per row, 64/P rows per wave), so
// every LDS exchange of a row is wave-local and needs no work-group barrier.
// All global loads of a row (half spectrum and the real operand) are issued
// before any arithmetic.

// Forward: complex row z (registers, natural order) -> FFT -> split into the
// half spectrum X[0..M] and store.  `row` is this row's wave-private LDS.
// Offset of column kx inside a row of the tiled half spectrum.
__device__ __forceinline__ long long col_off(int kx, long long tstride) {
  return (long long)(kx >> 4) * tstride + (kx & (kTile - 1));
}

template <int E, int PREC, int CM = 0>
__device__ __forceinline__ void r2c_store(float2 (&v)[E], int M, int P, const Sched& sc, int i,
                                          const float2* tw, float2* row, bool ok,
                                          float2* __restrict__ out, long long ts, float* stg) {
  fft_row<E, -1, PREC, CM>(v, sc, i, P, tw, row, stg);
#pragma unroll
  for (int m = 0; m < E; ++m) row[lslot<kXPad>(i + P * m)] = v[m];
  wave_sync();
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int k = i + P * m;
    const float2 A = v[m];
    const float2 B = conjf2(row[lslot<kXPad>(k == 0 ? 0 : M - k)]);
    const float2 ev = make_float2(0.5f * (A.x + B.x), 0.5f * (A.y + B.y));
    const float2 dd = csub(A, B);
    const float2 od = make_float2(0.5f * dd.y, -0.5f * dd.x);  // -i/2 * (A - B)
    const float2 X = cadd(ev, cmul(tw[k], od));
    if (ok) out[col_off(k, ts)] = X;
  }
  if (ok && i == 0) out[col_off(M, ts)] = make_float2(v[0].x - v[0].y, 0.f);
}

// Pairs X[k] with X[M-k] and forms z[k] = A + iB, the half-length complex
// spectrum whose inverse FFT interleaves the even and odd real samples.
template <int E>
__device__ __forceinline__ void c2r_prepare(float2 (&v)[E], float2 nyq, int M, int P, int i,
                                            const float2* tw, float2* row) {
#pragma unroll
  for (int m = 0; m < E; ++m) row[lslot<kXPad>(i + P * m)] = v[m];
  if (i == 0) row[lslot<kXPad>(M)] = nyq;
  wave_sync();
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int k = i + P * m;
    const float2 X = v[m];
    const float2 Y = conjf2(row[lslot<kXPad>(M - k)]);
    const float2 A = cadd(X, Y);
    const float2 B = cmulc(csub(X, Y), tw[k]);  // (X - conj X[M-k]) * exp(+2 pi i k / 2M)
    v[m] = make_float2(A.x - B.y, A.y + B.x);   // A + i B
  }
  wave_sync();
}

// Extrapolated point max(x + al * h, 0) with one rounding; a NaN passes through
// (the comparison is false) so that non-finite data still reach the flux check.
// Both passes that need y evaluate it with this function, so the estimate that
// is updated is bit for bit the one that was blurred.
__device__ __forceinline__ float predict1(float x, float h, float al) {
  const float y = __builtin_fmaf(al, h, x);
  return y < 0.f ? 0.f : y;
}

__device__ __forceinline__ float2 predict2(float2 x, float2 h, float al) {
  return make_float2(predict1(x.x, h.x, al), predict1(x.y, h.y, al));
}

// The volumes' rows are reached through pointers read from per-volume tables,
// which the compiler cannot place in an address space: it would emit flat
// accesses, each waited for on both the vector-memory and the LDS counter.  Rows
// are therefore addressed as global memory explicitly (an aligned float pair
// moves as one 8-byte scalar).
typedef __attribute__((address_space(1))) const double gcdouble;
typedef __attribute__((address_space(1))) double gdouble;
typedef __attribute__((address_space(1))) const float gcfloat;
typedef __attribute__((address_space(1))) float gfloat;

__device__ __forceinline__ float2 gload_pair(const float* row, int q) {
  return __builtin_bit_cast(float2, ((gcdouble*)row)[q]);  // C-style: changes address space
}

__device__ __forceinline__ void gstore_pair(float* row, int q, float2 v) {
  ((gdouble*)row)[q] = __builtin_bit_cast(double, v);
}

// Pair q (elements 2q, 2q+1) of a real row of `vx` floats; zero beyond the row
// or when `on` is false.  `row` must point at a readable row even when `on` is
// false: rows of even length are read unconditionally (pair 0 stands in for
// pairs beyond the row) and the zero selected afterwards, so that the loads of a
// row issue back to back.  Rows of odd length are not 8-byte aligned, so they are
// read one float at a time.
__device__ __forceinline__ float2 load_pair(const float* row, int q, int vx, bool on) {
  const int x = 2 * q;
  if ((vx & 1) == 0) {
    const float2 t = gload_pair(row, x < vx ? q : 0);
    return (on && x < vx) ? t : make_float2(0.f, 0.f);
  }
  if (!on || x >= vx) return make_float2(0.f, 0.f);
  const gcfloat* r = (gcfloat*)row;
  return make_float2(r[x], x + 1 < vx ? r[x + 1] : 0.f);
}

// Pairs i + P*m (m < E) of a row, as load_pair, for a row length whose parity
// is known (EVEN): no branch between the loads, so that they issue back to back.
// (EVEN: the loads only; zero_pairs selects the zeros once the values are needed)
template <bool EVEN, int E>
__device__ __forceinline__ void load_pairs_p(float2 (&w)[E], const float* row, int i, int P,
                                             int vx, bool on) {
  if constexpr (EVEN) {
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int q = i + P * m;
      w[m] = gload_pair(row, 2 * q < vx ? q : 0);
    }
  } else {
#pragma unroll
    for (int m = 0; m < E; ++m) w[m] = load_pair(row, i + P * m, vx, on);
  }
}

// Zeros of the pairs load_pairs_p<true> read but the row does not have (or all
// of them when `on` is false); a no-op for pairs load_pair already zeroed.
template <int E>
__device__ __forceinline__ void zero_pairs(float2 (&w)[E], int i, int P, int vx, bool on) {
#pragma unroll
  for (int m = 0; m < E; ++m) w[m] = (on && 2 * (i + P * m) < vx) ? w[m] : make_float2(0.f, 0.f);
}

// The same with the parity decided once, outside the loads, and the zeros selected.
template <int E>
__device__ __forceinline__ void load_pairs(float2 (&w)[E], const float* row, int i, int P,
                                           int vx, bool on) {
  if ((vx & 1) == 0) load_pairs_p<true>(w, row, i, P, vx, on);
  else load_pairs_p<false>(w, row, i, P, vx, on);
  zero_pairs(w, i, P, vx, on);
}

template <bool B>
struct BoolC {
  static constexpr bool value = B;
};

__device__ __forceinline__ void store_pair(float* row, int q, int vx, bool on, float2 v) {
  const int x = 2 * q;
  if (!on || x >= vx) return;
  if ((vx & 1) == 0) {
    gstore_pair(row, q, v);
  } else {
    gfloat* r = (gfloat*)row;
    r[x] = v.x;
    if (x + 1 < vx) r[x + 1] = v.y;
  }
}

// Work-group FP64 reduction of K values per thread (op per value: 0 sum, 1 min,
// 2 max): wavefront butterfly, then the waves in order; row r of the result goes
// to out[r * gridDim.x + blockIdx.x].  All threads of the work-group call it.
template <int K>
__device__ __forceinline__ void wg_reduce_rows(double (&v)[K], const int (&op)[K], double* out) {
  __shared__ double red[K][kXMaxThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int r = 0; r < K; ++r) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_xor(v[r], off, 64);
      v[r] = op[r] == 0 ? v[r] + o : op[r] == 1 ? fmin(v[r], o) : fmax(v[r], o);
    }
    if (lane == 0) red[r][wave] = v[r];
  }
  __syncthreads();
  if (tid == 0) {
    const int nw = blockDim.x >> 6;
#pragma unroll
    for (int r = 0; r < K; ++r) {
      double t = red[r][0];
      for (int q = 1; q < nw; ++q)
        t = op[r] == 0 ? t + red[r][q] : op[r] == 1 ? fmin(t, red[r][q]) : fmax(t, red[r][q]);
      out[(long long)r * gridDim.x + blockIdx.x] = t;
    }
  }
}

// One work-group tile of an X pass: gx is the tile's index among the ngx tiles of
// a volume, vol the volume (all threads of the work-group call it).  CM > 0: the
// row length M = CM is known at compile time (compile-time schedule).
template <int E, int MODE, int PREC = 0, int CM = 0>
__device__ __forceinline__ void xrow_tile(const XArgs& a, const Sched& sc,
                                          const float2* __restrict__ twg, int gx, int vol,
                                          int ngx, float2* lds) {
  const int M = CM > 0 ? CM : a.M, P = CM > 0 ? CM / E : a.P;
  const int tid = threadIdx.x;
  float2* tw = lds;  // 2M entries: exp(-2 pi i k / (2M))
  // The twiddle table (and the split-precision operand table) is copied after the
  // row's loads are issued, so that they are not held back behind its loads; the
  // barrier after the copy orders it before use.  Rows of compile-time length
  // above 512 copy it first instead: held through their long copy, the loaded
  // row would cost them occupancy.
  constexpr bool kTwFirst = !(CM > 0 && CM <= 512);
  auto fill_tw = [&]() {
    if constexpr (!kTwFirst) {
      for (int t = tid; t < 2 * M; t += blockDim.x) tw[t] = twg[t];
      if constexpr (PREC > 0) split_atab_fill<PREC>();
    }
  };
  if constexpr (kTwFirst) {
    for (int t = tid; t < 2 * M; t += blockDim.x) tw[t] = twg[t];
    if constexpr (PREC > 0) split_atab_fill<PREC>();
  }
  const int rpw = 64 / P;                       // rows per wavefront
  // the wave index is uniform across the wavefront: in a scalar register, rows of
  // a whole wavefront (P = 64) get scalar row addresses
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int rw = lane / P, i = lane - rw * P;
  const int lrow = wave * rpw + rw;             // row within the work-group
  const int rowi = gx * a.RPW + lrow;
  const bool inrow = rowi < a.nrows;
  const long long rix = inrow ? rowi : 0;
  float2* row = lds + 2 * M + lrow * a.RS;
  // split-precision stages: the wave's rows double as its staging area (>= 64 * 32
  // floats, 16-byte aligned: the host admits only even rows-per-wave * RS there)
  float* stg = reinterpret_cast<float*>(lds + 2 * M + wave * rpw * a.RS);
  const int zz = (int)(rix / a.ny), yy = (int)(rix - (long long)zz * a.ny);
  // rows of the caller's volume (vz, vy, vx) inside the transform grid; grid rows
  // outside it are neither read nor written (the pencil passes read them as zero)
  const bool ok = inrow && zz < a.vz && yy < a.vy;
  const bool rv = ok;
  const long long rr = rv ? (long long)zz * a.vy + yy : 0;
  const int vx = a.vx;
  float2* srow = a.spec + (long long)vol * a.vstride + (long long)zz * a.zstride + yy * kTile;
  const long long ts = a.tstride;

  float2 v[E];
  if constexpr (MODE == XM_R2C) {
    const float* rin = (a.rin_tab ? a.rin_tab[vol] : a.rin) + rr * a.rin_stride;
    load_pairs<E>(v, rin, i, P, vx, rv);
    fill_tw();
    __syncthreads();  // twiddles in LDS
    r2c_store<E, PREC, CM>(v, M, P, sc, i, tw, row, ok, srow, ts, stg);
  } else if constexpr (MODE == XM_PREDICT) {
    const long long ro = rr * vx;
    const bool hist = a.iter > 0;
    const float al = hist ? a.alpha[a.iter] : 0.f;
    float2 hv[E];
    load_pairs<E>(v, a.u + ro, i, P, vx, rv);
    if (hist) {
      load_pairs<E>(hv, a.hstep + ro, i, P, vx, rv);
    } else {
#pragma unroll
      for (int m = 0; m < E; ++m) hv[m] = make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = predict2(v[m], hv[m], al);
    fill_tw();
    __syncthreads();  // twiddles in LDS
    r2c_store<E, PREC, CM>(v, M, P, sc, i, tw, row, ok, srow, ts, stg);
  } else {
    constexpr bool kAcc = MODE == XM_UPDATE_ACC;
    // issue every global load of the row first
    // the metric variants of the ratio and update passes are separate kernels so
    // that the plain ones keep their register budget
    constexpr bool kRatio = MODE == XM_RATIO || MODE == XM_RATIO_LL;
    constexpr bool kUpdate = MODE == XM_UPDATE || MODE == XM_UPDATE_CHG || MODE == XM_UPDATE_PSNR;
    float2 w[(kRatio || kUpdate || kAcc) ? E : 1];
    float2 hv[kAcc ? E : 1], gv[kAcc ? E : 1];
    // srow is a row of the spectrum for every thread (row 0 where the row is not
    // wanted) and the real row pointers are valid likewise: every load of the row
    // issues unconditionally, in one branch per row parity, and the zeros are
    // selected afterwards
    float2 nyq;
    auto load_row = [&](auto even) {
      constexpr bool kEven = decltype(even)::value;
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = srow[col_off(i + P * m, ts)];
      nyq = srow[col_off(M, ts)];
      if constexpr (kRatio) {
        const float* dr = (a.d_tab ? a.d_tab[vol] : a.d) + rr * vx;
        load_pairs_p<kEven>(w, dr, i, P, vx, rv);
      } else if constexpr (kUpdate) {
        const float* ur = (a.u_tab ? a.u_tab[vol] : a.u) + rr * vx;
        load_pairs_p<kEven>(w, ur, i, P, vx, rv);
      } else if constexpr (kAcc) {
        load_pairs_p<kEven>(w, a.u + rr * vx, i, P, vx, rv);
      }
      // long rows select right away (fewer live registers), short ones after the
      // table copy's loads have joined the row's
      if constexpr (kTwFirst && (kRatio || kUpdate || kAcc)) zero_pairs(w, i, P, vx, rv);
    };
    if ((vx & 1) == 0) load_row(BoolC<true>{});
    else load_row(BoolC<false>{});
    fill_tw();  // (short rows) its loads join the row's in flight
    if constexpr (!kTwFirst && (kRatio || kUpdate || kAcc)) zero_pairs(w, i, P, vx, rv);
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = ok ? v[m] : make_float2(0.f, 0.f);
    nyq = (ok && i == 0) ? nyq : make_float2(0.f, 0.f);
    if constexpr (kAcc) {
      const long long ro = rr * vx;
      if (a.iter > 0) {
#pragma unroll
        for (int m = 0; m < E; ++m) {
          hv[m] = load_pair(a.hstep + ro, i + P * m, vx, rv);
          gv[m] = load_pair(a.gchg + ro, i + P * m, vx, rv);
        }
      } else {
#pragma unroll
        for (int m = 0; m < E; ++m) hv[m] = gv[m] = make_float2(0.f, 0.f);
      }
    }
    __syncthreads();  // twiddles in LDS
    c2r_prepare<E>(v, nyq, M, P, i, tw, row);
    fft_row<E, +1, PREC, CM>(v, sc, i, P, tw, row, stg);
    // v[m] holds (x[2n], x[2n+1]) for n = i + P*m (unnormalised; the 1/N is in the OTF)
    if constexpr (MODE == XM_C2R) {
      float* rout = (a.rout_tab ? a.rout_tab[vol] : a.rout) + rr * a.rout_stride;
#pragma unroll
      for (int m = 0; m < E; ++m) store_pair(rout, i + P * m, vx, rv, v[m]);
    } else if constexpr (kRatio) {
      // Poisson log-likelihood of the caller's voxels (XM_RATIO_LL): FP32 terms and
      // per-thread sums, FP64 across threads
      float ll = 0.f;
      constexpr bool want_ll = MODE == XM_RATIO_LL;
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const float2 q = v[m];
        if (want_ll && rv) {
          const int x0 = 2 * (i + P * m);
          if (x0 < vx && q.x > 1e-12f) ll += (w[m].x > 0.f ? w[m].x * logf(q.x) : 0.f) - q.x;
          if (x0 + 1 < vx && q.y > 1e-12f) ll += (w[m].y > 0.f ? w[m].y * logf(q.y) : 0.f) - q.y;
        }
        // d / q as d times the hardware reciprocal (at most 1.5 ulp from the
        // correctly rounded quotient; the pass is bound by vector instruction
        // issue, and the IEEE division sequence costs about ten instructions)
        v[m] = make_float2(q.x > 1e-12f ? w[m].x * __builtin_amdgcn_rcpf(q.x) : 0.f,
                           q.y > 1e-12f ? w[m].y * __builtin_amdgcn_rcpf(q.y) : 0.f);
      }
      wave_sync();  // row buffer reuse
      r2c_store<E, PREC, CM>(v, M, P, sc, CM > 0 ? opaque_int(i) : i, tw, row, ok, srow, ts, stg);
      if constexpr (want_ll) {
        double r[1] = {(double)ll};
        constexpr int ops[1] = {0};
        wg_reduce_rows<1>(r, ops, a.met_partials);
      }
    } else if constexpr (kAcc) {
      // x_{k+1} = y_k * max(c, 0) from the prediction y_k; keep h and g for the next
      // extrapolation and accumulate the flux and the two inner products of alpha
      const long long ro = rr * vx;
      const float al = a.iter > 0 ? a.alpha[a.iter] : 0.f;
      double acc = 0.0, sgg = 0.0, spp = 0.0;
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const float2 c = v[m];
        const float2 y = predict2(w[m], hv[m], al);
        const float2 xn = make_float2(y.x * (c.x < 0.f ? 0.f : c.x), y.y * (c.y < 0.f ? 0.f : c.y));
        const float2 g = make_float2(xn.x - y.x, xn.y - y.y);
        const float2 hn = make_float2(xn.x - w[m].x, xn.y - w[m].y);
        store_pair(a.u + ro, i + P * m, vx, rv, xn);
        store_pair(a.hstep + ro, i + P * m, vx, rv, hn);
        store_pair(a.gchg + ro, i + P * m, vx, rv, g);
        acc += (double)xn.x + (double)xn.y;
        sgg += (double)g.x * (double)gv[m].x + (double)g.y * (double)gv[m].y;
        spp += (double)gv[m].x * (double)gv[m].x + (double)gv[m].y * (double)gv[m].y;
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        acc += __shfl_xor(acc, off, 64);
        sgg += __shfl_xor(sgg, off, 64);
        spp += __shfl_xor(spp, off, 64);
      }
      __shared__ double wacc[3][kXMaxThreads / 64];
      if (lane == 0) {
        wacc[0][wave] = acc;
        wacc[1][wave] = sgg;
        wacc[2][wave] = spp;
      }
      __syncthreads();
      if (tid == 0) {
        double t0 = 0.0, t1 = 0.0, t2 = 0.0;
        const int nw = blockDim.x >> 6;
        for (int q = 0; q < nw; ++q) {
          t0 += wacc[0][q];
          t1 += wacc[1][q];
          t2 += wacc[2][q];
        }
        a.partials[(long long)a.iter * ngx + gx] = t0;
        a.acc_partials[gx] = t1;
        a.acc_partials[ngx + gx] = t2;
      }
    } else {  // XM_UPDATE
      float* ur = (a.u_tab ? a.u_tab[vol] : a.u) + rr * vx;
      double acc = 0.0;
      // stopping metrics of the new estimate: FP32 per-thread sums, FP64 across threads
      constexpr bool want_change = MODE == XM_UPDATE_CHG, want_psnr = MODE == XM_UPDATE_PSNR;
      float met[kMetRows] = {0.f, 0.f, 0.f, 0.f, 0.f, 3.0e38f, -3.0e38f};
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const float2 c = v[m];
        // clamp c < 0 to 0; a NaN passes through (as max(c, 0) does in the oracle) so
        // that non-finite inputs reach the flux check instead of being silently zeroed
        const float2 un = make_float2(w[m].x * (c.x < 0.f ? 0.f : c.x),
                                      w[m].y * (c.y < 0.f ? 0.f : c.y));
        store_pair(ur, i + P * m, vx, rv, un);
        acc += (double)un.x + (double)un.y;
        if constexpr (want_change) {
          const float dx = un.x - w[m].x, dy = un.y - w[m].y;
          met[0] += dx * dx + dy * dy;
          met[1] += w[m].x * w[m].x + w[m].y * w[m].y;
        } else if constexpr (want_psnr) {
          if (rv) {
            const float2 g = load_pair(a.ref + rr * vx, i + P * m, vx, true);
            const int x0 = 2 * (i + P * m);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              if (x0 + h < vx) {
                const float uu = h ? un.y : un.x, gg = h ? g.y : g.x;
                met[0] += uu;
                met[1] += uu * uu;
                met[2] += uu * gg;
                met[3] += gg;
                met[4] += gg * gg;
                met[5] = fminf(met[5], gg);
                met[6] = fmaxf(met[6], gg);
              }
            }
          }
        }
        v[m] = un;
      }
      if (a.do_fwd) {
        wave_sync();
        r2c_store<E, PREC, CM>(v, M, P, sc, CM > 0 ? opaque_int(i) : i, tw, row, ok, srow, ts,
                               stg);
      }
      // work-group partial of the flux: wavefront butterfly, then the waves in order
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
      __shared__ double wsum[kXMaxThreads / 64];
      if (lane == 0) wsum[wave] = acc;
      __syncthreads();
      if (tid == 0) {
        double t = 0.0;
        const int nw = blockDim.x >> 6;
        for (int q = 0; q < nw; ++q) t += wsum[q];
        const int it = a.iter_ptr ? *a.iter_ptr : a.iter;
        a.partials[((long long)it * a.nvol + vol) * ngx + gx] = t;
      }
      if constexpr (want_change) {
        double r[2] = {(double)met[0], (double)met[1]};
        constexpr int ops[2] = {0, 0};
        wg_reduce_rows<2>(r, ops, a.met_partials);
      } else if constexpr (want_psnr) {
        double r[kMetRows];
#pragma unroll
        for (int q = 0; q < kMetRows; ++q) r[q] = (double)met[q];
        r[5] = met[5] >= 3.0e38f ? 1.0e300 : r[5];
        r[6] = met[6] <= -3.0e38f ? -1.0e300 : r[6];
        constexpr int ops[kMetRows] = {0, 0, 0, 0, 0, 1, 2};
        wg_reduce_rows<kMetRows>(r, ops, a.met_partials);
      }
    }
  }
}

// The metric variants (XM_RATIO_LL, XM_UPDATE_CHG / PSNR) write their partials
// with wg_reduce_rows, indexed by the launch's own block and grid.
template <int E, int MODE, int PREC = 0, int CM = 0>
__global__ void __launch_bounds__(kXMaxThreads) k_xrow(XArgs a, Sched sc, const float2* __restrict__ twg) {
  if (a.stop && *a.stop) return;  // stopped: the whole work-group leaves together
  extern __shared__ __attribute__((aligned(16))) float2 lds[];
  xrow_tile<E, MODE, PREC, CM>(a, sc, twg, blockIdx.x, blockIdx.y, gridDim.x, lds);
}

// Metric and stop decision of iteration `it` (one work-group; fixed summation order).
__global__ void __launch_bounds__(256) k_metric(const double* __restrict__ mp, int groups,
                                                int metric, int it, double threshold,
                                                int min_iter, long long nvox,
                                                double* __restrict__ hist, int* __restrict__ stop) {
  if (stop[0]) return;
  const int tid = threadIdx.x;
  const int rows = (metric == MET_LOGLIK || metric == MET_SSIM || metric == MET_FSC) ? 1
                   : metric == MET_CHANGE                                            ? 2
                                                                                     : kMetRows;
  __shared__ double ws[kMetRows][4];
  for (int r = 0; r < rows; ++r) {
    const int op = (metric == MET_PSNR && r == 5) ? 1 : (metric == MET_PSNR && r == 6) ? 2 : 0;
    double t = op == 1 ? 1.0e300 : op == 2 ? -1.0e300 : 0.0;
    for (int g = tid; g < groups; g += blockDim.x) {
      const double x = mp[(long long)r * groups + g];
      t = op == 0 ? t + x : op == 1 ? fmin(t, x) : fmax(t, x);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_xor(t, off, 64);
      t = op == 0 ? t + o : op == 1 ? fmin(t, o) : fmax(t, o);
    }
    if ((tid & 63) == 0) ws[r][tid >> 6] = t;
  }
  __syncthreads();
  if (tid != 0) return;
  double s[kMetRows];
  for (int r = 0; r < rows; ++r) {
    const int op = (metric == MET_PSNR && r == 5) ? 1 : (metric == MET_PSNR && r == 6) ? 2 : 0;
    double t = ws[r][0];
    for (int q = 1; q < 4; ++q)
      t = op == 0 ? t + ws[r][q] : op == 1 ? fmin(t, ws[r][q]) : fmax(t, ws[r][q]);
    s[r] = t;
  }
  double m;
  bool halt = false;
  int done = it + 1;  // iterations carried out if the iteration stops here
  if (metric == MET_LOGLIK) {
    // likelihood of the estimate entering iteration it; stopping skips that iteration
    m = s[0];
    done = it;
    halt = it >= 1 && it >= min_iter && (m - hist[it - 1]) / fabs(m) < threshold;
  } else if (metric == MET_CHANGE) {
    m = sqrt(s[0] / s[1]);
    halt = done >= min_iter && m < threshold;
  } else if (metric == MET_SSIM) {
    m = s[0] / (double)nvox;  // nvox: number of windows
    halt = it >= 1 && done >= min_iter && m - hist[it - 1] < threshold;
  } else if (metric == MET_FSC) {
    m = s[0];  // resolution of the single-image FSC
    halt = it >= 1 && done >= min_iter && m - hist[it - 1] < threshold;
  } else {
    const double n = (double)nvox;
    const double cuu = s[1] - s[0] * s[0] / n, cug = s[2] - s[0] * s[3] / n;
    const double cgg = s[4] - s[3] * s[3] / n;
    double sse = cgg - (cuu > 0.0 ? cug * cug / cuu : 0.0);
    if (sse < 0.0) sse = 0.0;
    m = 20.0 * log10(s[6] - s[5]) - 10.0 * log10(sse / n);
    halt = it >= 1 && done >= min_iter && m - hist[it - 1] < threshold;
  }
  hist[it] = m;
  stop[2] = it + 1;
  if (halt) {
    stop[1] = done;
    stop[0] = 1;
  }
}

// flux[r] = sum of the work-group partials of row r (one iteration of one
// volume), in a fixed order.
__global__ void __launch_bounds__(256) k_flux_reduce(const double* __restrict__ partials, int groups,
                                                     double* __restrict__ flux) {
  const int it = blockIdx.x, tid = threadIdx.x;
  const double* p = partials + (long long)it * groups;
  double t = 0.0;
  for (int g = tid; g < groups; g += blockDim.x) t += p[g];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
  __shared__ double ws[4];
  if ((tid & 63) == 0) ws[tid >> 6] = t;
  __syncthreads();
  if (tid == 0) flux[it] = ((ws[0] + ws[1]) + ws[2]) + ws[3];
}

// alpha of the next extrapolated iteration from the two inner-product rows.
__global__ void __launch_bounds__(256) k_accel_alpha(const double* __restrict__ accp, int groups,
                                                     int it, float* __restrict__ alpha32,
                                                     double* __restrict__ alpha64) {
  const int tid = threadIdx.x;
  double num = 0.0, den = 0.0;
  for (int g = tid; g < groups; g += blockDim.x) {
    num += accp[g];
    den += accp[groups + g];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    num += __shfl_xor(num, off, 64);
    den += __shfl_xor(den, off, 64);
  }
  __shared__ double ws[2][4];
  if ((tid & 63) == 0) {
    ws[0][tid >> 6] = num;
    ws[1][tid >> 6] = den;
  }
  __syncthreads();
  if (tid == 0) {
    const double n = ((ws[0][0] + ws[0][1]) + ws[0][2]) + ws[0][3];
    const double d = ((ws[1][0] + ws[1][1]) + ws[1][2]) + ws[1][3];
    double al = 0.0;
    if (it > 0 && d > 0.0) {
      al = n / d;  // a NaN stays NaN and surfaces in the flux
      if (al < 0.0) al = 0.0;
      if (al > 1.0) al = 1.0;
    }
    alpha32[it + 1] = (float)al;
    alpha64[it + 1] = al;
    if (it == 0) {
      alpha32[0] = 0.f;
      alpha64[0] = 0.0;
    }
  }
}

// ---------------------------------------------------------------------------
// Fourier shell correlation
// ---------------------------------------------------------------------------
// a[z][y][x] = u[2z][2y][2x], b[z][y][x] = u[2z+1][2y+1][2x+1] (half-size volumes).
__global__ void k_split_diag(const float* __restrict__ u, int nz, int ny, int nx,
                             float* __restrict__ a, float* __restrict__ b, const int* stop) {
  if (stop && *stop) return;
  const int hz = nz / 2, hy = ny / 2, hx = nx / 2;
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
  if (x >= hx) return;
  const long long o = ((long long)z * hy + y) * hx + x;
  a[o] = u[((long long)(2 * z) * ny + 2 * y) * nx + 2 * x];
  b[o] = u[((long long)(2 * z + 1) * ny + 2 * y + 1) * nx + 2 * x + 1];
}

// |signed DFT index| of bin j of length n: j below ceil(n/2), n - j above.
__device__ __forceinline__ long long abs_index(int j, int n) {
  return j < (n + 1) / 2 ? j : n - j;
}

// One work-group per tile column (z, 16 kx columns, all ny rows) of two half
// spectra F and G: per shell s = floor(2 nbins rho) (nbins for rho >= 0.5),
// rho^2 = sum_i (k_i / n_i)^2, the sums of Re(F conj G), |F|^2, |G|^2, each column
// kx in 1 .. M-1 counted twice (it stands for its conjugate partner too).  The
// shell is exact: with L = lcm(n_i) and m_i = L / n_i, Q = sum_i (k_i m_i)^2 and
// s is the largest integer with s^2 L^2 <= 4 nbins^2 Q (all below 2^63 for
// L < 2^21).  Work-group partials go to
// part[((z * XT + tile) * (nbins + 1) + s) * 3 + {0, 1, 2}].
__global__ void __launch_bounds__(256) k_shell(const float2* __restrict__ F,
                                               const float2* __restrict__ G, int nz, int ny,
                                               int nx, int xt, int nbins, long long lcm,
                                               double* __restrict__ part, const int* stop) {
  if (stop && *stop) return;  // stopped: the whole work-group leaves together
  extern __shared__ double hist[];  // (nbins + 1) * 3
  const int tid = threadIdx.x;
  const int nb1 = nbins + 1;
  for (int t = tid; t < nb1 * 3; t += blockDim.x) hist[t] = 0.0;
  __syncthreads();
  const int tile = blockIdx.x, z = blockIdx.y;
  const int M = nx / 2;
  const long long base = ((long long)z * xt + tile) * ny * kTile;
  const unsigned long long D = (unsigned long long)lcm * (unsigned long long)lcm;
  const unsigned long long four = 4ull * (unsigned long long)nbins * (unsigned long long)nbins;
  const unsigned long long kz = (unsigned long long)(abs_index(z, nz) * (lcm / nz));
  for (int e = tid; e < ny * kTile; e += blockDim.x) {
    const int y = e >> 4, c = e & (kTile - 1);
    const int kx = tile * kTile + c;
    if (kx > M) continue;
    const unsigned long long ky = (unsigned long long)(abs_index(y, ny) * (lcm / ny));
    const unsigned long long kxx = (unsigned long long)kx * (unsigned long long)(lcm / nx);
    const unsigned long long Q = kz * kz + ky * ky + kxx * kxx;
    const unsigned long long A = four * Q;
    long long sh = (long long)(2.0 * nbins * sqrt((double)Q) / (double)lcm);
    while (sh > 0 && (unsigned long long)(sh * sh) * D > A) --sh;
    while ((unsigned long long)((sh + 1) * (sh + 1)) * D <= A) ++sh;
    if (sh > nbins) sh = nbins;
    const double w = (kx == 0 || kx == M) ? 1.0 : 2.0;
    const float2 f = F[base + e], g = G[base + e];
    const double fr = f.x, fi = f.y, gr = g.x, gi = g.y;
    atomicAdd(&hist[sh * 3 + 0], w * (fr * gr + fi * gi));
    atomicAdd(&hist[sh * 3 + 1], w * (fr * fr + fi * fi));
    atomicAdd(&hist[sh * 3 + 2], w * (gr * gr + gi * gi));
  }
  __syncthreads();
  double* out = part + ((long long)z * xt + tile) * nb1 * 3;
  for (int t = tid; t < nb1 * 3; t += blockDim.x) out[t] = hist[t];
}

// Sums the work-group partials per shell in a fixed order and writes
// out = [curve (nbins + 1), sums Re(F conj G), |F|^2, |G|^2 (nbins + 1 each),
// resolution]: the first shell s >= 1 whose FSC is below `threshold`, crossing
// interpolated between the centres of shells s-1 and s; 0.5 if none.
__global__ void __launch_bounds__(256) k_fsc_final(const double* __restrict__ part, int groups,
                                                   int nbins, double threshold,
                                                   double* __restrict__ out, const int* stop) {
  if (stop && *stop) return;
  const int nb1 = nbins + 1;
  for (int sh = threadIdx.x; sh < nb1; sh += blockDim.x) {
    double n = 0.0, d1 = 0.0, d2 = 0.0;
    for (int g = 0; g < groups; ++g) {
      const double* q = part + ((long long)g * nb1 + sh) * 3;
      n += q[0];
      d1 += q[1];
      d2 += q[2];
    }
    const double den = sqrt(d1 * d2);
    out[sh] = den > 0.0 ? n / den : 0.0;
    out[nb1 + sh] = n;
    out[2 * nb1 + sh] = d1;
    out[3 * nb1 + sh] = d2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double res = 0.5;
    for (int sh = 1; sh < nbins; ++sh) {
      if (out[sh] < threshold) {
        const double c0 = out[sh - 1], c1 = out[sh];
        const double t = c0 != c1 ? (c0 - threshold) / (c0 - c1) : 0.0;
        const double f0 = (sh - 0.5) * 0.5 / nbins, f1 = (sh + 0.5) * 0.5 / nbins;
        res = f0 + t * (f1 - f0);
        break;
      }
    }
    out[4 * nb1] = res;
  }
}

// ---------------------------------------------------------------------------
// Structural similarity (7x7x7 windows lying inside the volume)
// ---------------------------------------------------------------------------
constexpr int kSsimWin = 7;

// Per-block min and max of g; part[2 * block] = min, part[2 * block + 1] = max.
__global__ void __launch_bounds__(256) k_range(const float* __restrict__ g, long long n,
                                               double* __restrict__ part) {
  double mn = 1.0e300, mx = -1.0e300;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (long long)gridDim.x * blockDim.x) {
    const double v = g[t];
    mn = fmin(mn, v);
    mx = fmax(mx, v);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    mn = fmin(mn, __shfl_xor(mn, off, 64));
    mx = fmax(mx, __shfl_xor(mx, off, 64));
  }
  __shared__ double ws[2][4];
  const int tid = threadIdx.x;
  if ((tid & 63) == 0) {
    ws[0][tid >> 6] = mn;
    ws[1][tid >> 6] = mx;
  }
  __syncthreads();
  if (tid == 0) {
    for (int q = 1; q < (int)(blockDim.x >> 6); ++q) {
      ws[0][0] = fmin(ws[0][0], ws[0][q]);
      ws[1][0] = fmax(ws[1][0], ws[1][q]);
    }
    part[2 * blockIdx.x] = ws[0][0];
    part[2 * blockIdx.x + 1] = ws[1][0];
  }
}

// range[0] = max - min over the block partials (one thread, fixed order).
__global__ void k_range_final(const double* __restrict__ part, int blocks,
                              double* __restrict__ range) {
  if (threadIdx.x != 0) return;
  double mn = part[0], mx = part[1];
  for (int b = 1; b < blocks; ++b) {
    mn = fmin(mn, part[2 * b]);
    mx = fmax(mx, part[2 * b + 1]);
  }
  range[0] = mx - mn;
}

// X window sums of u, g, u^2, g^2, u g (FP64) for every row and every x0 whose
// window [x0, x0 + 7) lies inside the row: out[c][z][y][x0], c = 0..4.
__global__ void __launch_bounds__(256) k_ssim_x(const float* __restrict__ u,
                                                const float* __restrict__ g, int nz, int ny,
                                                int nx, double* __restrict__ out,
                                                const int* stop) {
  if (stop && *stop) return;
  const int nxo = nx - kSsimWin + 1;
  const int x0 = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
  if (x0 >= nxo) return;
  const long long row = ((long long)z * ny + y) * nx + x0;
  double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < kSsimWin; ++k) {
    const double a = u[row + k], b = g[row + k];
    s[0] += a;
    s[1] += b;
    s[2] += a * a;
    s[3] += b * b;
    s[4] += a * b;
  }
  const long long plane = (long long)nz * ny * nxo;
  const long long o = ((long long)z * ny + y) * nxo + x0;
#pragma unroll
  for (int c = 0; c < 5; ++c) out[c * plane + o] = s[c];
}

// Y window sums of the five X sums: in[c][z][y][x0] (ny rows) -> out[c][z][y0][x0].
// Each thread slides a window over kSsimChunk consecutive outputs (running sums),
// so each input is read about once instead of seven times.
constexpr int kSsimChunk = 32;
__global__ void __launch_bounds__(256) k_ssim_y(const double* __restrict__ in, int nz, int ny,
                                                int nxo, double* __restrict__ out,
                                                const int* stop) {
  if (stop && *stop) return;
  const int nyo = ny - kSsimWin + 1;
  const int x0 = blockIdx.x * blockDim.x + threadIdx.x, z = blockIdx.z;
  const int ya = blockIdx.y * kSsimChunk, yb = min(ya + kSsimChunk, nyo);
  if (x0 >= nxo) return;
  const long long pin = (long long)nz * ny * nxo, pout = (long long)nz * nyo * nxo;
  for (int c = 0; c < 5; ++c) {
    const double* src = in + c * pin + (long long)z * ny * nxo + x0;
    double* dst = out + c * pout + (long long)z * nyo * nxo + x0;
    double t = 0.0;
    for (int k = 0; k < kSsimWin; ++k) t += src[(long long)(ya + k) * nxo];
    dst[(long long)ya * nxo] = t;
    for (int y0 = ya + 1; y0 < yb; ++y0) {
      t += src[(long long)(y0 + kSsimWin - 1) * nxo] - src[(long long)(y0 - 1) * nxo];
      dst[(long long)y0 * nxo] = t;
    }
  }
}

// Z window sums (sliding over kSsimChunk outputs per thread), then the SSIM of
// each window (sample statistics, W = 343, C1 = (0.01 L)^2, C2 = (0.03 L)^2 with
// L = *range) summed per work-group into
// part[(blockIdx.z * nyo + y0) * gridDim.x + blockIdx.x].
__global__ void __launch_bounds__(256) k_ssim_z(const double* __restrict__ in, int nz, int nyo,
                                                int nxo, const double* __restrict__ range,
                                                double* __restrict__ part, const int* stop) {
  if (stop && *stop) return;
  const int nzo = nz - kSsimWin + 1;
  const int x0 = blockIdx.x * blockDim.x + threadIdx.x, y0 = blockIdx.y;
  const int za = blockIdx.z * kSsimChunk, zb = min(za + kSsimChunk, nzo);
  const long long pin = (long long)nz * nyo * nxo, zs = (long long)nyo * nxo;
  double val = 0.0;
  if (x0 < nxo) {
    const double* src = in + (long long)y0 * nxo + x0;
    double s[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      double t = 0.0;
      for (int k = 0; k < kSsimWin; ++k) t += src[c * pin + (long long)(za + k) * zs];
      s[c] = t;
    }
    const double W = (double)(kSsimWin * kSsimWin * kSsimWin), cn = W / (W - 1.0);
    const double L = range[0], c1 = (0.01 * L) * (0.01 * L), c2 = (0.03 * L) * (0.03 * L);
    for (int z0 = za; z0 < zb; ++z0) {
      if (z0 > za) {
#pragma unroll
        for (int c = 0; c < 5; ++c)
          s[c] += src[c * pin + (long long)(z0 + kSsimWin - 1) * zs] -
                  src[c * pin + (long long)(z0 - 1) * zs];
      }
      const double mu = s[0] / W, mg = s[1] / W;
      const double vu = cn * (s[2] / W - mu * mu), vg = cn * (s[3] / W - mg * mg);
      const double cug = cn * (s[4] / W - mu * mg);
      val += ((2.0 * mu * mg + c1) * (2.0 * cug + c2)) /
             ((mu * mu + mg * mg + c1) * (vu + vg + c2));
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) val += __shfl_xor(val, off, 64);
  __shared__ double ws[4];
  const int tid = threadIdx.x;
  if ((tid & 63) == 0) ws[tid >> 6] = val;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += ws[q];
    part[((long long)blockIdx.z * nyo + y0) * gridDim.x + blockIdx.x] = t;
  }
}

// ---------------------------------------------------------------------------
// small kernels: twiddles, PSF statistics and preparation, copy probe
// ---------------------------------------------------------------------------
// tab[m] = exp(-2 pi i m / n), evaluated in FP64 from the exact integer m / n
// and rounded once to FP32.
__global__ void k_twiddles(float2* tab, int n) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n) return;
  double s, c;
  sincospi(2.0 * (double)m / (double)n, &s, &c);
  tab[m] = make_float2((float)c, (float)(-s));
}

// FP64 sum, min and non-finite count of h; partial per block, last block finishes.
__global__ void __launch_bounds__(256) k_psf_stats(const float* __restrict__ h, long long n,
                                                   double* partials, unsigned* counter,
                                                   double* out) {
  __shared__ double ssum[4], smin[4], snf[4];
  __shared__ bool last_block;
  const int tid = threadIdx.x;
  double s = 0.0, mn = 1.0e300, nf = 0.0;
  for (long long t = (long long)blockIdx.x * blockDim.x + tid; t < n;
       t += (long long)gridDim.x * blockDim.x) {
    const float v = h[t];
    if (!isfinite(v)) {
      nf += 1.0;
    } else {
      s += (double)v;
      mn = fmin(mn, (double)v);
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    s += __shfl_xor(s, off, 64);
    mn = fmin(mn, __shfl_xor(mn, off, 64));
    nf += __shfl_xor(nf, off, 64);
  }
  if ((tid & 63) == 0) {
    ssum[tid >> 6] = s;
    smin[tid >> 6] = mn;
    snf[tid >> 6] = nf;
  }
  __syncthreads();
  if (tid == 0) {
    double a = 0.0, b = 1.0e300, c = 0.0;
    for (int w = 0; w < 4; ++w) {
      a += ssum[w];
      b = fmin(b, smin[w]);
      c += snf[w];
    }
    partials[3 * blockIdx.x + 0] = a;
    partials[3 * blockIdx.x + 1] = b;
    partials[3 * blockIdx.x + 2] = c;
    __threadfence();
    last_block = (atomicAdd(counter, 1u) == gridDim.x - 1);
  }
  __syncthreads();
  if (last_block && tid == 0) {
    __threadfence();
    const unsigned long long* pp = reinterpret_cast<const unsigned long long*>(partials);
    double a = 0.0, b = 1.0e300, c = 0.0;
    for (unsigned g = 0; g < gridDim.x; ++g) {
      a += __longlong_as_double((long long)__hip_atomic_load(pp + 3 * g + 0, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT));
      b = fmin(b, __longlong_as_double((long long)__hip_atomic_load(
                      pp + 3 * g + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)));
      c += __longlong_as_double((long long)__hip_atomic_load(pp + 3 * g + 2, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT));
    }
    out[0] = a;
    out[1] = b;
    out[2] = c;
    __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// PSF index along one axis that lands on grid index o once the PSF (length p,
// centre p/2) is centred on voxel 0 of a periodic grid of length n >= p:
// offsets 0 .. p-1-c sit at o = offset, offsets -c .. -1 at o = n + offset.
// -1: no PSF entry lands on o.
__device__ __forceinline__ int psf_src(int o, int n, int p) {
  const int c = p / 2;
  if (o < p - c) return o + c;
  if (o >= n - c) return o - n + c;
  return -1;
}

// out[z][y][x] (rows `out_row_stride` floats apart) = the PSF entry that lands on
// grid voxel (z, y, x) times `scale` (product in FP64), else 0: the PSF with its
// centre floor(p/2) moved to voxel 0.
__global__ void k_psf_prep(const float* __restrict__ h, float* __restrict__ out, int nz, int ny,
                           int nx, int pz, int py, int px, long long out_row_stride,
                           double scale) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  const int z = blockIdx.z;
  if (x >= nx) return;
  const int sx = psf_src(x, nx, px), sy = psf_src(y, ny, py), sz = psf_src(z, nz, pz);
  float v = 0.f;
  if (sx >= 0 && sy >= 0 && sz >= 0) v = h[((long long)sz * py + sy) * px + sx];
  out[((long long)z * ny + y) * out_row_stride + x] = (float)((double)v * scale);
}

// Streaming copy of n 16-byte words: each thread loads kCopyUnroll words a
// work-group width apart, then stores them (all loads in flight at once).
constexpr int kCopyUnroll = 4;
__global__ void __launch_bounds__(256) k_copy(const float4* __restrict__ src,
                                              float4* __restrict__ dst, long long n) {
  const long long base = (long long)blockIdx.x * blockDim.x * kCopyUnroll + threadIdx.x;
  float4 v[kCopyUnroll];
#pragma unroll
  for (int u = 0; u < kCopyUnroll; ++u) {
    const long long t = base + (long long)u * blockDim.x;
    if (t < n) v[u] = src[t];
  }
#pragma unroll
  for (int u = 0; u < kCopyUnroll; ++u) {
    const long long t = base + (long long)u * blockDim.x;
    if (t < n) dst[t] = v[u];
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// With `launch` false only the LDS attribute is set (work-groups above 64 KB).
// Launch on `s`; with timing events the dispatch packet itself stamps them
// (hipExtLaunchKernelGGL), so they bracket exactly the kernel's execution.
#define RL_LAUNCH(K, G, B, LDS, S, EV0, EV1, ...)                            \
  do {                                                                       \
    if (EV0)                                                                 \
      hipExtLaunchKernelGGL(K, G, B, LDS, S, EV0, EV1, 0, __VA_ARGS__);      \
    else                                                                     \
      hipLaunchKernelGGL(K, G, B, LDS, S, __VA_ARGS__);                      \
  } while (0)

template <int MODE, int MAXT, int EV, int PREC = 0>
static hipError_t pencil_one(dim3 g, dim3 b, size_t lds, hipStream_t s, float2* data,
                             const float2* otf, const float2* tw, const PencilArgs& a,
                             const Sched& sc, bool launch = true, hipEvent_t ev0 = nullptr,
                             hipEvent_t ev1 = nullptr) {
  if (lds > 65536 - (PREC > 0 ? kSplitTabBytes : 0)) {
    static bool attr_done = false;  // once per instantiation
    if (!attr_done) {
      hipError_t e =
          hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pencil<EV, MODE, MAXT, PREC>),
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              163840 - (PREC > 0 ? kSplitTabBytes : 0));
      if (e != hipSuccess) return e;
      attr_done = true;
    }
  }
  if (!launch) return hipSuccess;
  RL_LAUNCH((k_pencil<EV, MODE, MAXT, PREC>), g, b, lds, s, ev0, ev1, data, otf, tw, a, sc);
  return hipGetLastError();
}

template <int MODE, int E, int L, int PREC>
static hipError_t pencil_ct_one(dim3 g, dim3 b, size_t lds, hipStream_t s, float2* data,
                                const float2* otf, const float2* tw, const PencilArgs& a,
                                bool launch, hipEvent_t ev0, hipEvent_t ev1) {
  if (lds > 65536 - (PREC > 0 ? kSplitTabBytes : 0)) {
    static bool attr_done = false;  // once per instantiation
    if (!attr_done) {
      hipError_t e =
          hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pencil_ct<E, MODE, PREC, L>),
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              163840 - (PREC > 0 ? kSplitTabBytes : 0));
      if (e != hipSuccess) return e;
      attr_done = true;
    }
  }
  if (!launch) return hipSuccess;
  RL_LAUNCH((k_pencil_ct<E, MODE, PREC, L>), g, b, lds, s, ev0, ev1, data, otf, tw, a);
  return hipGetLastError();
}

template <int MODE, int L>
static hipError_t pencil_ct_prec(int prec, dim3 g, dim3 b, size_t lds, hipStream_t s,
                                 float2* data, const float2* otf, const float2* tw,
                                 const PencilArgs& a, bool launch, hipEvent_t ev0, hipEvent_t ev1) {
  switch (prec) {
    case 0: return pencil_ct_one<MODE, 16, L, 0>(g, b, lds, s, data, otf, tw, a, launch, ev0, ev1);
    case 1: return pencil_ct_one<MODE, 16, L, 1>(g, b, lds, s, data, otf, tw, a, launch, ev0, ev1);
    case 2: return pencil_ct_one<MODE, 16, L, 2>(g, b, lds, s, data, otf, tw, a, launch, ev0, ev1);
    default: return hipErrorInvalidValue;
  }
}

template <int MODE>
static hipError_t pencil_e(int E, int prec, dim3 g, dim3 b, size_t lds, hipStream_t s,
                           float2* data, const float2* otf, const float2* tw, const PencilArgs& a,
                           const Sched& sc, bool launch = true, hipEvent_t ev0 = nullptr,
                           hipEvent_t ev1 = nullptr) {
  if (b.x > 1024) return hipErrorInvalidValue;
  if (b.x % 64 != 0) prec = 0;  // MFMA stages need whole wavefronts
  // split-precision work-groups have at most 512 threads (their register budget)
  if (E == 16 && prec > 0 && b.x > 512) return hipErrorInvalidValue;
  if (pencil_compiled_len(E, a.L, (int)b.x) > 0 && a.P * E == a.L) {
    // lengths without 16-point stages: FP32 arithmetic in every precision
#define RL_PCT(EV, LV)                                                                  \
    if (E == EV && a.L == LV)                                                           \
      return pencil_ct_one<MODE, EV, LV, 0>(g, b, lds, s, data, otf, tw, a, launch, ev0, ev1);
    RL_PCT(30, 2160) RL_PCT(6, 24) RL_PCT(6, 48) RL_PCT(6, 96) RL_PCT(12, 48) RL_PCT(12, 96)
    RL_PCT(12, 192) RL_PCT(8, 32) RL_PCT(8, 64) RL_PCT(8, 128) RL_PCT(8, 256) RL_PCT(8, 512)
#undef RL_PCT
    switch (a.L) {
      case 128: return pencil_ct_prec<MODE, 128>(prec, g, b, lds, s, data, otf, tw, a, launch, ev0, ev1);
      case 256: return pencil_ct_prec<MODE, 256>(prec, g, b, lds, s, data, otf, tw, a, launch, ev0, ev1);
      case 512: return pencil_ct_prec<MODE, 512>(prec, g, b, lds, s, data, otf, tw, a, launch, ev0, ev1);
      default: return hipErrorInvalidValue;
    }
  }
  if (E == 16 && prec == 1)
    return pencil_one<MODE, 512, 16, 1>(g, b, lds, s, data, otf, tw, a, sc, launch, ev0, ev1);
  if (E == 16 && prec == 2)
    return pencil_one<MODE, 512, 16, 2>(g, b, lds, s, data, otf, tw, a, sc, launch, ev0, ev1);
  if (b.x > 512) {
    switch (E) {
      case 8: return pencil_one<MODE, 1024, 8>(g, b, lds, s, data, otf, tw, a, sc, launch, ev0, ev1);
      case 16: return pencil_one<MODE, 1024, 16>(g, b, lds, s, data, otf, tw, a, sc, launch, ev0, ev1);
      default: return hipErrorInvalidValue;
    }
  }
  switch (E) {
#define RL_CASE(EV) \
  case EV: return pencil_one<MODE, 512, EV>(g, b, lds, s, data, otf, tw, a, sc, launch, ev0, ev1);
    RL_CASE(1) RL_CASE(2) RL_CASE(3) RL_CASE(4) RL_CASE(6) RL_CASE(8) RL_CASE(12) RL_CASE(16)
    RL_CASE(24) RL_CASE(5) RL_CASE(10) RL_CASE(20) RL_CASE(7) RL_CASE(14) RL_CASE(9) RL_CASE(18)
    RL_CASE(15) RL_CASE(30)
#undef RL_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t prepare_pencil(int mode, int E, int L, int prec, dim3 block, size_t lds) {
  PencilArgs a{};
  a.L = L;
  a.P = E > 0 ? L / E : 0;
  const Sched sc{};
  const dim3 g(1);
  switch (mode) {
    case PM_FWD: return pencil_e<PM_FWD>(E, prec, g, block, lds, 0, nullptr, nullptr, nullptr, a, sc, false);
    case PM_INV: return pencil_e<PM_INV>(E, prec, g, block, lds, 0, nullptr, nullptr, nullptr, a, sc, false);
    case PM_FKI: return pencil_e<PM_FKI>(E, prec, g, block, lds, 0, nullptr, nullptr, nullptr, a, sc, false);
    case PM_FCKI: return pencil_e<PM_FCKI>(E, prec, g, block, lds, 0, nullptr, nullptr, nullptr, a, sc, false);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pencil(int mode, int E, int prec, dim3 grid, dim3 block, size_t lds,
                         hipStream_t s, float2* data, const float2* otf, const float2* tw,
                         const PencilArgs& a, const Sched& sc, hipEvent_t ev0, hipEvent_t ev1) {
  switch (mode) {
    case PM_FWD:
      return pencil_e<PM_FWD>(E, prec, grid, block, lds, s, data, otf, tw, a, sc, true, ev0, ev1);
    case PM_INV:
      return pencil_e<PM_INV>(E, prec, grid, block, lds, s, data, otf, tw, a, sc, true, ev0, ev1);
    case PM_FKI:
      return pencil_e<PM_FKI>(E, prec, grid, block, lds, s, data, otf, tw, a, sc, true, ev0, ev1);
    case PM_FCKI:
      return pencil_e<PM_FCKI>(E, prec, grid, block, lds, s, data, otf, tw, a, sc, true, ev0,
                               ev1);
    default: return hipErrorInvalidValue;
  }
}

// The per-iteration passes of power-of-two rows with 4 or 8 elements per thread
// (P = M / E <= 64) run on compile-time schedules.
template <int MODE, int E>
static bool xrow_ct(int M, dim3 g, dim3 b, size_t lds, hipStream_t s, const XArgs& a,
                    const Sched& sc, const float2* tw, hipEvent_t ev0, hipEvent_t ev1) {
  switch (M) {
#define RL_CM(MV)                                                                \
  case MV:                                                                       \
    if constexpr (xrow_compiled_len(MODE, E, MV, 0) == MV) {                     \
      RL_LAUNCH((k_xrow<E, MODE, 0, MV>), g, b, lds, s, ev0, ev1, a, sc, tw);    \
      return true;                                                               \
    }                                                                            \
    return false;
    RL_CM(24) RL_CM(48) RL_CM(96) RL_CM(64) RL_CM(128) RL_CM(256) RL_CM(512) RL_CM(1280)
#undef RL_CM
    default:
      return false;
  }
}

template <int MODE>
static hipError_t xrow_e(int E, int prec, dim3 g, dim3 b, size_t lds, hipStream_t s,
                         const XArgs& a, const Sched& sc, const float2* tw, hipEvent_t ev0,
                         hipEvent_t ev1) {
  if constexpr (MODE == XM_RATIO || MODE == XM_UPDATE) {
    if (xrow_compiled_len(MODE, E, a.M, E == 16 ? prec : 0) > 0) {  // PREC of the instance
      const bool ok = E == 4    ? xrow_ct<MODE, 4>(a.M, g, b, lds, s, a, sc, tw, ev0, ev1)
                      : E == 6  ? xrow_ct<MODE, 6>(a.M, g, b, lds, s, a, sc, tw, ev0, ev1)
                      : E == 8  ? xrow_ct<MODE, 8>(a.M, g, b, lds, s, a, sc, tw, ev0, ev1)
                                : xrow_ct<MODE, 20>(a.M, g, b, lds, s, a, sc, tw, ev0, ev1);
      return ok ? hipGetLastError() : hipErrorInvalidValue;
    }
  }
  if (E == 16 && prec == 1) {
    RL_LAUNCH((k_xrow<16, MODE, 1>), g, b, lds, s, ev0, ev1, a, sc, tw);
    return hipGetLastError();
  }
  if (E == 16 && prec == 2) {
    RL_LAUNCH((k_xrow<16, MODE, 2>), g, b, lds, s, ev0, ev1, a, sc, tw);
    return hipGetLastError();
  }
  switch (E) {
#define RL_CASE(EV)                                                      \
  case EV:                                                               \
    RL_LAUNCH((k_xrow<EV, MODE>), g, b, lds, s, ev0, ev1, a, sc, tw);    \
    break;
    RL_CASE(1) RL_CASE(2) RL_CASE(3) RL_CASE(4) RL_CASE(6) RL_CASE(8) RL_CASE(12) RL_CASE(16)
    RL_CASE(24) RL_CASE(5) RL_CASE(10) RL_CASE(20) RL_CASE(7) RL_CASE(14) RL_CASE(9) RL_CASE(18)
    RL_CASE(15) RL_CASE(30)
#undef RL_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_xrow(int mode, int E, int prec, dim3 grid, dim3 block, size_t lds,
                       hipStream_t s, const XArgs& a, const Sched& sc, const float2* tw,
                       hipEvent_t ev0, hipEvent_t ev1) {
  switch (mode) {
    case XM_R2C: return xrow_e<XM_R2C>(E, prec, grid, block, lds, s, a, sc, tw, ev0, ev1);
    case XM_C2R: return xrow_e<XM_C2R>(E, prec, grid, block, lds, s, a, sc, tw, ev0, ev1);
    case XM_RATIO: return xrow_e<XM_RATIO>(E, prec, grid, block, lds, s, a, sc, tw, ev0, ev1);
    case XM_UPDATE: return xrow_e<XM_UPDATE>(E, prec, grid, block, lds, s, a, sc, tw, ev0, ev1);
    case XM_RATIO_LL:
      return xrow_e<XM_RATIO_LL>(E, prec, grid, block, lds, s, a, sc, tw, ev0, ev1);
    case XM_UPDATE_CHG:
      return xrow_e<XM_UPDATE_CHG>(E, prec, grid, block, lds, s, a, sc, tw, ev0, ev1);
    case XM_UPDATE_PSNR:
      return xrow_e<XM_UPDATE_PSNR>(E, prec, grid, block, lds, s, a, sc, tw, ev0, ev1);
    case XM_PREDICT: return xrow_e<XM_PREDICT>(E, prec, grid, block, lds, s, a, sc, tw, ev0, ev1);
    case XM_UPDATE_ACC:
      return xrow_e<XM_UPDATE_ACC>(E, prec, grid, block, lds, s, a, sc, tw, ev0, ev1);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_metric(const double* met_partials, int groups, int metric, int it,
                         double threshold, int min_iter, long long nvox, double* hist, int* stop,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_metric, dim3(1), dim3(256), 0, s, met_partials, groups, metric, it,
                     threshold, min_iter, nvox, hist, stop);
  return hipGetLastError();
}

hipError_t launch_ssim(const float* u, const float* g, int nz, int ny, int nx, double* buf_a,
                       double* buf_b, double* range_part, int range_blocks, double* range,
                       double* part, bool want_range, const int* stop, hipStream_t s) {
  const long long n = (long long)nz * ny * nx;
  const int nxo = nx - kSsimWin + 1, nyo = ny - kSsimWin + 1, nzo = nz - kSsimWin + 1;
  const unsigned bx = (unsigned)((nxo + 255) / 256);
  hipError_t e;
  if (want_range) {
    hipLaunchKernelGGL(k_range, dim3((unsigned)range_blocks), dim3(256), 0, s, g, n, range_part);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_range_final, dim3(1), dim3(64), 0, s, range_part, range_blocks, range);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_ssim_x, dim3(bx, (unsigned)ny, (unsigned)nz), dim3(256), 0, s, u, g, nz, ny,
                     nx, buf_a, stop);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const unsigned cy = (unsigned)((nyo + kSsimChunk - 1) / kSsimChunk);
  const unsigned cz = (unsigned)((nzo + kSsimChunk - 1) / kSsimChunk);
  hipLaunchKernelGGL(k_ssim_y, dim3(bx, cy, (unsigned)nz), dim3(256), 0, s, buf_a, nz, ny, nxo,
                     buf_b, stop);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_ssim_z, dim3(bx, (unsigned)nyo, cz), dim3(256), 0, s, buf_b, nz, nyo, nxo,
                     range, part, stop);
  return hipGetLastError();
}

hipError_t launch_split_diag(const float* u, int nz, int ny, int nx, float* a, float* b,
                             hipStream_t s, const int* stop) {
  dim3 g((unsigned)((nx / 2 + 255) / 256), (unsigned)(ny / 2), (unsigned)(nz / 2));
  hipLaunchKernelGGL(k_split_diag, g, dim3(256), 0, s, u, nz, ny, nx, a, b, stop);
  return hipGetLastError();
}

hipError_t launch_fsc(const float2* F, const float2* G, int nz, int ny, int nx, int xt, int nbins,
                      long long lcm, double threshold, double* part, double* out,
                      hipStream_t s, const int* stop) {
  const size_t lds = (size_t)(nbins + 1) * 3 * sizeof(double);
  hipLaunchKernelGGL(k_shell, dim3((unsigned)xt, (unsigned)nz), dim3(256), lds, s, F, G, nz, ny,
                     nx, xt, nbins, lcm, part, stop);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fsc_final, dim3(1), dim3(256), 0, s, part, nz * xt, nbins, threshold, out,
                     stop);
  return hipGetLastError();
}

hipError_t launch_accel_alpha(const double* acc_partials, int groups, int it, float* alpha32,
                              double* alpha64, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  RL_LAUNCH(k_accel_alpha, dim3(1), dim3(256), 0, s, ev0, ev1, acc_partials, groups, it, alpha32,
            alpha64);
  return hipGetLastError();
}

hipError_t launch_flux_reduce(const double* partials, int groups, int rows, double* flux,
                              hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  RL_LAUNCH(k_flux_reduce, dim3(rows), dim3(256), 0, s, ev0, ev1, partials, groups, flux);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Persistent batched iteration (see PersistArgs)
// ---------------------------------------------------------------------------
// Index of the XCD (accelerator complex die) this wave runs on.
__device__ __forceinline__ int xcc_id() {
  return (int)(__builtin_amdgcn_s_getreg((3 << 11) | 20) & 15);  // hwreg(HW_REG_XCC_ID, 0, 4)
}

// Current value of a counter or flag that only ever holds values >= 0, read with
// an atomic compare-and-swap (against -1, so it never stores): the read is
// performed where the atomic increments are.  An atomic add of zero would not do:
// the compiler folds it into a plain load.
__device__ __forceinline__ int poll_int(int* p) {
  int v = -1;
  __hip_atomic_compare_exchange_strong(p, &v, -1, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
  return v;
}

template <int MODE>
__device__ __forceinline__ void persist_pencil(const PersistClass& c, const PencilArgs& a,
                                               const Sched& sc, const float2* tw, int E, int gx,
                                               int gy, int vol, float2* lds) {
  switch (E) {
#define RL_PE(EV) \
  case EV: pencil_tile<EV, MODE>(c.spec, c.otf, tw, a, sc, gx, gy, vol, lds); break;
    RL_PE(4) RL_PE(6) RL_PE(8) RL_PE(12)
#undef RL_PE
    default: break;
  }
}

template <int MODE>
__device__ __forceinline__ void persist_xrow(const PersistClass& c, const XArgs& a, int gx,
                                             int vol, float2* lds) {
  switch (c.ex) {
#define RL_XE(EV) \
  case EV: xrow_tile<EV, MODE>(a, c.sx, c.twx, gx, vol, c.xtiles, lds); break;
    RL_XE(2) RL_XE(4) RL_XE(6)
#undef RL_XE
    default: break;
  }
}

__global__ void __launch_bounds__(kPersistThreads) k_persist(PersistArgs pa) {
  extern __shared__ __attribute__((aligned(16))) float2 lds[];
  __shared__ int s_seg, s_tile;
  const int q = xcc_id();
  if (q >= pa.nq) return;  // no work is queued for this XCD
  const int it = *pa.iter_ptr;
  int* tickets = pa.tickets + (long long)it * pa.nq;
  int* done = pa.done + (long long)it * pa.nvrow * kPersistPasses;
  const int s0 = pa.qseg[q], s1 = pa.qseg[q + 1];
  if (s1 <= s0) return;
  const int total = pa.segs[s1 - 1].first + pa.segs[s1 - 1].tiles;
  // Counters and the error flag of queue q are only touched by this XCD's
  // work-groups, and only with atomic read-modify-writes (poll_int reads too).
  int* err = pa.error + q;
  for (;;) {
    if (threadIdx.x == 0) {
      const int t = __hip_atomic_fetch_add(&tickets[q], 1, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
      int seg = -1, tile = 0;
      if (t < total && !poll_int(err)) {
        int lo = s0, hi = s1 - 1;  // last segment with first <= t
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (pa.segs[mid].first <= t) lo = mid;
          else hi = mid - 1;
        }
        seg = lo;
        const PersistSeg g = pa.segs[seg];
        tile = t - g.first;
        if (g.pass > 0) {  // every tile of the previous pass of this volume
          const PersistClass& c = pa.cls[g.cls];
          const int pp = g.pass - 1, kind = pp & 3;
          const int need = kind == 0 ? c.xtiles : (kind == 2 ? c.ztiles : c.ytiles);
          int* ctr = done + (long long)g.vrow * kPersistPasses + pp;
          int n = 0;
          while (poll_int(ctr) < need) {
            __builtin_amdgcn_s_sleep(2);
            if (++n >= pa.spin_limit || poll_int(err)) {
              __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              seg = -1;
              break;
            }
          }
          // the producers' stores are in this XCD's L2: drop this CU's L1 copies
          asm volatile("buffer_inv sc0" ::: "memory");
        }
      }
      s_seg = seg;
      s_tile = tile;
    }
    __syncthreads();
    const int seg = s_seg, tile = s_tile;
    if (seg < 0) break;
    const PersistSeg g = pa.segs[seg];
    const PersistClass& c = pa.cls[g.cls];
    switch (g.pass) {
      case 0: persist_xrow<XM_RATIO>(c, c.xr, tile, g.vol, lds); break;
      case 1: case 5:
        persist_pencil<PM_FWD>(c, c.py, c.sy, c.twy, c.ey, tile % c.ygx, tile / c.ygx, g.vol, lds);
        break;
      case 2:
        persist_pencil<PM_FCKI>(c, c.pz, c.sz, c.twz, c.ez, tile % c.zgx, tile / c.zgx, g.vol, lds);
        break;
      case 3: case 7:
        persist_pencil<PM_INV>(c, c.py, c.sy, c.twy, c.ey, tile % c.ygx, tile / c.ygx, g.vol, lds);
        break;
      case 4: {  // the last iteration's update skips the forward transform
        XArgs xu = c.xu;
        xu.do_fwd = pa.npass > 5 ? 1 : 0;
        persist_xrow<XM_UPDATE>(c, xu, tile, g.vol, lds);
        break;
      }
      case 6:
        persist_pencil<PM_FKI>(c, c.pz, c.sz, c.twz, c.ez, tile % c.zgx, tile / c.zgx, g.vol, lds);
        break;
      default: break;
    }
    // completion: every wave's stores acknowledged by the L2, then one increment
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0)
      __hip_atomic_fetch_add(done + (long long)g.vrow * kPersistPasses + g.pass, 1,
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

hipError_t launch_persist(const PersistArgs& a, int grid, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL(k_persist, dim3((unsigned)grid), dim3(kPersistThreads), lds, s, a);
  return hipGetLastError();
}

hipError_t persist_occupancy(size_t lds, int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_persist, kPersistThreads,
                                                      lds);
}

__global__ void k_zero_ints(int* p, long long n) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = 0;
}

__global__ void k_otf_zmajor(const float2* __restrict__ in, float2* __restrict__ out, long long n,
                             int nz, int ny, int xt, int ncols) {
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (long long)gridDim.x * blockDim.x) {
    const int col = (int)(idx & (kTile - 1));
    long long r = idx >> 4;  // ((v * nz + z) * xt + t) * ny + y
    const int y = (int)(r % ny);
    r /= ny;
    const int t = (int)(r % xt);
    r /= xt;
    const int z = (int)(r % nz);
    const long long v = r / nz;
    const int w = min(kTile, ncols - t * kTile);  // the tile's stored width
    if (col >= w) continue;                       // padding: not stored
    out[((v * xt + t) * ny * nz) * kTile + ((long long)y * nz + z) * w + col] = in[idx];
  }
}

hipError_t launch_otf_zmajor(const float2* in, float2* out, int nvol, int nz, int ny, int xt,
                             int ncols, hipStream_t s) {
  const long long n = (long long)nvol * nz * ny * xt * kTile;
  if (n <= 0) return hipSuccess;
  if (ncols <= (xt - 1) * kTile || ncols > xt * kTile) return hipErrorInvalidValue;
  const long long blocks = std::min<long long>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_otf_zmajor, dim3((unsigned)blocks), dim3(256), 0, s, in, out, n, nz, ny,
                     xt, ncols);
  return hipGetLastError();
}

hipError_t launch_zero_ints(int* p, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_ints, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

__global__ void k_advance(int* counter) {
  if (threadIdx.x == 0) counter[0] += 1;
}

__global__ void k_set_counter(int* counter, int value) {
  if (threadIdx.x == 0) counter[0] = value;
}

hipError_t launch_advance(int* counter, hipStream_t s) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, counter);
  return hipGetLastError();
}

hipError_t launch_set_counter(int* counter, int value, hipStream_t s) {
  hipLaunchKernelGGL(k_set_counter, dim3(1), dim3(64), 0, s, counter, value);
  return hipGetLastError();
}

hipError_t launch_twiddles(float2* tab, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_twiddles, dim3((n + 255) / 256), dim3(256), 0, s, tab, n);
  return hipGetLastError();
}

hipError_t launch_psf_stats(const float* h, long long n, double* partials, int nblk,
                            unsigned* counter, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_psf_stats, dim3(nblk), dim3(256), 0, s, h, n, partials, counter, out);
  return hipGetLastError();
}

hipError_t launch_psf_prep(const float* h, int pz, int py, int px, float* out, int nz, int ny,
                           int nx, long long out_row_stride, double scale, hipStream_t s) {
  dim3 g((nx + 255) / 256, ny, nz);
  hipLaunchKernelGGL(k_psf_prep, g, dim3(256), 0, s, h, out, nz, ny, nx, pz, py, px,
                     out_row_stride, scale);
  return hipGetLastError();
}

hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s) {
  const long long n = (long long)(bytes / 16);
  long long blocks = (n + 256LL * kCopyUnroll - 1) / (256LL * kCopyUnroll);
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, s,
                     reinterpret_cast<const float4*>(src), reinterpret_cast<float4*>(dst), n);
  return hipGetLastError();
}

}  // namespace rlmi
