// MFMA flavours of the opposite-spin contraction D * (pq|rs) * E, shared by
// the full-size sigma kernels (sigma.hip) and the batch solver (batch.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sbci {
namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

// MFMA flavours of the opposite-spin contraction.
//   A     element type of the ERI tile in LDS (and of the B fragments)
//   Acc   accumulation type of sigma's row in LDS (FP64 in every flavour:
//         measured on gfx950, ds_add_f64 sustains several times the rate of
//         ds_add_f32 for this scatter, and it is more accurate)
//   KSTEP K per MFMA, KPL K elements per lane
//   orow  output row held by lane group g, register r (measured on gfx950:
//         the f64 16x16x4 result interleaves its rows across lane groups)
struct MF64 {
  using A = double;
  using Acc = double;
  using Frag = double;
  using Out = d4_t;
  static constexpr int KSTEP = 4, KPL = 1, PAD = 1;
  __device__ static int orow(int g, int r) { return g + 4 * r; }
  template <typename T> __device__ static A cvt(T x) { return (A)x; }
  __device__ static Frag load_a(const A *p) { return *p; }
  template <typename T>
  __device__ static Frag load_b(const T *cv, const uint32_t *off, uint32_t J) {
    return (Frag)cv[off[0] + J];
  }
  __device__ static Out mma(Frag a, Frag b, Out c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
struct MF32 {
  using A = float;
  using Acc = double;  // FP64 LDS atomics are far faster than FP32 ones on gfx950
  using Frag = float;
  using Out = f4_t;
  static constexpr int KSTEP = 4, KPL = 1, PAD = 1;
  __device__ static int orow(int g, int r) { return 4 * g + r; }
  template <typename T> __device__ static A cvt(T x) { return (A)x; }
  __device__ static Frag load_a(const A *p) { return *p; }
  template <typename T>
  __device__ static Frag load_b(const T *cv, const uint32_t *off, uint32_t J) {
    return (Frag)cv[off[0] + J];
  }
  __device__ static Out mma(Frag a, Frag b, Out c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
struct MBF16 {
  using A = __bf16;
  using Acc = double;
  using Frag = bf8_t;
  using Out = f4_t;
  static constexpr int KSTEP = 32, KPL = 8, PAD = 0;
  __device__ static int orow(int g, int r) { return 4 * g + r; }
  template <typename T> __device__ static A cvt(T x) { return (__bf16)(float)x; }
  __device__ static Frag load_a(const A *p) { return *reinterpret_cast<const bf8_t *>(p); }
  template <typename T>
  __device__ static Frag load_b(const T *cv, const uint32_t *off, uint32_t J) {
    Frag f;
#pragma unroll
    for (int t = 0; t < 8; ++t) f[t] = (__bf16)(float)cv[off[t] + J];
    return f;
  }
  __device__ static Out mma(Frag a, Frag b, Out c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

__device__ __forceinline__ int pair_index(int p, int q) {
  int k = p > q ? p : q, l = p > q ? q : p;
  return k * (k + 1) / 2 + l;
}

// Reproducible FP64 scatter of the opposite-spin kernels.  A row of sigma
// accumulates in 64-bit fixed point: integer additions are exact, so the row
// does not depend on the order in which waves add.  The scale is a power of
// two chosen per row from a bound bnd on every partial sum (bnd < 2^62 after
// scaling); bad (a non-finite bound) makes the row NaN.
__device__ __forceinline__ void fix_scale_from_bound(double bnd, double &scale, double &inv,
                                                     bool &bad) {
  bad = !(bnd < INFINITY);
  scale = inv = 1.0;
  if (bnd > 0 && !bad) {
    int x = 0;
    frexp(bnd, &x);  // bnd < 2^x
    int ex = 62 - x;
    ex = ex > 900 ? 900 : (ex < -900 ? -900 : ex);
    scale = ldexp(1.0, ex);
    inv = ldexp(1.0, -ex);
  }
}

// Add one contribution to a row slot: in fixed point (FIX) v is already in
// fixed-point units (|v| < 2^62, the scale folded into the operands) and is
// taken to floor(v) by a split at 2^32, hi = floor(v / 2^32), lo = v - hi 2^32
// in [0, 2^32), both exact; otherwise an FP64 atomic add.
template <bool FIX>
__device__ __forceinline__ void scatter_add(double *slot, double v) {
  if constexpr (FIX) {
    const double hi = floor(v * 0x1p-32);
    const double lo = fma(hi, -0x1p32, v);
    const unsigned long long q =
        ((unsigned long long)(unsigned)(int)hi << 32) + (unsigned long long)(unsigned)lo;
    atomicAdd(reinterpret_cast<unsigned long long *>(slot), q);
  } else {
    atomicAdd(slot, v);
  }
}

// Row write-back value of slot j: fixed point scaled back (or NaN), or the
// FP64 sum.
template <bool FIX, typename T>
__device__ __forceinline__ T row_value(const double *acc, int64_t j, double inv, bool bad) {
  if constexpr (FIX) {
    const long long q = (long long)reinterpret_cast<const unsigned long long *>(acc)[j];
    return bad ? (T)NAN : (T)((double)q * inv);
  } else {
    return (T)acc[j];
  }
}

}  // namespace
}  // namespace sbci
