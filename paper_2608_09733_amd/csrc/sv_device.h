#pragma once
// gfx950 kernels of the state-vector library.
//
// State layout in HBM: two planes (re, im) of 2^n elements (double for
// complex128, float for complex64).  Gate action follows the paper's gather /
// multiply / scatter over the amplitudes that differ only on the targets
// (Section 5.3), but indices are computed by bit insertion instead of an index
// table, and many gates are applied per HBM round trip (see sv_internal.h).
#include <hip/hip_runtime.h>

#include <type_traits>
#include <stdint.h>

#include "sv_internal.h"

namespace svk {

template <typename T> struct C2T;
template <> struct C2T<double> { using type = double2; };
template <> struct C2T<float> { using type = float2; };

template <typename T> struct V4T;   // 16-byte global vector of T
template <> struct V4T<double> { using type = double2; static constexpr int N = 2; };
template <> struct V4T<float> { using type = float4; static constexpr int N = 4; };

// Read-only views in the constant address space: the data (plan descriptors,
// coefficients) is written before the kernel and never during it, so loads
// through these pointers are invariant and go to the scalar cache (SGPRs)
// when the address is wave-uniform.
#define SVI_CONST __attribute__((address_space(4)))
template <typename T>
__device__ __forceinline__ const SVI_CONST T *cptr(const T *p) {
  return (const SVI_CONST T *)p;
}

// Workgroup barrier that orders LDS only: the fences are scoped to the local
// address space, so outstanding global loads (the next tile's prefetch) are
// not waited for, unlike __syncthreads().
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <typename T>
__device__ __forceinline__ int swz(int i) {
  return svi_swz(i, sizeof(T) == 8 ? 3 : 4);
}

// Insert a zero bit at each position of pos[0..np) (ascending).
__device__ __forceinline__ uint64_t insert_zeros64(uint64_t x, const int32_t *pos, int np) {
  for (int k = 0; k < np; k++) {
    const int p = pos[k];
    const uint64_t lo = x & ((1ull << p) - 1ull);
    x = ((x >> p) << (p + 1)) | lo;
  }
  return x;
}

__device__ __forceinline__ int insert_zeros32c(int x, const SVI_CONST int32_t *pos, int np) {
  for (int k = 0; k < np; k++) {
    const int p = pos[k];
    const int lo = x & ((1 << p) - 1);
    x = ((x >> p) << (p + 1)) | lo;
  }
  return x;
}

// Micro-op o, read through the constant address space (uniform index:
// scalar loads, not vector loads whose waits would also wait for other
// memory traffic in flight).
__device__ __forceinline__ MicroOp op_at(const MicroOp *ops, int o) {
  const SVI_CONST MicroOp &s = cptr(ops)[o];
  MicroOp m;
  m.type = s.type;
  m.t0 = s.t0;
  m.t1 = s.t1;
  m.mask = s.mask;
  m.cm = s.cm;
  m.cv = s.cv;
  m.coef = s.coef;
  m.gz = s.gz;
  m.galpha = s.galpha;
  m.gbeta = s.gbeta;
  return m;
}

// Tile-local base index of thread tid in a stage: thread-index bit k placed
// on tile bit tpos[k] (the group bits stay zero).
template <int M, int R>
__device__ __forceinline__ int stage_base(int tid, const SVI_CONST StageDesc &sd) {
  // tpos read as aligned 32-bit words (scalar loads; byte loads of the
  // descriptor would become vector loads, whose waits also wait for the
  // tile prefetch in flight), bytes extracted with scalar shifts
  const SVI_CONST int32_t *w = (const SVI_CONST int32_t *)sd.tpos;
  int b = 0;
#pragma unroll
  for (int k = 0; k < M - R; k++) {
    const int pos = (w[k >> 2] >> (8 * (k & 3))) & 0xff;
    b |= ((tid >> k) & 1) << pos;
  }
  return b;
}

__device__ __forceinline__ int insert_zeros32(int x, const int32_t *pos, int np) {
  for (int k = 0; k < np; k++) {
    const int p = pos[k];
    const int lo = x & ((1 << p) - 1);
    x = ((x >> p) << (p + 1)) | lo;
  }
  return x;
}

// Global offset of tile row r: bit k of r goes to qubit hb[k].
__device__ __forceinline__ uint64_t spread_row(int r, const int32_t *hb, int nh) {
  uint64_t o = 0;
  for (int k = 0; k < nh; k++) o |= (uint64_t)((r >> k) & 1) << hb[k];
  return o;
}

// Offset of tile element i from its tile's base: the low c bits stay, bit
// c + k goes to qubit hb[k].
__device__ __forceinline__ uint64_t tile_off(int i, int c, const int32_t *hb, int nh) {
  return spread_row(i >> c, hb, nh) + (uint64_t)(i & ((1 << c) - 1));
}

// Base index of tile `tile`: zeros inserted at the tile's qubits (0..c-1 and hb).
__device__ __forceinline__ uint64_t tile_base(int64_t tile, int c, const int32_t *hb, int nh) {
  uint64_t x = (uint64_t)tile << c;
  return insert_zeros64(x, hb, nh);
}

// Tile-local index whose bits land on output index i under the output bit
// permutation pm (output bit k <- bit pm[k]).
__device__ __forceinline__ int perm_bits(int i, const int32_t *pm, int m) {
  int j = 0;
  for (int b = 0; b < m; b++) j |= ((i >> b) & 1) << pm[b];
  return j;
}

// ------------------------------------------------------------ micro-ops
// All group arrays are indexed with compile-time indices only.

template <typename T, int R, int TB>
__device__ __forceinline__ void mo_u(T *re, T *im, const double *cf, uint32_t cm, uint32_t cv) {
  const T a0r = (T)cf[0], a0i = (T)cf[1], a1r = (T)cf[2], a1i = (T)cf[3];
  const T b0r = (T)cf[4], b0i = (T)cf[5], b1r = (T)cf[6], b1i = (T)cf[7];
  if (cm == 0) {
#pragma unroll
    for (int j = 0; j < (1 << R); j++) {
      if (j & (1 << TB)) continue;
      const int k = j | (1 << TB);
      const T xr = re[j], xi = im[j], yr = re[k], yi = im[k];
      re[j] = a0r * xr - a0i * xi + a1r * yr - a1i * yi;
      im[j] = a0r * xi + a0i * xr + a1r * yi + a1i * yr;
      re[k] = b0r * xr - b0i * xi + b1r * yr - b1i * yi;
      im[k] = b0r * xi + b0i * xr + b1r * yi + b1i * yr;
    }
  } else {
#pragma unroll
    for (int j = 0; j < (1 << R); j++) {
      if (j & (1 << TB)) continue;
      if ((j & cm) != cv) continue;
      const int k = j | (1 << TB);
      const T xr = re[j], xi = im[j], yr = re[k], yi = im[k];
      re[j] = a0r * xr - a0i * xi + a1r * yr - a1i * yi;
      im[j] = a0r * xi + a0i * xr + a1r * yi + a1i * yr;
      re[k] = b0r * xr - b0i * xi + b1r * yr - b1i * yi;
      im[k] = b0r * xi + b0i * xr + b1r * yi + b1i * yr;
    }
  }
}

template <typename T, int R, int TB>
__device__ __forceinline__ void mo_r(T *re, T *im, const double *cf, uint32_t cm, uint32_t cv) {
  const T r00 = (T)cf[0], r01 = (T)cf[1], r10 = (T)cf[2], r11 = (T)cf[3];
  if (cm == 0) {
#pragma unroll
    for (int j = 0; j < (1 << R); j++) {
      if (j & (1 << TB)) continue;
      const int k = j | (1 << TB);
      const T xr = re[j], xi = im[j], yr = re[k], yi = im[k];
      re[j] = r00 * xr + r01 * yr;
      im[j] = r00 * xi + r01 * yi;
      re[k] = r10 * xr + r11 * yr;
      im[k] = r10 * xi + r11 * yi;
    }
  } else {
#pragma unroll
    for (int j = 0; j < (1 << R); j++) {
      if (j & (1 << TB)) continue;
      if ((j & cm) != cv) continue;
      const int k = j | (1 << TB);
      const T xr = re[j], xi = im[j], yr = re[k], yi = im[k];
      re[j] = r00 * xr + r01 * yr;
      im[j] = r00 * xi + r01 * yi;
      re[k] = r10 * xr + r11 * yr;
      im[k] = r10 * xi + r11 * yi;
    }
  }
}

template <typename T, int R>
__device__ __forceinline__ void mo_p(T *re, T *im, const double *cf, uint32_t mask, uint32_t cm,
                                     uint32_t cv) {
  const T d0r = (T)cf[0], d0i = (T)cf[1], d1r = (T)cf[2], d1i = (T)cf[3];
#pragma unroll
  for (int j = 0; j < (1 << R); j++) {
    if ((j & cm) != cv) continue;
    const bool odd = __builtin_popcount((uint32_t)j & mask) & 1;
    const T dr = odd ? d1r : d0r;
    const T di = odd ? d1i : d0i;
    const T xr = re[j], xi = im[j];
    re[j] = xr * dr - xi * di;
    im[j] = xr * di + xi * dr;
  }
}

template <typename T, int R, int TB>
__device__ __forceinline__ void mo_x(T *re, T *im, uint32_t cm, uint32_t cv) {
#pragma unroll
  for (int j = 0; j < (1 << R); j++) {
    if (j & (1 << TB)) continue;
    if ((j & cm) != cv) continue;
    const int k = j | (1 << TB);
    T t = re[j]; re[j] = re[k]; re[k] = t;
    t = im[j]; im[j] = im[k]; im[k] = t;
  }
}

template <typename T, int R, int A, int B>
__device__ __forceinline__ void mo_swap(T *re, T *im, uint32_t cm, uint32_t cv) {
#pragma unroll
  for (int j = 0; j < (1 << R); j++) {
    if (!((j >> A) & 1) || ((j >> B) & 1)) continue;
    if ((j & cm) != cv) continue;
    const int k = j ^ (1 << A) ^ (1 << B);
    T t = re[j]; re[j] = re[k]; re[k] = t;
    t = im[j]; im[j] = im[k]; im[k] = t;
  }
}

template <typename T, int R>
__device__ __forceinline__ void mo_neg(T *re, T *im, uint32_t cm, uint32_t cv) {
#pragma unroll
  for (int j = 0; j < (1 << R); j++) {
    if ((j & cm) != cv) continue;
    re[j] = -re[j];
    im[j] = -im[j];
  }
}

// 4x4 on (bit A = low local bit, bit B = high local bit).
template <typename T, int R, int A, int B>
__device__ __forceinline__ void mo_q(T *re, T *im, const double *cf, uint32_t cm, uint32_t cv) {
  T u[32];
#pragma unroll
  for (int q = 0; q < 32; q++) u[q] = (T)cf[q];
#pragma unroll
  for (int j = 0; j < (1 << R); j++) {
    if ((j >> A) & 1) continue;
    if ((j >> B) & 1) continue;
    if ((j & cm) != cv) continue;
    constexpr int a1 = 1 << A, b1 = 1 << B;
    const T x0r = re[j], x0i = im[j], x1r = re[j | a1], x1i = im[j | a1];
    const T x2r = re[j | b1], x2i = im[j | b1], x3r = re[j | a1 | b1], x3i = im[j | a1 | b1];
#define SVI_ROW(r, dst)                                                                   \
    {                                                                                     \
      const T ar = u[8 * r + 0] * x0r - u[8 * r + 1] * x0i + u[8 * r + 2] * x1r -         \
                   u[8 * r + 3] * x1i + u[8 * r + 4] * x2r - u[8 * r + 5] * x2i +         \
                   u[8 * r + 6] * x3r - u[8 * r + 7] * x3i;                               \
      const T ai = u[8 * r + 0] * x0i + u[8 * r + 1] * x0r + u[8 * r + 2] * x1i +         \
                   u[8 * r + 3] * x1r + u[8 * r + 4] * x2i + u[8 * r + 5] * x2r +         \
                   u[8 * r + 6] * x3i + u[8 * r + 7] * x3r;                               \
      re[dst] = ar;                                                                       \
      im[dst] = ai;                                                                       \
    }
    SVI_ROW(0, j) SVI_ROW(1, j | a1) SVI_ROW(2, j | b1) SVI_ROW(3, j | a1 | b1)
#undef SVI_ROW
  }
}

// Real rotation between the two local patterns of a two-level subspace:
// for every j with (j & tm) == pa, partner k = j ^ XM:
//   (x_j, x_k) <- (r00 x_j + r01 x_k, r10 x_j + r11 x_k).
template <typename T, int R, int XM>
__device__ __forceinline__ void mo_2l(T *re, T *im, const double *cf, uint32_t tm, uint32_t pa,
                                      uint32_t cm, uint32_t cv) {
  const T r00 = (T)cf[0], r01 = (T)cf[1], r10 = (T)cf[2], r11 = (T)cf[3];
#pragma unroll
  for (int j = 0; j < (1 << R); j++) {
    if (((uint32_t)j & tm) != pa) continue;
    if ((j & cm) != cv) continue;
    const int k = j ^ XM;
    const T xr = re[j], xi = im[j], yr = re[k], yi = im[k];
    re[j] = r00 * xr + r01 * yr;
    im[j] = r00 * xi + r01 * yi;
    re[k] = r10 * xr + r11 * yr;
    im[k] = r10 * xi + r11 * yi;
  }
}

// 2^K x 2^K on group bits 0..K-1.
template <typename T, int R, int K>
__device__ __forceinline__ void mo_dense(T *re, T *im, const double *cf, uint32_t cm,
                                         uint32_t cv) {
  constexpr int D = 1 << K;
#pragma clang loop unroll(full)
  for (int o = 0; o < (1 << (R - K)); o++) {
    const int base = o << K;
    if ((base & cm) != cv) continue;
    T xr[D], xi[D];
#pragma unroll
    for (int q = 0; q < D; q++) { xr[q] = re[base + q]; xi[q] = im[base + q]; }
#pragma unroll
    for (int r = 0; r < D; r++) {
      T ar = 0, ai = 0;
#pragma unroll
      for (int q = 0; q < D; q++) {
        const T ur = (T)cf[(r * D + q) * 2], ui = (T)cf[(r * D + q) * 2 + 1];
        ar += ur * xr[q] - ui * xi[q];
        ai += ur * xi[q] + ui * xr[q];
      }
      re[base + r] = ar;
      im[base + r] = ai;
    }
  }
}

template <typename T, int R, typename CP = const double *>
__device__ __forceinline__ void mo_diagt(T *re, T *im, CP cf) {
#pragma unroll
  for (int j = 0; j < (1 << R); j++) {
    const T dr = (T)cf[2 * j], di = (T)cf[2 * j + 1];
    const T xr = re[j], xi = im[j];
    re[j] = xr * dr - xi * di;
    im[j] = xr * di + xi * dr;
  }
}

// Im <lam| G |psi> over one group from the generator's per-slot table (see
// GRAD_ODD / GRAD_BETA in sv_internal.h); XM is the generator's x-mask.
template <typename T, int R, int XM, bool ODD, typename CP>
__device__ __forceinline__ double mo_grad(const T *pr, const T *pi, const T *lr, const T *li,
                                          CP tab) {
  constexpr int G = 1 << R;
  double acc = 0.0;
#pragma unroll
  for (int j = 0; j < G; j++) {
    const int k = j ^ XM;
    const double ljr = (double)lr[j], lji = (double)li[j];
    const double f = ODD ? ljr * (double)pr[k] + lji * (double)pi[k]
                         : ljr * (double)pi[k] - lji * (double)pr[k];
    acc += (double)tab[j] * f;
  }
  return acc;
}

// Fast-Givens rotation on group bit TB (record {form, k, scale, 0}, form 0 or
// 1, always 0 for FP64; the scale is applied separately).  Gentleman's scaled
// rotation: each output is one FMA with a +-1 coefficient on one input.
template <typename T, int R, int TB, typename CP>
__device__ __forceinline__ void mo_fastr(T *re, T *im, CP cf) {
  const T k = (T)cf[1];
#define SVI_FR(XR, XI, YR, YI)                                   \
  _Pragma("unroll") for (int j = 0; j < (1 << R); j++) {         \
    if (j & (1 << TB)) continue;                                 \
    const int l = j | (1 << TB);                                 \
    const T xr = re[j], xi = im[j], yr = re[l], yi = im[l];      \
    re[j] = XR; im[j] = XI; re[l] = YR; im[l] = YI;              \
  }
  if constexpr (sizeof(T) == 8) {
    // FP64 coefficients are always form 0 (CF_FORM0): straight-line FMAs,
    // with no branch whose two arms the compiler would merge with copies
    SVI_FR(xr - k * yr, xi - k * yi, k * xr + yr, k * xi + yi)
  } else {
    const int form = (int)cf[0];
    if (form == 0) {
      SVI_FR(xr - k * yr, xi - k * yi, k * xr + yr, k * xi + yi)
    } else {
      SVI_FR(k * xr - yr, k * xi - yi, xr + k * yr, xi + k * yi)
    }
  }
#undef SVI_FR
}

// Static Kronecker stage: s * D_after * (R~_{R-1} (x) ... (x) R~_0) * D_before,
// in three parts so that gradient terms can be taken between them.
template <typename T, int R, typename CP>
__device__ __forceinline__ void kron_pre(T *re, T *im, CP cf, int dflags) {
  if (dflags & 1) mo_diagt<T, R>(re, im, cf + 4 * R);
}

template <typename T, int R, typename CP>
__device__ __forceinline__ void kron_rot(T *re, T *im, CP cf, uint32_t rmask) {
  if (rmask & 1u) mo_fastr<T, R, 0>(re, im, cf + 0);
  if (rmask & 2u) mo_fastr<T, R, 1>(re, im, cf + 4);
  if constexpr (R > 2) { if (rmask & 4u) mo_fastr<T, R, 2>(re, im, cf + 8); }
  if constexpr (R > 3) { if (rmask & 8u) mo_fastr<T, R, 3>(re, im, cf + 12); }
  if constexpr (R > 4) { if (rmask & 16u) mo_fastr<T, R, 4>(re, im, cf + 16); }
}

// Every group bit rotated (rmask full), no conditionals.
template <typename T, int R, typename CP>
__device__ __forceinline__ void kron_rot_all(T *re, T *im, CP cf) {
  mo_fastr<T, R, 0>(re, im, cf + 0);
  mo_fastr<T, R, 1>(re, im, cf + 4);
  if constexpr (R > 2) mo_fastr<T, R, 2>(re, im, cf + 8);
  if constexpr (R > 3) mo_fastr<T, R, 3>(re, im, cf + 12);
  if constexpr (R > 4) mo_fastr<T, R, 4>(re, im, cf + 16);
}

template <typename T, int R, typename CP>
__device__ __forceinline__ void kron_post(T *re, T *im, CP cf, int dflags) {
  constexpr int G = 1 << R;
  CP ta = cf + 4 * R + 2 * G;
  if (dflags & 2) mo_diagt<T, R>(re, im, ta);
  if (dflags & 4) {
    const T sc = (T)ta[2 * G];
#pragma unroll
    for (int j = 0; j < G; j++) { re[j] *= sc; im[j] *= sc; }
  }
}

template <typename T, int R, typename CP>
__device__ __forceinline__ void kron_stage(T *re, T *im, CP cf, uint32_t rmask, int dflags) {
  kron_pre<T, R>(re, im, cf, dflags);
  kron_rot<T, R>(re, im, cf, rmask);
  kron_post<T, R>(re, im, cf, dflags);
}

#define SVI_T5(F, t, ...)                                   \
  switch (t) {                                              \
    case 0: F<T, R, 0>(__VA_ARGS__); break;                 \
    case 1: F<T, R, 1>(__VA_ARGS__); break;                 \
    case 2: if constexpr (R > 2) F<T, R, 2>(__VA_ARGS__); break; \
    case 3: if constexpr (R > 3) F<T, R, 3>(__VA_ARGS__); break; \
    case 4: if constexpr (R > 4) F<T, R, 4>(__VA_ARGS__); break; \
    default: break;                                         \
  }

template <typename T, int R>
__device__ __forceinline__ void dispatch_swap(int a, int b, T *re, T *im, uint32_t cm, uint32_t cv) {
#define SVI_SW(A, B) if (a == A && b == B) { if constexpr (A < R && B < R) mo_swap<T, R, A, B>(re, im, cm, cv); return; }
  SVI_SW(0, 1) SVI_SW(0, 2) SVI_SW(0, 3) SVI_SW(0, 4) SVI_SW(1, 0) SVI_SW(1, 2) SVI_SW(1, 3)
  SVI_SW(1, 4) SVI_SW(2, 0) SVI_SW(2, 1) SVI_SW(2, 3) SVI_SW(2, 4) SVI_SW(3, 0) SVI_SW(3, 1)
  SVI_SW(3, 2) SVI_SW(3, 4) SVI_SW(4, 0) SVI_SW(4, 1) SVI_SW(4, 2) SVI_SW(4, 3)
#undef SVI_SW
}

template <typename T, int R>
__device__ __forceinline__ void dispatch_q(int a, int b, T *re, T *im, const double *cf,
                                           uint32_t cm, uint32_t cv) {
#define SVI_Q(A, B) if (a == A && b == B) { if constexpr (A < R && B < R) mo_q<T, R, A, B>(re, im, cf, cm, cv); return; }
  SVI_Q(0, 1) SVI_Q(0, 2) SVI_Q(0, 3) SVI_Q(0, 4) SVI_Q(1, 0) SVI_Q(1, 2) SVI_Q(1, 3)
  SVI_Q(1, 4) SVI_Q(2, 0) SVI_Q(2, 1) SVI_Q(2, 3) SVI_Q(2, 4) SVI_Q(3, 0) SVI_Q(3, 1)
  SVI_Q(3, 2) SVI_Q(3, 4) SVI_Q(4, 0) SVI_Q(4, 1) SVI_Q(4, 2) SVI_Q(4, 3)
#undef SVI_Q
}

template <typename T, int R>
__device__ __forceinline__ void apply_op(const MicroOp &op, T *re, T *im, const double *coef) {
  const double *cf = coef + op.coef;
  switch (op.type) {
    case MO_U: SVI_T5(mo_u, op.t0, re, im, cf, op.cm, op.cv) break;
    case MO_R: SVI_T5(mo_r, op.t0, re, im, cf, op.cm, op.cv) break;
    case MO_P: mo_p<T, R>(re, im, cf, op.mask, op.cm, op.cv); break;
    case MO_X:
      switch (op.t0) {
        case 0: mo_x<T, R, 0>(re, im, op.cm, op.cv); break;
        case 1: mo_x<T, R, 1>(re, im, op.cm, op.cv); break;
        case 2: if constexpr (R > 2) mo_x<T, R, 2>(re, im, op.cm, op.cv); break;
        case 3: if constexpr (R > 3) mo_x<T, R, 3>(re, im, op.cm, op.cv); break;
        case 4: if constexpr (R > 4) mo_x<T, R, 4>(re, im, op.cm, op.cv); break;
        default: break;
      }
      break;
    case MO_SWAP: dispatch_swap<T, R>(op.t0, op.t1, re, im, op.cm, op.cv); break;
    case MO_NEG: mo_neg<T, R>(re, im, op.cm, op.cv); break;
    case MO_Q: dispatch_q<T, R>(op.t0, op.t1, re, im, cf, op.cm, op.cv); break;
    case MO_DENSE:
      switch (op.mask) {
        case 1: mo_dense<T, R, 1>(re, im, cf, op.cm, op.cv); break;
        case 2: mo_dense<T, R, 2>(re, im, cf, op.cm, op.cv); break;
        case 3: if constexpr (R >= 3) mo_dense<T, R, 3>(re, im, cf, op.cm, op.cv); break;
        default: break;
      }
      break;
    case MO_DIAGT: mo_diagt<T, R>(re, im, cf); break;
    case MO_2L:
      switch (op.t1) {
#define SVI_L(XV) case XV: if constexpr (XV < (1 << R)) mo_2l<T, R, XV>(re, im, cf, op.mask, op.gz, op.cm, op.cv); break;
        SVI_L(1) SVI_L(2) SVI_L(3) SVI_L(4) SVI_L(5) SVI_L(6) SVI_L(7) SVI_L(8) SVI_L(9) SVI_L(10)
        SVI_L(11) SVI_L(12) SVI_L(13) SVI_L(14) SVI_L(15) SVI_L(16) SVI_L(17) SVI_L(18) SVI_L(19)
        SVI_L(20) SVI_L(21) SVI_L(22) SVI_L(23) SVI_L(24) SVI_L(25) SVI_L(26) SVI_L(27) SVI_L(28)
        SVI_L(29) SVI_L(30) SVI_L(31)
#undef SVI_L
        default: break;
      }
      break;
    default: break;
  }
}

// Im <lam| G |psi> over one group for the generator of a two-level rotation
// between the slot patterns a ((j & tm) == pa) and b = a ^ XM: G a = i b,
// G b = -i a, so the term is Re(conj(lam_b) psi_a) - Re(conj(lam_a) psi_b).
template <typename T, int R, int XM>
__device__ __forceinline__ double mo_grad2l(const T *pr, const T *pi, const T *lr, const T *li,
                                            uint32_t tm, uint32_t pa, uint32_t cm, uint32_t cv) {
  double acc = 0.0;
#pragma unroll
  for (int j = 0; j < (1 << R); j++) {
    if (((uint32_t)j & tm) != pa) continue;
    if ((j & cm) != cv) continue;
    const int k = j ^ XM;
    acc += ((double)lr[k] * (double)pr[j] + (double)li[k] * (double)pi[j]) -
           ((double)lr[j] * (double)pr[k] + (double)li[j] * (double)pi[k]);
  }
  return acc;
}

// MO_GRAD: generator alpha * (Pauli string) + beta * I on the control subspace,
// through its per-slot table in the coefficient buffer.
template <typename T, int R>
__device__ __forceinline__ double grad_op(const MicroOp &op, const T *pr, const T *pi, const T *lr,
                                          const T *li, const double *coef) {
  const SVI_CONST double *tab = cptr(coef) + op.t0;
  const uint32_t x = op.mask;   // x-mask over group bits
  // diagonal generators (Z strings, phases): one table, the even form on j itself
  if (x == 0) return mo_grad<T, R, 0, false>(pr, pi, lr, li, tab);
  const bool odd = (op.t1 & GRAD_ODD) != 0;
  switch (x) {
#define SVI_G(XV) case XV: if constexpr (XV < (1 << R)) { \
      if (odd) return mo_grad<T, R, XV, true>(pr, pi, lr, li, tab); \
      return mo_grad<T, R, XV, false>(pr, pi, lr, li, tab); } break;
    SVI_G(1) SVI_G(2) SVI_G(3) SVI_G(4) SVI_G(5) SVI_G(6) SVI_G(7) SVI_G(8) SVI_G(9)
    SVI_G(10) SVI_G(11) SVI_G(12) SVI_G(13) SVI_G(14) SVI_G(15) SVI_G(16) SVI_G(17) SVI_G(18)
    SVI_G(19) SVI_G(20) SVI_G(21) SVI_G(22) SVI_G(23) SVI_G(24) SVI_G(25) SVI_G(26) SVI_G(27)
    SVI_G(28) SVI_G(29) SVI_G(30) SVI_G(31)
#undef SVI_G
    default: break;
  }
  return 0.0;
}

// MO_GRAD inside a Kronecker stage: the planner admits only diagonal
// generators (x = 0) and the Y of an uncontrolled RY (x = one group bit,
// n_Y = 1), so only those forms are compiled here (fewer code paths, fewer
// live registers in the two-state kernel).
template <typename T, int R>
__device__ __forceinline__ double grad_kron(const MicroOp &op, const T *pr, const T *pi,
                                            const T *lr, const T *li, const double *coef) {
  const SVI_CONST double *tab = cptr(coef) + op.t0;
  switch (op.mask) {
    case 0: return mo_grad<T, R, 0, false>(pr, pi, lr, li, tab);
    case 1: return mo_grad<T, R, 1, true>(pr, pi, lr, li, tab);
    case 2: return mo_grad<T, R, 2, true>(pr, pi, lr, li, tab);
    case 4: if constexpr (R > 2) return mo_grad<T, R, 4, true>(pr, pi, lr, li, tab); break;
    case 8: if constexpr (R > 3) return mo_grad<T, R, 8, true>(pr, pi, lr, li, tab); break;
    case 16: if constexpr (R > 4) return mo_grad<T, R, 16, true>(pr, pi, lr, li, tab); break;
    default: break;
  }
  return 0.0;
}

// MO_GRAD or MO_GRAD2L (the micro-op interpreter; Kronecker stages hold MO_GRAD only).
template <typename T, int R>
__device__ __forceinline__ double grad_any(const MicroOp &op, const T *pr, const T *pi,
                                           const T *lr, const T *li, const double *coef) {
  if (op.type == MO_GRAD2L) {
    switch (op.t1) {
#define SVI_G2(XV) case XV: if constexpr (XV < (1 << R)) return mo_grad2l<T, R, XV>(pr, pi, lr, li, op.mask, op.gz, op.cm, op.cv); break;
      SVI_G2(3) SVI_G2(5) SVI_G2(6) SVI_G2(9) SVI_G2(10) SVI_G2(12) SVI_G2(15) SVI_G2(17)
      SVI_G2(18) SVI_G2(20) SVI_G2(23) SVI_G2(24) SVI_G2(27) SVI_G2(29) SVI_G2(30)
#undef SVI_G2
      default: break;
    }
    return 0.0;
  }
  return grad_op<T, R>(op, pr, pi, lr, li, coef);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ------------------------------------------------------------ tile sweep
// One persistent workgroup loops over tiles.  NS = 1 (forward) or 2 (adjoint:
// state 0 = psi, state 1 = lambda, micro-ops applied to both, MO_GRAD
// accumulates gradient partials).

#define SVI_GSLOTS 256
#define SVI_GSLOTS_WIDE 128  // gradient slots per sweep of the two-state Kronecker kernel

// Sum of v over the 64 lanes of a wave, valid in lane 63, by DPP lane moves
// (VALU only): partial sums within rows of 16 lanes (shifts by 1, 2, 4, 8),
// then row 0 into row 1 and row 2 into row 3 (broadcast of lane 15), then
// rows 0-1 into rows 2-3 (broadcast of lane 31).  Lanes outside a shift's row
// read 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, ROW_MASK, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double wave_total63(double v) {
  v += dpp_d<0x111, 0xf>(v);   // row_shr:1
  v += dpp_d<0x112, 0xf>(v);   // row_shr:2
  v += dpp_d<0x114, 0xf>(v);   // row_shr:4
  v += dpp_d<0x118, 0xf>(v);   // row_shr:8
  v += dpp_d<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp_d<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
  return v;
}

// Swaps the upper 32 lanes of x with the lower 32 lanes of y (64-bit values,
// v_permlane32_swap on each half).
__device__ __forceinline__ void swap32_d(double &x, double &y) {
  const long long xb = __double_as_longlong(x), yb = __double_as_longlong(y);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)xb, (unsigned)yb, false, false);
  const auto hi =
      __builtin_amdgcn_permlane32_swap((unsigned)(xb >> 32), (unsigned)(yb >> 32), false, false);
  x = __longlong_as_double(((long long)hi[0] << 32) | (unsigned)lo[0]);
  y = __longlong_as_double(((long long)hi[1] << 32) | (unsigned)lo[1]);
}

// Sums over the 64 lanes of a wave of two per-lane values in one chain: the
// halves exchange and add, so that lanes 0-31 hold half-sums of v0 and lanes
// 32-63 of v1; row shifts by 1, 2, 4, 8 sum each row of 16 lanes, and the
// broadcast of lane 15 into rows 1 and 3 adds row 0 to row 1 and row 2 to
// row 3.  The total of v0 is valid in lane 31, that of v1 in lane 63: 18 VALU
// instructions for both, against 18 for each through wave_total63.  Needs
// every lane of the wave active.
__device__ __forceinline__ double wave_total2(double v0, double v1) {
  swap32_d(v0, v1);
  double t = v0 + v1;
  t += dpp_d<0x111, 0xf>(t);   // row_shr:1
  t += dpp_d<0x112, 0xf>(t);   // row_shr:2
  t += dpp_d<0x114, 0xf>(t);   // row_shr:4
  t += dpp_d<0x118, 0xf>(t);   // row_shr:8
  t += dpp_d<0x142, 0xa>(t);   // row_bcast:15 into rows 1 and 3
  return t;
}

// Adds the two wave totals of wave_total2 to slots s0 and s1 of the wave's LDS
// row (a slot < 0: none) with adds that return nothing, lanes 31 and 63.
__device__ __forceinline__ void wave_deposit2(double *row, int s0, int s1, double t, int lane) {
  const int slot = lane == 31 ? s0 : s1;
  if ((lane == 31 || lane == 63) && slot >= 0) atomicAdd(&row[slot], t);
}

template <typename T, int M, int R, int NS>
__global__ void __launch_bounds__(1 << (M - R)) k_sweep(SweepArgs a) {
  constexpr int NT = 1 << (M - R);
  constexpr int G = 1 << R;
  constexpr int VN = V4T<T>::N;
  constexpr int LV = VN == 2 ? 1 : 2;
  constexpr int NIT = (1 << M) / (VN * NT);   // vector loads per thread per plane (full tile)
  constexpr int NWAVE = (NT + 63) / 64;
  using C2 = typename C2T<T>::type;
  using V4 = typename V4T<T>::type;
  __shared__ C2 lds[NS][1 << M];
  __shared__ double wsum[NS == 2 ? NWAVE : 1][NS == 2 ? SVI_GSLOTS : 1];
  __shared__ double gacc[NS == 2 ? SVI_GSLOTS : 1];
  __shared__ int32_t hb_s[SVI_MMAX];

  const int tid = threadIdx.x;
  const int m = a.m, c = a.c, nh = a.nh;
  const int mm = m > R ? m : R;              // tile bits including phantom padding
  const int ntile_el = 1 << m;               // real amplitudes per tile
  const int ngroups = 1 << (mm - R);
  const bool vec = c >= LV;                  // rows hold whole 16-byte vectors

  if (tid < SVI_MMAX) hb_s[tid] = a.hb[tid < nh ? tid : 0];
  if constexpr (NS == 2) {
    for (int s = tid; s < SVI_GSLOTS; s += NT) gacc[s] = 0.0;
  }
  __syncthreads();

  // Row offsets of this thread's elements, the same for every tile.
  uint64_t roff[NIT];
#pragma unroll
  for (int k = 0; k < NIT; k++) {
    const int i = (tid + k * NT) * (vec ? VN : 1);
    roff[k] = spread_row(i >> c, hb_s, nh) + (uint64_t)(i & ((1 << c) - 1));
  }

  const int tsw = swz<T>(tid * VN);          // swizzled slot of this thread's first element
  T *const pre0 = (T *)a.re, *const pim0 = (T *)a.im;
  T *const pre1 = (T *)a.re2, *const pim1 = (T *)a.im2;

  for (int64_t tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
    const uint64_t base = tile_base(tile, c, hb_s, nh);
    // ---- load tile (rows of 2^c contiguous amplitudes) into LDS
    if (mm > m) {
      for (int i = tid; i < (1 << mm); i += NT) {
        lds[0][swz<T>(i)] = C2{0, 0};
        if constexpr (NS == 2) lds[1][swz<T>(i)] = C2{0, 0};
      }
      __syncthreads();
    }
#pragma unroll
    for (int s = 0; s < NS; s++) {
      const T *pr = s == 0 ? pre0 : pre1;
      const T *pi = s == 0 ? pim0 : pim1;
      if (s == 0 && (a.flags & SW_INIT_ZERO)) {
        for (int i = tid; i < ntile_el; i += NT) {
          const T v = (base == 0 && i == 0) ? (T)1 : (T)0;
          lds[0][swz<T>(i)] = C2{v, 0};
        }
      } else if (vec) {
#pragma unroll
        for (int k = 0; k < NIT; k++) {
          const int i = (tid + k * NT) * VN;
          if (i < ntile_el) {
            const uint64_t g = base + roff[k];
            const V4 vr = *(const V4 *)(pr + g);
            const V4 vi = *(const V4 *)(pi + g);
            const int si = tsw ^ swz<T>(k * NT * VN);
            if constexpr (VN == 2) {
              lds[s][si] = C2{vr.x, vi.x};
              lds[s][si ^ 1] = C2{vr.y, vi.y};
            } else {
              lds[s][si] = C2{vr.x, vi.x};
              lds[s][si ^ 1] = C2{vr.y, vi.y};
              lds[s][si ^ 2] = C2{vr.z, vi.z};
              lds[s][si ^ 3] = C2{vr.w, vi.w};
            }
          }
        }
      } else {
        for (int i = tid; i < ntile_el; i += NT) {
          const uint64_t g = base + spread_row(i >> c, hb_s, nh) + (uint64_t)(i & ((1 << c) - 1));
          lds[s][swz<T>(i)] = C2{pr[g], pi[g]};
        }
      }
    }
    __syncthreads();

    // ---- stages
    for (int st = a.stage_begin; st < a.stage_end; st++) {
      const SVI_CONST StageDesc &sd = cptr(a.stages)[st];
      // Every thread runs the stage (keeps wave shuffles uniform).  Threads
      // beyond the tile's groups work on LDS slots above 2^mm, which are
      // never written back.
      const bool active = tid < ngroups;
      const int gbs = swz<T>(stage_base<M, R>(tid, sd)) * (int)sizeof(C2);
      T re[NS][G], im[NS][G];
#pragma unroll
      for (int s = 0; s < NS; s++) {
        const char *lb = (const char *)lds[s];
#pragma unroll
        for (int j = 0; j < G; j++) {
          const C2 v = *(const C2 *)(lb + (gbs ^ sd.ld_off[j]));
          re[s][j] = v.x;
          im[s][j] = v.y;
        }
      }
      if (sd.kind == ST_KRON) {
        const SVI_CONST double *kc = cptr(a.coef) + sd.kcoef;
        if constexpr (NS == 2) {
          // gradient terms Im <lam| G |psi> at the stage point where each
          // record's generator commutes with the rest of the stage; terms taken
          // after the fast-Givens rotations see both states divided by the
          // stage scale s, so they are multiplied by s^2
          auto grads = [&](int b, int e, double mult) {
            for (int o = b; o < e; o++) {
              const MicroOp op = op_at(a.ops, o);
              double v = active ? mult * grad_kron<T, R>(op, re[0], im[0], re[1], im[1], a.coef) : 0.0;
              v = wave_sum(v);
              if ((tid & 63) == 0) wsum[tid >> 6][op.coef] = v;
            }
          };
          grads(sd.op_begin, sd.g1, 1.0);
          kron_pre<T, R>(re[0], im[0], kc, sd.dflags);
          kron_pre<T, R>(re[1], im[1], kc, sd.dflags);
          grads(sd.g1, sd.g2, 1.0);
          kron_rot<T, R>(re[0], im[0], kc, sd.rmask);
          kron_rot<T, R>(re[1], im[1], kc, sd.rmask);
          if (sd.g2 < sd.op_end) {
            const double sc = kc[4 * R + 4 * G];
            grads(sd.g2, sd.op_end, sc * sc);
          }
          kron_post<T, R>(re[0], im[0], kc, sd.dflags);
          kron_post<T, R>(re[1], im[1], kc, sd.dflags);
        } else {
          kron_stage<T, R>(re[0], im[0], kc, sd.rmask, sd.dflags);
        }
      } else
      for (int o = sd.op_begin; o < sd.op_end; o++) {
        const MicroOp op = op_at(a.ops, o);
        if constexpr (NS == 2) {
          if (op.type == MO_GRAD || op.type == MO_GRAD2L) {
            double v = active ? grad_any<T, R>(op, re[0], im[0], re[1], im[1], a.coef) : 0.0;
            v = wave_sum(v);
            if ((tid & 63) == 0) wsum[tid >> 6][op.coef] = v;
            continue;
          }
        }
        apply_op<T, R>(op, re[0], im[0], a.coef);
        if constexpr (NS == 2) apply_op<T, R>(op, re[1], im[1], a.coef);
      }
      if (sd.dflags & SD_XCHG) lds_barrier();
#pragma unroll
      for (int s = 0; s < NS; s++) {
        char *lb = (char *)lds[s];
#pragma unroll
        for (int j = 0; j < G; j++) *(C2 *)(lb + (gbs ^ sd.st_off[j])) = C2{re[s][j], im[s][j]};
      }
      __syncthreads();
    }

    if constexpr (NS == 2) {
      // fold this tile's per-wave sums into the workgroup accumulators
      for (int s = tid; s < a.n_gslots; s += NT) {
        double v = 0.0;
        for (int w = 0; w < NWAVE; w++) v += wsum[w][s];
        gacc[s] += v;
      }
    }

    // ---- store tile (through the output bit permutation of a remapping sweep)
    const bool operm = (a.flags & SW_OPERM) != 0;
#pragma unroll
    for (int s = 0; s < NS; s++) {
      T *pr = s == 0 ? pre0 : pre1;
      T *pi = s == 0 ? pim0 : pim1;
      if (vec) {
        const int so1 = operm ? swz<T>(perm_bits(1, a.operm, m)) : 1;
        const int so2 = operm ? swz<T>(perm_bits(2, a.operm, m)) : 2;
#pragma unroll
        for (int k = 0; k < NIT; k++) {
          const int i = (tid + k * NT) * VN;
          if (i < ntile_el) {
            const uint64_t g = base + roff[k];
            const int si = operm ? swz<T>(perm_bits(i, a.operm, m)) : tsw ^ swz<T>(k * NT * VN);
            V4 vr, vi;
            if constexpr (VN == 2) {
              const C2 p0 = lds[s][si], p1 = lds[s][si ^ so1];
              vr = V4{p0.x, p1.x};
              vi = V4{p0.y, p1.y};
            } else {
              const C2 p0 = lds[s][si], p1 = lds[s][si ^ so1];
              const C2 p2 = lds[s][si ^ so2], p3 = lds[s][si ^ so1 ^ so2];
              vr = V4{p0.x, p1.x, p2.x, p3.x};
              vi = V4{p0.y, p1.y, p2.y, p3.y};
            }
            *(V4 *)(pr + g) = vr;
            *(V4 *)(pi + g) = vi;
          }
        }
      } else {
        for (int i = tid; i < ntile_el; i += NT) {
          const uint64_t g = base + spread_row(i >> c, hb_s, nh) + (uint64_t)(i & ((1 << c) - 1));
          const C2 p = lds[s][swz<T>(operm ? perm_bits(i, a.operm, m) : i)];
          pr[g] = p.x;
          pi[g] = p.y;
        }
      }
    }
    __syncthreads();
  }

  if constexpr (NS == 2) {
    for (int s = tid; s < a.n_gslots; s += NT)
      a.gpart[(int64_t)(a.gslot_begin + s) * gridDim.x + blockIdx.x] = gacc[s];
  }
}


// ------------------------------------------------- Kronecker-only sweep
// Lean variant for sweeps whose every stage is a Kronecker stage.  Stage
// descriptors and coefficients are uniform and read with scalar loads; LDS
// holds only the tile, and the code holds only the static stage body, so the
// register groups stay in VGPRs with no interpreter paths competing for them.

// Tile order: XCD-aware.  Workgroup b runs on XCD b % 8; in every round the
// workgroups of one XCD take a contiguous run of tiles, so tiles that share
// HBM lines and DRAM pages are fetched through the same L2 at the same time.
__device__ __forceinline__ int64_t tile_of(int64_t round_base, int b, int grid) {
  const int per = grid >> 3;
  return grid >= 8 && (grid & 7) == 0 ? round_base + (int64_t)(b & 7) * per + (b >> 3)
                                      : round_base + b;
}

template <typename T, int M, int R>
__global__ void __launch_bounds__(1 << (M - R)) k_sweep_kron(SweepArgs a) {
  constexpr int NT = 1 << (M - R);
  constexpr int G = 1 << R;
  using C2 = typename C2T<T>::type;
  // Per-stage thread bases (tile-local slot offset of the thread's register
  // group) depend on the thread and the stage, not on the tile: the first
  // GTAB stages take theirs from a table built once per launch in the LDS
  // the tile leaves free (sized so the workgroups per CU stay as they are).
  constexpr int TILE_BYTES = (1 << M) * (int)sizeof(C2);
  constexpr int GTAB_BYTES = TILE_BYTES >= 131072 ? 30720 : TILE_BYTES >= 65536 ? 14336 : 6144;
  constexpr int GTAB = GTAB_BYTES / (2 * NT) > 0 ? GTAB_BYTES / (2 * NT) : 1;
  __shared__ C2 lds[1 << M];
  __shared__ int32_t hb_s[SVI_MMAX];
  __shared__ uint16_t gtab[GTAB * NT];   // swizzled element index (tiles hold <= 2^14)

  const int tid = threadIdx.x;
  const int m = a.m, c = a.c, nh = a.nh;
  const int ntile_el = 1 << m;
  const bool init0 = (a.flags & SW_INIT_ZERO) != 0;
  const SVI_CONST StageDesc *stages = cptr(a.stages + a.stage_begin);
  const int nst = a.stage_end - a.stage_begin;
  const SVI_CONST double *coef = cptr(a.coef);

  if (tid < SVI_MMAX) hb_s[tid] = a.hb[tid < nh ? tid : 0];
  const int ntab = nst < GTAB ? nst : GTAB;
  for (int st = 0; st < ntab; st++)   // each thread reads back only its own entries
    gtab[st * NT + tid] = (uint16_t)swz<T>(stage_base<M, R>(tid, stages[st]));
  __syncthreads();

  // Lane tid moves tile elements i = tid + k * NT (k < G) between HBM and
  // LDS, one amplitude per access: consecutive lanes take consecutive
  // addresses along the tile's contiguous qubits, and every loaded value is
  // already the register that the (re, im) LDS write takes.  (Loading pairs
  // of amplitudes of one plane would need a register shuffle into (re, im)
  // pairs, which the compiler places, with a wait for the load, right after
  // the load.)
  //
  // Element i sits at tile_base + tile_off(i); tile_off is a bit deposit, so
  // it splits over the disjoint bit fields of tid and k * NT into a per-lane
  // part and wave-uniform parts.  Past the end of a small tile (i >= 2^m) the
  // deposit drops the missing tile bits, so the address stays inside the tile:
  // loads there are issued (and discarded) rather than branched around, and
  // stores are skipped.
  const uint64_t loff = tile_off(tid, c, hb_s, nh);
  uint64_t kb[R];
#pragma unroll
  for (int r = 0; r < R; r++) kb[r] = tile_off(NT << r, c, a.hb, nh);
  uint64_t loff_p;
  auto goff = [&](int k) {
    uint64_t o = loff_p;
#pragma unroll
    for (int r = 0; r < R; r++)
      if ((k >> r) & 1) o += kb[r];
    return o;
  };
  // LDS slots: element i is written to swz(i) and, for the store, read from
  // swz(P(i)) with P the identity or the output bit permutation of a
  // remapping sweep; swz and P are linear over XOR, so each is a per-lane
  // slot XOR wave-uniform parts.
  const bool operm = (a.flags & SW_OPERM) != 0;
  const int tsl = swz<T>(tid);
  const int ssl = swz<T>(operm ? perm_bits(tid, a.operm, m) : tid);
  int wsb[R], ssb[R];
#pragma unroll
  for (int r = 0; r < R; r++) {
    wsb[r] = swz<T>(NT << r);
    ssb[r] = swz<T>(operm ? perm_bits(NT << r, a.operm, m) : NT << r);
  }
  auto slot = [&](int base, const int *sb, int k) {
    int o = base;
#pragma unroll
    for (int r = 0; r < R; r++)
      if ((k >> r) & 1) o ^= sb[r];
    return o;
  };
  T *const pre = (T *)a.re, *const pim = (T *)a.im;
  char *const lb = (char *)lds;
  // tile t's base: t's bits deposited on the qubits outside the tile (for a
  // sparse sweep, on those of them inside the support only)
  const bool sparse = (a.flags & SW_SPARSE) != 0;
  auto tbase = [&](int64_t t) {
    return sparse ? tile_base(t, c, a.bz, a.nbz) : tile_base(t, c, hb_s, nh);
  };
  // The per-lane bases are re-declared opaque before each phase, so the
  // compiler recomputes the (cheap) per-element addresses next to their use
  // instead of hoisting all of them out of the tile loop and spilling them:
  // a scratch reload would wait on every outstanding HBM access.
  loff_p = loff;
  int tsl_p = tsl, ssl_p = ssl;
  auto opaque = [](auto &v) { asm volatile("" : "+v"(v)); };

  // Software pipeline: the next tile's HBM loads are issued into registers
  // before the current tile's stages run, so their latency hides behind the
  // LDS / VALU work, and the current tile's stores drain behind the next
  // tile's stages.  Inside the loop the next tile enters LDS after this
  // tile's stores, on one straight path: every HBM access sits in fixed-count
  // unrolled code, so the wait for the loads leaves the stores (issued after
  // them) in flight.  The loop is instantiated separately for a sweep that
  // synthesises |0..0> (no loads), so neither copy merges a path with loads
  // in flight into one without.  A full tile (m == M, every n >= M) takes a
  // copy with no per-element guards, so no HBM access or LDS write sits
  // under a lane branch whose skipped path would make the waits conservative.
  auto run = [&](auto synth, auto full) {
    constexpr bool I0 = decltype(synth)::value;
    constexpr bool FULL = decltype(full)::value;
    T nr[G], ni[G];
    auto fetch = [&](int64_t t) {
      const uint64_t b0 = tbase(t);
#pragma unroll
      for (int k = 0; k < G; k++) {
        const uint64_t g = b0 + goff(k);
        nr[k] = pre[g];
        ni[k] = pim[g];
      }
    };
    auto tile_in = [&](int64_t t) {
      opaque(tsl_p);
#pragma unroll
      for (int k = 0; k < G; k++) {
        if (FULL || tid + k * NT < ntile_el) {
          if constexpr (I0) {
            const T v = (t == 0 && tid + k * NT == 0) ? (T)1 : (T)0;
            lds[slot(tsl_p, wsb, k)] = C2{v, 0};
          } else {
            lds[slot(tsl_p, wsb, k)] = C2{nr[k], ni[k]};
          }
        }
      }
    };
    // Prefetch distance one tile: the loads of tile t+1 are issued right after
    // tile t enters LDS (in the same straight-line block that consumed the
    // previous prefetch registers, so no wait precedes them) and run behind
    // tile t's stages; tile t's stores drain behind tile t+1's stages.
    int64_t r0 = 0;
    int64_t tile = tile_of(0, blockIdx.x, gridDim.x);
    if (tile >= a.ntiles) return;
    int64_t next = tile_of(r0 + gridDim.x, blockIdx.x, gridDim.x);
    if constexpr (!I0) fetch(tile);
    tile_in(tile);
    lds_barrier();
    if constexpr (!I0) {
      if (next < a.ntiles) {
        opaque(loff_p);
        fetch(next);
      }
    }

    while (true) {
      const uint64_t base = tbase(tile);
      // From |0..0> only tile 0 holds a nonzero amplitude, and a sweep's
      // gates act within tiles, so every other tile stays zero: it skips the
      // stages and is written as zeros (uniform over the workgroup).
      const bool live = !I0 || tile == 0;
      // ---- stages
      for (int st = 0; live && st < nst; st++) {
        const SVI_CONST StageDesc &sd = stages[st];
        const int gbs =
            (st < ntab ? (int)gtab[st * NT + tid] : swz<T>(stage_base<M, R>(tid, sd))) * (int)sizeof(C2);
        // The common stage (every group bit rotated, then D_after) runs as its
        // own straight-line body from loads to stores; the general body
        // branches on the stage's parts.  Separate bodies leave nothing to
        // merge, so neither pays register copies for the other's branches.
        auto body = [&](auto full_stage) {
          T re[G], im[G];
#pragma unroll
          for (int j = 0; j < G; j++) {
            const C2 v = *(const C2 *)(lb + (gbs ^ sd.ld_off[j]));
            re[j] = v.x;
            im[j] = v.y;
          }
          if constexpr (decltype(full_stage)::value) {
            kron_rot_all<T, R>(re, im, coef + sd.kcoef);
            mo_diagt<T, R>(re, im, coef + sd.kcoef + 4 * R + 2 * G);
          } else {
            kron_stage<T, R>(re, im, coef + sd.kcoef, sd.rmask, sd.dflags);
          }
          if (sd.dflags & SD_XCHG) lds_barrier();
#pragma unroll
          for (int j = 0; j < G; j++) *(C2 *)(lb + (gbs ^ sd.st_off[j])) = C2{re[j], im[j]};
        };
        if (sd.rmask == (1u << R) - 1 && (sd.dflags & 7) == 2)
          body(std::true_type{});
        else
          body(std::false_type{});
        if (sd.dflags & SD_WLOCAL) {
          // the next stage reads only slots this wave wrote: keep the wave's
          // LDS accesses in order, no workgroup barrier
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
        } else {
          lds_barrier();
        }
      }
      // ---- LDS to HBM
      opaque(ssl_p);
      opaque(loff_p);
      if (live) {
#pragma unroll
        for (int k = 0; k < G; k++) {
          if (FULL || tid + k * NT < ntile_el) {
            const C2 p = lds[slot(ssl_p, ssb, k)];
            const uint64_t g = base + goff(k);
            pre[g] = p.x;
            pim[g] = p.y;
          }
        }
      } else {
#pragma unroll
        for (int k = 0; k < G; k++) {
          if (FULL || tid + k * NT < ntile_el) {
            const uint64_t g = base + goff(k);
            pre[g] = (T)0;
            pim[g] = (T)0;
          }
        }
      }
      lds_barrier();
      if (next >= a.ntiles) break;
      // ---- next tile into LDS (a synthesised sweep's later tiles are zero:
      // nothing to stage), then the prefetch of the one after
      if (!I0) tile_in(next);
      lds_barrier();
      r0 += gridDim.x;
      tile = next;
      next = tile_of(r0 + gridDim.x, blockIdx.x, gridDim.x);
      if constexpr (!I0) {
        if (next < a.ntiles) {
          opaque(loff_p);
          fetch(next);
        }
      }
    }
  };
  if (m == M) {
    if (init0)
      run(std::true_type{}, std::true_type{});
    else
      run(std::false_type{}, std::true_type{});
  } else {
    if (init0)
      run(std::true_type{}, std::false_type{});
    else
      run(std::false_type{}, std::false_type{});
  }
}

// ------------------------------------------------ tile sweep, one workgroup
// Tiles [t0, t1) of one sweep of one state, run by one workgroup of 2^(M-R)
// threads through the LDS tile `lt` (2^M amplitudes) with the tile's
// high-bit table staged in `hb` (LDS, SVI_MMAX entries).  No qubit remapping
// on the way out (SW_OPERM is not taken).  KO: every stage is a Kronecker
// stage (no micro-op interpreter in the caller's kernel).
template <typename T, int M, int R, bool KO>
__device__ void sweep_tiles(const SVI_CONST SweepArgs &a, int64_t t0, int64_t t1,
                            typename C2T<T>::type *lt, int32_t *hb) {
  constexpr int NT = 1 << (M - R);
  constexpr int G = 1 << R;
  constexpr int VN = V4T<T>::N;
  constexpr int LV = VN == 2 ? 1 : 2;
  constexpr int NIT = (1 << M) / (VN * NT);
  using C2 = typename C2T<T>::type;
  using V4 = typename V4T<T>::type;
  const int tid = threadIdx.x;
  const int m = a.m, c = a.c, nh = a.nh;
  const int mm = m > R ? m : R;
  const int ntile_el = 1 << m;
  const bool vec = c >= LV;
  const bool init0 = (a.flags & SW_INIT_ZERO) != 0;
  const int st_begin = a.stage_begin, st_end = a.stage_end;
  const SVI_CONST StageDesc *stages = cptr(a.stages);
  const MicroOp *ops = a.ops;
  const double *coef = a.coef;
  T *const pre = (T *)a.re, *const pim = (T *)a.im;

  if (tid < SVI_MMAX) hb[tid] = a.hb[tid < nh ? tid : 0];
  __syncthreads();
  uint64_t roff[NIT];
#pragma unroll
  for (int k = 0; k < NIT; k++) {
    const int i = (tid + k * NT) * (vec ? VN : 1);
    roff[k] = spread_row(i >> c, hb, nh) + (uint64_t)(i & ((1 << c) - 1));
  }
  const int tsw = swz<T>(tid * VN);
  char *const lb = (char *)lt;

  // tile bases: a sparse sweep deposits the tile index on the support's
  // qubits outside the tile only (bz, read from the descriptor)
  const bool sparse = (a.flags & SW_SPARSE) != 0;
  for (int64_t tile = t0; tile < t1; tile++) {
    uint64_t base;
    if (sparse) {
      base = (uint64_t)tile << c;
      for (int k = 0; k < a.nbz; k++) {
        const int p = a.bz[k];
        base = ((base >> p) << (p + 1)) | (base & ((1ull << p) - 1ull));
      }
    } else {
      base = tile_base(tile, c, hb, nh);
    }
    if (init0 && base != 0) {
      // From |0..0> every tile but the one holding index 0 stays zero (a
      // sweep's gates act within tiles): it is written as zeros, with no
      // stages and no LDS (uniform over the workgroup)
      if (vec) {
        V4 z;
        if constexpr (VN == 2) z = V4{(T)0, (T)0};
        else z = V4{(T)0, (T)0, (T)0, (T)0};
#pragma unroll
        for (int k = 0; k < NIT; k++) {
          const int i = (tid + k * NT) * VN;
          if (i < ntile_el) {
            *(V4 *)(pre + base + roff[k]) = z;
            *(V4 *)(pim + base + roff[k]) = z;
          }
        }
      } else {
        for (int i = tid; i < ntile_el; i += NT) {
          const uint64_t g = base + spread_row(i >> c, hb, nh) + (uint64_t)(i & ((1 << c) - 1));
          pre[g] = (T)0;
          pim[g] = (T)0;
        }
      }
      continue;
    }
    if (mm > m) {
      // tiles smaller than one register group: padding slots hold zeros
      for (int i = tid; i < (1 << mm); i += NT) lt[swz<T>(i)] = C2{0, 0};
      __syncthreads();
    }
    if (init0) {
      for (int i = tid; i < ntile_el; i += NT) {
        const T v = (base == 0 && i == 0) ? (T)1 : (T)0;
        lt[swz<T>(i)] = C2{v, 0};
      }
    } else if (vec) {
#pragma unroll
      for (int k = 0; k < NIT; k++) {
        const int i = (tid + k * NT) * VN;
        if (i < ntile_el) {
          const uint64_t g = base + roff[k];
          const V4 vr = *(const V4 *)(pre + g);
          const V4 vi = *(const V4 *)(pim + g);
          const int si = tsw ^ swz<T>(k * NT * VN);
          if constexpr (VN == 2) {
            lt[si] = C2{vr.x, vi.x};
            lt[si ^ 1] = C2{vr.y, vi.y};
          } else {
            lt[si] = C2{vr.x, vi.x};
            lt[si ^ 1] = C2{vr.y, vi.y};
            lt[si ^ 2] = C2{vr.z, vi.z};
            lt[si ^ 3] = C2{vr.w, vi.w};
          }
        }
      }
    } else {
      for (int i = tid; i < ntile_el; i += NT) {
        const uint64_t g = base + spread_row(i >> c, hb, nh) + (uint64_t)(i & ((1 << c) - 1));
        lt[swz<T>(i)] = C2{pre[g], pim[g]};
      }
    }
    __syncthreads();

    for (int st = st_begin; st < st_end; st++) {
      const SVI_CONST StageDesc &sd = stages[st];
      const int gbs = swz<T>(stage_base<M, R>(tid, sd)) * (int)sizeof(C2);
      // a full Kronecker stage (every group bit rotated, then D_after) runs as
      // its own straight-line body, loads to stores; the general body branches
      auto body = [&](auto full_stage) {
        T re[G], im[G];
#pragma unroll
        for (int j = 0; j < G; j++) {
          const C2 v = *(const C2 *)(lb + (gbs ^ sd.ld_off[j]));
          re[j] = v.x;
          im[j] = v.y;
        }
        if constexpr (decltype(full_stage)::value) {
          kron_rot_all<T, R>(re, im, cptr(coef) + sd.kcoef);
          mo_diagt<T, R>(re, im, cptr(coef) + sd.kcoef + 4 * R + 2 * G);
        } else if (KO || sd.kind == ST_KRON) {
          kron_stage<T, R>(re, im, cptr(coef) + sd.kcoef, sd.rmask, sd.dflags);
        } else {
          for (int o = sd.op_begin; o < sd.op_end; o++) {
            const MicroOp op = op_at(ops, o);
            apply_op<T, R>(op, re, im, coef);
          }
        }
        if (sd.dflags & SD_XCHG) __syncthreads();
#pragma unroll
        for (int j = 0; j < G; j++) *(C2 *)(lb + (gbs ^ sd.st_off[j])) = C2{re[j], im[j]};
      };
      if (sd.kind == ST_KRON && sd.rmask == (1u << R) - 1 && (sd.dflags & 7) == 2)
        body(std::true_type{});
      else
        body(std::false_type{});
      __syncthreads();
    }

    if (vec) {
#pragma unroll
      for (int k = 0; k < NIT; k++) {
        const int i = (tid + k * NT) * VN;
        if (i < ntile_el) {
          const uint64_t g = base + roff[k];
          const int si = tsw ^ swz<T>(k * NT * VN);
          V4 vr, vi;
          if constexpr (VN == 2) {
            const C2 p0 = lt[si], p1 = lt[si ^ 1];
            vr = V4{p0.x, p1.x};
            vi = V4{p0.y, p1.y};
          } else {
            const C2 p0 = lt[si], p1 = lt[si ^ 1], p2 = lt[si ^ 2], p3 = lt[si ^ 3];
            vr = V4{p0.x, p1.x, p2.x, p3.x};
            vi = V4{p0.y, p1.y, p2.y, p3.y};
          }
          *(V4 *)(pre + g) = vr;
          *(V4 *)(pim + g) = vi;
        }
      }
    } else {
      for (int i = tid; i < ntile_el; i += NT) {
        const uint64_t g = base + spread_row(i >> c, hb, nh) + (uint64_t)(i & ((1 << c) - 1));
        const C2 p = lt[swz<T>(i)];
        pre[g] = p.x;
        pim[g] = p.y;
      }
    }
    __syncthreads();
  }
  // a zero tile ends without the barrier above, and a caller's next sweep
  // starts by rewriting hb, which the last tiles' addresses were read from
  if (init0) __syncthreads();
}

// ------------------------------------------- two-state Kronecker stage
// One Kronecker stage applied to the psi and lambda tiles held side by side in
// LDS (lb0, lb1), with the gradient terms Im <lam| G |psi> of the stage's
// gradient micro-ops taken at the three stage points (stage input, after
// D_before, after the rotations).  Terms go through in pairs: sink(s0, s1, t)
// receives the pair's wave_total2 result t and the pair's slots (s1 = -1: a
// single term), uniform across the wave.  Ends with the barrier (or the wave
// fence of a wave-local stage) that makes the stores visible to the next stage.
template <typename T, int R, typename Sink>
__device__ __forceinline__ void kron2_stage(char *lb0, char *lb1, int gbs,
                                            const SVI_CONST StageDesc &sd,
                                            const SVI_CONST double *coef, const MicroOp *ops,
                                            const double *gcoef, bool active, Sink &&sink) {
  constexpr int G = 1 << R;
  using C2 = typename C2T<T>::type;
  char *const lb[2] = {lb0, lb1};
  T re[2][G], im[2][G];
#pragma unroll
  for (int s = 0; s < 2; s++) {
#pragma unroll
    for (int j = 0; j < G; j++) {
      const C2 v = *(const C2 *)(lb[s] + (gbs ^ sd.ld_off[j]));
      re[s][j] = v.x;
      im[s][j] = v.y;
    }
  }
  const SVI_CONST double *kc = coef + sd.kcoef;
  auto grads = [&](int b, int e, double mult, int point) {
    // two terms at a time, summed over the wave in one chain of lane moves
    // (groups of four, in any arrangement, measured slower)
    if ((sd.gdiag >> point) & 1) {
      // every generator here is diagonal: one array of the products
      // Im(conj(lam_j) psi_j), then a dot product with each term's table
      double fz[G];
#pragma unroll
      for (int j = 0; j < G; j++)
        fz[j] = (double)re[1][j] * (double)im[0][j] - (double)im[1][j] * (double)re[0][j];
      auto dot = [&](const MicroOp &op) {
        const SVI_CONST double *tab = cptr(gcoef) + op.t0;
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < G; j++) acc += (double)tab[j] * fz[j];
        return acc;
      };
      int o = b;
#pragma clang loop unroll(disable)
      for (; o + 1 < e; o += 2) {
        const MicroOp op0 = op_at(ops, o), op1 = op_at(ops, o + 1);
        const double v0 = active ? mult * dot(op0) : 0.0;
        const double v1 = active ? mult * dot(op1) : 0.0;
        sink(op0.coef, op1.coef, wave_total2(v0, v1));
      }
      if (o < e) {
        const MicroOp op = op_at(ops, o);
        sink(op.coef, -1, wave_total2(active ? mult * dot(op) : 0.0, 0.0));
      }
      return;
    }
    int o = b;
#pragma clang loop unroll(disable)
    for (; o + 1 < e; o += 2) {
      const MicroOp op0 = op_at(ops, o), op1 = op_at(ops, o + 1);
      const double v0 = active ? mult * grad_kron<T, R>(op0, re[0], im[0], re[1], im[1], gcoef) : 0.0;
      const double v1 = active ? mult * grad_kron<T, R>(op1, re[0], im[0], re[1], im[1], gcoef) : 0.0;
      sink(op0.coef, op1.coef, wave_total2(v0, v1));
    }
    if (o < e) {
      const MicroOp op = op_at(ops, o);
      const double v = active ? mult * grad_kron<T, R>(op, re[0], im[0], re[1], im[1], gcoef) : 0.0;
      sink(op.coef, -1, wave_total2(v, 0.0));
    }
  };
  grads(sd.op_begin, sd.g1, 1.0, 0);
  kron_pre<T, R>(re[0], im[0], kc, sd.dflags);
  kron_pre<T, R>(re[1], im[1], kc, sd.dflags);
  grads(sd.g1, sd.g2, 1.0, 1);
  kron_rot<T, R>(re[0], im[0], kc, sd.rmask);
  kron_rot<T, R>(re[1], im[1], kc, sd.rmask);
  if (sd.g2 < sd.op_end) {
    const double sc = kc[4 * R + 4 * G];
    grads(sd.g2, sd.op_end, sc * sc, 2);
  }
  kron_post<T, R>(re[0], im[0], kc, sd.dflags);
  kron_post<T, R>(re[1], im[1], kc, sd.dflags);
  if (sd.dflags & SD_XCHG) lds_barrier();
#pragma unroll
  for (int s = 0; s < 2; s++) {
#pragma unroll
    for (int j = 0; j < G; j++) *(C2 *)(lb[s] + (gbs ^ sd.st_off[j])) = C2{re[s][j], im[s][j]};
  }
  if (sd.dflags & SD_WLOCAL) {
    // the next stage reads only slots this wave wrote
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
  } else {
    lds_barrier();
  }
}

// One micro-op stage (the interpreter) applied to the psi and lambda tiles
// in LDS: each gate micro-op acts on both states, each gradient micro-op sends
// its term Im <lam| G |psi> to sink(slot, -1, wave total) at its place in the
// stage.
// Ends with the barrier that makes the stores visible to the next stage.
template <typename T, int R, typename Sink>
__device__ __forceinline__ void ops2_stage(char *lb0, char *lb1, int gbs,
                                           const SVI_CONST StageDesc &sd, const MicroOp *ops,
                                           const double *coef, bool active, Sink &&sink) {
  constexpr int G = 1 << R;
  using C2 = typename C2T<T>::type;
  char *const lb[2] = {lb0, lb1};
  T re[2][G], im[2][G];
#pragma unroll
  for (int s = 0; s < 2; s++) {
#pragma unroll
    for (int j = 0; j < G; j++) {
      const C2 v = *(const C2 *)(lb[s] + (gbs ^ sd.ld_off[j]));
      re[s][j] = v.x;
      im[s][j] = v.y;
    }
  }
  for (int o = sd.op_begin; o < sd.op_end; o++) {
    const MicroOp op = op_at(ops, o);
    if (op.type == MO_GRAD || op.type == MO_GRAD2L) {
      const double v = active ? grad_any<T, R>(op, re[0], im[0], re[1], im[1], coef) : 0.0;
      sink(op.coef, -1, wave_total2(v, 0.0));
      continue;
    }
    apply_op<T, R>(op, re[0], im[0], coef);
    apply_op<T, R>(op, re[1], im[1], coef);
  }
  if (sd.dflags & SD_XCHG) lds_barrier();
#pragma unroll
  for (int s = 0; s < 2; s++) {
#pragma unroll
    for (int j = 0; j < G; j++) *(C2 *)(lb[s] + (gbs ^ sd.st_off[j])) = C2{re[s][j], im[s][j]};
  }
  lds_barrier();
}

// ------------------------------------------- two-state Kronecker sweep
// Adjoint backward sweeps whose every stage is a Kronecker stage: psi and
// lambda tiles side by side in LDS, the stage applied to both, and the
// gradient terms Im <lam| G |psi> taken at the three stage points (stage
// input, after D_before, after the rotations) and reduced per workgroup.
template <typename T, int M, int R>
__global__ void __launch_bounds__(1 << (M - R)) k_sweep_kron2(SweepArgs a) {
  constexpr int NT = 1 << (M - R);
  constexpr int G = 1 << R;
  constexpr int VN = V4T<T>::N;
  constexpr int NIT = (1 << M) / (VN * NT);
  constexpr int NWAVE = NT / 64;
  using C2 = typename C2T<T>::type;
  using V4 = typename V4T<T>::type;
  // per-stage thread bases from a table built once per launch (as in
  // k_sweep_kron), in the LDS left by the tiles and the per-wave sums within
  // the workgroup's share of the CU (one workgroup per CU for 128 KiB of
  // tiles, two for 64 KiB)
  constexpr int TILE_BYTES = 2 * (1 << M) * (int)sizeof(C2);
  constexpr int WG_LDS = TILE_BYTES >= 131072 ? 163840 : TILE_BYTES >= 65536 ? 81920 : 40960;
  constexpr int GTAB_BYTES = WG_LDS - TILE_BYTES - NWAVE * SVI_GSLOTS_WIDE * 8 - 4 * SVI_MMAX - 256;
  constexpr int GTAB = GTAB_BYTES / (4 * NT) > 0 ? GTAB_BYTES / (4 * NT) : 1;
  __shared__ C2 lds[2][1 << M];
  __shared__ double wacc[NWAVE][SVI_GSLOTS_WIDE];   // per-wave sums of the gradient slots
  __shared__ int32_t hb_s[SVI_MMAX];
  __shared__ int32_t gtab[GTAB * NT];

  const int tid = threadIdx.x;
  const int m = a.m, c = a.c, nh = a.nh;
  const int ntile_el = 1 << m;
  const bool vec = c >= (VN == 2 ? 1 : 2);
  const SVI_CONST StageDesc *stages = cptr(a.stages + a.stage_begin);
  const int nst = a.stage_end - a.stage_begin;
  const SVI_CONST double *coef = cptr(a.coef);

  if (tid < SVI_MMAX) hb_s[tid] = a.hb[tid < nh ? tid : 0];
  const int ntab = nst < GTAB ? nst : GTAB;
  for (int st = 0; st < ntab; st++)   // each thread reads back only its own entries
    gtab[st * NT + tid] = swz<T>(stage_base<M, R>(tid, stages[st])) * (int)sizeof(C2);
  for (int k = tid; k < NWAVE * SVI_GSLOTS_WIDE; k += NT) (&wacc[0][0])[k] = 0.0;
  __syncthreads();

  uint64_t roff[NIT];
#pragma unroll
  for (int k = 0; k < NIT; k++) {
    const int i = (tid + k * NT) * (vec ? VN : 1);
    roff[k] = spread_row(i >> c, hb_s, nh) + (uint64_t)(i & ((1 << c) - 1));
  }
  const int tsw = swz<T>(tid * VN);
  T *const pr[2] = {(T *)a.re, (T *)a.re2};
  T *const pi[2] = {(T *)a.im, (T *)a.im2};

  int64_t r0 = 0;
  for (int64_t tile = tile_of(0, blockIdx.x, gridDim.x); tile < a.ntiles;) {
    const uint64_t base = tile_base(tile, c, hb_s, nh);
    // ---- both tiles into LDS
#pragma unroll
    for (int s = 0; s < 2; s++) {
      if (vec) {
#pragma unroll
        for (int k = 0; k < NIT; k++) {
          const int i = (tid + k * NT) * VN;
          if (i < ntile_el) {
            const uint64_t g = base + roff[k];
            const V4 vr = *(const V4 *)(pr[s] + g);
            const V4 vi = *(const V4 *)(pi[s] + g);
            const int si = tsw ^ swz<T>(k * NT * VN);
            if constexpr (VN == 2) {
              lds[s][si] = C2{vr.x, vi.x};
              lds[s][si ^ 1] = C2{vr.y, vi.y};
            } else {
              lds[s][si] = C2{vr.x, vi.x};
              lds[s][si ^ 1] = C2{vr.y, vi.y};
              lds[s][si ^ 2] = C2{vr.z, vi.z};
              lds[s][si ^ 3] = C2{vr.w, vi.w};
            }
          }
        }
      } else {
        for (int i = tid; i < ntile_el; i += NT) {
          const uint64_t g = base + spread_row(i >> c, hb_s, nh) + (uint64_t)(i & ((1 << c) - 1));
          lds[s][swz<T>(i)] = C2{pr[s][g], pi[s][g]};
        }
      }
    }
    lds_barrier();
    // ---- stages
    for (int st = 0; st < nst; st++) {
      const SVI_CONST StageDesc &sd = stages[st];
      const int gbs =
          st < ntab ? gtab[st * NT + tid] : swz<T>(stage_base<M, R>(tid, sd)) * (int)sizeof(C2);
      const bool active = tid < (1 << (m > R ? m - R : 0));
      kron2_stage<T, R>((char *)lds[0], (char *)lds[1], gbs, sd, coef, a.ops, a.coef, active,
                        [&](int s0, int s1, double t) {
        // this tile's wave totals into the wave's LDS rows of their slots
        // (LDS adds without return: the wave does not wait)
        wave_deposit2(wacc[tid >> 6], s0, s1, t, tid & 63);
      });
    }
    // ---- LDS to HBM
#pragma unroll
    for (int s = 0; s < 2; s++) {
      if (vec) {
#pragma unroll
        for (int k = 0; k < NIT; k++) {
          const int i = (tid + k * NT) * VN;
          if (i < ntile_el) {
            const uint64_t g = base + roff[k];
            const int si = tsw ^ swz<T>(k * NT * VN);
            V4 vr, vi;
            if constexpr (VN == 2) {
              const C2 p0 = lds[s][si], p1 = lds[s][si ^ 1];
              vr = V4{p0.x, p1.x};
              vi = V4{p0.y, p1.y};
            } else {
              const C2 p0 = lds[s][si], p1 = lds[s][si ^ 1], p2 = lds[s][si ^ 2], p3 = lds[s][si ^ 3];
              vr = V4{p0.x, p1.x, p2.x, p3.x};
              vi = V4{p0.y, p1.y, p2.y, p3.y};
            }
            *(V4 *)(pr[s] + g) = vr;
            *(V4 *)(pi[s] + g) = vi;
          }
        }
      } else {
        for (int i = tid; i < ntile_el; i += NT) {
          const uint64_t g = base + spread_row(i >> c, hb_s, nh) + (uint64_t)(i & ((1 << c) - 1));
          const C2 p = lds[s][swz<T>(i)];
          pr[s][g] = p.x;
          pi[s][g] = p.y;
        }
      }
    }
    __syncthreads();
    r0 += gridDim.x;
    tile = tile_of(r0, blockIdx.x, gridDim.x);
  }
  __syncthreads();
  for (int sl = tid; sl < a.n_gslots; sl += NT) {
    double v = 0.0;
    for (int w = 0; w < NWAVE; w++) v += wacc[w][sl];
    a.gpart[(int64_t)(a.gslot_begin + sl) * gridDim.x + blockIdx.x] = v;
  }
}

}  // namespace svk
