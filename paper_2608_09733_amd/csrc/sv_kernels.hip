// gfx950 kernels of the state-vector library.
//
// State layout in HBM: two planes (re, im) of 2^n elements (double for
// complex128, float for complex64).  Gate action follows the paper's gather /
// multiply / scatter over the amplitudes that differ only on the targets
// (Section 5.3), but indices are computed by bit insertion instead of an index
// table, and many gates are applied per HBM round trip (see sv_internal.h).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sv_internal.h"

namespace {

template <typename T> struct C2T;
template <> struct C2T<double> { using type = double2; };
template <> struct C2T<float> { using type = float2; };

template <typename T> struct V4T;   // 16-byte global vector of T
template <> struct V4T<double> { using type = double2; static constexpr int N = 2; };
template <> struct V4T<float> { using type = float4; static constexpr int N = 4; };

// LDS swizzle: xor the low B bits of the element index with a fold of its
// higher bits, so that lanes whose indices differ only in higher bits land in
// different banks.  Bijective because the higher bits are unchanged.
template <typename T>
__device__ __forceinline__ int swz(int i) {
  constexpr int B = sizeof(T) == 8 ? 3 : 4;
  constexpr int MSK = (1 << B) - 1;
  int h = (i >> B) ^ (i >> (2 * B)) ^ (i >> (3 * B)) ^ (i >> (4 * B));
  return i ^ (h & MSK);
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

// Base index of tile `tile`: zeros inserted at the tile's qubits (0..c-1 and hb).
__device__ __forceinline__ uint64_t tile_base(int64_t tile, int c, const int32_t *hb, int nh) {
  uint64_t x = (uint64_t)tile << c;
  return insert_zeros64(x, hb, nh);
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

template <typename T, int R>
__device__ __forceinline__ void mo_diagt(T *re, T *im, const double *cf) {
#pragma unroll
  for (int j = 0; j < (1 << R); j++) {
    const T dr = (T)cf[2 * j], di = (T)cf[2 * j + 1];
    const T xr = re[j], xi = im[j];
    re[j] = xr * dr - xi * di;
    im[j] = xr * di + xi * dr;
  }
}

// Im <lam| G |psi> over one group, G = alpha * (Pauli string x,z) + beta * I
// on the control subspace.  XM is the compile-time x-mask (group bits).
template <typename T, int R, int XM>
__device__ __forceinline__ double mo_grad(const T *pr, const T *pi, const T *lr, const T *li,
                                          uint32_t z, uint32_t cm, uint32_t cv, double alpha,
                                          double beta) {
  const int ny = __builtin_popcount((uint32_t)XM & z) & 3;
  double acc = 0.0;
#pragma unroll
  for (int j = 0; j < (1 << R); j++) {
    if ((j & cm) != cv) continue;
    const int k = j ^ XM;
    // (P psi)_j = i^ny (-1)^{popcount(k & z)} psi_k
    const bool neg = __builtin_popcount((uint32_t)k & z) & 1;
    double wr = (double)pr[k], wi = (double)pi[k];
    double tr, ti;
    switch (ny) {
      case 0: tr = wr; ti = wi; break;
      case 1: tr = -wi; ti = wr; break;
      case 2: tr = -wr; ti = -wi; break;
      default: tr = wi; ti = -wr; break;
    }
    if (neg) { tr = -tr; ti = -ti; }
    const double gr = alpha * tr + beta * (double)pr[j];
    const double gi = alpha * ti + beta * (double)pi[j];
    // Im(conj(l) * g) = lr*gi - li*gr
    acc += (double)lr[j] * gi - (double)li[j] * gr;
  }
  return acc;
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

template <typename T, int R>
__device__ __forceinline__ double grad_op(const MicroOp &op, const T *pr, const T *pi, const T *lr,
                                          const T *li) {
  // op.mask = x-mask (0, one bit, or two bits) over group bits.
  const uint32_t x = op.mask;
  switch (x) {
#define SVI_G(XV) case XV: if constexpr (XV < (1 << R)) return mo_grad<T, R, XV>(pr, pi, lr, li, op.gz, op.cm, op.cv, op.galpha, op.gbeta); break;
    SVI_G(0) SVI_G(1) SVI_G(2) SVI_G(3) SVI_G(4) SVI_G(5) SVI_G(6) SVI_G(7) SVI_G(8) SVI_G(9)
    SVI_G(10) SVI_G(11) SVI_G(12) SVI_G(13) SVI_G(14) SVI_G(15) SVI_G(16) SVI_G(17) SVI_G(18)
    SVI_G(19) SVI_G(20) SVI_G(21) SVI_G(22) SVI_G(23) SVI_G(24) SVI_G(25) SVI_G(26) SVI_G(27)
    SVI_G(28) SVI_G(29) SVI_G(30) SVI_G(31)
#undef SVI_G
    default: break;
  }
  return 0.0;
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
            if constexpr (VN == 2) {
              lds[s][swz<T>(i)] = C2{vr.x, vi.x};
              lds[s][swz<T>(i + 1)] = C2{vr.y, vi.y};
            } else {
              lds[s][swz<T>(i)] = C2{vr.x, vi.x};
              lds[s][swz<T>(i + 1)] = C2{vr.y, vi.y};
              lds[s][swz<T>(i + 2)] = C2{vr.z, vi.z};
              lds[s][swz<T>(i + 3)] = C2{vr.w, vi.w};
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
      const StageDesc &sd = a.stages[st];
      // Every thread runs the stage (keeps wave shuffles uniform).  Threads
      // beyond the tile's groups work on LDS slots above 2^mm, which are
      // never written back.
      const bool active = tid < ngroups;
      const int gb = insert_zeros32(tid, sd.sbits, R);
      T re[NS][G], im[NS][G];
#pragma unroll
      for (int s = 0; s < NS; s++) {
#pragma unroll
        for (int j = 0; j < G; j++) {
          const C2 v = lds[s][swz<T>(gb + sd.ld_off[j])];
          re[s][j] = v.x;
          im[s][j] = v.y;
        }
      }
      for (int o = sd.op_begin; o < sd.op_end; o++) {
        const MicroOp op = a.ops[o];
        if constexpr (NS == 2) {
          if (op.type == MO_GRAD) {
            double v = active ? grad_op<T, R>(op, re[0], im[0], re[1], im[1]) : 0.0;
            v = wave_sum(v);
            if ((tid & 63) == 0) wsum[tid >> 6][op.coef] = v;
            continue;
          }
        }
        apply_op<T, R>(op, re[0], im[0], a.coef);
        if constexpr (NS == 2) apply_op<T, R>(op, re[1], im[1], a.coef);
      }
#pragma unroll
      for (int s = 0; s < NS; s++) {
#pragma unroll
        for (int j = 0; j < G; j++) lds[s][swz<T>(gb + sd.st_off[j])] = C2{re[s][j], im[s][j]};
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

    // ---- store tile
#pragma unroll
    for (int s = 0; s < NS; s++) {
      T *pr = s == 0 ? pre0 : pre1;
      T *pi = s == 0 ? pim0 : pim1;
      if (vec) {
#pragma unroll
        for (int k = 0; k < NIT; k++) {
          const int i = (tid + k * NT) * VN;
          if (i < ntile_el) {
            const uint64_t g = base + roff[k];
            V4 vr, vi;
            if constexpr (VN == 2) {
              const C2 p0 = lds[s][swz<T>(i)], p1 = lds[s][swz<T>(i + 1)];
              vr = V4{p0.x, p1.x};
              vi = V4{p0.y, p1.y};
            } else {
              const C2 p0 = lds[s][swz<T>(i)], p1 = lds[s][swz<T>(i + 1)];
              const C2 p2 = lds[s][swz<T>(i + 2)], p3 = lds[s][swz<T>(i + 3)];
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
          const C2 p = lds[s][swz<T>(i)];
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

// ------------------------------------------------- single-gate sweeps
// One work item per group of amplitudes that the gate mixes; the control
// bits are inserted as constants, so only the firing subspace is touched.

struct GateArgs {
  void *re, *im;
  const double *coef;
  int32_t type;          // MO_U, MO_R, MO_P, MO_X, MO_SWAP, MO_NEG, MO_Q
  int32_t t0, t1;        // target qubits (t1 for 2-target types)
  int32_t npos;          // inserted positions (targets + controls, ascending)
  int32_t pos[SVI_RMAX + 5];
  uint64_t cval;         // control bits that must be set (others zero)
  uint64_t pmask;        // MO_P: parity mask (global)
  int64_t nitems;
};

template <typename T>
__global__ void __launch_bounds__(256) k_gate(GateArgs a) {
  T *re = (T *)a.re, *im = (T *)a.im;
  const double *cf = a.coef;
  for (int64_t it = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; it < a.nitems;
       it += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t b = insert_zeros64((uint64_t)it, a.pos, a.npos) | a.cval;
    switch (a.type) {
      case MO_U: case MO_R: {
        const uint64_t k = b | (1ull << a.t0);
        const T xr = re[b], xi = im[b], yr = re[k], yi = im[k];
        if (a.type == MO_U) {
          re[b] = (T)cf[0] * xr - (T)cf[1] * xi + (T)cf[2] * yr - (T)cf[3] * yi;
          im[b] = (T)cf[0] * xi + (T)cf[1] * xr + (T)cf[2] * yi + (T)cf[3] * yr;
          re[k] = (T)cf[4] * xr - (T)cf[5] * xi + (T)cf[6] * yr - (T)cf[7] * yi;
          im[k] = (T)cf[4] * xi + (T)cf[5] * xr + (T)cf[6] * yi + (T)cf[7] * yr;
        } else {
          re[b] = (T)cf[0] * xr + (T)cf[1] * yr;
          im[b] = (T)cf[0] * xi + (T)cf[1] * yi;
          re[k] = (T)cf[2] * xr + (T)cf[3] * yr;
          im[k] = (T)cf[2] * xi + (T)cf[3] * yi;
        }
        break;
      }
      case MO_X: {
        const uint64_t k = b | (1ull << a.t0);
        const T xr = re[b], xi = im[b];
        re[b] = re[k]; im[b] = im[k];
        re[k] = xr; im[k] = xi;
        break;
      }
      case MO_SWAP: {
        const uint64_t j = b | (1ull << a.t0), k = b | (1ull << a.t1);
        const T xr = re[j], xi = im[j];
        re[j] = re[k]; im[j] = im[k];
        re[k] = xr; im[k] = xi;
        break;
      }
      case MO_P: {
        const bool odd = __builtin_popcountll(b & a.pmask) & 1;
        const T dr = (T)cf[odd ? 2 : 0], di = (T)cf[odd ? 3 : 1];
        const T xr = re[b], xi = im[b];
        re[b] = xr * dr - xi * di;
        im[b] = xr * di + xi * dr;
        break;
      }
      case MO_NEG:
        re[b] = -re[b];
        im[b] = -im[b];
        break;
      case MO_Q: {
        const uint64_t id[4] = {b, b | (1ull << a.t0), b | (1ull << a.t1),
                                b | (1ull << a.t0) | (1ull << a.t1)};
        T xr[4], xi[4];
#pragma unroll
        for (int q = 0; q < 4; q++) { xr[q] = re[id[q]]; xi[q] = im[id[q]]; }
#pragma unroll
        for (int r = 0; r < 4; r++) {
          T ar = 0, ai = 0;
#pragma unroll
          for (int q = 0; q < 4; q++) {
            const T ur = (T)cf[(r * 4 + q) * 2], ui = (T)cf[(r * 4 + q) * 2 + 1];
            ar += ur * xr[q] - ui * xi[q];
            ai += ur * xi[q] + ui * xr[q];
          }
          re[id[r]] = ar;
          im[id[r]] = ai;
        }
        break;
      }
      default: break;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_init_zero(T *re, T *im, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    re[i] = (i == 0) ? (T)1 : (T)0;
    im[i] = (T)0;
  }
}

// ------------------------------------------------ coefficient builder
// Gate matrices in FP64 from the parameter vector (paper Section 5.2: build at
// the widest precision, narrow only at the boundary).  Kinds follow sv.h.

enum { K_I = 0, K_X, K_Y, K_Z, K_H, K_S, K_SDG, K_T, K_TDG, K_SX, K_RX, K_RY, K_RZ, K_P, K_U2,
       K_U3, K_SWAP, K_RXX, K_RYY, K_RZZ, K_GIVENS, K_DEXC, K_UNITARY };

__device__ void gate_local(int kind, const double *th, double *m /* interleaved, row-major */) {
  const double h = 0.5 * th[0];
  double s, c;
  sincos(h, &s, &c);
  const double r2 = 0.70710678118654752440;
  for (int i = 0; i < 8; i++) m[i] = 0.0;
  switch (kind) {
    case K_X: m[2] = 1; m[4] = 1; break;
    case K_Y: m[3] = -1; m[5] = 1; break;
    case K_Z: m[0] = 1; m[6] = -1; break;
    case K_H: m[0] = r2; m[2] = r2; m[4] = r2; m[6] = -r2; break;
    case K_S: m[0] = 1; m[7] = 1; break;
    case K_SDG: m[0] = 1; m[7] = -1; break;
    case K_T: m[0] = 1; m[6] = r2; m[7] = r2; break;
    case K_TDG: m[0] = 1; m[6] = r2; m[7] = -r2; break;
    case K_SX: m[0] = 0.5; m[1] = 0.5; m[2] = 0.5; m[3] = -0.5;
               m[4] = 0.5; m[5] = -0.5; m[6] = 0.5; m[7] = 0.5; break;
    case K_RX: m[0] = c; m[3] = -s; m[5] = -s; m[6] = c; break;
    case K_RY: m[0] = c; m[2] = -s; m[4] = s; m[6] = c; break;
    case K_RZ: m[0] = c; m[1] = -s; m[6] = c; m[7] = s; break;
    case K_P: { double sp, cp; sincos(th[0], &sp, &cp); m[0] = 1; m[6] = cp; m[7] = sp; break; }
    case K_U2: case K_U3: {
      double t, f, l;
      if (kind == K_U3) { t = th[0]; f = th[1]; l = th[2]; }
      else { t = 1.57079632679489661923; f = th[0]; l = th[1]; }
      double st, ct, sf, cf, sl, cl, sfl, cfl;
      sincos(0.5 * t, &st, &ct);
      sincos(f, &sf, &cf);
      sincos(l, &sl, &cl);
      sincos(f + l, &sfl, &cfl);
      m[0] = ct; m[1] = 0;
      m[2] = -cl * st; m[3] = -sl * st;
      m[4] = cf * st; m[5] = sf * st;
      m[6] = cfl * ct; m[7] = sfl * ct;
      break;
    }
    default: m[0] = 1; m[6] = 1; break;
  }
}

__global__ void k_build_coefs(const CoefDesc *d, int nd, const double *params, const double *statics,
                              double *coef) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nd; i += gridDim.x * blockDim.x) {
    const CoefDesc cd = d[i];
    const int fmt = cd.fmt & 0xff;
    const bool dag = (cd.fmt & CF_DAGGER) != 0;
    double th[3] = {0, 0, 0};
    for (int k = 0; k < 3; k++)
      if (cd.pidx[k] >= 0) th[k] = params[cd.pidx[k]];
    double *out = coef + cd.dst;
    if (fmt == CF_U2X2 || fmt == CF_R2X2 || fmt == CF_DIAG) {
      double m[8];
      gate_local(cd.kind, th, m);
      if (dag) {
        // conjugate transpose
        double t0 = m[2], t1 = m[3];
        m[2] = m[4]; m[3] = -m[5];
        m[4] = t0; m[5] = -t1;
        m[1] = -m[1]; m[7] = -m[7];
      }
      if (fmt == CF_U2X2) {
        for (int k = 0; k < 8; k++) out[k] = m[k];
      } else if (fmt == CF_R2X2) {
        out[0] = m[0]; out[1] = m[2]; out[2] = m[4]; out[3] = m[6];
      } else {
        out[0] = m[0]; out[1] = m[1]; out[2] = m[6]; out[3] = m[7];
      }
    } else if (fmt == CF_Q4X4 || fmt == CF_D16) {
      const int D = fmt == CF_Q4X4 ? 4 : 16;
      for (int k = 0; k < 2 * D * D; k++) out[k] = 0.0;
      double s, c;
      sincos(0.5 * th[0], &s, &c);
      if (cd.kind == K_RXX || cd.kind == K_RYY) {
        // c I - i s P(x)P; XX maps j -> 3-j; YY has sign -1 on |00>,|11>
        for (int j = 0; j < 4; j++) {
          out[(j * 4 + j) * 2] = c;
          const double ph = (cd.kind == K_RYY && (j == 0 || j == 3)) ? -1.0 : 1.0;
          out[((3 - j) * 4 + j) * 2 + 1] = -s * ph;
        }
      } else if (cd.kind == K_GIVENS || cd.kind == K_DEXC) {
        const int lo = cd.kind == K_GIVENS ? 1 : 3, hi = cd.kind == K_GIVENS ? 2 : 12;
        for (int j = 0; j < D; j++) out[(j * D + j) * 2] = 1.0;
        out[(lo * D + lo) * 2] = c;
        out[(lo * D + hi) * 2] = -s;
        out[(hi * D + lo) * 2] = s;
        out[(hi * D + hi) * 2] = c;
      } else if (cd.kind == K_SWAP) {
        out[(0 * 4 + 0) * 2] = 1; out[(1 * 4 + 2) * 2] = 1;
        out[(2 * 4 + 1) * 2] = 1; out[(3 * 4 + 3) * 2] = 1;
      } else if (cd.kind == K_RZZ) {
        for (int j = 0; j < 4; j++) {
          const int par = (j ^ (j >> 1)) & 1;
          out[(j * 4 + j) * 2] = c;
          out[(j * 4 + j) * 2 + 1] = par ? s : -s;
        }
      }
      if (dag) {
        for (int r = 0; r < D; r++)
          for (int q = r; q < D; q++) {
            const double ar = out[(r * D + q) * 2], ai = out[(r * D + q) * 2 + 1];
            const double br = out[(q * D + r) * 2], bi = out[(q * D + r) * 2 + 1];
            out[(r * D + q) * 2] = br; out[(r * D + q) * 2 + 1] = -bi;
            out[(q * D + r) * 2] = ar; out[(q * D + r) * 2 + 1] = -ai;
          }
      }
    } else if (fmt == CF_COPY) {
      // user matrix, 2^k x 2^k, len = 2 * 4^k
      int D = 1;
      while (2 * D * D < cd.len) D <<= 1;
      for (int k = 0; k < cd.len; k++) out[k] = statics[cd.src + k];
      if (dag) {
        for (int r = 0; r < D; r++)
          for (int q = r; q < D; q++) {
            const double ar = out[(r * D + q) * 2], ai = out[(r * D + q) * 2 + 1];
            const double br = out[(q * D + r) * 2], bi = out[(q * D + r) * 2 + 1];
            out[(r * D + q) * 2] = br; out[(r * D + q) * 2 + 1] = -bi;
            out[(q * D + r) * 2] = ar; out[(q * D + r) * 2 + 1] = -ai;
          }
      }
    }
  }
}

// --------------------------------------------------- Pauli tile pass
// Expectation values <P_j> and (optionally) lam = sum_j c_j P_j psi for the
// terms whose x-mask lies inside the tile (paper Section 4.4 Pauli action:
// P|b> = i^{nY} (-1)^{popcount(b & z)} |b ^ x>).

#define SVI_PTERMS 64

template <typename T, int M>
__global__ void __launch_bounds__(256) k_pauli(PauliPassArgs a) {
  constexpr int NT = 256;
  constexpr int EPT = (1 << M) / NT;   // elements per thread
  constexpr int NWAVE = NT / 64;
  using C2 = typename C2T<T>::type;
  __shared__ C2 lds[1 << M];
  __shared__ double wsum[NWAVE][SVI_PTERMS];
  __shared__ double tacc[SVI_PTERMS];
  __shared__ uint32_t xl_s[SVI_PTERMS], zl_s[SVI_PTERMS];

  const int tid = threadIdx.x;
  const int m = a.m, c = a.c, nh = a.nh;
  const int nel = 1 << m;
  const int nterm = a.t_end - a.t_begin;
  const T *pre = (const T *)a.re, *pim = (const T *)a.im;
  T *lre = (T *)a.lre, *lim = (T *)a.lim;

  // tile-local masks of every term of this pass
  for (int t = tid; t < nterm; t += NT) {
    const PauliTermDev pt = a.terms[a.t_begin + t];
    uint32_t xl = 0, zl = 0;
    for (int b = 0; b < c; b++) {
      xl |= (uint32_t)((pt.x >> b) & 1) << b;
      zl |= (uint32_t)((pt.z >> b) & 1) << b;
    }
    for (int k = 0; k < nh; k++) {
      xl |= (uint32_t)((pt.x >> a.hb[k]) & 1) << (c + k);
      zl |= (uint32_t)((pt.z >> a.hb[k]) & 1) << (c + k);
    }
    xl_s[t] = xl;
    zl_s[t] = zl;
    tacc[t] = 0.0;
  }
  __syncthreads();

  for (int64_t tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
    const uint64_t base = tile_base(tile, c, a.hb, nh);
    for (int i = tid; i < nel; i += NT) {
      const uint64_t g = base + spread_row(i >> c, a.hb, nh) + (uint64_t)(i & ((1 << c) - 1));
      lds[swz<T>(i)] = C2{pre[g], pim[g]};
    }
    __syncthreads();
    T lr[EPT], li[EPT];
#pragma unroll
    for (int k = 0; k < EPT; k++) { lr[k] = 0; li[k] = 0; }
    for (int t = 0; t < nterm; t++) {
      const PauliTermDev pt = a.terms[a.t_begin + t];
      const uint32_t xl = xl_s[t], zl = zl_s[t];
      const int ny = __builtin_popcountll(pt.x & pt.z) & 3;
      const bool bneg = __builtin_popcountll(base & pt.z) & 1;   // non-tile bits' sign
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < EPT; k++) {
        const int i = tid + k * NT;
        if (i < nel) {
          const C2 pb = lds[swz<T>(i)];
          const C2 pp = lds[swz<T>(i ^ (int)xl)];
          // t1 = conj(psi_{b^x}) * i^ny * s(b) * psi_b
          double wr = (double)pb.x, wi = (double)pb.y, tr, ti;
          switch (ny) {
            case 0: tr = wr; ti = wi; break;
            case 1: tr = -wi; ti = wr; break;
            case 2: tr = -wr; ti = -wi; break;
            default: tr = wi; ti = -wr; break;
          }
          const bool neg = bneg ^ (bool)(__builtin_popcount((uint32_t)i & zl) & 1);
          if (neg) { tr = -tr; ti = -ti; }
          acc += (double)pp.x * tr + (double)pp.y * ti;   // Re(conj(pp) * t)
          if (lre) {
            // (P psi)[b] = i^ny (-1)^{popcount((b^x) & z)} psi[b^x]
            double ur = (double)pp.x, ui = (double)pp.y, vr, vi;
            switch (ny) {
              case 0: vr = ur; vi = ui; break;
              case 1: vr = -ui; vi = ur; break;
              case 2: vr = -ur; vi = -ui; break;
              default: vr = ui; vi = -ur; break;
            }
            const bool neg2 = bneg ^ (bool)(__builtin_popcount((uint32_t)(i ^ xl) & zl) & 1);
            if (neg2) { vr = -vr; vi = -vi; }
            lr[k] += (T)(pt.c * vr);
            li[k] += (T)(pt.c * vi);
          }
        }
      }
      acc = wave_sum(acc);
      if ((tid & 63) == 0) wsum[tid >> 6][t] = acc;
    }
    __syncthreads();
    for (int t = tid; t < nterm; t += NT) {
      double v = 0.0;
      for (int w = 0; w < NWAVE; w++) v += wsum[w][t];
      tacc[t] += v;
    }
    if (lre) {
#pragma unroll
      for (int k = 0; k < EPT; k++) {
        const int i = tid + k * NT;
        if (i < nel) {
          const uint64_t g = base + spread_row(i >> c, a.hb, nh) + (uint64_t)(i & ((1 << c) - 1));
          if (a.accumulate) {
            lre[g] += lr[k];
            lim[g] += li[k];
          } else {
            lre[g] = lr[k];
            lim[g] = li[k];
          }
        }
      }
    }
    __syncthreads();
  }
  for (int t = tid; t < nterm; t += NT) a.part[(int64_t)t * gridDim.x + blockIdx.x] = tacc[t];
}

// Sum each slot's partials in a fixed order: out[s] = sum_w part[s * np + w].
__global__ void k_reduce_rows(const double *part, int nslots, int np, double *out) {
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < nslots; s += gridDim.x * blockDim.x) {
    double v = 0.0;
    for (int w = 0; w < np; w++) v += part[(int64_t)s * np + w];
    out[s] = v;
  }
}

// grad[p] = sum over slots mapped to p in ascending slot order (CSR).
__global__ void k_gather_grad(const double *slot_sum, const int32_t *row_ptr, const int32_t *slots,
                              int np, double *grad) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < np; p += gridDim.x * blockDim.x) {
    double v = 0.0;
    for (int k = row_ptr[p]; k < row_ptr[p + 1]; k++) v += slot_sum[slots[k]];
    grad[p] = v;
  }
}

// E = sum_j c_j <P_j> in term order.
__global__ void k_energy(const double *terms, const double *coef, int nt, double *out) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double e = 0.0;
    for (int j = 0; j < nt; j++) e += coef[j] * terms[j];
    out[0] = e;
  }
}

// ------------------------------------------------------------ sampling
// Fixed-order specification (see sv.h): p_b = fma(x, x, y*y); chunk sums by
// pairwise tree; sequential prefix; counter-based SplitMix64 uniforms.

#pragma clang fp contract(off)

template <typename T>
__device__ __forceinline__ double prob_at(const T *re, const T *im, uint64_t b) {
  const double x = (double)re[b], y = (double)im[b];
  return __fma_rn(x, x, y * y);
}

template <typename T>
__global__ void __launch_bounds__(256) k_chunk_sums(const T *re, const T *im, int cbits, int64_t K,
                                                    double *S) {
  __shared__ double v[2][1024];
  const int C = 1 << cbits;
  for (int64_t k = blockIdx.x; k < K; k += gridDim.x) {
    for (int i = threadIdx.x; i < C; i += blockDim.x) v[0][i] = prob_at(re, im, (uint64_t)k * C + i);
    __syncthreads();
    int src = 0;
    // pairwise tree: level by level, adjacent pairs
    for (int len = C; len > 1; len >>= 1) {
      const int h = len >> 1;
      for (int i = threadIdx.x; i < h; i += blockDim.x) v[src ^ 1][i] = v[src][2 * i] + v[src][2 * i + 1];
      src ^= 1;
      __syncthreads();
    }
    if (threadIdx.x == 0) S[k] = v[src][0];
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) k_prefix(const double *S, int64_t K, double *P) {
  __shared__ double buf[4096];
  __shared__ double carry;
  if (threadIdx.x == 0) { P[0] = 0.0; carry = 0.0; }
  __syncthreads();
  for (int64_t b0 = 0; b0 < K; b0 += 4096) {
    const int len = (int)((K - b0) < 4096 ? (K - b0) : 4096);
    for (int i = threadIdx.x; i < len; i += blockDim.x) buf[i] = S[b0 + i];
    __syncthreads();
    if (threadIdx.x == 0) {
      double acc = carry;
      for (int i = 0; i < len; i++) {
        acc = acc + buf[i];
        buf[i] = acc;
      }
      carry = acc;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < len; i += blockDim.x) P[b0 + i + 1] = buf[i];
    __syncthreads();
  }
}

__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t s) {
  uint64_t z = seed + (s + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct SampleArgs {
  const void *re, *im;
  const double *S, *P;
  int64_t K;
  int32_t cbits;
  int32_t nq;
  int32_t qubits[64];
  uint64_t seed;
  int64_t shots;
  uint64_t *out;
};

template <typename T>
__global__ void __launch_bounds__(256) k_sample(SampleArgs a) {
  const T *re = (const T *)a.re, *im = (const T *)a.im;
  const int64_t C = 1ll << a.cbits;
  const double Tot = a.P[a.K];
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < a.shots;
       s += (int64_t)gridDim.x * blockDim.x) {
    const double u = (double)(splitmix64(a.seed, (uint64_t)s) >> 11) * 0x1.0p-53;
    const double t = u * Tot;
    // first k with P[k+1] > t (P non-decreasing)
    int64_t lo = 0, hi = a.K;   // answer in [0, K]; K means none
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (a.P[mid + 1] > t) hi = mid; else lo = mid + 1;
    }
    int64_t ks = lo;
    if (ks >= a.K) {
      ks = -1;
      for (int64_t k = a.K - 1; k >= 0; k--)
        if (a.S[k] > 0.0) { ks = k; break; }
      if (ks < 0) ks = 0;
    }
    const double r = t - a.P[ks];
    double acc = 0.0;
    int64_t pick = -1, lastpos = -1;
    for (int64_t i = 0; i < C; i++) {
      const uint64_t b = (uint64_t)(ks * C + i);
      const double p = prob_at(re, im, b);
      acc = acc + p;
      if (p > 0.0) lastpos = (int64_t)b;
      if (acc > r) { pick = (int64_t)b; break; }
    }
    if (pick < 0) pick = lastpos >= 0 ? lastpos : ks * C;
    uint64_t o = 0;
    for (int i = 0; i < a.nq; i++) o |= (((uint64_t)pick >> a.qubits[i]) & 1ull) << i;
    a.out[s] = o;
  }
}

#pragma clang fp contract(on)

}  // namespace

// ------------------------------------------------------------ launchers
// Host-callable wrappers (C++ linkage, used by sv_host.cpp).

#include "sv_launch.h"

template <typename T, int M, int R, int NS>
static hipError_t launch_sweep_t(const SweepArgs &a, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_sweep<T, M, R, NS>), dim3(grid), dim3(1 << (M - R)), 0, s, a);
  return hipGetLastError();
}

template <typename T, int M, int R, int NS>
static int occ_sweep_t() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sweep<T, M, R, NS>, 1 << (M - R), 0) !=
      hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

#define SVI_VARIANTS(X)      \
  X(double, 13, 5, 1)        \
  X(double, 12, 5, 1)        \
  X(double, 13, 4, 1)        \
  X(double, 12, 4, 1)        \
  X(double, 11, 5, 1)        \
  X(double, 12, 4, 2)        \
  X(double, 11, 4, 2)        \
  X(float, 14, 5, 1)         \
  X(float, 13, 5, 1)         \
  X(float, 13, 4, 2)

hipError_t svk_launch_sweep(int dbl, int M, int R, int NS, const SweepArgs &a, int grid,
                            hipStream_t s) {
#define X(T, MM, RR, NN)                                                        \
  if ((dbl == (sizeof(T) == 8)) && M == MM && R == RR && NS == NN)              \
    return launch_sweep_t<T, MM, RR, NN>(a, grid, s);
  SVI_VARIANTS(X)
#undef X
  return hipErrorInvalidValue;
}

int svk_sweep_occupancy(int dbl, int M, int R, int NS) {
#define X(T, MM, RR, NN)                                                        \
  if ((dbl == (sizeof(T) == 8)) && M == MM && R == RR && NS == NN)              \
    return occ_sweep_t<T, MM, RR, NN>();
  SVI_VARIANTS(X)
#undef X
  return 0;
}

int svk_has_sweep(int dbl, int M, int R, int NS) {
#define X(T, MM, RR, NN)                                                        \
  if ((dbl == (sizeof(T) == 8)) && M == MM && R == RR && NS == NN) return 1;
  SVI_VARIANTS(X)
#undef X
  return 0;
}

hipError_t svk_launch_gate(int dbl, const GateArgsHost &h, hipStream_t s) {
  GateArgs a;
  a.re = h.re; a.im = h.im; a.coef = h.coef; a.type = h.type; a.t0 = h.t0; a.t1 = h.t1;
  a.npos = h.npos;
  for (int i = 0; i < SVI_RMAX + 5; i++) a.pos[i] = i < h.npos ? h.pos[i] : 0;
  a.cval = h.cval; a.pmask = h.pmask; a.nitems = h.nitems;
  int64_t blocks = (h.nitems + 255) / 256;
  int grid = (int)(blocks < 65536 ? blocks : 65536);
  if (grid < 1) grid = 1;
  if (dbl) hipLaunchKernelGGL(k_gate<double>, dim3(grid), dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_gate<float>, dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t svk_launch_init_zero(int dbl, void *re, void *im, int64_t n, hipStream_t s) {
  int64_t blocks = (n + 255) / 256;
  int grid = (int)(blocks < 65536 ? blocks : 65536);
  if (dbl) hipLaunchKernelGGL(k_init_zero<double>, dim3(grid), dim3(256), 0, s, (double *)re, (double *)im, n);
  else hipLaunchKernelGGL(k_init_zero<float>, dim3(grid), dim3(256), 0, s, (float *)re, (float *)im, n);
  return hipGetLastError();
}

hipError_t svk_launch_coefs(const CoefDesc *d, int nd, const double *params, const double *statics,
                            double *coef, hipStream_t s) {
  if (nd <= 0) return hipSuccess;
  int grid = (nd + 127) / 128;
  hipLaunchKernelGGL(k_build_coefs, dim3(grid), dim3(128), 0, s, d, nd, params, statics, coef);
  return hipGetLastError();
}

hipError_t svk_launch_pauli(int dbl, int M, const PauliPassArgs &a, int grid, hipStream_t s) {
  if (dbl && M == 13) hipLaunchKernelGGL((k_pauli<double, 13>), dim3(grid), dim3(256), 0, s, a);
  else if (!dbl && M == 13) hipLaunchKernelGGL((k_pauli<float, 13>), dim3(grid), dim3(256), 0, s, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

int svk_pauli_occupancy(int dbl) {
  int nb = 0;
  hipError_t e = dbl ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_pauli<double, 13>, 256, 0)
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_pauli<float, 13>, 256, 0);
  return (e == hipSuccess && nb > 0) ? nb : 1;
}

hipError_t svk_launch_reduce_rows(const double *part, int nslots, int np, double *out,
                                  hipStream_t s) {
  if (nslots <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_rows, dim3((nslots + 127) / 128), dim3(128), 0, s, part, nslots, np, out);
  return hipGetLastError();
}

hipError_t svk_launch_gather_grad(const double *slot_sum, const int32_t *row_ptr,
                                  const int32_t *slots, int np, double *grad, hipStream_t s) {
  if (np <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_grad, dim3((np + 127) / 128), dim3(128), 0, s, slot_sum, row_ptr, slots, np, grad);
  return hipGetLastError();
}

hipError_t svk_launch_energy(const double *terms, const double *coef, int nt, double *out,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_energy, dim3(1), dim3(64), 0, s, terms, coef, nt, out);
  return hipGetLastError();
}

hipError_t svk_launch_sampling(int dbl, const void *re, const void *im, int n, double *S, double *P,
                               uint64_t seed, int64_t shots, const int32_t *qubits, int nq,
                               uint64_t *out, hipStream_t s) {
  const int cbits = n < 10 ? n : 10;
  const int64_t K = (1ll << n) >> cbits;
  int grid = (int)(K < 4096 ? K : 4096);
  if (dbl) hipLaunchKernelGGL(k_chunk_sums<double>, dim3(grid), dim3(256), 0, s, (const double *)re, (const double *)im, cbits, K, S);
  else hipLaunchKernelGGL(k_chunk_sums<float>, dim3(grid), dim3(256), 0, s, (const float *)re, (const float *)im, cbits, K, S);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_prefix, dim3(1), dim3(256), 0, s, S, K, P);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (shots <= 0) return hipSuccess;
  SampleArgs a;
  a.re = re; a.im = im; a.S = S; a.P = P; a.K = K; a.cbits = cbits; a.nq = nq;
  for (int i = 0; i < 64; i++) a.qubits[i] = i < nq ? qubits[i] : 0;
  a.seed = seed; a.shots = shots; a.out = out;
  int64_t blocks = (shots + 255) / 256;
  int g2 = (int)(blocks < 4096 ? blocks : 4096);
  if (dbl) hipLaunchKernelGGL(k_sample<double>, dim3(g2), dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_sample<float>, dim3(g2), dim3(256), 0, s, a);
  return hipGetLastError();
}
