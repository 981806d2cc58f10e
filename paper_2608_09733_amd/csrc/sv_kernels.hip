// gfx950 kernels of the state-vector library (everything except the tile
// sweep variants, which live in sv_sweep_variant.hip and are compiled once per
// variant).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "sv_device.h"

namespace {
using namespace svk;

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

// Fast-Givens factorisation of a real orthogonal 2x2 r = [[r0, r1], [r2, r3]]
// (Gentleman 1973): out = {form, k, scale, 0}, r = scale * (form matrix).
// form0: a rotation always takes form 0 (k = s / c; c is never exactly zero
// for a rotation angle that is a double, so k is finite, and the error of
// (x - k y) c stays within a few ulps of |x c| + |y s|).
__device__ void fast_givens(const double *r, double *out, bool form0 = false) {
  // rotation [[c,-s],[s,c]] vs reflection [[a,b],[b,-a]]
  const bool rot = fabs(r[0] - r[3]) + fabs(r[1] + r[2]) <= fabs(r[0] + r[3]) + fabs(r[1] - r[2]);
  if (rot) {
    // [[c, -s], [s, c]]
    const double c = r[0], s = r[2];
    if (form0 || fabs(c) >= fabs(s)) { out[0] = 0; out[1] = s / c; out[2] = c; }
    else { out[0] = 1; out[1] = c / s; out[2] = s; }
  } else {
    // [[a, b], [b, -a]]
    const double a = r[0], b = r[1];
    if (fabs(a) >= fabs(b)) { out[0] = 2; out[1] = b / a; out[2] = a; }
    else { out[0] = 3; out[1] = a / b; out[2] = b; }
  }
  out[3] = 0.0;
}

// Coefficients of one descriptor, written at coef + cd.dst.
__device__ void build_coef(const CoefDesc &cd, const double *params, const double *statics,
                           const TabFactor *fac, double *coef) {
  const int fmt = cd.fmt & 0xff;
  const bool dag = (cd.fmt & CF_DAGGER) != 0;
  const bool f0 = (cd.fmt & CF_FORM0) != 0;
  double th[3] = {0, 0, 0};
  // pidx holds parameter indices except for the table / scale formats,
  // where pidx[0] counts factors
  const bool takes_params = fmt != CF_TABLE && fmt != CF_SCALE && fmt != CF_COPY &&
                            fmt != CF_IDENT2 && fmt != CF_CONSTS;
  if (takes_params)
    for (int k = 0; k < 3; k++)
      if (cd.pidx[k] >= 0) th[k] = params[cd.pidx[k]];
  double *out = coef + cd.dst;
  if (fmt == CF_CONSTS) {
    for (int k = 0; k < cd.len; k++) out[k] = params[cd.src + k];
  } else if (fmt == CF_FASTR) {
    double m[8];
    gate_local(cd.kind, th, m);
    double r[4] = {m[0], m[2], m[4], m[6]};   // real 2x2
    if (dag) { const double t = r[1]; r[1] = r[2]; r[2] = t; }
    fast_givens(r, out, f0);
  } else if (fmt == CF_SCALE) {
    // product of the fast-Givens scales of the (daggered, if flagged) real gates
    double sc = 1.0;
    for (int f = cd.src; f < cd.src + cd.pidx[0]; f++) {
      const TabFactor tf = fac[f];
      double m[8], rec[4];
      double tt[3] = {tf.pidx >= 0 ? params[tf.pidx] : 0.0, 0.0, 0.0};
      gate_local(tf.kind, tt, m);
      double r[4] = {m[0], m[2], m[4], m[6]};
      if (dag) { const double t = r[1]; r[1] = r[2]; r[2] = t; }
      fast_givens(r, rec, f0);
      sc *= rec[2];
    }
    out[0] = sc;
  } else if (fmt == CF_IDENT2) {
    out[0] = 1.0; out[1] = 0.0; out[2] = 0.0; out[3] = 1.0;
  } else if (fmt == CF_TABLE) {
    const int G = 1 << cd.len;
    for (int j = 0; j < G; j++) { out[2 * j] = 1.0; out[2 * j + 1] = 0.0; }
    for (int f = cd.src; f < cd.src + cd.pidx[0]; f++) {
      const TabFactor tf = fac[f];
      double m[8];
      double tt[3] = {tf.pidx >= 0 ? params[tf.pidx] : 0.0, 0.0, 0.0};
      gate_local(tf.kind, tt, m);
      double gsc = 1.0;
      if (tf.neg == 2) {
        double r[4] = {m[0], m[2], m[4], m[6]}, rec[4];
        if (dag) { const double t = r[1]; r[1] = r[2]; r[2] = t; }
        fast_givens(r, rec, f0);
        gsc = rec[2];
      }
      for (int j = 0; j < G; j++) {
        if (((uint32_t)j & tf.cm) != tf.cv) continue;
        double dr, di;
        if (tf.neg == 2) { dr = gsc; di = 0.0; }
        else if (tf.neg) { dr = -1.0; di = 0.0; }
        else if (__builtin_popcount((uint32_t)j & tf.mask) & 1) { dr = m[6]; di = m[7]; }
        else { dr = m[0]; di = m[1]; }
        const double xr = out[2 * j], xi = out[2 * j + 1];
        out[2 * j] = xr * dr - xi * di;
        out[2 * j + 1] = xr * di + xi * dr;
      }
    }
    if (dag)
      for (int j = 0; j < G; j++) out[2 * j + 1] = -out[2 * j + 1];
  } else if (fmt == CF_U2X2 || fmt == CF_R2X2 || fmt == CF_DIAG) {
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

__global__ void k_build_coefs(const CoefDesc *d, int nd, const double *params, const double *statics,
                              const TabFactor *fac, double *coef) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nd; i += gridDim.x * blockDim.x)
    build_coef(d[i], params, statics, fac, coef);
}

// --------------------------------------------------- Pauli tile pass
// Expectation values <P_j> and (optionally) lam = sum_j c_j P_j psi for the
// terms whose x-mask lies inside the tile (paper Section 4.4 Pauli action:
// P|b> = i^{nY} (-1)^{popcount(b & z)} |b ^ x>).

#define SVI_PTERMS 64

// Term t, read through the constant address space (uniform index: scalar
// loads instead of vector loads and their waits inside the tile loop).
__device__ __forceinline__ PauliTermDev term_at(const PauliTermDev *terms, int t) {
  const SVI_CONST PauliTermDev &s = cptr(terms)[t];
  PauliTermDev p;
  p.x = s.x;
  p.z = s.z;
  p.c = s.c;
  p.term = s.term;
  p.pad = 0;
  return p;
}

// In-place Walsh-Hadamard transform of N register values (N a power of two):
// v[z] becomes sum_k (-1)^{popcount(k & z)} v[k].
template <int N>
__device__ __forceinline__ void wht_regs(double (&v)[N]) {
#pragma unroll
  for (int h = 1; h < N; h <<= 1)
#pragma unroll
    for (int k = 0; k < N; k++)
      if (!(k & h)) {
        const double x = v[k], y = v[k | h];
        v[k] = x + y;
        v[k | h] = x - y;
      }
}

// LAM: the pass also builds (or adds into) lambda = sum_j c_j P_j psi.
// Eight elements per thread: 1024 threads for a 13-bit tile, 512 for 12.
template <typename T, int M, bool LAM>
__global__ void __launch_bounds__((1 << M) / 8) k_pauli(PauliPassArgs a) {
  constexpr int NT = (1 << M) / 8;
  constexpr int EPT = (1 << M) / NT;   // elements per thread: i = tid + k * NT
  constexpr int NWAVE = NT / 64;
  using C2 = typename C2T<T>::type;
  __shared__ C2 lds[1 << M];
  __shared__ double wsum[NWAVE][SVI_PTERMS];
  __shared__ double tacc[SVI_PTERMS];
  __shared__ uint32_t xl_s[SVI_PTERMS], zl_s[SVI_PTERMS];
  __shared__ int32_t hb_s[SVI_MMAX];

  const int tid = threadIdx.x;
  const int m = a.m, c = a.c, nh = a.nh;
  const int nel = 1 << m;
  const int nterm = a.t_end - a.t_begin;
  const T *pre = (const T *)a.re, *pim = (const T *)a.im;
  T *lre = (T *)a.lre, *lim = (T *)a.lim;

  // tile-local masks of every term of this pass
  if (tid < SVI_MMAX) hb_s[tid] = a.hb[tid < nh ? tid : 0];
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
  // element tid + k * NT of a tile sits at tile_base + loff + koff[k]
  // (tile_off is a bit deposit: per-lane part plus wave-uniform parts)
  const uint64_t loff = tile_off(tid, c, hb_s, nh);
  uint64_t koff[EPT];
#pragma unroll
  for (int k = 0; k < EPT; k++) koff[k] = tile_off(k * NT, c, a.hb, nh);   // kernel arguments: scalar

  for (int64_t tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
    const uint64_t base = tile_base(tile, c, hb_s, nh);
#pragma unroll
    for (int k = 0; k < EPT; k++) {
      const int i = tid + k * NT;
      if (i < nel) {
        const uint64_t g = base + (loff | koff[k]);
        lds[swz<T>(i)] = C2{pre[g], pim[g]};
      }
    }
    __syncthreads();
    // |psi|^2 of this thread's elements (0 beyond the tile)
    double pn[EPT], zs[EPT];
#pragma unroll
    for (int k = 0; k < EPT; k++) {
      const int i = tid + k * NT;
      double v = 0.0;
      if (i < nel) {
        const C2 pb = lds[swz<T>(i)];
        v = (double)pb.x * (double)pb.x + (double)pb.y * (double)pb.y;
      }
      pn[k] = v;
      zs[k] = 0.0;
    }
    // one term's sum over this tile and wave (DPP lane moves, in lane 63)
    auto put = [&](int t, double acc) {
      acc = wave_total63(acc);
      if ((tid & 63) == 63) wsum[tid >> 6][t] = acc;
    };
    // Z-only terms: sign(i) = parity(base & z) ^ parity(tid & zl) ^ parity(k & zk)
    // with zk = zl / NT the term's bits among the element bits k.  After one
    // Walsh-Hadamard transform over k, pn[zk] is sum_k (-1)^{popcount(k & zk)}
    // |psi_k|^2, so a term reads one entry; for lambda, each term adds its
    // signed coefficient to bin zk, and the same transform of the bins gives
    // the diagonal factor of every element.
    wht_regs<EPT>(pn);
    for (int t = 0; t < nterm; t++) {
      if (xl_s[t] != 0) continue;
      const PauliTermDev pt = term_at(a.terms, a.t_begin + t);
      const uint32_t zl = zl_s[t];
      const bool sneg = (__builtin_popcountll(base & pt.z) ^ __builtin_popcount((uint32_t)tid & zl)) & 1;
      const uint32_t zk = zl / NT;
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < EPT; q++)
        if (zk == (uint32_t)q) {
          acc = pn[q];
          if constexpr (LAM) zs[q] += sneg ? -pt.c : pt.c;
        }
      put(t, sneg ? -acc : acc);
    }
    if constexpr (LAM) wht_regs<EPT>(zs);
    // terms with an X / Y part: partner amplitudes from LDS; the thread's own
    // amplitudes are kept in registers when no lambda is built (its
    // accumulators' registers are free then), else re-read from LDS
    T ownr[LAM ? 1 : EPT], owni[LAM ? 1 : EPT];
    if constexpr (!LAM) {
#pragma unroll
      for (int k = 0; k < EPT; k++) {
        const int i = tid + k * NT;
        ownr[k] = 0;
        owni[k] = 0;
        if (i < nel) {
          const C2 pb = lds[swz<T>(i)];
          ownr[k] = pb.x;
          owni[k] = pb.y;
        }
      }
    }
    auto own = [&](int k, int i) -> C2 {
      if constexpr (LAM) return lds[swz<T>(i)];
      else return C2{ownr[k], owni[k]};
    };
    T lr[EPT], li[EPT];
    if constexpr (LAM) {
#pragma unroll
      for (int k = 0; k < EPT; k++) {
        const int i = tid + k * NT;
        lr[k] = 0;
        li[k] = 0;
        if (i < nel) {
          const C2 pb = lds[swz<T>(i)];
          lr[k] = (T)(zs[k] * (double)pb.x);
          li[k] = (T)(zs[k] * (double)pb.y);
        }
      }
    }
    for (int t = 0; t < nterm; t++) {
      const uint32_t xl = xl_s[t];
      if (xl == 0) continue;
      const PauliTermDev pt = term_at(a.terms, a.t_begin + t);
      const uint32_t zl = zl_s[t];
      const int ny = __builtin_popcountll(pt.x & pt.z) & 3;
      const bool bneg = __builtin_popcountll(base & pt.z) & 1;   // non-tile bits' sign
      if (zl == 0) {
        // no Z bit inside the tile, hence no Y (every X bit is a tile bit):
        // the sign (-1)^bneg is the same for every element, so the term is
        // s Re sum conj(psi_{b^x}) psi_b, and lambda adds s c psi_{b^x}
        const double s1 = bneg ? -1.0 : 1.0, cs = s1 * pt.c;
        double sr = 0.0;
#pragma unroll
        for (int k = 0; k < EPT; k++) {
          const int i = tid + k * NT;
          if (i < nel) {
            const C2 pb = own(k, i);
            const C2 pp = lds[swz<T>(i ^ (int)xl)];
            const double ur = (double)pp.x, ui = (double)pp.y;
            sr += ur * (double)pb.x + ui * (double)pb.y;
            if constexpr (LAM) {
              lr[k] += (T)(cs * ur);
              li[k] += (T)(cs * ui);
            }
          }
        }
        put(t, s1 * sr);
        continue;
      }
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < EPT; k++) {
        const int i = tid + k * NT;
        if (i < nel) {
          const C2 pb = own(k, i);
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
          if constexpr (LAM) {
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
      put(t, acc);
    }
    __syncthreads();
    for (int t = tid; t < nterm; t += NT) {
      double v = 0.0;
      for (int w = 0; w < NWAVE; w++) v += wsum[w][t];
      tacc[t] += v;
    }
    if constexpr (LAM) {
#pragma unroll
      for (int k = 0; k < EPT; k++) {
        const int i = tid + k * NT;
        if (i < nel) {
          const uint64_t g = base + (loff | koff[k]);
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

// Diagonal (Z-only) terms, expectation only: one streaming read of the state
// for up to SVI_ZTERMS terms.  Each thread holds K = J * VN probabilities per
// iteration at fixed "register" bit positions (the VN elements of a 16-byte
// vector and J vector slots NT * VN apart); a Walsh-Hadamard transform over
// them gives, for every z pattern on those bits, the signed sum
// sum_x (-1)^{popcount(z & x)} p_x, so each term costs one indexed read plus
// a sign from the thread's and the chunk's bits.
#define SVI_ZTERMS 32

template <typename T>
__global__ void __launch_bounds__(256) k_zexp(const T *re, const T *im, int64_t nchunks,
                                              const PauliTermDev *terms, int nt, double *part) {
  constexpr int NT = 256;
  constexpr int VN = V4T<T>::N;
  constexpr int LV = VN == 2 ? 1 : 2;            // log2 VN
  constexpr int J = 4;
  constexpr int K = J * VN;
  constexpr int CH = NT * VN * J;                // amplitudes per chunk
  constexpr int LCH = LV + 8 + 2;                // log2 CH
  using V4 = typename V4T<T>::type;
  __shared__ double wsum[NT / 64][SVI_ZTERMS];
  __shared__ double wl[K][NT];                   // this thread's transform, column tid
  const int tid = threadIdx.x;
  const SVI_CONST PauliTermDev *tm = cptr(terms);
  // per term, hoisted out of the chunk loop: the z bits on the chunk index,
  // the transform slot of its z bits on the register positions, and the sign
  // from this thread's index bits (applied once at the end)
  uint32_t zc[SVI_ZTERMS];
  int zr[SVI_ZTERMS];
  uint32_t tpar = 0;
#pragma unroll
  for (int t = 0; t < SVI_ZTERMS; t++) {
    const uint64_t z = t < nt ? tm[t].z : 0;
    zc[t] = (uint32_t)(z >> LCH);
    zr[t] = (int)(z & (VN - 1)) | (int)(((z >> (LV + 8)) & (J - 1)) << LV);
    tpar |= (uint32_t)(__builtin_popcountll(z & ((uint64_t)tid * VN)) & 1) << t;
  }
  double acc[SVI_ZTERMS];
#pragma unroll
  for (int t = 0; t < SVI_ZTERMS; t++) acc[t] = 0.0;
  // software pipeline: the next chunk's loads are in flight while the
  // current chunk's transform and term sums run
  V4 nr[J], ni[J];
  auto fetch = [&](int64_t ch) {
    const uint64_t cb = (uint64_t)ch * CH;
#pragma unroll
    for (int j = 0; j < J; j++) {
      const uint64_t g = cb + (uint64_t)j * (NT * VN) + (uint64_t)tid * VN;
      nr[j] = *(const V4 *)(re + g);
      ni[j] = *(const V4 *)(im + g);
    }
  };
  if (blockIdx.x < nchunks) fetch(blockIdx.x);
  for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
    double p[K];
#pragma unroll
    for (int j = 0; j < J; j++) {
      auto sq = [](T a, T b) { return (double)a * (double)a + (double)b * (double)b; };
      if constexpr (VN == 2) {
        p[j * 2] = sq(nr[j].x, ni[j].x);
        p[j * 2 + 1] = sq(nr[j].y, ni[j].y);
      } else {
        p[j * 4] = sq(nr[j].x, ni[j].x);
        p[j * 4 + 1] = sq(nr[j].y, ni[j].y);
        p[j * 4 + 2] = sq(nr[j].z, ni[j].z);
        p[j * 4 + 3] = sq(nr[j].w, ni[j].w);
      }
    }
    if (ch + gridDim.x < nchunks) fetch(ch + gridDim.x);
#pragma unroll
    for (int h = 1; h < K; h <<= 1)
#pragma unroll
      for (int x = 0; x < K; x++)
        if (!(x & h)) {
          const double a = p[x], b = p[x + h];
          p[x] = a + b;
          p[x + h] = a - b;
        }
    // the transform goes through this thread's own LDS column, so each term
    // picks its slot with one indexed read instead of a select chain
#pragma unroll
    for (int x = 0; x < K; x++) wl[x][tid] = p[x];
    const uint32_t chl = (uint32_t)ch;
    // all SVI_ZTERMS slots run unconditionally (slots >= nt read slot 0 and
    // are never written out), so the reads batch without branches
#pragma unroll
    for (int t = 0; t < SVI_ZTERMS; t++) {
      const double sg = (__builtin_popcount(chl & zc[t]) & 1) ? -1.0 : 1.0;
      acc[t] = fma(sg, wl[zr[t]][tid], acc[t]);
    }
  }
#pragma unroll
  for (int t = 0; t < SVI_ZTERMS; t++) {
    if (t < nt) {
      const double v = wave_sum((tpar >> t) & 1 ? -acc[t] : acc[t]);
      if ((tid & 63) == 0) wsum[tid >> 6][t] = v;
    }
  }
  __syncthreads();
  if (tid < nt) {
    double v = 0.0;
    for (int w = 0; w < NT / 64; w++) v += wsum[w][tid];
    part[(int64_t)tid * gridDim.x + blockIdx.x] = v;
  }
}

// One Pauli term with an arbitrary x-mask, untiled: every work item reads
// psi_b and psi_{b^x} from HBM.  Used for terms whose X/Y support does not fit
// in a tile.  Expectation partial sums per workgroup in part[blockIdx];
// lam_b (+)= c (P psi)_b when lre is set.
template <typename T>
__global__ void __launch_bounds__(256) k_pauli_wide(const T *re, const T *im, T *lre, T *lim,
                                                    uint64_t x, uint64_t z, double cf, int64_t N,
                                                    int accumulate, double *part) {
  __shared__ double ws[4];
  const int ny = __builtin_popcountll(x & z) & 3;
  double acc = 0.0;
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < N;
       b += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t u = (uint64_t)b, p = u ^ x;
    const double br = (double)re[u], bi = (double)im[u], pr = (double)re[p], pi = (double)im[p];
    double tr, ti;
    switch (ny) {
      case 0: tr = br; ti = bi; break;
      case 1: tr = -bi; ti = br; break;
      case 2: tr = -br; ti = -bi; break;
      default: tr = bi; ti = -br; break;
    }
    if (__builtin_popcountll(u & z) & 1) { tr = -tr; ti = -ti; }
    acc += pr * tr + pi * ti;
    if (lre) {
      double vr, vi;
      switch (ny) {
        case 0: vr = pr; vi = pi; break;
        case 1: vr = -pi; vi = pr; break;
        case 2: vr = -pr; vi = -pi; break;
        default: vr = pi; vi = -pr; break;
      }
      if (__builtin_popcountll(p & z) & 1) { vr = -vr; vi = -vi; }
      const T ar = (T)(cf * vr), ai = (T)(cf * vi);
      if (accumulate) { lre[u] += ar; lim[u] += ai; }
      else { lre[u] = ar; lim[u] = ai; }
    }
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

// Tr(rho P) partial sums for a density matrix held as a 2n-qubit vector
// (rho_{rc} at index r 2^n + c): term t = blockIdx.y, rows r strided over the
// x-blocks; value = Re(i^nY (-1)^{|r & z|} rho_{r, r ^ x}).  Each block writes
// one partial, summed in a fixed order afterwards.
template <typename T>
__global__ void __launch_bounds__(256) k_dm_pauli(const T *re, const T *im, int n,
                                                  const PauliTermDev *terms, double *part) {
  __shared__ double ws[4];
  const PauliTermDev tm = terms[blockIdx.y];
  const int ny = __popcll(tm.x & tm.z) & 3;
  const int64_t R = 1ll << n;
  double acc = 0.0;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < R;
       r += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t idx = ((uint64_t)r << n) | ((uint64_t)r ^ tm.x);
    const double a = (double)re[idx], b = (double)im[idx];
    double v = ny == 0 ? a : ny == 1 ? -b : ny == 2 ? -a : b;
    if (__popcll((uint64_t)r & tm.z) & 1) v = -v;
    acc += v;
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

// One-qubit channel on a density matrix held as a vector: the 4x4 complex
// superoperator S (row-major, local index l = c + 2 r for column bit qc and
// row bit qr, qc < qr) acts on the four entries of each group; one read and
// one write of the vector.
struct ChannelArgs {
  void *re, *im;
  int64_t groups;     // 2^(N - 2)
  int qc, qr;
  double s[32];       // interleaved (re, im)
};

template <typename T>
__global__ void __launch_bounds__(256) k_dm_channel(ChannelArgs a) {
  T *re = (T *)a.re, *im = (T *)a.im;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < a.groups;
       g += (int64_t)gridDim.x * blockDim.x) {
    // insert zero bits at qc, then at qr
    uint64_t b = (uint64_t)g;
    b = ((b >> a.qc) << (a.qc + 1)) | (b & ((1ull << a.qc) - 1));
    b = ((b >> a.qr) << (a.qr + 1)) | (b & ((1ull << a.qr) - 1));
    uint64_t idx[4];
    double xr[4], xi[4];
#pragma unroll
    for (int l = 0; l < 4; l++) {
      idx[l] = b | ((uint64_t)(l & 1) << a.qc) | ((uint64_t)(l >> 1) << a.qr);
      xr[l] = (double)re[idx[l]];
      xi[l] = (double)im[idx[l]];
    }
#pragma unroll
    for (int o = 0; o < 4; o++) {
      double yr = 0.0, yi = 0.0;
#pragma unroll
      for (int l = 0; l < 4; l++) {
        const double sr = a.s[2 * (4 * o + l)], si = a.s[2 * (4 * o + l) + 1];
        yr += sr * xr[l] - si * xi[l];
        yi += sr * xi[l] + si * xr[l];
      }
      re[idx[o]] = (T)yr;
      im[idx[o]] = (T)yi;
    }
  }
}

// Two one-qubit channels in one pass: qubits a and b (column bits qa, qb,
// row bits qa + off, qb + off); each thread takes the 16 entries those four
// bits span, applies S_a to each group of four that differs only in a's bits,
// then S_b likewise, and writes once.
struct Channel2Args {
  void *re, *im;
  int64_t groups;     // 2^(N - 4)
  int qa, qb, off;
  int pos[4];         // the four bit positions, ascending
  double sa[32], sb[32];
};

template <typename T>
__global__ void __launch_bounds__(256) k_dm_channel2(Channel2Args a) {
  T *re = (T *)a.re, *im = (T *)a.im;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < a.groups;
       g += (int64_t)gridDim.x * blockDim.x) {
    uint64_t b = (uint64_t)g;
#pragma unroll
    for (int k = 0; k < 4; k++) b = ((b >> a.pos[k]) << (a.pos[k] + 1)) | (b & ((1ull << a.pos[k]) - 1));
    // entry e: bit 0 = a column, 1 = a row, 2 = b column, 3 = b row
    uint64_t idx[16];
    double xr[16], xi[16];
#pragma unroll
    for (int e = 0; e < 16; e++) {
      idx[e] = b | ((uint64_t)(e & 1) << a.qa) | ((uint64_t)((e >> 1) & 1) << (a.qa + a.off)) |
               ((uint64_t)((e >> 2) & 1) << a.qb) | ((uint64_t)((e >> 3) & 1) << (a.qb + a.off));
      xr[e] = (double)re[idx[e]];
      xi[e] = (double)im[idx[e]];
    }
#pragma unroll
    for (int hi = 0; hi < 4; hi++) {        // S_a on entries hi * 4 + la
      double yr[4], yi[4];
#pragma unroll
      for (int o = 0; o < 4; o++) {
        yr[o] = 0.0; yi[o] = 0.0;
#pragma unroll
        for (int l = 0; l < 4; l++) {
          const double sr = a.sa[2 * (4 * o + l)], si = a.sa[2 * (4 * o + l) + 1];
          yr[o] += sr * xr[4 * hi + l] - si * xi[4 * hi + l];
          yi[o] += sr * xi[4 * hi + l] + si * xr[4 * hi + l];
        }
      }
#pragma unroll
      for (int o = 0; o < 4; o++) { xr[4 * hi + o] = yr[o]; xi[4 * hi + o] = yi[o]; }
    }
#pragma unroll
    for (int lo = 0; lo < 4; lo++) {        // S_b on entries lb * 4 + lo
      double yr[4], yi[4];
#pragma unroll
      for (int o = 0; o < 4; o++) {
        yr[o] = 0.0; yi[o] = 0.0;
#pragma unroll
        for (int l = 0; l < 4; l++) {
          const double sr = a.sb[2 * (4 * o + l)], si = a.sb[2 * (4 * o + l) + 1];
          yr[o] += sr * xr[4 * l + lo] - si * xi[4 * l + lo];
          yi[o] += sr * xi[4 * l + lo] + si * xr[4 * l + lo];
        }
      }
#pragma unroll
      for (int o = 0; o < 4; o++) { xr[4 * o + lo] = yr[o]; xi[4 * o + lo] = yi[o]; }
    }
#pragma unroll
    for (int e = 0; e < 16; e++) {
      re[idx[e]] = (T)xr[e];
      im[idx[e]] = (T)xi[e];
    }
  }
}

// A two-qubit channel: the 16x16 complex superoperator S (device memory,
// row-major, interleaved; entry index e = column bits (q0, q1) + 4 * row bits
// (q0 + off, q1 + off)) on the 16 entries each thread takes; one read and one
// write of the vector.
struct Channel16Args {
  void *re, *im;
  const double *S;
  int64_t groups;     // 2^(N - 4)
  int q[4];           // bit of entry bits 0..3: q0, q1, q0 + off, q1 + off
  int pos[4];         // the same positions, ascending
};

template <typename T>
__global__ void __launch_bounds__(256) k_dm_channel16(Channel16Args a) {
  T *re = (T *)a.re, *im = (T *)a.im;
  const SVI_CONST double *S = cptr(a.S);
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < a.groups;
       g += (int64_t)gridDim.x * blockDim.x) {
    uint64_t b = (uint64_t)g;
#pragma unroll
    for (int k = 0; k < 4; k++) b = ((b >> a.pos[k]) << (a.pos[k] + 1)) | (b & ((1ull << a.pos[k]) - 1));
    uint64_t idx[16];
    double xr[16], xi[16];
#pragma unroll
    for (int e = 0; e < 16; e++) {
      idx[e] = b | ((uint64_t)(e & 1) << a.q[0]) | ((uint64_t)((e >> 1) & 1) << a.q[1]) |
               ((uint64_t)((e >> 2) & 1) << a.q[2]) | ((uint64_t)((e >> 3) & 1) << a.q[3]);
      xr[e] = (double)re[idx[e]];
      xi[e] = (double)im[idx[e]];
    }
    for (int o = 0; o < 16; o++) {
      double yr = 0.0, yi = 0.0;
#pragma unroll
      for (int l = 0; l < 16; l++) {
        const double sr = S[2 * (16 * o + l)], si = S[2 * (16 * o + l) + 1];
        yr += sr * xr[l] - si * xi[l];
        yi += sr * xi[l] + si * xr[l];
      }
      re[idx[o]] = (T)yr;
      im[idx[o]] = (T)yi;
    }
  }
}

// Up to five one-qubit channels in one pass through an LDS tile of 2^TB
// entries (TB = 12: up to four channels, 256 threads, two tiles per CU;
// TB = 13: five, 1024 threads, one tile per CU): the tile's vector bits are
// the channels' column and row bits and the lowest vector bits the channels
// leave free, and tile-index bit j is the j-th lowest of them (pos[j]), so a
// wave's loads run over the longest consecutive stretches; each channel's
// 4x4 superoperator is applied to the 2^(TB-2) groups of four entries that
// differ in its two bits, one channel after another, and the tile is written
// back once.
struct ChannelTileArgs {
  void *re, *im;
  int64_t tiles;      // 2^(N - TB)
  int k;              // channels in this pass (1..5)
  int pos[13];        // vector bit of tile-index bit j (TB of them)
  int sorted[13];     // pos, ascending
  int ci[5], ri[5];   // tile-index bits of channel i's column and row bits
  int real;           // every imaginary part of s is zero
  double s[32];
};

template <typename T, int TB>
__global__ void __launch_bounds__(TB == 13 ? 1024 : 256) k_dm_channel_tile(ChannelTileArgs a) {
  constexpr int NT = TB == 13 ? 1024 : 256;
  constexpr int LT = TB == 13 ? 10 : 8;   // tile-index bits of the thread
  constexpr int KB = TB - LT;              // tile-index bits of the unrolled element
  constexpr int EPT = 1 << KB;             // entries per thread
  __shared__ double2 lds[1 << TB];
  T *re = (T *)a.re, *im = (T *)a.im;
  const int tid = threadIdx.x;
  // Tile entry e = tid + NT k sits at base | loff | koff[k]: the deposit of
  // e's bits on pos[] splits into the thread's part (bits below LT) and a
  // part that depends only on the unrolled k (uniform: scalar).
  uint64_t loff = 0;
#pragma unroll
  for (int j = 0; j < LT; j++) loff |= (uint64_t)((tid >> j) & 1) << a.pos[j];
  uint64_t koff[EPT];
#pragma unroll
  for (int k = 0; k < EPT; k++) {
    koff[k] = 0;
#pragma unroll
    for (int j = 0; j < KB; j++) koff[k] |= (uint64_t)((k >> j) & 1) << a.pos[LT + j];
  }
  auto tile_base = [&](int64_t t) {
    uint64_t base = (uint64_t)t;
#pragma unroll
    for (int j = 0; j < TB; j++)
      base = ((base >> a.sorted[j]) << (a.sorted[j] + 1)) | (base & ((1ull << a.sorted[j]) - 1));
    return base | loff;
  };
  // With one 13-bit tile per CU no other tile's work hides the loads, so the
  // next tile is fetched into registers while this one's channels run; two
  // 12-bit tiles per CU overlap each other instead.
  constexpr bool PRE = TB == 13;
  T pr[PRE ? EPT : 1], pim[PRE ? EPT : 1];
  if constexpr (PRE) {
    if (blockIdx.x < a.tiles) {
      const uint64_t lb = tile_base(blockIdx.x);
#pragma unroll
      for (int k = 0; k < EPT; k++) {
        pr[k] = re[lb | koff[k]];
        pim[k] = im[lb | koff[k]];
      }
    }
  }
  for (int64_t t = blockIdx.x; t < a.tiles; t += gridDim.x) {
    const uint64_t lb = tile_base(t);
#pragma unroll
    for (int k = 0; k < EPT; k++) {
      if constexpr (PRE) {
        lds[tid + NT * k] = make_double2((double)pr[k], (double)pim[k]);
      } else {
        const uint64_t g = lb | koff[k];
        lds[tid + NT * k] = make_double2((double)re[g], (double)im[g]);
      }
    }
    __syncthreads();
    if constexpr (PRE) {
      const int64_t tn = t + gridDim.x;
      if (tn < a.tiles) {
        const uint64_t lbn = tile_base(tn);
#pragma unroll
        for (int k = 0; k < EPT; k++) {
          pr[k] = re[lbn | koff[k]];
          pim[k] = im[lbn | koff[k]];
        }
      }
    }
    for (int i = 0; i < a.k; i++) {
      const int c = a.ci[i], r = a.ri[i];
      const int lo = c < r ? c : r, hi = c < r ? r : c;
      for (int gi = tid; gi < (1 << (TB - 2)); gi += NT) {
        int e0 = ((gi >> lo) << (lo + 1)) | (gi & ((1 << lo) - 1));
        e0 = ((e0 >> hi) << (hi + 1)) | (e0 & ((1 << hi) - 1));
        int ix[4];
        double xr[4], xi[4];
#pragma unroll
        for (int l = 0; l < 4; l++) {
          ix[l] = e0 | ((l & 1) << c) | ((l >> 1) << r);
          const double2 v = lds[ix[l]];
          xr[l] = v.x;
          xi[l] = v.y;
        }
        // a real superoperator (depolarizing, dephasing, amplitude damping
        // and every other channel with real Kraus operators) takes half the
        // multiply-adds
        auto apply = [&](auto real) {
#pragma unroll
          for (int o = 0; o < 4; o++) {
            double yr = 0.0, yi = 0.0;
#pragma unroll
            for (int l = 0; l < 4; l++) {
              const double sr = a.s[2 * (4 * o + l)];
              if constexpr (decltype(real)::value) {
                yr += sr * xr[l];
                yi += sr * xi[l];
              } else {
                const double si = a.s[2 * (4 * o + l) + 1];
                yr += sr * xr[l] - si * xi[l];
                yi += sr * xi[l] + si * xr[l];
              }
            }
            lds[ix[o]] = make_double2(yr, yi);
          }
        };
        if (a.real) apply(std::true_type{});
        else apply(std::false_type{});
      }
      __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < EPT; k++) {
      const uint64_t g = lb | koff[k];
      const double2 v = lds[tid + NT * k];
      re[g] = (T)v.x;
      im[g] = (T)v.y;
    }
    __syncthreads();
  }
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
// E = sum_k c_k <P_k> with the coefficients taken from the device term list
// (pass order), so no host data is involved.
__global__ void k_energy_terms(const double *vals, const PauliTermDev *terms, int nt, double *out) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double e = 0.0;
    for (int k = 0; k < nt; k++) e += terms[k].c * vals[k];
    out[0] = e;
  }
}

__global__ void k_energy(const double *terms, const double *coef, int nt, double *out) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double e = 0.0;
    for (int j = 0; j < nt; j++) e += coef[j] * terms[j];
    out[0] = e;
  }
}

// ------------------------------------------------------------ sampling
// Fixed-order specification (see sv.h): p_b = fma(x, x, y*y); chunk sums by
// pairwise tree; blocked prefix; counter-based SplitMix64 uniforms.

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

// Prefix over the K chunk sums in blocks of G = min(K, 1024) chunks: the
// local exclusive prefix L_k of each block runs left to right, the block
// totals Q_j are prefixed left to right into the offsets E_j, and
// P_k = E_j + L_k, P_K = E_J.  Each chain is one lane's sequence of dependent
// additions, read from LDS in batches so the reads overlap the adds.
__device__ __forceinline__ double chain_lds(const double *v, double *w, int len, double acc) {
  for (int i0 = 0; i0 < len; i0 += 8) {
    double x[8];
#pragma unroll
    for (int j = 0; j < 8; j++) x[j] = (i0 + j < len) ? v[i0 + j] : 0.0;
#pragma unroll
    for (int j = 0; j < 8; j++)
      if (i0 + j < len) {
        w[i0 + j] = acc;
        acc = acc + x[j];
      }
  }
  return acc;
}

// One wave per block of G chunk sums: P[jG + i] <- L, Q[j] <- block total.
// Chunk sums for 1024-amplitude chunks, one wave per chunk and no LDS: lane l
// reads amplitudes 128 j + 2 l, +1 of each of the chunk's eight 128-wide
// slabs (coalesced), adds each pair (tree level 1), combines adjacent blocks
// across lanes with shuffle-downs by 1..32 (levels 2-7: lane 0 then holds
// each slab's sum), and lane 0 adds the eight slab sums pairwise (levels
// 8-10): the same pairwise tree as k_chunk_sums.
template <typename T>
__global__ void __launch_bounds__(256) k_chunk_sums_wave(const T *re, const T *im, int64_t K,
                                                         double *S) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = (int64_t)gridDim.x * 4;
  for (int64_t k = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); k < K; k += nw) {
    const uint64_t base = (uint64_t)k * 1024 + 2 * lane;
    double v[8];
#pragma unroll
    for (int j = 0; j < 8; j++) {
      const uint64_t b = base + 128 * j;
      v[j] = prob_at(re, im, b) + prob_at(re, im, b + 1);
    }
#pragma unroll
    for (int d = 1; d < 64; d <<= 1)
#pragma unroll
      for (int j = 0; j < 8; j++) v[j] = v[j] + __shfl_down(v[j], d);
    if (lane == 0) S[k] = ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
  }
}

__global__ void __launch_bounds__(64) k_prefix_local(const double *S, int G, double *P, double *Q) {
  __shared__ double v[1024], w[1024];
  const int64_t base = (int64_t)blockIdx.x * G;
  for (int i = threadIdx.x; i < G; i += 64) v[i] = S[base + i];
  __syncthreads();
  if (threadIdx.x == 0) Q[blockIdx.x] = chain_lds(v, w, G, 0.0);
  __syncthreads();
  for (int i = threadIdx.x; i < G; i += 64) P[base + i] = w[i];
}

// One wave: E[j] = sum of Q[0..j) left to right (J + 1 entries), P[K] = E[J].
__global__ void __launch_bounds__(64) k_prefix_blocks(const double *Q, int64_t J, double *E,
                                                      double *P, int64_t K) {
  __shared__ double v[1024], w[1024];
  __shared__ double carry;
  if (threadIdx.x == 0) carry = 0.0;
  for (int64_t b0 = 0; b0 < J; b0 += 1024) {
    const int len = (int)((J - b0) < 1024 ? (J - b0) : 1024);
    __syncthreads();
    for (int i = threadIdx.x; i < len; i += 64) v[i] = Q[b0 + i];
    __syncthreads();
    if (threadIdx.x == 0) carry = chain_lds(v, w, len, carry);
    __syncthreads();
    for (int i = threadIdx.x; i < len; i += 64) E[b0 + i] = w[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    E[J] = carry;
    P[K] = carry;
  }
}

// P_k = E_j + L_k for the G chunks of block j.
__global__ void __launch_bounds__(256) k_prefix_add(const double *E, int G, double *P) {
  const double e = E[blockIdx.x];
  const int64_t base = (int64_t)blockIdx.x * G;
  for (int i = threadIdx.x; i < G; i += 256) P[base + i] = e + P[base + i];
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
    const int64_t b0 = ks * C;
    if (C >= 16) {
      // same left-to-right accumulation, with the chunk's amplitudes read 16
      // at a time (independent loads) instead of one per dependent step
      for (int64_t i0 = 0; i0 < C && pick < 0; i0 += 16) {
        double p[16];
#pragma unroll
        for (int j = 0; j < 16; j++) p[j] = prob_at(re, im, (uint64_t)(b0 + i0 + j));
#pragma unroll
        for (int j = 0; j < 16; j++)
          if (pick < 0) {
            acc = acc + p[j];
            if (p[j] > 0.0) lastpos = b0 + i0 + j;
            if (acc > r) pick = b0 + i0 + j;
          }
      }
    } else {
      for (int64_t i = 0; i < C; i++) {
        const double p = prob_at(re, im, (uint64_t)(b0 + i));
        acc = acc + p;
        if (p > 0.0) lastpos = b0 + i;
        if (acc > r) { pick = b0 + i; break; }
      }
    }
    if (pick < 0) pick = lastpos >= 0 ? lastpos : b0;
    uint64_t o = 0;
    for (int i = 0; i < a.nq; i++) o |= (((uint64_t)pick >> a.qubits[i]) & 1ull) << i;
    a.out[s] = o;
  }
}

// FP64 draws with chunks of >= 8 amplitudes, done cooperatively: the 64
// shots of a wave walk their chunks together, 8 amplitudes per shot per step.
// Eight lanes fetch one shot's 8 re and 8 im values as 16-byte pieces (a
// 64-byte run per plane, so a load instruction covers 8 shots' runs instead
// of 64 scattered words), the pieces pass through LDS, and each lane then
// runs the same left-to-right accumulation as k_sample for its own shot.
__global__ void __launch_bounds__(256) k_sample_coop(SampleArgs a) {
  __shared__ double2 stage[4][64 * 9];  // per wave: 64 shots x 8 pieces, +1 pad
  const double *re = (const double *)a.re, *im = (const double *)a.im;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double2 *buf = stage[w];
  const int64_t C = 1ll << a.cbits;
  const double Tot = a.P[a.K];
  const int part = lane & 7;  // 0..3: pieces of re, 4..7: pieces of im
  const double *plane = part < 4 ? re : im;
  const int q2 = 2 * (part & 3);
  for (int64_t s0 = ((int64_t)blockIdx.x * 4 + w) * 64; s0 < a.shots;
       s0 += (int64_t)gridDim.x * 256) {
    const int64_t s = s0 + lane;
    const bool live = s < a.shots;
    int64_t ks = 0;
    double r = 0.0;
    if (live) {
      const double u = (double)(splitmix64(a.seed, (uint64_t)s) >> 11) * 0x1.0p-53;
      const double t = u * Tot;
      int64_t lo = 0, hi = a.K;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a.P[mid + 1] > t) hi = mid; else lo = mid + 1;
      }
      ks = lo;
      if (ks >= a.K) {
        ks = -1;
        for (int64_t k = a.K - 1; k >= 0; k--)
          if (a.S[k] > 0.0) { ks = k; break; }
        if (ks < 0) ks = 0;
      }
      r = t - a.P[ks];
    }
    const int64_t b0 = ks * C;
    double acc = 0.0;
    int64_t pick = live ? -1 : 0, lastpos = -1;
    long long src[8];
#pragma unroll
    for (int i = 0; i < 8; i++) src[i] = __shfl((long long)b0, 8 * i + (lane >> 3));
    for (int64_t i0 = 0; i0 < C; i0 += 8) {
      const unsigned long long todo = __ballot(pick < 0);
      if (todo == 0) break;
#pragma unroll
      for (int i = 0; i < 8; i++) {
        const int T = 8 * i + (lane >> 3);
        if ((todo >> T) & 1ull) buf[T * 9 + part] = *(const double2 *)(plane + src[i] + i0 + q2);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
      if (pick < 0) {
#pragma unroll
        for (int j = 0; j < 8; j++) {
          const double2 vr = buf[lane * 9 + (j >> 1)], vi = buf[lane * 9 + 4 + (j >> 1)];
          const double x = (j & 1) ? vr.y : vr.x, y = (j & 1) ? vi.y : vi.x;
          const double p = __fma_rn(x, x, y * y);
          if (pick < 0) {
            acc = acc + p;
            if (p > 0.0) lastpos = b0 + i0 + j;
            if (acc > r) pick = b0 + i0 + j;
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
    }
    if (live) {
      if (pick < 0) pick = lastpos >= 0 ? lastpos : b0;
      uint64_t o = 0;
      for (int i = 0; i < a.nq; i++) o |= (((uint64_t)pick >> a.qubits[i]) & 1ull) << i;
      a.out[s] = o;
    }
  }
}

// ------------------------------------------------------------ shot readout
// Integer counting over device samples: exact and independent of the order
// in which threads add their counts.

__global__ void __launch_bounds__(256) k_zero_u64(unsigned long long *p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

// counts[b] += number of samples equal to b (b < 2^nq)
__global__ void __launch_bounds__(256) k_histogram(const uint64_t *samples, int64_t shots,
                                                   unsigned long long *counts) {
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < shots;
       s += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&counts[samples[s]], 1ull);
}

// odd[m] += number of samples in this block's slice whose bits under
// masks[m] have odd parity (one thread per mask, slices along blockIdx.y)
__global__ void __launch_bounds__(256) k_parity_counts(const uint64_t *samples, int64_t shots,
                                                       const uint64_t *masks, int nm,
                                                       unsigned long long *odd) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (shots + gridDim.y - 1) / gridDim.y;
  const int64_t s0 = (int64_t)blockIdx.y * per;
  const int64_t s1 = s0 + per < shots ? s0 + per : shots;
  if (m >= nm || s0 >= s1) return;
  const uint64_t mask = masks[m];
  unsigned long long c = 0;
  for (int64_t s = s0; s < s1; s++) c += (unsigned long long)(__popcll(samples[s] & mask) & 1);
  atomicAdd(&odd[m], c);
}

#pragma clang fp contract(on)

}  // namespace

// ------------------------------------------------------------ launchers
// Host-callable wrappers (C++ linkage, used by sv_host.cpp).

#include "sv_launch.h"

// Sweep variants, one translation unit each (sv_sweep_variant.hip).
#include "sv_variants.h"

#define X(T, MM, RR, NN)                                                       \
  hipError_t SVI_VNAME(launch, T, MM, RR, NN)(const SweepArgs &, int, hipStream_t); \
  int SVI_VNAME(occ, T, MM, RR, NN)();                                            \
  hipError_t SVI_VNAME(launchk, T, MM, RR, NN)(const SweepArgs &, int, hipStream_t); \
  int SVI_VNAME(occk, T, MM, RR, NN)();
SVI_VARIANTS(X)
#undef X

hipError_t svk_launch_sweep_kron(int dbl, int M, int R, int NS, const SweepArgs &a, int grid,
                                 hipStream_t s) {
#define X(T, MM, RR, NN)                                                        \
  if (NN == NS && (dbl == (sizeof(T) == 8)) && M == MM && R == RR)              \
    return SVI_VNAME(launchk, T, MM, RR, NN)(a, grid, s);
  SVI_VARIANTS(X)
#undef X
  return hipErrorInvalidValue;
}

int svk_sweep_kron_occupancy(int dbl, int M, int R, int NS) {
#define X(T, MM, RR, NN)                                                        \
  if (NN == NS && (dbl == (sizeof(T) == 8)) && M == MM && R == RR)              \
    return SVI_VNAME(occk, T, MM, RR, NN)();
  SVI_VARIANTS(X)
#undef X
  return 0;
}

hipError_t svk_launch_sweep(int dbl, int M, int R, int NS, const SweepArgs &a, int grid,
                            hipStream_t s) {
#define X(T, MM, RR, NN)                                                        \
  if ((dbl == (sizeof(T) == 8)) && M == MM && R == RR && NS == NN)              \
    return SVI_VNAME(launch, T, MM, RR, NN)(a, grid, s);
  SVI_VARIANTS(X)
#undef X
  return hipErrorInvalidValue;
}

int svk_sweep_occupancy(int dbl, int M, int R, int NS) {
#define X(T, MM, RR, NN)                                                        \
  if ((dbl == (sizeof(T) == 8)) && M == MM && R == RR && NS == NN)              \
    return SVI_VNAME(occ, T, MM, RR, NN)();
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
                            const TabFactor *fac, double *coef, hipStream_t s) {
  if (nd <= 0) return hipSuccess;
  int grid = (nd + 127) / 128;
  hipLaunchKernelGGL(k_build_coefs, dim3(grid), dim3(128), 0, s, d, nd, params, statics, fac, coef);
  return hipGetLastError();
}

hipError_t svk_launch_pauli(int dbl, int M, const PauliPassArgs &a, int grid, hipStream_t s) {
  if (M != 12) return hipErrorInvalidValue;
  const bool lam = a.lre != nullptr;
  const dim3 blk((1 << 12) / 8);
  if (dbl && lam) hipLaunchKernelGGL((k_pauli<double, 12, true>), dim3(grid), blk, 0, s, a);
  else if (dbl) hipLaunchKernelGGL((k_pauli<double, 12, false>), dim3(grid), blk, 0, s, a);
  else if (lam) hipLaunchKernelGGL((k_pauli<float, 12, true>), dim3(grid), blk, 0, s, a);
  else hipLaunchKernelGGL((k_pauli<float, 12, false>), dim3(grid), blk, 0, s, a);
  return hipGetLastError();
}

hipError_t svk_launch_pauli_wide(int dbl, const void *re, const void *im, void *lre, void *lim,
                                 uint64_t x, uint64_t z, double c, int64_t N, int accumulate,
                                 double *part, int grid, hipStream_t s) {
  if (dbl)
    hipLaunchKernelGGL(k_pauli_wide<double>, dim3(grid), dim3(256), 0, s, (const double *)re,
                       (const double *)im, (double *)lre, (double *)lim, x, z, c, N, accumulate, part);
  else
    hipLaunchKernelGGL(k_pauli_wide<float>, dim3(grid), dim3(256), 0, s, (const float *)re,
                       (const float *)im, (float *)lre, (float *)lim, x, z, c, N, accumulate, part);
  return hipGetLastError();
}

int svk_pauli_occupancy(int dbl) {
  int nb = 0;
  hipError_t e = dbl ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_pauli<double, 12, true>, (1 << 12) / 8, 0)
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_pauli<float, 12, true>, (1 << 12) / 8, 0);
  return (e == hipSuccess && nb > 0) ? nb : 1;
}

hipError_t svk_launch_dm_channel(int dbl, void *re, void *im, int nq, int qc, int qr,
                                 const double *s32, hipStream_t s) {
  ChannelArgs a;
  a.re = re; a.im = im;
  a.groups = 1ll << (nq - 2);
  a.qc = qc; a.qr = qr;
  for (int i = 0; i < 32; i++) a.s[i] = s32[i];
  const int grid = (int)std::min<int64_t>((a.groups + 255) / 256, 16384);
  if (dbl) hipLaunchKernelGGL(k_dm_channel<double>, dim3(grid), dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_dm_channel<float>, dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t svk_launch_dm_channel2(int dbl, void *re, void *im, int nq, int qa, int qb, int off,
                                  const double *sa, const double *sb, hipStream_t s) {
  Channel2Args a;
  a.re = re; a.im = im;
  a.groups = 1ll << (nq - 4);
  a.qa = qa; a.qb = qb; a.off = off;
  int p[4] = {qa, qb, qa + off, qb + off};
  std::sort(p, p + 4);
  for (int k = 0; k < 4; k++) a.pos[k] = p[k];
  for (int i = 0; i < 32; i++) { a.sa[i] = sa[i]; a.sb[i] = sb[i]; }
  const int grid = (int)std::min<int64_t>((a.groups + 255) / 256, 16384);
  if (dbl) hipLaunchKernelGGL(k_dm_channel2<double>, dim3(grid), dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_dm_channel2<float>, dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t svk_launch_dm_channel16(int dbl, void *re, void *im, int nq, int q0, int q1, int off,
                                   const double *d_S, hipStream_t s) {
  Channel16Args a;
  a.re = re; a.im = im; a.S = d_S;
  a.groups = 1ll << (nq - 4);
  a.q[0] = q0; a.q[1] = q1; a.q[2] = q0 + off; a.q[3] = q1 + off;
  int p[4] = {a.q[0], a.q[1], a.q[2], a.q[3]};
  std::sort(p, p + 4);
  for (int k = 0; k < 4; k++) a.pos[k] = p[k];
  const int grid = (int)std::min<int64_t>((a.groups + 255) / 256, 16384);
  if (dbl) hipLaunchKernelGGL(k_dm_channel16<double>, dim3(grid), dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_dm_channel16<float>, dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t svk_launch_dm_channel_tile(int dbl, void *re, void *im, int nq, int off,
                                      const int *qubits, int k, const double *s32, hipStream_t s) {
  const int TB = k == 5 ? 13 : 12;
  if (nq < TB || k < 1 || k > 5) return hipErrorInvalidValue;
  ChannelTileArgs a;
  a.re = re; a.im = im;
  a.tiles = 1ll << (nq - TB);
  a.k = k;
  uint64_t used = 0;
  for (int i = 0; i < k; i++) used |= (1ull << qubits[i]) | (1ull << (qubits[i] + off));
  int chan[10], nc = 0;
  for (int b = 0; b < nq; b++)
    if (used >> b & 1) chan[nc++] = b;
  if (nc != 2 * k) return hipErrorInvalidValue;   // the qubits must be distinct
  int np = 0;
  for (int b = 0; b < nq && np < TB - nc; b++)
    if (!(used >> b & 1)) a.pos[np++] = b;
  if (np + nc != TB) return hipErrorInvalidValue;
  for (int j = 0; j < nc; j++) a.pos[np + j] = chan[j];
  std::sort(a.pos, a.pos + TB);   // lanes run over the lowest of the tile's vector bits
  for (int j = 0; j < TB; j++) a.sorted[j] = a.pos[j];
  for (int j = TB; j < 13; j++) a.pos[j] = a.sorted[j] = 0;
  for (int i = 0; i < k; i++)
    for (int j = 0; j < TB; j++) {
      if (a.pos[j] == qubits[i]) a.ci[i] = j;
      if (a.pos[j] == qubits[i] + off) a.ri[i] = j;
    }
  a.real = 1;
  for (int i = 0; i < 32; i++) {
    a.s[i] = s32[i];
    if ((i & 1) && s32[i] != 0.0) a.real = 0;
  }
  if (TB == 13) {
    // one persistent workgroup per CU, each walking its tiles with the
    // register prefetch
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const int grid = (int)std::min<int64_t>(a.tiles, std::max(cus, 1));
    if (dbl) hipLaunchKernelGGL((k_dm_channel_tile<double, 13>), dim3(grid), dim3(1024), 0, s, a);
    else hipLaunchKernelGGL((k_dm_channel_tile<float, 13>), dim3(grid), dim3(1024), 0, s, a);
  } else {
    const int grid = (int)std::min<int64_t>(a.tiles, 8192);
    if (dbl) hipLaunchKernelGGL((k_dm_channel_tile<double, 12>), dim3(grid), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_dm_channel_tile<float, 12>), dim3(grid), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t svk_launch_dm_pauli(int dbl, const void *re, const void *im, int n,
                               const PauliTermDev *terms, int nt, int nb, double *part,
                               hipStream_t s) {
  if (dbl) hipLaunchKernelGGL(k_dm_pauli<double>, dim3(nb, nt), dim3(256), 0, s, (const double *)re, (const double *)im, n, terms, part);
  else hipLaunchKernelGGL(k_dm_pauli<float>, dim3(nb, nt), dim3(256), 0, s, (const float *)re, (const float *)im, n, terms, part);
  return hipGetLastError();
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

hipError_t svk_launch_zexp(int dbl, const void *re, const void *im, int n, const PauliTermDev *terms,
                           int nt, double *part, int grid, hipStream_t s) {
  if (nt < 1 || nt > SVI_ZTERMS) return hipErrorInvalidValue;
  const int64_t ch = dbl ? 2048 : 4096;
  const int64_t N = (int64_t)1 << n;
  if (N < ch) return hipErrorInvalidValue;
  if (dbl)
    hipLaunchKernelGGL(k_zexp<double>, dim3(grid), dim3(256), 0, s, (const double *)re,
                       (const double *)im, N / ch, terms, nt, part);
  else
    hipLaunchKernelGGL(k_zexp<float>, dim3(grid), dim3(256), 0, s, (const float *)re,
                       (const float *)im, N / ch, terms, nt, part);
  return hipGetLastError();
}

int svk_zexp_occupancy(int dbl) {
  int nb = 0;
  hipError_t e = dbl ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_zexp<double>, 256, 0)
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_zexp<float>, 256, 0);
  return (e == hipSuccess && nb > 0) ? nb : 1;
}

hipError_t svk_launch_energy_terms(const double *vals, const PauliTermDev *terms, int nt,
                                   double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_energy_terms, dim3(1), dim3(64), 0, s, vals, terms, nt, out);
  return hipGetLastError();
}

hipError_t svk_launch_sampling(int dbl, const void *re, const void *im, int n, double *S, double *P,
                               double *QE, uint64_t seed, int64_t shots, const int32_t *qubits,
                               int nq, uint64_t *out, hipStream_t s) {
  const int cbits = n < 10 ? n : 10;
  const int64_t K = (1ll << n) >> cbits;
  int grid = (int)(K < 4096 ? K : 4096);
  if (cbits == 10) {
    const int gw = (int)std::min<int64_t>((K + 3) / 4, 8192);
    if (dbl) hipLaunchKernelGGL(k_chunk_sums_wave<double>, dim3(gw), dim3(256), 0, s, (const double *)re, (const double *)im, K, S);
    else hipLaunchKernelGGL(k_chunk_sums_wave<float>, dim3(gw), dim3(256), 0, s, (const float *)re, (const float *)im, K, S);
  } else if (dbl) {
    hipLaunchKernelGGL(k_chunk_sums<double>, dim3(grid), dim3(256), 0, s, (const double *)re, (const double *)im, cbits, K, S);
  } else {
    hipLaunchKernelGGL(k_chunk_sums<float>, dim3(grid), dim3(256), 0, s, (const float *)re, (const float *)im, cbits, K, S);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int G = (int)(K < 1024 ? K : 1024);
  const int64_t J = K / G;
  double *Q = QE, *E = QE + J;
  hipLaunchKernelGGL(k_prefix_local, dim3((unsigned)J), dim3(64), 0, s, S, G, P, Q);
  hipLaunchKernelGGL(k_prefix_blocks, dim3(1), dim3(64), 0, s, Q, J, E, P, K);
  hipLaunchKernelGGL(k_prefix_add, dim3((unsigned)J), dim3(256), 0, s, E, G, P);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (shots <= 0) return hipSuccess;
  SampleArgs a;
  a.re = re; a.im = im; a.S = S; a.P = P; a.K = K; a.cbits = cbits; a.nq = nq;
  for (int i = 0; i < 64; i++) a.qubits[i] = i < nq ? qubits[i] : 0;
  a.seed = seed; a.shots = shots; a.out = out;
  int64_t blocks = (shots + 255) / 256;
  int g2 = (int)(blocks < 4096 ? blocks : 4096);
  // both kernels draw the same indices; the cooperative one pays off once
  // there are enough waves to keep the memory system busy
  if (dbl && cbits >= 3 && shots >= 4096)
    hipLaunchKernelGGL(k_sample_coop, dim3(g2), dim3(256), 0, s, a);
  else if (dbl) hipLaunchKernelGGL(k_sample<double>, dim3(g2), dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_sample<float>, dim3(g2), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t svk_launch_histogram(const uint64_t *samples, int64_t shots, int nq,
                                uint64_t *counts, hipStream_t s) {
  const int64_t nb = 1ll << nq;
  unsigned long long *c = (unsigned long long *)counts;
  hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)std::min<int64_t>((nb + 255) / 256, 4096)), dim3(256), 0,
                     s, c, nb);
  if (shots > 0)
    hipLaunchKernelGGL(k_histogram, dim3((unsigned)std::min<int64_t>((shots + 255) / 256, 4096)),
                       dim3(256), 0, s, samples, shots, c);
  return hipGetLastError();
}

hipError_t svk_launch_parity_counts(const uint64_t *samples, int64_t shots, const uint64_t *masks,
                                    int nm, uint64_t *odd, hipStream_t s) {
  unsigned long long *o = (unsigned long long *)odd;
  hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)std::min<int64_t>((nm + 255) / 256, 4096)), dim3(256), 0,
                     s, o, (int64_t)nm);
  if (shots > 0 && nm > 0) {
    const unsigned gx = (unsigned)((nm + 255) / 256);
    // enough slices along y for a few hundred blocks, each at least 1024 shots long
    int64_t gy = std::max<int64_t>(1, std::min<int64_t>((shots + 1023) / 1024, 1024 / (int64_t)gx));
    hipLaunchKernelGGL(k_parity_counts, dim3(gx, (unsigned)gy), dim3(256), 0, s, samples, shots,
                       masks, nm, o);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------ ragged batch
// Persistent batch kernel variants (sv_batch_variant.hip) and the two small
// kernels around it: queue reset (a kernel rather than a memset, so a captured
// graph replays it reliably) and the per-circuit observable reduction.

#define X(T, MM, RR)                                                                     \
  hipError_t SVB_VNAME(launch, T, MM, RR)(const BatchKernelArgs &, int, int, hipStream_t); \
  int SVB_VNAME(occ, T, MM, RR)(int);
SVB_VARIANTS(X)
#undef X

hipError_t svk_launch_batch(int dbl, int M, int R, int kron_only, const BatchKernelArgs &a,
                            int grid, hipStream_t s) {
#define X(T, MM, RR)                                                  \
  if ((dbl == (sizeof(T) == 8)) && M == MM && R == RR)                \
    return SVB_VNAME(launch, T, MM, RR)(a, grid, kron_only, s);
  SVB_VARIANTS(X)
#undef X
  return hipErrorInvalidValue;
}

int svk_batch_occupancy(int dbl, int M, int R, int kron_only) {
#define X(T, MM, RR)                                                  \
  if ((dbl == (sizeof(T) == 8)) && M == MM && R == RR) return SVB_VNAME(occ, T, MM, RR)(kron_only);
  SVB_VARIANTS(X)
#undef X
  return 0;
}

int svk_has_batch(int dbl, int M, int R) {
#define X(T, MM, RR)                                                  \
  if ((dbl == (sizeof(T) == 8)) && M == MM && R == RR) return 1;
  SVB_VARIANTS(X)
#undef X
  return 0;
}

namespace {

__global__ void k_batch_reset(int32_t *head, int32_t *done, int32_t *err, int nc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    *head = 0;
    *err = 0;
  }
  if (i < nc) done[i] = 0;
}

// out[c] = sum over entries k of circuit c (rows rowptr[c]..rowptr[c+1]) of
// coef[k] * part[slot[k]], in entry order.
__global__ void k_batch_reduce(const int32_t *rowptr, const int32_t *slot, const double *coef,
                               const double *part, double *out, int nc) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  double e = 0.0;
  for (int k = rowptr[c]; k < rowptr[c + 1]; k++) e += coef[k] * part[slot[k]];
  out[c] = e;
}

}  // namespace

hipError_t svk_launch_batch_reset(int32_t *head, int32_t *done, int32_t *err, int nc,
                                  hipStream_t s) {
  const int n = nc > 1 ? nc : 1;
  hipLaunchKernelGGL(k_batch_reset, dim3((n + 255) / 256), dim3(256), 0, s, head, done, err, nc);
  return hipGetLastError();
}

hipError_t svk_launch_batch_reduce(const int32_t *rowptr, const int32_t *slot, const double *coef,
                                   const double *part, double *out, int nc, hipStream_t s) {
  if (nc <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_reduce, dim3((nc + 255) / 256), dim3(256), 0, s, rowptr, slot, coef,
                     part, out, nc);
  return hipGetLastError();
}

// ------------------------------------------------------------- serving
// Small adjoint requests, one workgroup each (see ServeReq).  The tiling is
// fixed: 12-qubit tiles of 8-amplitude register groups, 512 threads; psi and
// lambda tiles side by side take 128 KiB of LDS, so one workgroup runs per CU
// and a request of n <= 12 qubits is one tile per sweep.
#define SVS_M 12
#define SVS_R 3

namespace {

// Coefficients of every request: blockIdx.y = request, both plans.
__global__ void __launch_bounds__(256) k_serve_coefs(const ServeReq *reqs) {
  const ServeReq &q = reqs[blockIdx.y];
  const int nd = q.f_ndesc + q.b_ndesc;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nd; i += gridDim.x * blockDim.x) {
    if (i < q.f_ndesc) build_coef(q.f_desc[i], q.f_params, nullptr, q.f_fac, q.f_coef);
    else build_coef(q.b_desc[i - q.f_ndesc], q.b_params, nullptr, q.b_fac, q.b_coef);
  }
}

// GEN: the requests' plans hold micro-op (interpreter) stages; without it
// every stage of every sweep is a Kronecker stage and the kernel is leaner.
template <typename T, int M, int R, bool GEN>
__global__ void __launch_bounds__(1 << (M - R)) k_serve(ServeArgs sa) {
  constexpr int NT = 1 << (M - R);
  constexpr int NWAVE = NT / 64;
  using C2 = typename C2T<T>::type;
  __shared__ __align__(16) char tiles[2 * (1 << M) * sizeof(C2)];
  __shared__ double wacc[NWAVE][SVI_GSLOTS_MAX];
  __shared__ double wred[NWAVE];
  __shared__ int32_t hb_s[SVI_MMAX];
  __shared__ int32_t req_s;
  C2 *const lt = (C2 *)tiles;
  const int tid = threadIdx.x;
  // the queue counter is taken by wave 0 as a whole wave (one lane adds 1)
  const bool wave0 = __builtin_amdgcn_readfirstlane(tid) == 0;
  const int one = tid == 0 ? 1 : 0;
  for (;;) {
    if (wave0) {
      const int v = __hip_atomic_fetch_add(sa.head, one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (tid == 0) req_s = v;
    }
    __syncthreads();
    const int r = __builtin_amdgcn_readfirstlane(req_s);
    __syncthreads();
    if (r >= sa.nreq) break;
    const ServeReq &q = sa.reqs[r];

    // ---- forward: the circuit from |0..0> (the first sweep synthesises it)
    for (int s = 0; s < q.f_nsweeps; s++) {
      const SVI_CONST SweepArgs &a = cptr(sa.sweeps)[q.f_sweep + s];
      sweep_tiles<T, M, R, !GEN>(a, 0, a.ntiles, lt, hb_s);
    }
    __syncthreads();

    // ---- lambda = H psi and E = Re <psi|lambda> (paper Section 4.4 Pauli
    // action: P|b> = i^{nY} (-1)^{popcount(b & z)} |b ^ x>)
    double e = 0.0;
    {
      const int64_t N = (int64_t)1 << q.n;
      const T *pr = (const T *)q.re, *pim = (const T *)q.im;
      T *lr = (T *)q.lre, *li = (T *)q.lim;
      for (int64_t b = tid; b < N; b += NT) {
        double ar = 0.0, ai = 0.0;
        for (int t = 0; t < q.n_terms; t++) {
          const uint64_t x = q.terms[t].x, z = q.terms[t].z;
          const double c = q.terms[t].c;
          const uint64_t src = (uint64_t)b ^ x;
          const double sr = (double)pr[src], si = (double)pim[src];
          double tr, ti;
          switch (__builtin_popcountll(x & z) & 3) {   // i^{nY}
            case 0: tr = sr; ti = si; break;
            case 1: tr = -si; ti = sr; break;
            case 2: tr = -sr; ti = -si; break;
            default: tr = si; ti = -sr; break;
          }
          if (__builtin_popcountll(src & z) & 1) { tr = -tr; ti = -ti; }
          ar += c * tr;
          ai += c * ti;
        }
        lr[b] = (T)ar;
        li[b] = (T)ai;
        e += (double)pr[b] * ar + (double)pim[b] * ai;
      }
      e = wave_sum(e);
      if ((tid & 63) == 0) wred[tid >> 6] = e;
      __syncthreads();
      e = 0.0;
      for (int w = 0; w < NWAVE; w++) e += wred[w];
    }
    __syncthreads();

    // ---- backward: two-state sweeps; each gradient term is summed over the
    // wave, then added to the wave's LDS row of its slot (in tile and stage
    // order: deterministic), and the rows are summed per sweep
    for (int s = 0; s < q.b_nsweeps; s++) {
      const SVI_CONST SweepArgs &a = cptr(sa.sweeps)[q.b_sweep + s];
      const int m = a.m, c = a.c, nh = a.nh;
      const int ntile_el = 1 << m;
      const int nst = a.stage_end - a.stage_begin;
      const SVI_CONST StageDesc *stages = cptr(a.stages + a.stage_begin);
      const SVI_CONST double *coef = cptr(a.coef);
      T *const pr[2] = {(T *)a.re, (T *)a.re2};
      T *const pi[2] = {(T *)a.im, (T *)a.im2};
      if (tid < SVI_MMAX) hb_s[tid] = a.hb[tid < nh ? tid : 0];
      for (int k = tid; k < NWAVE * SVI_GSLOTS_MAX; k += NT) (&wacc[0][0])[k] = 0.0;
      __syncthreads();
      const bool active = tid < (1 << (m > R ? m - R : 0));
      for (int64_t tile = 0; tile < a.ntiles; tile++) {
        const uint64_t base = tile_base(tile, c, hb_s, nh);
        for (int st2 = 0; st2 < 2; st2++)
          for (int i = tid; i < ntile_el; i += NT) {
            const uint64_t g = base + spread_row(i >> c, hb_s, nh) + (uint64_t)(i & ((1 << c) - 1));
            lt[st2 * (1 << M) + swz<T>(i)] = C2{pr[st2][g], pi[st2][g]};
          }
        __syncthreads();
        for (int st = 0; st < nst; st++) {
          const SVI_CONST StageDesc &sd = stages[st];
          const int gbs = swz<T>(stage_base<M, R>(tid, sd)) * (int)sizeof(C2);
          auto sink = [&](int s0, int s1, double t) {
            wave_deposit2(wacc[tid >> 6], s0, s1, t, tid & 63);
          };
          if (!GEN || sd.kind == ST_KRON)
            kron2_stage<T, R>((char *)lt, (char *)(lt + (1 << M)), gbs, sd, coef, a.ops, a.coef, active,
                              sink);
          else if constexpr (GEN)
            ops2_stage<T, R>((char *)lt, (char *)(lt + (1 << M)), gbs, sd, a.ops, a.coef, active, sink);
        }
        for (int st2 = 0; st2 < 2; st2++)
          for (int i = tid; i < ntile_el; i += NT) {
            const uint64_t g = base + spread_row(i >> c, hb_s, nh) + (uint64_t)(i & ((1 << c) - 1));
            const C2 p = lt[st2 * (1 << M) + swz<T>(i)];
            pr[st2][g] = p.x;
            pi[st2][g] = p.y;
          }
        __syncthreads();
      }
      for (int sl = tid; sl < a.n_gslots; sl += NT) {
        double v = 0.0;
        for (int w = 0; w < NWAVE; w++) v += wacc[w][sl];
        q.slots[a.gslot_begin + sl] = v;
      }
      __syncthreads();
    }

    // ---- dE/dtheta_p: the parameter's slots in slot order
    for (int p = tid; p < q.n_params; p += NT) {
      double g = 0.0;
      for (int k = q.rowptr[p]; k < q.rowptr[p + 1]; k++) g += q.slots[q.gslots[k]];
      q.out[1 + p] = g;
    }
    if (tid == 0) q.out[0] = e;
    __syncthreads();
  }
}

}  // namespace

// Requests of up to 16 qubits: beyond the 12-qubit tile a request's planes
// (at most 4 x 512 KiB) stay in the L2 and last-level caches between sweeps.
int svk_serve_max_qubits() { return 16; }

hipError_t svk_launch_serve_coefs(const ServeReq *d_reqs, int nreq, int max_desc, hipStream_t s) {
  if (nreq <= 0) return hipSuccess;
  const int bx = max_desc > 0 ? (max_desc + 255) / 256 : 1;
  hipLaunchKernelGGL(k_serve_coefs, dim3(bx < 64 ? bx : 64, nreq), dim3(256), 0, s, d_reqs);
  return hipGetLastError();
}

hipError_t svk_launch_serve(const ServeReq *d_reqs, const SweepArgs *d_sweeps, int32_t *d_head,
                            int nreq, int general, int grid, hipStream_t s) {
  if (nreq <= 0) return hipSuccess;
  ServeArgs a;
  a.reqs = d_reqs;
  a.sweeps = d_sweeps;
  a.head = d_head;
  a.nreq = nreq;
  if (general)
    hipLaunchKernelGGL((k_serve<double, SVS_M, SVS_R, true>), dim3(grid), dim3(1 << (SVS_M - SVS_R)), 0,
                       s, a);
  else
    hipLaunchKernelGGL((k_serve<double, SVS_M, SVS_R, false>), dim3(grid), dim3(1 << (SVS_M - SVS_R)), 0,
                       s, a);
  return hipGetLastError();
}

int svk_serve_tiling(int *M, int *R) {
  *M = SVS_M;
  *R = SVS_R;
  return 1 << (SVS_M - SVS_R);
}
