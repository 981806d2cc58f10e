/*
 * CPU oracle for the state-vector path -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain C99 with interleaved complex128, no fusion, no SIMD intrinsics, built
 * with -O2 -ffp-contract=off.  Gates are applied one at a time exactly as the
 * gather / multiply / scatter of the paper's gate-application equation
 * (Section 5.3): for every basis index whose target bits are zero and whose
 * control bits match, gather the 2^k amplitudes, multiply by the local matrix,
 * scatter back.  The only parallelism is an optional OpenMP loop over those
 * independent groups, used when timing large states.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.
 */
#include "sv_oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

static const double PI = 3.14159265358979323846;

int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

static int n_params_of(int kind) {
  switch (kind) {
    case ORC_RX: case ORC_RY: case ORC_RZ: case ORC_P:
    case ORC_RXX: case ORC_RYY: case ORC_RZZ: case ORC_GIVENS: case ORC_DEXC:
      return 1;
    case ORC_U2: return 2;
    case ORC_U3: return 3;
    default: return 0;
  }
}

static int n_targets_of(const orc_op *op) {
  switch (op->kind) {
    case ORC_SWAP: case ORC_RXX: case ORC_RYY: case ORC_RZZ: case ORC_GIVENS: return 2;
    case ORC_DEXC: return 4;
    case ORC_UNITARY: return op->n_targets;
    default: return 1;
  }
}

/* ------------------------------------------------------------ gate matrices
 * Written entry by entry from the textbook definitions (paper Section 4.2 gate
 * table; rotation convention exp(-i theta P / 2), Section 9.1).  m is d x d,
 * row-major, d = 2^k. */

static void set_identity(cplx *m, int d) {
  for (int i = 0; i < d * d; i++) m[i] = 0.0;
  for (int i = 0; i < d; i++) m[i * d + i] = 1.0;
}

/* Rotation within the 2-dim subspace spanned by local indices a and b:
 * |a> -> c|a> + s|b>, |b> -> -s|a> + c|b>. */
static void subspace_rotation(cplx *m, int d, int a, int b, double cth, double sth) {
  set_identity(m, d);
  m[a * d + a] = cth;
  m[a * d + b] = -sth;
  m[b * d + a] = sth;
  m[b * d + b] = cth;
}

static int build_matrix(const orc_op *op, const double *params, int dwhich, cplx *m) {
  /* dwhich < 0: the matrix itself.  dwhich >= 0: derivative w.r.t. that
   * parameter slot, entry by entry. */
  double th[3] = {0, 0, 0};
  int np_ = n_params_of(op->kind);
  for (int i = 0; i < np_; i++) th[i] = params[op->param_index[i]];
  int k = n_targets_of(op);
  int d = 1 << k;
  const int der = dwhich >= 0;
  if (der && dwhich >= np_) return -1;
  double h = th[0] / 2.0;
  double c = cos(h), s = sin(h);
  /* dc/dtheta = -s/2, ds/dtheta = c/2 */
  double dc = -s / 2.0, ds = c / 2.0;
  double cc = der ? dc : c, ss = der ? ds : s;
  const double r2 = 1.0 / sqrt(2.0);
  for (int i = 0; i < d * d; i++) m[i] = 0.0;
  switch (op->kind) {
    case ORC_I: set_identity(m, 2); break;
    case ORC_X: m[1] = 1; m[2] = 1; break;
    case ORC_Y: m[1] = -I; m[2] = I; break;
    case ORC_Z: m[0] = 1; m[3] = -1; break;
    case ORC_H: m[0] = r2; m[1] = r2; m[2] = r2; m[3] = -r2; break;
    case ORC_S: m[0] = 1; m[3] = I; break;
    case ORC_SDG: m[0] = 1; m[3] = -I; break;
    case ORC_T: m[0] = 1; m[3] = cexp(I * PI / 4.0); break;
    case ORC_TDG: m[0] = 1; m[3] = cexp(-I * PI / 4.0); break;
    case ORC_SX:
      m[0] = 0.5 * (1 + I); m[1] = 0.5 * (1 - I);
      m[2] = 0.5 * (1 - I); m[3] = 0.5 * (1 + I);
      break;
    case ORC_RX: m[0] = cc; m[1] = -I * ss; m[2] = -I * ss; m[3] = cc; break;
    case ORC_RY: m[0] = cc; m[1] = -ss; m[2] = ss; m[3] = cc; break;
    case ORC_RZ:
      if (!der) { m[0] = cexp(-I * h); m[3] = cexp(I * h); }
      else { m[0] = -0.5 * I * cexp(-I * h); m[3] = 0.5 * I * cexp(I * h); }
      break;
    case ORC_P:
      if (!der) { m[0] = 1; m[3] = cexp(I * th[0]); }
      else { m[0] = 0; m[3] = I * cexp(I * th[0]); }
      break;
    case ORC_U2: case ORC_U3: {
      /* U3(t, f, l) = [[cos(t/2), -e^{il} sin(t/2)], [e^{if} sin(t/2), e^{i(f+l)} cos(t/2)]];
       * U2(f, l) = U3(pi/2, f, l). */
      double t, f, l;
      int wt, wf, wl; /* which slot each angle came from */
      if (op->kind == ORC_U3) { t = th[0]; f = th[1]; l = th[2]; wt = 0; wf = 1; wl = 2; }
      else { t = PI / 2.0; f = th[0]; l = th[1]; wt = -1; wf = 0; wl = 1; }
      double ct = cos(t / 2.0), st = sin(t / 2.0);
      cplx ef = cexp(I * f), el = cexp(I * l), efl = cexp(I * (f + l));
      if (!der) {
        m[0] = ct; m[1] = -el * st; m[2] = ef * st; m[3] = efl * ct;
      } else if (dwhich == wt) {
        m[0] = -st / 2.0; m[1] = -el * ct / 2.0; m[2] = ef * ct / 2.0; m[3] = -efl * st / 2.0;
      } else if (dwhich == wf) {
        m[0] = 0; m[1] = 0; m[2] = I * ef * st; m[3] = I * efl * ct;
      } else if (dwhich == wl) {
        m[0] = 0; m[1] = -I * el * st; m[2] = 0; m[3] = I * efl * ct;
      } else {
        return -1;
      }
      break;
    }
    case ORC_SWAP:
      m[0 * 4 + 0] = 1; m[1 * 4 + 2] = 1; m[2 * 4 + 1] = 1; m[3 * 4 + 3] = 1;
      break;
    case ORC_RXX: case ORC_RYY: {
      /* exp(-i h P(x)P) = c I - i s P(x)P.  XX maps j -> 3 - j with phase 1;
       * YY maps j -> 3 - j with phase -1 on |00>,|11> and +1 on |01>,|10>. */
      for (int j = 0; j < 4; j++) {
        m[j * 4 + j] = cc;
        double ph = 1.0;
        if (op->kind == ORC_RYY) ph = (j == 0 || j == 3) ? -1.0 : 1.0;
        m[(3 - j) * 4 + j] = -I * ss * ph;
      }
      break;
    }
    case ORC_RZZ:
      for (int j = 0; j < 4; j++) {
        int par = (j & 1) ^ ((j >> 1) & 1);
        /* parity 0: e^{-ih}; parity 1: e^{+ih} */
        double sg = par ? 1.0 : -1.0;
        m[j * 4 + j] = der ? (sg * 0.5 * I * cexp(sg * I * h)) : cexp(sg * I * h);
      }
      break;
    case ORC_GIVENS:
      if (!der) subspace_rotation(m, 4, 1, 2, c, s);
      else {
        for (int i = 0; i < 16; i++) m[i] = 0.0;
        m[1 * 4 + 1] = dc; m[1 * 4 + 2] = -ds; m[2 * 4 + 1] = ds; m[2 * 4 + 2] = dc;
      }
      break;
    case ORC_DEXC:
      if (!der) subspace_rotation(m, 16, 3, 12, c, s);
      else {
        for (int i = 0; i < 256; i++) m[i] = 0.0;
        m[3 * 16 + 3] = dc; m[3 * 16 + 12] = -ds; m[12 * 16 + 3] = ds; m[12 * 16 + 12] = dc;
      }
      break;
    case ORC_UNITARY:
      if (der) return -1;
      if (!op->matrix || k < 1 || k > 5) return -1;
      for (int i = 0; i < d * d; i++) m[i] = op->matrix[2 * i] + I * op->matrix[2 * i + 1];
      break;
    default:
      return -1;
  }
  if (der && np_ == 0) return -1;
  return 0;
}

int orc_gate_matrix(const orc_op *op, const double *params, double *m) {
  cplx buf[1024];
  if (build_matrix(op, params, -1, buf)) return -1;
  int d = 1 << n_targets_of(op);
  for (int i = 0; i < d * d; i++) { m[2 * i] = creal(buf[i]); m[2 * i + 1] = cimag(buf[i]); }
  return 0;
}

int orc_gate_dmatrix(const orc_op *op, const double *params, int which, double *m) {
  cplx buf[1024];
  if (build_matrix(op, params, which, buf)) return -1;
  int d = 1 << n_targets_of(op);
  for (int i = 0; i < d * d; i++) { m[2 * i] = creal(buf[i]); m[2 * i + 1] = cimag(buf[i]); }
  return 0;
}

/* ----------------------------------------------------------- gate action */

/* out <- M acting on the op's targets of `in` where the controls match, and
 * either the untouched amplitude (zero_rest = 0) or zero (zero_rest = 1)
 * elsewhere.  in == out is allowed. */
static int act(int n, const cplx *in, cplx *out, const orc_op *op, const cplx *M, int zero_rest) {
  int k = n_targets_of(op);
  int d = 1 << k;
  uint64_t N = 1ull << n;
  uint64_t tmask = 0, cmask = 0, cval = 0;
  for (int i = 0; i < k; i++) {
    if (op->targets[i] < 0 || op->targets[i] >= n) return -1;
    if (tmask & (1ull << op->targets[i])) return -1;
    tmask |= 1ull << op->targets[i];
  }
  for (int i = 0; i < op->n_controls; i++) {
    int q = op->controls[i];
    if (q < 0 || q >= n) return -1;
    if ((tmask | cmask) & (1ull << q)) return -1;
    cmask |= 1ull << q;
    if ((op->control_states >> i) & 1u) cval |= 1ull << q;
  }
  if (zero_rest) {
    /* first clear everything outside the firing subspace */
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < (int64_t)N; b++)
      if (((uint64_t)b & cmask) != cval) out[b] = 0.0;
  } else if (in != out) {
    memcpy(out, in, sizeof(cplx) * N);
  }
#pragma omp parallel for schedule(static)
  for (int64_t bb = 0; bb < (int64_t)N; bb++) {
    uint64_t b = (uint64_t)bb;
    if (b & tmask) continue;
    if ((b & cmask) != cval) continue;
    uint64_t idx[32];
    cplx v[32];
    for (int j = 0; j < d; j++) {
      uint64_t a = b;
      for (int i = 0; i < k; i++)
        if ((j >> i) & 1) a |= 1ull << op->targets[i];
      idx[j] = a;
      v[j] = in[a];
    }
    for (int r = 0; r < d; r++) {
      cplx acc = 0.0;
      for (int col = 0; col < d; col++) acc += M[r * d + col] * v[col];
      out[idx[r]] = acc;
    }
  }
  return 0;
}

int orc_apply(int n, double *psi_, const orc_op *ops, int n_ops, const double *params) {
  cplx *psi = (cplx *)psi_;
  cplx M[1024];
  for (int g = 0; g < n_ops; g++) {
    if (build_matrix(&ops[g], params, -1, M)) return -1 - g;
    if (act(n, psi, psi, &ops[g], M, 0)) return -1 - g;
  }
  return 0;
}

int orc_run(int n, double *psi_, const orc_op *ops, int n_ops, const double *params) {
  cplx *psi = (cplx *)psi_;
  uint64_t N = 1ull << n;
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < (int64_t)N; b++) psi[b] = 0.0;
  psi[0] = 1.0;
  return orc_apply(n, psi_, ops, n_ops, params);
}

/* ------------------------------------------------------ Pauli observables
 * Matrix-free Pauli action (paper Section 4.4): P|b> = i^{nY} (-1)^{popcount(b & z)} |b ^ x>,
 * with x marking X or Y and z marking Z or Y, nY = popcount(x & z). */

static cplx ipow(int e) {
  switch (e & 3) {
    case 0: return 1.0;
    case 1: return I;
    case 2: return -1.0;
    default: return -I;
  }
}

static int parity64(uint64_t v) { return __builtin_popcountll(v) & 1; }

int orc_expect_pauli(int n, const double *psi_, const uint64_t *x, const uint64_t *z,
                     const double *c, int n_terms, double *out_terms, double *out_im,
                     double *out_sum) {
  const cplx *psi = (const cplx *)psi_;
  uint64_t N = 1ull << n;
  double total = 0.0;
  for (int j = 0; j < n_terms; j++) {
    if ((x[j] | z[j]) >> n) return -1;
    cplx ph = ipow(__builtin_popcountll(x[j] & z[j]));
    double sre = 0.0, sim = 0.0;
    /* <psi|P|psi> = sum_b conj(psi[b ^ x]) * phase(b) * psi[b] */
#pragma omp parallel for reduction(+ : sre, sim) schedule(static)
    for (int64_t bb = 0; bb < (int64_t)N; bb++) {
      uint64_t b = (uint64_t)bb;
      double sg = parity64(b & z[j]) ? -1.0 : 1.0;
      cplx t = conj(psi[b ^ x[j]]) * ph * sg * psi[b];
      sre += creal(t);
      sim += cimag(t);
    }
    if (out_terms) out_terms[j] = sre;
    if (out_im) out_im[j] = sim;
    total += c[j] * sre;
  }
  if (out_sum) *out_sum = total;
  return 0;
}

int orc_apply_pauli_sum(int n, const double *psi_, const uint64_t *x, const uint64_t *z,
                        const double *c, int n_terms, double *lam_) {
  const cplx *psi = (const cplx *)psi_;
  cplx *lam = (cplx *)lam_;
  uint64_t N = 1ull << n;
  for (int j = 0; j < n_terms; j++)
    if ((x[j] | z[j]) >> n) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t bb = 0; bb < (int64_t)N; bb++) lam[bb] = 0.0;
  for (int j = 0; j < n_terms; j++) {
    cplx ph = ipow(__builtin_popcountll(x[j] & z[j]));
    /* (P psi)[b ^ x] = phase(b) psi[b] */
#pragma omp parallel for schedule(static)
    for (int64_t bb = 0; bb < (int64_t)N; bb++) {
      uint64_t b = (uint64_t)bb;
      double sg = parity64(b & z[j]) ? -1.0 : 1.0;
      lam[b ^ x[j]] += c[j] * ph * sg * psi[b];
    }
  }
  return 0;
}

/* ------------------------------------------------------------ gradients
 * psi_j = U_j psi_{j-1}, E = <psi_m|H|psi_m>.  With lam_j = U_{j+1}^dag ...
 * U_m^dag H psi_m, the chain rule gives dE/dtheta = 2 Re <lam_j| dU_j/dtheta |psi_{j-1}>
 * summed over every gate that reads theta (a parameter used by several gates
 * sums their contributions, paper Section 4.2). */

static void dagger(const cplx *M, cplx *Md, int d) {
  for (int r = 0; r < d; r++)
    for (int c = 0; c < d; c++) Md[c * d + r] = conj(M[r * d + c]);
}

int orc_adjoint_grad(int n, const orc_op *ops, int n_ops, const double *params, int n_params,
                     const uint64_t *x, const uint64_t *z, const double *c, int n_terms,
                     double *energy, double *grad) {
  uint64_t N = 1ull << n;
  cplx *psi = (cplx *)malloc(sizeof(cplx) * N);
  cplx *lam = (cplx *)malloc(sizeof(cplx) * N);
  cplx *tmp = (cplx *)malloc(sizeof(cplx) * N);
  int rc = 0;
  if (!psi || !lam || !tmp) { rc = -100; goto done; }
  for (int p = 0; p < n_params; p++) grad[p] = 0.0;
  rc = orc_run(n, (double *)psi, ops, n_ops, params);
  if (rc) goto done;
  rc = orc_expect_pauli(n, (const double *)psi, x, z, c, n_terms, NULL, NULL, energy);
  if (rc) goto done;
  rc = orc_apply_pauli_sum(n, (const double *)psi, x, z, c, n_terms, (double *)lam);
  if (rc) goto done;
  for (int g = n_ops - 1; g >= 0; g--) {
    cplx M[1024], Md[1024], D[1024];
    const orc_op *op = &ops[g];
    int d = 1 << n_targets_of(op);
    if (build_matrix(op, params, -1, M)) { rc = -1 - g; goto done; }
    dagger(M, Md, d);
    /* psi <- psi_{g-1} */
    if (act(n, psi, psi, op, Md, 0)) { rc = -1 - g; goto done; }
    int np_ = n_params_of(op->kind);
    for (int w = 0; w < np_; w++) {
      int p = op->param_index[w];
      if (p < 0 || p >= n_params) { rc = -1 - g; goto done; }
      if (build_matrix(op, params, w, D)) { rc = -1 - g; goto done; }
      if (act(n, psi, tmp, op, D, 1)) { rc = -1 - g; goto done; }
      double acc = 0.0;
      for (uint64_t b = 0; b < N; b++) acc += creal(conj(lam[b]) * tmp[b]);
      grad[p] += 2.0 * acc;
    }
    /* lam <- lam_{g-1} */
    if (act(n, lam, lam, op, Md, 0)) { rc = -1 - g; goto done; }
  }
done:
  free(psi);
  free(lam);
  free(tmp);
  return rc;
}

/* --------------------------------------------------------------- sampling
 * The paper states only that basis indices are drawn from p_b = x_b^2 + y_b^2
 * on the device and counted (Section 5.3).  The fixed-order specification
 * implemented here (every floating-point operation in a stated order):
 *   1. p_b = fma(x_b, x_b, y_b * y_b) in binary64.
 *   2. Chunks of C = 2^min(n,10) consecutive indices; S_k = pairwise tree sum
 *      of chunk k (adjacent pairs, level by level).
 *   3. Blocks of G = 2^10 consecutive chunks (a single block when K <= G).
 *      Inside block j: L_k = S of the block's chunks before k, added left to
 *      right from 0.0; Q_j = the same sum over the whole block.  Block
 *      offsets E_0 = 0, E_{j+1} = E_j + Q_j, left to right.  P_k = E_j + L_k
 *      for k in block j, and T = P_K = E_J.  With one block this is the plain
 *      left-to-right prefix P_{k+1} = P_k + S_k.
 *   4. u_s = (splitmix64(seed, s) >> 11) * 2^-53.
 *   5. t = u_s * T; k* = first k with P_{k+1} > t, else the last k with S_k > 0.
 *   6. r = t - P_{k*}; a += p_b left to right inside chunk k*; pick the first
 *      b with a > r, else the last b in the chunk with p_b > 0.
 *   7. Output bit i = bit qubits[i] of b.
 * SplitMix64 is the generator published by Steele, Lea and Flood (OOPSLA
 * 2014): state advances by the golden-gamma constant; the output mixes with
 * two xor-shift-multiply rounds and a final xor-shift. */

uint64_t orc_splitmix64(uint64_t seed, uint64_t s) {
  uint64_t zz = seed + (s + 1u) * 0x9E3779B97F4A7C15ull;
  zz = (zz ^ (zz >> 30)) * 0xBF58476D1CE4E5B9ull;
  zz = (zz ^ (zz >> 27)) * 0x94D049BB133111EBull;
  return zz ^ (zz >> 31);
}

static double prob_of(const cplx *psi, uint64_t b) {
  double xr = creal(psi[b]), yi = cimag(psi[b]);
  return fma(xr, xr, yi * yi);
}

static double tree_sum(const double *v, uint64_t len) {
  if (len == 1) return v[0];
  uint64_t h = len / 2;
  return tree_sum(v, h) + tree_sum(v + h, h);
}

int orc_sample_prefix(int n, const double *psi_, double *S, double *P) {
  const cplx *psi = (const cplx *)psi_;
  int cbits = n < 10 ? n : 10;
  uint64_t C = 1ull << cbits, K = (1ull << n) >> cbits;
  double *buf = (double *)malloc(sizeof(double) * C);
  if (!buf) return -100;
  for (uint64_t k = 0; k < K; k++) {
    for (uint64_t i = 0; i < C; i++) buf[i] = prob_of(psi, k * C + i);
    S[k] = tree_sum(buf, C);
  }
  free(buf);
  const uint64_t G = K < 1024 ? K : 1024, J = K / G;
  double E = 0.0;  /* E_j, the sum of the block totals before block j */
  for (uint64_t j = 0; j < J; j++) {
    double Lk = 0.0;
    for (uint64_t k = j * G; k < (j + 1) * G; k++) {
      P[k] = E + Lk;
      Lk = Lk + S[k];
    }
    E = E + Lk;
  }
  P[K] = E;
  return 0;
}

/* Steps 5 and 6 for one target value t: the drawn basis index. */
static int64_t draw_index(const cplx *psi, const double *S, const double *P, uint64_t K, uint64_t C,
                          double t) {
  int64_t ks = -1;
  for (uint64_t k = 0; k < K; k++)
    if (P[k + 1] > t) { ks = (int64_t)k; break; }
  if (ks < 0)
    for (int64_t k = (int64_t)K - 1; k >= 0; k--)
      if (S[k] > 0.0) { ks = k; break; }
  if (ks < 0) ks = 0;  /* all-zero state: index 0 by convention */
  double r = t - P[ks];
  double a = 0.0;
  int64_t pick = -1, lastpos = -1;
  for (uint64_t i = 0; i < C; i++) {
    uint64_t b = (uint64_t)ks * C + i;
    double p = prob_of(psi, b);
    a += p;
    if (p > 0.0) lastpos = (int64_t)b;
    if (a > r) { pick = (int64_t)b; break; }
  }
  if (pick < 0) pick = lastpos >= 0 ? lastpos : (int64_t)ks * (int64_t)C;
  return pick;
}

int orc_sample_at(int n, const double *psi_, const double *t, int64_t count, uint64_t *out) {
  const cplx *psi = (const cplx *)psi_;
  int cbits = n < 10 ? n : 10;
  uint64_t C = 1ull << cbits, K = (1ull << n) >> cbits;
  double *S = (double *)malloc(sizeof(double) * K);
  double *P = (double *)malloc(sizeof(double) * (K + 1));
  if (!S || !P) { free(S); free(P); return -100; }
  orc_sample_prefix(n, psi_, S, P);
  for (int64_t s = 0; s < count; s++) out[s] = (uint64_t)draw_index(psi, S, P, K, C, t[s]);
  free(S);
  free(P);
  return 0;
}

int orc_sample(int n, const double *psi_, uint64_t seed, int64_t shots, const int32_t *qubits,
               int n_measured, uint64_t *out) {
  const cplx *psi = (const cplx *)psi_;
  for (int i = 0; i < n_measured; i++)
    if (qubits[i] < 0 || qubits[i] >= n) return -1;
  int cbits = n < 10 ? n : 10;
  uint64_t C = 1ull << cbits, K = (1ull << n) >> cbits;
  double *S = (double *)malloc(sizeof(double) * K);
  double *P = (double *)malloc(sizeof(double) * (K + 1));
  if (!S || !P) { free(S); free(P); return -100; }
  orc_sample_prefix(n, psi_, S, P);
  double T = P[K];
  for (int64_t s = 0; s < shots; s++) {
    double u = (double)(orc_splitmix64(seed, (uint64_t)s) >> 11) * 0x1.0p-53;
    int64_t pick = draw_index(psi, S, P, K, C, u * T);
    uint64_t o = 0;
    for (int i = 0; i < n_measured; i++)
      o |= (((uint64_t)pick >> qubits[i]) & 1u) << i;
    out[s] = o;
  }
  free(S);
  free(P);
  return 0;
}

/* ------------------------------------------------------------ fusion plan
 * One open block S; for an op on qubits Q: if S is non-empty and |S u Q| > k,
 * emit S and start a new one; then S <- S u Q.  Op order is preserved (paper
 * Section 9.2: fusion joins consecutive operations without reordering). */

int orc_fuse_greedy(int k, const orc_op *ops, int n_ops, int32_t *block_of) {
  uint64_t open = 0;
  int nblocks = 0;
  for (int g = 0; g < n_ops; g++) {
    uint64_t q = 0;
    for (int i = 0; i < n_targets_of(&ops[g]); i++) q |= 1ull << ops[g].targets[i];
    for (int i = 0; i < ops[g].n_controls; i++) q |= 1ull << ops[g].controls[i];
    if (open && __builtin_popcountll(open | q) > k) {
      open = 0;
    }
    if (!open) nblocks++;
    open |= q;
    block_of[g] = nblocks - 1;
  }
  return nblocks;
}
