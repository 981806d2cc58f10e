/*
 * CPU oracle for the state-vector path -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, deliberately unoptimised FP64 simulator written from the
 * paper's definitions.  It is used only by the tests, by the smoke check and
 * by the CPU-baseline timing leg of the benchmark.  It shares no code, header,
 * table or helper with the HIP library, and the HIP library never calls it.
 *
 * Conventions (all stated in the paper or chosen where it is silent):
 *   - Qubit q is bit q of the basis index (little-endian).
 *   - A k-target gate's local index is j = sum_i bit(t_i) * 2^i, so the first
 *     target is the least-significant bit of the gate's matrix index
 *     (paper Section 4.2: targets before controls).
 *   - control_states bit i set: control i fires on |1>; clear: on |0>
 *     (paper Section 4.2: a control may trigger on |0>).
 *   - Rotations are R_P(theta) = exp(-i theta P / 2) (paper Section 9.1).
 *   - Amplitudes are interleaved complex128 (re, im) pairs.
 */
#ifndef SV_ORACLE_H
#define SV_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORC_I = 0, ORC_X, ORC_Y, ORC_Z, ORC_H, ORC_S, ORC_SDG, ORC_T, ORC_TDG, ORC_SX,
  ORC_RX, ORC_RY, ORC_RZ, ORC_P, ORC_U2, ORC_U3,
  ORC_SWAP, ORC_RXX, ORC_RYY, ORC_RZZ, ORC_GIVENS, ORC_DEXC, ORC_UNITARY,
  ORC_NKINDS
};

typedef struct {
  int32_t kind;
  int32_t n_targets;
  int32_t targets[5];
  int32_t n_controls;
  int32_t controls[5];
  uint32_t control_states;
  int32_t param_index[3];
  const double *matrix;   /* ORC_UNITARY: row-major 2^k x 2^k, interleaved re/im */
} orc_op;

/* Apply ops[0..n_ops) in order to psi (2^n interleaved complex128), in place. */
int orc_apply(int n, double *psi, const orc_op *ops, int n_ops, const double *params);

/* psi <- |0...0> then orc_apply. */
int orc_run(int n, double *psi, const orc_op *ops, int n_ops, const double *params);

/* The gate's local 2^k x 2^k matrix (targets only) into m (interleaved). */
int orc_gate_matrix(const orc_op *op, const double *params, double *m);

/* d(matrix)/d(param slot `which`) into m. */
int orc_gate_dmatrix(const orc_op *op, const double *params, int which, double *m);

/* <P_j> for each term (x_mask, z_mask) and sum_j c_j <P_j>.  out_im gets the
 * imaginary parts (zero for a Hermitian P up to rounding); may be NULL. */
int orc_expect_pauli(int n, const double *psi, const uint64_t *x, const uint64_t *z,
                     const double *c, int n_terms, double *out_terms, double *out_im,
                     double *out_sum);

/* lam <- H psi = sum_j c_j P_j psi. */
int orc_apply_pauli_sum(int n, const double *psi, const uint64_t *x, const uint64_t *z,
                        const double *c, int n_terms, double *lam);

/* E = <psi|H|psi> with psi = U(params)|0>, and dE/dparams by reverse-mode
 * accumulation through each gate's derivative matrix. */
int orc_adjoint_grad(int n, const orc_op *ops, int n_ops, const double *params, int n_params,
                     const uint64_t *x, const uint64_t *z, const double *c, int n_terms,
                     double *energy, double *grad);

/* Counter-based SplitMix64 output for counter s under seed. */
uint64_t orc_splitmix64(uint64_t seed, uint64_t s);

/* Terminal Z-basis sampling by the fixed-order specification. */
int orc_sample(int n, const double *psi, uint64_t seed, int64_t shots, const int32_t *qubits,
               int n_measured, uint64_t *out);

/* Steps 5-6 of the specification for given target values: out[s] = the basis
 * index drawn for t[s] (the sampler draws t = u_s * T; tests may pass any t,
 * including t >= T, which reaches the fallbacks). */
int orc_sample_at(int n, const double *psi, const double *t, int64_t count, uint64_t *out);

/* Probability-prefix quantities of the sampling specification (for tests):
 * chunk sums S (K entries) and prefixes P (K+1 entries), K = 2^n / 2^min(n,10). */
int orc_sample_prefix(int n, const double *psi, double *S, double *P);

/* Greedy in-order fusion: one open block; an op whose qubits would push the
 * open block past k qubits closes it.  block_of[i] gets op i's block id.
 * Returns the number of blocks. */
int orc_fuse_greedy(int k, const orc_op *ops, int n_ops, int32_t *block_of);

/* Number of OpenMP threads the oracle uses (1 when built without OpenMP). */
int orc_threads(void);

#ifdef __cplusplus
}
#endif
#endif
