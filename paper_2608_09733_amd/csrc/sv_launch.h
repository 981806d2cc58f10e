// Host-side entry points of the kernels in sv_kernels.hip (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sv_internal.h"

struct GateArgsHost {
  void *re, *im;
  const double *coef;
  int32_t type;
  int32_t t0, t1;
  int32_t npos;
  int32_t pos[SVI_RMAX + 5];
  uint64_t cval;
  uint64_t pmask;
  int64_t nitems;
};

hipError_t svk_launch_sweep(int dbl, int M, int R, int NS, const SweepArgs &a, int grid,
                            hipStream_t s);
int svk_sweep_occupancy(int dbl, int M, int R, int NS);
hipError_t svk_launch_sweep_kron(int dbl, int M, int R, int NS, const SweepArgs &a, int grid,
                                 hipStream_t s);
int svk_sweep_kron_occupancy(int dbl, int M, int R, int NS);
int svk_has_sweep(int dbl, int M, int R, int NS);
hipError_t svk_launch_gate(int dbl, const GateArgsHost &a, hipStream_t s);
hipError_t svk_launch_init_zero(int dbl, void *re, void *im, int64_t n, hipStream_t s);
hipError_t svk_launch_coefs(const CoefDesc *d, int nd, const double *params,
                            const double *statics, const TabFactor *fac, double *coef,
                            hipStream_t s);
hipError_t svk_launch_pauli(int dbl, int M, const PauliPassArgs &a, int grid, hipStream_t s);
int svk_pauli_occupancy(int dbl);
hipError_t svk_launch_pauli_wide(int dbl, const void *re, const void *im, void *lre, void *lim,
                                 uint64_t x, uint64_t z, double c, int64_t N, int accumulate,
                                 double *part, int grid, hipStream_t s);
hipError_t svk_launch_reduce_rows(const double *part, int nslots, int np, double *out,
                                  hipStream_t s);
// one-qubit channel: 4x4 superoperator s32 (row-major, interleaved, local index
// c + 2 r) on column bit qc < row bit qr of an nq-qubit vector
hipError_t svk_launch_dm_channel(int dbl, void *re, void *im, int nq, int qc, int qr,
                                 const double *s32, hipStream_t s);
// two one-qubit channels (same layout) on qubits qa != qb, row bits at + off
hipError_t svk_launch_dm_channel2(int dbl, void *re, void *im, int nq, int qa, int qb, int off,
                                  const double *sa, const double *sb, hipStream_t s);
// two-qubit channel: 16x16 superoperator in device memory on qubits q0 != q1
hipError_t svk_launch_dm_channel16(int dbl, void *re, void *im, int nq, int q0, int q1, int off,
                                   const double *d_S, hipStream_t s);
// up to four one-qubit channels (same superoperator) in one LDS-tile pass; nq >= 12
hipError_t svk_launch_dm_channel_tile(int dbl, void *re, void *im, int nq, int off,
                                      const int *qubits, int k, const double *s32, hipStream_t s);
// part[t * nb + b] <- block b's partial of Tr(rho P_t), rho of n qubits as a 2n-qubit vector
hipError_t svk_launch_dm_pauli(int dbl, const void *re, const void *im, int n,
                               const PauliTermDev *terms, int nt, int nb, double *part,
                               hipStream_t s);
hipError_t svk_launch_gather_grad(const double *slot_sum, const int32_t *row_ptr,
                                  const int32_t *slots, int np, double *grad, hipStream_t s);
hipError_t svk_launch_zexp(int dbl, const void *re, const void *im, int n, const PauliTermDev *terms,
                           int nt, double *part, int grid, hipStream_t s);
int svk_zexp_occupancy(int dbl);
#define SVI_ZTERMS_HOST 32
hipError_t svk_launch_energy_terms(const double *vals, const PauliTermDev *terms, int nt,
                                   double *out, hipStream_t s);
hipError_t svk_launch_energy(const double *terms, const double *coef, int nt, double *out,
                             hipStream_t s);
// QE: 2 * (K / min(K, 1024)) + 1 doubles of device scratch (block totals and offsets).
hipError_t svk_launch_sampling(int dbl, const void *re, const void *im, int n, double *S,
                               double *P, double *QE, uint64_t seed, int64_t shots,
                               const int32_t *qubits, int nq, uint64_t *out, hipStream_t s);

// counts[0 .. 2^nq) <- histogram of samples (zeroed first)
hipError_t svk_launch_histogram(const uint64_t *samples, int64_t shots, int nq, uint64_t *counts,
                                hipStream_t s);
// odd[m] <- number of samples with odd parity under masks[m] (zeroed first)
hipError_t svk_launch_parity_counts(const uint64_t *samples, int64_t shots, const uint64_t *masks,
                                    int nm, uint64_t *odd, hipStream_t s);

#define SVI_GSLOTS_MAX 128   // gradient slots per backward sweep of the two-state Kronecker kernel
#define SVI_GSLOTS_HARD 256  // gradient slots of the general two-state kernel (LDS)
#define SVI_PTERMS_MAX 64
#define SVI_KMAX_STAGES_HOST 16

hipError_t svk_launch_batch(int dbl, int M, int R, int kron_only, const BatchKernelArgs &a,
                            int grid, hipStream_t s);
int svk_batch_occupancy(int dbl, int M, int R, int kron_only);
int svk_has_batch(int dbl, int M, int R);
hipError_t svk_launch_batch_reset(int32_t *head, int32_t *done, int32_t *err, int nc,
                                  hipStream_t s);
hipError_t svk_launch_batch_reduce(const int32_t *rowptr, const int32_t *slot, const double *coef,
                                   const double *part, double *out, int nc, hipStream_t s);

// Serving (whole small requests, one workgroup each): coefficients of every
// request (max_desc: most descriptors of one request), then the persistent
// request kernel over reqs[0 .. nreq); *d_head must be zero.  general: some
// plan holds micro-op stages.
hipError_t svk_launch_serve_coefs(const ServeReq *d_reqs, int nreq, int max_desc, hipStream_t s);
hipError_t svk_launch_serve(const ServeReq *d_reqs, const SweepArgs *d_sweeps, int32_t *d_head,
                            int nreq, int general, int grid, hipStream_t s);
int svk_serve_max_qubits();
int svk_serve_tiling(int *M, int *R);   // returns threads per workgroup
