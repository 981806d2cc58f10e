// Internal descriptors shared by the host planner (sv_host.cpp) and the
// gfx950 kernels (sv_kernels.hip).  Not part of the public ABI.
//
// Execution model
//   A *sweep* reads and writes every amplitude of a state once.  It works on
//   *tiles*: 2^m amplitudes whose indices differ only on the tile's qubits
//   (the c lowest qubits, which give contiguous rows in HBM, plus m-c others).
//   A tile is staged in LDS (re/im interleaved), then a sequence of *stages*
//   runs: in a stage every thread holds one *group* of 2^R amplitudes that
//   differ only on the stage's R tile bits in registers and applies the
//   stage's micro-ops to it (a fused block of <= R qubits).  Permutations at
//   the start or end of a stage are folded into its LDS load/store offsets.
#pragma once
#include <stdint.h>

#define SVI_MMAX 14          // largest tile (bits) of any kernel instantiation
#define SVI_RMAX 5           // largest register group (bits)
#define SVI_GMAX 32          // 1 << SVI_RMAX

// Micro-op types (register-level operations on one group).
enum {
  MO_NOP = 0,
  MO_U = 1,      // general 2x2 complex on group bit t0; coef: 8 doubles row-major (re,im)
  MO_R = 2,      // real 2x2 on bit t0; coef: 4 doubles
  MO_P = 3,      // parity diagonal: slot j *= (popcount(j & mask) odd ? d1 : d0); coef d0r,d0i,d1r,d1i
  MO_X = 4,      // swap slots j <-> j ^ (1 << t0)
  MO_SWAP = 5,   // swap slots with (bit t0, bit t1) = (1,0) <-> (0,1)
  MO_NEG = 6,    // negate slots whose control bits match (cm/cv); Z-type gates
  MO_Q = 7,      // 4x4 complex on bits (t0 = low, t1 = high); coef 32 doubles
  MO_DENSE = 8,  // 2^k x 2^k complex (k <= 3, in `mask`) on group bits 0..k-1; coef 2*4^k doubles
  MO_GRAD = 9,   // adjoint: accumulate Im<lam| G |psi> into gradient slot `coef`
  MO_DIAGT = 10, // slot j *= table[j] (2^R complex at coef)
  MO_2L = 11,    // real 2x2 rotation between local patterns: slots with (j & mask) == gz and
                 // their partners j ^ t1; coef r00,r01,r10,r11 (Givens, double excitation)
};

struct MicroOp {
  int32_t type;
  int32_t t0, t1;      // group-local bit indices
  uint32_t mask;       // MO_P parity mask; MO_DENSE: k; MO_GRAD: generator x-mask
  uint32_t cm, cv;     // control condition on the group-local index: (j & cm) == cv
  int32_t coef;        // offset (in doubles) into the coefficient buffer; MO_GRAD: slot
  uint32_t gz;         // MO_GRAD: generator z-mask (Y = bit in both masks)
  double galpha, gbeta;// MO_GRAD: G = alpha * PauliString + beta * I (on the control subspace)
};

struct StageDesc {
  int32_t sbits[SVI_RMAX];     // tile-local bit positions of the group bits (group bit i)
  int32_t op_begin, op_end;    // micro-ops [op_begin, op_end)
  int32_t pad;
  uint16_t ld_off[SVI_GMAX];   // tile-local offset loaded into slot j
  uint16_t st_off[SVI_GMAX];   // tile-local offset slot j is stored to
};

// Per-sweep launch arguments (passed by value).
struct SweepArgs {
  void *re, *im;             // planes of state 0 (psi)
  void *re2, *im2;           // planes of state 1 (lambda; adjoint only)
  const StageDesc *stages;
  const MicroOp *ops;
  const double *coef;
  double *gpart;             // adjoint: gradient partials [slot][grid]
  int32_t n;                 // qubits of the state
  int32_t m;                 // tile bits actually used (<= template M)
  int32_t c;                 // low contiguous tile bits
  int32_t nh;                // m - c
  int32_t hb[SVI_MMAX];      // qubit index of tile bit c+k (ascending)
  int32_t stage_begin, stage_end;
  int32_t flags;             // SW_INIT_ZERO ...
  int32_t gslot_begin, n_gslots;  // adjoint: gradient slots used by this sweep
  int64_t ntiles;
};

#define SW_INIT_ZERO 1       // synthesise |0..0> instead of loading state 0

// Coefficient descriptors (built on the device from the parameter vector).
enum {
  CF_U2X2 = 1,     // 8 doubles
  CF_R2X2 = 2,     // 4 doubles (real gates)
  CF_DIAG = 3,     // 4 doubles (d0, d1)
  CF_Q4X4 = 4,     // 32 doubles
  CF_D16 = 5,      // 512 doubles (4-target gate)
  CF_COPY = 6,     // copy `len` doubles from the static (user-matrix) area
};
#define CF_DAGGER 0x100

struct CoefDesc {
  int32_t kind;        // sv_gate_kind
  int32_t fmt;         // CF_* | CF_DAGGER
  int32_t pidx[3];
  int32_t dst;         // offset in doubles
  int32_t src;         // CF_COPY: offset into static area
  int32_t len;         // CF_COPY: doubles
};

// Expectation / H|psi> tile pass.
struct PauliTermDev {
  uint64_t x, z;
  double c;
  int32_t term;        // output slot
  int32_t pad;
};

struct PauliPassArgs {
  const void *re, *im;       // psi
  void *lre, *lim;           // lambda output (NULL: expectation only)
  const PauliTermDev *terms;
  double *part;              // partials [term_in_pass][grid]
  int32_t n, m, c, nh;
  int32_t hb[SVI_MMAX];
  int32_t t_begin, t_end;    // terms of this pass
  int32_t accumulate;        // lambda: add to existing values
  int64_t ntiles;
};
