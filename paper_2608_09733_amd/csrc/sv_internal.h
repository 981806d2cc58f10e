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
  MO_GRAD = 9,   // adjoint: accumulate Im<lam| G |psi> into gradient slot `coef` from the
                 // per-slot table at coefficient offset t0 (see GRAD_ODD / GRAD_BETA)
  MO_DIAGT = 10, // slot j *= table[j] (2^R complex at coef)
  MO_2L = 11,    // real 2x2 rotation between local patterns: slots with (j & mask) == gz and
                 // their partners j ^ t1; coef r00,r01,r10,r11 (Givens, double excitation)
  MO_GRAD2L = 12,// adjoint: accumulate Im<lam| G |psi> into slot `coef` for the generator of
                 // an MO_2L rotation (same mask / gz / t1 / cm / cv): G a = i b, G b = -i a
                 // for a = slot with (j & mask) == gz, b = a ^ t1, and G = 0 elsewhere
};

// MO_GRAD of a generator G = alpha P + beta I on the control subspace, P the
// Pauli string (x, z) of the group bits with n_Y = popcount(x & z):
//   Im <lam| G |psi> = sum_j c_j F(lam_j, psi_{j^x})
// with F = Re(conj(lam) psi') when n_Y is odd (GRAD_ODD in t1), Im(conj(lam)
// psi') when even; c_j = alpha (-1)^{popcount((j^x) & z)} (negated when n_Y
// mod 4 >= 2), plus beta when x = 0 (beta is nonzero only for phase gates,
// whose x is 0), and 0 outside the control subspace.  The table holds the
// 2^R values c_j.
#define GRAD_ODD 1

struct MicroOp {
  int32_t type;
  int32_t t0, t1;      // group-local bit indices
  uint32_t mask;       // MO_P parity mask; MO_DENSE: k; MO_GRAD: generator x-mask
  uint32_t cm, cv;     // control condition on the group-local index: (j & cm) == cv
  int32_t coef;        // offset (in doubles) into the coefficient buffer; MO_GRAD: slot
  uint32_t gz;         // MO_GRAD: generator z-mask (Y = bit in both masks)
  double galpha, gbeta;// MO_GRAD: G = alpha * PauliString + beta * I (on the control subspace)
};

// Stage kinds.
//   ST_OPS:  run the micro-op list [op_begin, op_end) on the group.
//   ST_KRON: the static form  P * s * D_after * (R~_{R-1} (x) ... (x) R~_0) * D_before
//            with R~_t a rotation on group bit t (present if bit t of rmask) in
//            fast-Givens form (one coefficient of each row is +-1, so each
//            output is one FMA; the factored-out scales multiply into s),
//            D_* diagonal tables of 2^R complex entries (present per dflags bit
//            0 / 1), s a real scalar (dflags bit 2; otherwise already folded
//            into D_after) and P folded into st_off.  Coefficients at kcoef:
//            [R_0 .. R_{R-1}: 4 doubles each][D_before: 2^(R+1)][D_after: 2^(R+1)][s].
//            Fast-Givens record of R_t: {form, k, scale, 0} with
//              form 0: x' = x - k y, y' = k x + y      (k = s/c, scale c)
//              form 1: x' = k x - y, y' = x + k y      (k = c/s, scale s)
//            FP64 plans always take form 0 (CF_FORM0); FP32 plans take form 1
//            when |s| > |c|, so that |k| <= 1.
enum { ST_OPS = 0, ST_KRON = 1 };

// Thread mapping of a stage: thread-index bit k sits on tile bit tpos[k]
// (k < tile bits - group bits); the lane bits (k < 6) hold every tile bit that
// the stage's slot offsets reach outside the group (an X controlled by group
// qubits whose target is another tile qubit: a thread then stores to slots
// that other threads load), so those exchanges stay inside one wave, whose
// loads complete before its stores (they feed them).
// dflags bits:
//   SD_XCHG:   the exchanged bits did not fit the lane bits: every load of the
//              stage completes (workgroup barrier) before any store.
//   SD_WLOCAL: the next stage of the sweep keeps this stage's wave bits
//              (tpos[6..]), so each wave reads there exactly the slots it
//              wrote here: no workgroup barrier is needed in between.
#define SD_XCHG 8
#define SD_WLOCAL 16

struct StageDesc {
  int32_t sbits[SVI_RMAX];     // tile-local bit positions of the group bits, ascending
  int32_t op_begin, op_end;    // micro-ops [op_begin, op_end)
  int32_t kind;                // ST_OPS / ST_KRON
  uint32_t rmask;              // ST_KRON: group bits carrying a real 2x2
  int32_t dflags;              // ST_KRON: 1 = D_before, 2 = D_after; SD_* (any kind)
  int32_t kcoef;               // ST_KRON: coefficient offset (doubles)
  int32_t g1, g2;              // ST_KRON: MO_GRAD ops [op_begin, g1) run on the stage input,
                               // [g1, g2) after D_before, [g2, op_end) after the rotations
  uint32_t gdiag;              // ST_KRON: bit p set when every MO_GRAD op of range p
                               // (0, 1, 2 as above) has a diagonal generator
  int8_t tpos[16] __attribute__((aligned(4)));   // tile bit of thread-index bit k (see above)
  int32_t ld_off[SVI_GMAX];    // swizzled tile-local BYTE offset loaded into slot j
  int32_t st_off[SVI_GMAX];    // swizzled tile-local BYTE offset slot j is stored to
};

// LDS swizzle of a tile-local element index (B = 3 for 16-byte complex
// elements, 4 for 8-byte ones): xor the low B bits with a fold of the higher
// bits.  It is linear over GF(2), so for disjoint bit sets
// swz(a | b) = swz(a) ^ swz(b), which lets offsets be swizzled ahead of time.
#if defined(__HIP__)
#define SVI_HD __host__ __device__
#else
#define SVI_HD
#endif
static inline SVI_HD int svi_swz(int i, int B) {
  const int msk = (1 << B) - 1;
  const int h = (i >> B) ^ (i >> (2 * B)) ^ (i >> (3 * B)) ^ (i >> (4 * B));
  return i ^ (h & msk);
}

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
  int32_t operm[SVI_MMAX];   // SW_OPERM: output tile bit k takes LDS tile bit operm[k]
  int32_t nbz;               // SW_SPARSE: tile bases take zeros at bz[0..nbz) (ascending):
  int32_t bz[32];            //   the tile's high bits and the qubits still outside the support
};

#define SW_INIT_ZERO 1       // synthesise |0..0> instead of loading state 0
#define SW_OPERM 2           // permute tile bits on the way out (qubit remapping)
// A sweep of a state evolved from |0..0> by earlier sweeps only: amplitudes
// are nonzero only where every qubit outside the earlier sweeps' tiles is 0
// (a sweep's gates act within tiles), so only the tiles whose outside qubits
// off that support are 0 are run (ntiles of them, bases from bz); the others
// hold zeros in memory, before and after.
#define SW_SPARSE 4

// Coefficient descriptors (built on the device from the parameter vector).
enum {
  CF_U2X2 = 1,     // 8 doubles
  CF_R2X2 = 2,     // 4 doubles (real gates)
  CF_DIAG = 3,     // 4 doubles (d0, d1)
  CF_Q4X4 = 4,     // 32 doubles
  CF_D16 = 5,      // 512 doubles (4-target gate)
  CF_COPY = 6,     // copy `len` doubles from the static (user-matrix) area
  CF_TABLE = 7,    // diagonal table of 2^len complex entries from factors [src, src+pidx[0])
  CF_IDENT2 = 8,   // 2x2 real identity (4 doubles)
  CF_FASTR = 9,    // fast-Givens record {form, k, scale, 0} of a real 1q gate (see CF_FORM0)
  CF_SCALE = 10,   // real scalar: product of the fast-Givens scales of factors [src, +pidx[0])
  CF_CONSTS = 11,  // copy `len` doubles from the parameter vector at `src` (plan constants)
};

// One factor of a diagonal table: entry j is multiplied, when (j & cm) == cv,
// by -1 (neg = 1), by the diagonal entry d0 / d1 of gate `kind` chosen by the
// parity of j & mask (neg = 0), or -- for every entry -- by the fast-Givens
// scale of the real 1q gate `kind` (neg = 2).
struct TabFactor {
  int32_t kind;
  int32_t pidx;
  uint32_t mask, cm, cv;
  int32_t neg;
};
#define CF_DAGGER 0x100
// CF_FASTR / CF_SCALE / CF_TABLE scale factors: a rotation always takes form 0
// (k = s / c, scale c; the FP64 kernels apply it without a form branch).
// Without the flag the form with |k| <= 1 is chosen (FP32, whose range a
// product of large k could leave).
#define CF_FORM0 0x200

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

// Ragged batch: one persistent launch drains a device queue of work units.
// A unit is a range of tiles of one sweep (or of one Pauli pass) of one
// circuit.  Units are queued in an order in which every unit depends only on
// units before it, so a workgroup that holds a unit never waits on a unit that
// has not been taken yet.
enum { UK_SWEEP = 0, UK_PAULI = 1 };

struct BatchUnit {
  int32_t kind;        // UK_SWEEP / UK_PAULI
  int32_t circ;        // circuit index (dependency counter)
  int32_t arg;         // index into the sweep or Pauli-pass argument array
  int32_t wait;        // units of this circuit that must be complete first
  int64_t t0, t1;      // tiles [t0, t1)
  int32_t part;        // UK_PAULI: first partial-sum slot (one per term of the pass)
  int32_t pad;
};

struct BatchKernelArgs {
  const BatchUnit *units;
  const SweepArgs *sweeps;
  const PauliPassArgs *passes;
  double *part;        // Pauli partial sums
  int32_t *head;       // next unit to take
  int32_t *done;       // completed units per circuit
  int32_t *err;        // bit 0: a dependency wait expired
  int32_t nunits;
  int32_t spin_limit;  // polls before a wait expires; < 0: every wait expires at once
};

// Serving: one workgroup takes one small request off the queue and runs its
// whole adjoint -- forward sweeps, lambda = H psi and E = <psi|H|psi>, the
// backward sweeps with their gradient slots, the gather into dE/dtheta --
// with the request's planes in L2.  Coefficients are built by a launch before.
struct ServeReq {
  int32_t n;                  // qubits
  int32_t n_params;           // user parameters (gradient length)
  int32_t f_sweep, f_nsweeps; // forward sweeps in ServeArgs::sweeps
  int32_t b_sweep, b_nsweeps; // backward sweeps
  int32_t f_ndesc, b_ndesc;   // coefficient descriptors of the two plans
  int32_t n_terms;            // observable terms
  int32_t pad;
  const CoefDesc *f_desc, *b_desc;
  const TabFactor *f_fac, *b_fac;
  const double *f_params, *b_params;  // user parameters, then the plan's constants
  double *f_coef, *b_coef;
  void *re, *im;              // psi (2^n elements each)
  void *lre, *lim;            // lambda
  const PauliTermDev *terms;  // x, z, c of each term
  double *slots;              // gradient slot sums of the backward plan
  const int32_t *rowptr;      // parameter p takes slots gslots[rowptr[p] .. rowptr[p+1])
  const int32_t *gslots;
  double *out;                // E, then dE/dtheta_p
};

struct ServeArgs {
  const ServeReq *reqs;
  const SweepArgs *sweeps;
  int32_t *head;              // next request to take (zero at launch)
  int32_t nreq;
};
