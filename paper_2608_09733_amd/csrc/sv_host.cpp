// Host runtime of libsv: argument validation, circuit lowering, the sweep /
// stage planner, plan cache, kernel launches and the C ABI of include/sv.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "sv.h"
#include "sv_internal.h"
#include "sv_launch.h"

// ------------------------------------------------------------------ errors

static thread_local std::string g_err;

static sv_status fail(sv_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIPCHK(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(SV_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));         \
  } while (0)

extern "C" const char *sv_last_error(void) { return g_err.c_str(); }

extern "C" const char *sv_version(void) {
  return "libsv gfx950 (tile sweeps M<=14, register blocks R<=5, FP64/FP32 planes)";
}

// ------------------------------------------------------------- device info

struct DevInfo {
  int cus = 0;
};
static std::mutex g_dev_mu;
static std::unordered_map<int, DevInfo> g_dev;

static sv_status device_info(DevInfo &out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_dev_mu);
  auto it = g_dev.find(dev);
  if (it == g_dev.end()) {
    DevInfo di;
    HIPCHK(hipDeviceGetAttribute(&di.cus, hipDeviceAttributeMultiprocessorCount, dev));
    it = g_dev.emplace(dev, di).first;
  }
  out = it->second;
  return SV_OK;
}

// --------------------------------------------------------------- lowering

static int arity_of(int kind) {
  switch (kind) {
    case SV_SWAP: case SV_RXX: case SV_RYY: case SV_RZZ: case SV_GIVENS: return 2;
    case SV_DEXC: return 4;
    case SV_UNITARY: return -1;
    default: return 1;
  }
}

static int nparams_of(int kind) {
  switch (kind) {
    case SV_RX: case SV_RY: case SV_RZ: case SV_P: case SV_RXX: case SV_RYY: case SV_RZZ:
    case SV_GIVENS: case SV_DEXC:
      return 1;
    case SV_U2: return 2;
    case SV_U3: return 3;
    default: return 0;
  }
}

// Kernel-side kind ids (sv_kernels.hip gate_local) equal sv_gate_kind values.

struct GateRec {
  int kind = 0;
  int nt = 0;
  int t[5] = {0, 0, 0, 0, 0};
  int nc = 0;
  int c[5] = {0, 0, 0, 0, 0};
  uint32_t cs = 0;
  int pidx[3] = {-1, -1, -1};
  uint64_t qmask = 0;        // targets | controls
  int mo = MO_NOP;
  int coef_kind = 0;         // kind used to build the coefficients
  int fmt = 0;               // CF_* (0 = none)
  int ncoef = 0;             // doubles
  int user_mat = -1;         // index of the user matrix (SV_UNITARY)
  bool dagger = false;
  // adjoint gradient micro-op (before the gate)
  bool grad = false;
  int gparam = -1;
  uint64_t gx = 0, gz = 0;   // generator masks (global qubits)
  double galpha = 1.0, gbeta = 0.0;
  bool grad2l = false;       // generator of the MO_2L rotation itself (Givens, double excitation)
  double cost = 0.0;         // VALU ops per amplitude (rough)
};

static sv_status validate_op(const sv_op &op, int idx, int n, int n_params) {
  if (op.kind < 0 || op.kind >= SV_NKINDS) return fail(SV_EINVAL, "op %d: bad kind %d", idx, op.kind);
  int ar = arity_of(op.kind);
  if (op.kind == SV_UNITARY) {
    if (op.n_targets < 1 || op.n_targets > 3)
      return fail(SV_EUNSUPPORTED, "op %d: user matrices on 1..3 targets are supported (got %d)",
                  idx, op.n_targets);
    if (!op.matrix) return fail(SV_EINVAL, "op %d: unitary without matrix", idx);
  } else if (op.n_targets != ar) {
    return fail(SV_EINVAL, "op %d: kind %d takes %d targets, got %d", idx, op.kind, ar, op.n_targets);
  }
  if (op.n_controls < 0 || op.n_controls > SV_MAX_CONTROLS)
    return fail(SV_EINVAL, "op %d: bad control count %d", idx, op.n_controls);
  uint64_t seen = 0;
  for (int i = 0; i < op.n_targets + op.n_controls; i++) {
    int q = i < op.n_targets ? op.targets[i] : op.controls[i - op.n_targets];
    if (q < 0 || q >= n) return fail(SV_EINVAL, "op %d: qubit %d out of range [0,%d)", idx, q, n);
    if (seen & (1ull << q)) return fail(SV_EINVAL, "op %d: qubit %d repeated", idx, q);
    seen |= 1ull << q;
  }
  if (op.n_controls < 32 && (op.control_states >> op.n_controls) != 0)
    return fail(SV_EINVAL, "op %d: control_states has bits beyond n_controls", idx);
  for (int i = 0; i < nparams_of(op.kind); i++)
    if (op.param_index[i] < 0 || op.param_index[i] >= n_params)
      return fail(SV_EUNBOUND, "op %d: parameter index %d unbound (n_params=%d)", idx,
                  op.param_index[i], n_params);
  if ((int)__builtin_popcountll(seen) > SVI_RMAX)
    return fail(SV_EUNSUPPORTED, "op %d: acts on %d qubits (max %d incl. controls)", idx,
                (int)__builtin_popcountll(seen), SVI_RMAX);
  return SV_OK;
}

// Largest state: 32 qubits (64 GiB of FP64 planes; the largest size the
// tests run).  Indices are 64-bit throughout.
#define SVI_NMAX 32

static void set_mo(GateRec &g) {
  switch (g.kind) {
    case SV_X: g.mo = MO_X; g.cost = 1; break;
    case SV_Z: g.mo = MO_NEG; g.cost = 1; break;
    case SV_Y: case SV_SX: case SV_RX: case SV_U2: case SV_U3:
      g.mo = MO_U; g.fmt = CF_U2X2; g.ncoef = 8; g.cost = 8; break;
    case SV_H: case SV_RY: g.mo = MO_R; g.fmt = CF_R2X2; g.ncoef = 4; g.cost = 4; break;
    case SV_S: case SV_SDG: case SV_T: case SV_TDG: case SV_RZ: case SV_P:
      g.mo = MO_P; g.fmt = CF_DIAG; g.ncoef = 4; g.cost = 4; break;
    case SV_RZZ: g.mo = MO_P; g.fmt = CF_DIAG; g.ncoef = 4; g.coef_kind = SV_RZ; g.cost = 4; break;
    case SV_SWAP: g.mo = MO_SWAP; g.cost = 1; break;
    case SV_RXX: case SV_RYY: g.mo = MO_Q; g.fmt = CF_Q4X4; g.ncoef = 32; g.cost = 16; break;
    case SV_GIVENS: case SV_DEXC:
      g.mo = MO_2L; g.fmt = CF_R2X2; g.ncoef = 4; g.coef_kind = SV_RY; g.cost = 2; break;
    case SV_UNITARY:
      if (g.nt == 1) { g.mo = MO_U; g.ncoef = 8; g.cost = 8; }
      else if (g.nt == 2) { g.mo = MO_Q; g.ncoef = 32; g.cost = 16; }
      else { g.mo = MO_DENSE; g.ncoef = 2 * 64; g.cost = 32; }
      g.fmt = CF_COPY;
      break;
    default: g.mo = MO_NOP; break;
  }
  if (g.coef_kind == 0) g.coef_kind = g.kind;
}

static GateRec lower_one(const sv_op &op, int user_mat) {
  GateRec g;
  g.kind = op.kind;
  g.nt = op.n_targets;
  for (int i = 0; i < g.nt; i++) { g.t[i] = op.targets[i]; g.qmask |= 1ull << g.t[i]; }
  g.nc = op.n_controls;
  for (int i = 0; i < g.nc; i++) { g.c[i] = op.controls[i]; g.qmask |= 1ull << g.c[i]; }
  g.cs = op.control_states;
  for (int i = 0; i < nparams_of(op.kind); i++) g.pidx[i] = op.param_index[i];
  g.user_mat = op.kind == SV_UNITARY ? user_mat : -1;
  set_mo(g);
  return g;
}

// Generator of a single-angle gate exp(-i theta G / 2): G = alpha P + beta I.
static bool generator_of(const GateRec &g, uint64_t &x, uint64_t &z, double &alpha, double &beta) {
  alpha = 1.0; beta = 0.0; x = z = 0;
  uint64_t b0 = 1ull << g.t[0];
  uint64_t b01 = g.nt >= 2 ? (b0 | (1ull << g.t[1])) : b0;
  switch (g.kind) {
    case SV_RX: x = b0; return true;
    case SV_RY: x = z = b0; return true;
    case SV_RZ: z = b0; return true;
    case SV_P: z = b0; beta = -1.0; return true;   // diag(1, e^{i l}) = exp(-i l (Z - I)/2)
    case SV_RXX: x = b01; return true;
    case SV_RYY: x = z = b01; return true;
    case SV_RZZ: z = b01; return true;
    default: return false;
  }
}

// --------------------------------------------------------------- planner

struct StageP {
  std::vector<int> recs;      // indices into the record list, program order
  int gq[SVI_RMAX];           // tile-local position of group bit i
  bool dense = false;
  bool kron = false;          // canonical Kronecker stage
  std::vector<int> lead, dbefore, rops, dafter, trail;   // kron: records by role
};

// Diagonal records (phases, Z-type gates, any controls) commute with each
// other, so an untaken diagonal record holds back only the non-diagonal
// records after it that share a qubit; any other untaken record holds back
// every later record sharing a qubit.  Taking a record then moves it only
// across records it commutes with.
static bool is_diag(const GateRec &g) { return g.mo == MO_P || g.mo == MO_NEG; }

// Records a Kronecker stage can hold: uncontrolled RY rotations, diagonal
// gates (any controls) and permutations (any controls).  A leading or trailing
// X whose controls are group qubits may target any tile qubit: the bit flip
// then depends on the register slot only, so it is a fixed XOR on the slot's
// LDS offset, whichever thread holds the slot.
// A gradient record (adjoint backward program) fits too when its generator
// commutes with everything the stage applies between the stage point where its
// gradient is evaluated and the gate itself: a diagonal generator for diagonal
// gates (evaluated on the stage input, or after the rotations for diagonal gates
// that follow a rotation), Y on the rotated qubit for an RY (evaluated after the
// leading diagonal table; the other rotations act on other qubits).
static bool kron_eligible(const GateRec &g) {
  if (g.mo == MO_R) return g.nc == 0 && g.nt == 1 && g.kind == SV_RY;
  if (g.grad) return g.mo == MO_P && g.gx == 0;
  return g.mo == MO_P || g.mo == MO_NEG || g.mo == MO_X || g.mo == MO_SWAP;
}

// Closure of records that fit  P_trail * D_after * (x) R * D_before * P_lead  inside S
// (an X of P_lead / P_trail: controls in S, target anywhere in the tile Tt).
// Returns a score: rotations weigh more than diagonal gates and permutations,
// which can ride along in many stages, while every rotation costs a stage slot.
static constexpr int kRotWeight = 4;
static int closure_kron(const std::vector<GateRec> &recs, const std::vector<int> &cand,
                        const std::vector<char> &done, uint64_t S, uint64_t Tt, StageP *st) {
  uint64_t blocked = 0, blocked_nd = 0, rq = 0, dA = 0, pq = 0;
  bool leading = true;
  int cnt = 0;
  for (int r : cand) {
    if (done[r]) continue;
    const GateRec &g = recs[r];
    const uint64_t q = g.qmask;
    const uint64_t tq = g.mo == MO_X ? 1ull << g.t[0] : 0;
    const bool fits = (q & ~S) == 0 || (tq && (q & ~tq & ~S) == 0 && (tq & Tt) != 0);
    const bool free = (q & blocked) == 0 && (is_diag(g) || (q & blocked_nd) == 0);
    bool ok = fits && free && kron_eligible(g);
    int role = -1;   // 0 lead, 1 dbefore, 2 r, 3 dafter, 4 trail
    if (ok) {
      if (g.mo == MO_X || g.mo == MO_SWAP) {
        role = leading ? 0 : 4;
        if (!leading) pq |= q;
      } else if (g.mo == MO_P || g.mo == MO_NEG) {
        if (q & pq) ok = false;
        else if (q & rq) { role = 3; dA |= q; }
        else role = 1;
      } else {
        if (q & (rq | dA | pq)) ok = false;
        else { role = 2; rq |= q; }
      }
    }
    if (ok) {
      if (role != 0) leading = false;
      cnt += role == 2 ? kRotWeight : 1;
      if (st) {
        st->recs.push_back(r);
        std::vector<int> *dst[5] = {&st->lead, &st->dbefore, &st->rops, &st->dafter, &st->trail};
        dst[role]->push_back(r);
      }
    } else {
      if (is_diag(g)) blocked_nd |= q;
      else blocked |= q;
      if ((blocked & S) == S) break;
    }
  }
  return cnt;
}

struct SweepP {
  int m = 0, c = 0, nh = 0;
  int hb[SVI_MMAX] = {0};     // physical bit positions of tile bits c..m-1
  int lq[SVI_MMAX] = {0};     // logical qubit held by each tile-local bit (input side)
  bool operm = false;         // the sweep permutes tile bits on output
  int perm[SVI_MMAX] = {0};   // output tile bit k takes input tile bit perm[k]
  std::vector<StageP> stages;
};

struct Tiling {
  int M = 13, c = 3, R = 5;
};

static int popc(uint64_t v) { return __builtin_popcountll(v); }

// Records of `cand` (program order, not yet done) that can run inside qubit set T:
// a record is taken iff its qubits lie in T and no earlier untaken record it
// does not commute with (see is_diag) shares a qubit with it.  Records flagged
// in `veto` block like untaken ones.
static int closure(const std::vector<GateRec> &recs, const std::vector<int> &cand,
                   const std::vector<char> &done, uint64_t T, std::vector<int> *take,
                   const std::vector<char> *veto = nullptr, double cost_cap = 1e300) {
  uint64_t blocked = 0, blocked_nd = 0;   // all records / non-diagonal records held back
  int cnt = 0;
  double cost = 0.0;
  for (int r : cand) {
    if (done[r]) continue;
    const uint64_t q = recs[r].qmask;
    const bool vetoed = veto && (*veto)[r];
    const bool diag = is_diag(recs[r]);
    const bool free = (q & blocked) == 0 && (diag || (q & blocked_nd) == 0);
    if (!vetoed && (q & ~T) == 0 && free && cost + recs[r].cost <= cost_cap) {
      cnt++;
      cost += recs[r].cost;
      if (take) take->push_back(r);
    } else {
      if (diag && !vetoed) blocked_nd |= q;
      else blocked |= q;
      if ((blocked & T) == T) break;
    }
  }
  return cnt;
}

// Qubits of the earliest pending record that is blocked w.r.t. T (tie-break).
static uint64_t first_blocked_qubits(const std::vector<GateRec> &recs, const std::vector<int> &cand,
                                     const std::vector<char> &done, uint64_t T) {
  uint64_t blocked = 0, blocked_nd = 0;
  for (int r : cand) {
    if (done[r]) continue;
    const uint64_t q = recs[r].qmask;
    const bool diag = is_diag(recs[r]);
    const bool free = (q & blocked) == 0 && (diag || (q & blocked_nd) == 0);
    if ((q & ~T) == 0 && free) continue;
    return q & ~T ? (q & ~T) : q;
  }
  return 0;
}

// Tile-local bit of logical qubit q (-1 if q is not in the tile).
static int tile_pos(const SweepP &sw, int q) {
  for (int p = 0; p < sw.m; p++)
    if (sw.lq[p] == q) return p;
  return -1;
}

// Tile over logical qubit set T with physical layout occ (physical position ->
// logical qubit; identity when null): the c lowest physical positions, whose
// occupants must lie in T, plus the physical positions of T's other qubits.
static void set_tile(SweepP &sw, int n, uint64_t T, int c, const int *occ = nullptr) {
  if (popc(T) > SVI_MMAX) abort();   // planner invariant: a tile holds at most SVI_MMAX qubits
  sw.c = c;
  sw.nh = 0;
  for (int p = 0; p < c; p++) sw.lq[p] = occ ? occ[p] : p;
  for (int p = c; p < n; p++) {
    const int q = occ ? occ[p] : p;
    if (T & (1ull << q)) {
      sw.hb[sw.nh] = p;
      sw.lq[c + sw.nh] = q;
      sw.nh++;
    }
  }
  sw.m = c + sw.nh;
}

// Logical qubits held by the tile, as a mask.
static uint64_t tile_mask(const SweepP &sw) {
  uint64_t T = 0;
  for (int p = 0; p < sw.m; p++) T |= 1ull << sw.lq[p];
  return T;
}

// Split one sweep's records into register stages of <= R qubits.
static void plan_stages(const std::vector<GateRec> &recs, const std::vector<int> &take, SweepP &sw,
                        int R, int n, bool allow_kron = false) {
  std::vector<char> done(recs.size(), 0);
  std::vector<char> veto(recs.size(), 0);
  for (int r : take)
    if (recs[r].mo == MO_DENSE) veto[r] = 1;
  const uint64_t Ttile = tile_mask(sw);
  size_t left = take.size();
  const int mm = std::max(sw.m, R);
  while (left) {
    int first = -1;
    for (int r : take)
      if (!done[r]) { first = r; break; }
    StageP st;
    std::vector<int> grp;   // qubits (global) in group order
    if (allow_kron && kron_eligible(recs[first])) {
      uint64_t S = recs[first].qmask;
      while (popc(S) < R) {
        int best = -1, bestv = closure_kron(recs, take, done, S, Ttile, nullptr);
        for (int q = 0; q < n; q++) {
          if (!(Ttile & (1ull << q)) || (S & (1ull << q))) continue;
          int v = closure_kron(recs, take, done, S | (1ull << q), Ttile, nullptr);
          if (v > bestv) { bestv = v; best = q; }
        }
        if (best < 0) break;
        S |= 1ull << best;
      }
      st.kron = true;
      closure_kron(recs, take, done, S, Ttile, &st);
      for (int r : st.recs) { done[r] = 1; left--; }
      for (int q = 0; q < n; q++)
        if (S & (1ull << q)) grp.push_back(q);
    } else if (recs[first].mo == MO_DENSE) {
      st.dense = true;
      st.recs.push_back(first);
      done[first] = 1;
      left--;
      for (int i = 0; i < recs[first].nt; i++) grp.push_back(recs[first].t[i]);
      for (int i = 0; i < recs[first].nc; i++) grp.push_back(recs[first].c[i]);
    } else {
      uint64_t S = recs[first].qmask;
      while (popc(S) < R) {
        int best = -1, bestv = closure(recs, take, done, S, nullptr, &veto);
        for (int q = 0; q < n; q++) {
          if (!(Ttile & (1ull << q)) || (S & (1ull << q))) continue;
          int v = closure(recs, take, done, S | (1ull << q), nullptr, &veto);
          if (v > bestv) { bestv = v; best = q; }
        }
        if (best < 0) {
          uint64_t fq = first_blocked_qubits(recs, take, done, S) & Ttile & ~S;
          // only grow by a record we can actually take later
          if (fq && popc(S | fq) <= R) {
            S |= fq;
            continue;
          }
          break;
        }
        S |= 1ull << best;
      }
      std::vector<int> got;
      closure(recs, take, done, S, &got, &veto);
      for (int r : got) { done[r] = 1; left--; }
      st.recs = got;
      for (int q = 0; q < n; q++)
        if (S & (1ull << q)) grp.push_back(q);
    }
    // group bit -> tile-local position; pad with the highest unused positions
    int used = 0;
    for (size_t i = 0; i < grp.size(); i++) st.gq[i] = tile_pos(sw, grp[i]);
    used = (int)grp.size();
    uint64_t taken = 0;
    for (int i = 0; i < used; i++) taken |= 1ull << st.gq[i];
    for (int p = mm - 1; p >= 0 && used < R; p--)
      if (!(taken & (1ull << p))) { st.gq[used++] = p; taken |= 1ull << p; }
    sw.stages.push_back(st);
  }
}

// Output layout of a remapping sweep: the tile's positions get the occupants
// in `want` (physical position -> logical qubit, tile positions only); records
// the tile-local output permutation in sw and applies it to occ.
static void set_output_layout(SweepP &sw, std::vector<int> &occ, const std::vector<int> &want) {
  bool change = false;
  for (int k = 0; k < sw.m; k++) {
    const int phys = k < sw.c ? k : sw.hb[k - sw.c];
    const int q = want[phys];
    sw.perm[k] = tile_pos(sw, q);
    if (sw.perm[k] != k) change = true;
  }
  sw.operm = change;
  for (int k = 0; k < sw.m; k++) {
    const int phys = k < sw.c ? k : sw.hb[k - sw.c];
    occ[phys] = want[phys];
  }
}

// Replays a plan's qubit layout: every tile's logical map matches the layout
// it reads, every output permutation is a bijection of the tile bits, and the
// plan ends in the identity layout.
static bool layout_consistent(const std::vector<SweepP> &sweeps, int n) {
  std::vector<int> occ(n);
  for (int p = 0; p < n; p++) occ[p] = p;
  for (const SweepP &sw : sweeps) {
    if (sw.m > SVI_MMAX || sw.m != sw.c + sw.nh) return false;
    std::vector<int> nxt = occ;
    uint32_t used = 0;
    for (int k = 0; k < sw.m; k++) {
      const int phys = k < sw.c ? k : sw.hb[k - sw.c];
      if (phys < 0 || phys >= n || sw.lq[k] != occ[phys]) return false;
      const int src = sw.operm ? sw.perm[k] : k;
      if (src < 0 || src >= sw.m || (used >> src) & 1) return false;
      used |= 1u << src;
      nxt[phys] = sw.lq[src];
    }
    occ = nxt;
  }
  for (int p = 0; p < n; p++)
    if (occ[p] != p) return false;
  return true;
}

// AUTO planner: DAG-aware tile clustering.  With `remap`, the c low physical
// positions (contiguous rows in HBM) are not tied to qubits 0..c-1: at the end
// of each sweep the tile's qubits are permuted so that the low positions hold
// the qubits the earliest pending gates need, and the last sweep (or one extra
// sweep) restores the identity layout.
static void plan_auto(const std::vector<GateRec> &recs, int n, const Tiling &tl,
                      std::vector<SweepP> &out, double cost_cap, bool kron = false,
                      bool remap = false) {
  const int M = std::min(tl.M, n);
  const int c = std::min(tl.c, n);
  std::vector<int> cand(recs.size());
  for (size_t i = 0; i < recs.size(); i++) cand[i] = (int)i;
  std::vector<char> done(recs.size(), 0);
  size_t left = recs.size();
  std::vector<int> occ(n);
  for (int p = 0; p < n; p++) occ[p] = p;
  // restoring the layout needs the low positions and the homes of their
  // occupants in one tile
  remap = remap && n > M && 2 * c <= M;
  size_t start = 0;
  while (left) {
    while (start < cand.size() && done[cand[start]]) start++;
    std::vector<int> sub(cand.begin() + start, cand.end());
    uint64_t T = 0;
    for (int p = 0; p < c; p++) T |= 1ull << occ[p];
    if (n <= M) {
      T = n >= 64 ? ~0ull : ((1ull << n) - 1);
    } else {
      for (int step = c; step < M; step++) {
        int best = -1, bestv = closure(recs, sub, done, T, nullptr, nullptr, cost_cap);
        for (int q = 0; q < n; q++) {
          if (T & (1ull << q)) continue;
          int v = closure(recs, sub, done, T | (1ull << q), nullptr, nullptr, cost_cap);
          if (v > bestv) { bestv = v; best = q; }
        }
        if (best < 0) {
          uint64_t fq = first_blocked_qubits(recs, sub, done, T) & ~T;
          if (!fq) break;
          // lowest qubit of the earliest blocked record
          best = __builtin_ctzll(fq);
        }
        T |= 1ull << best;
      }
      // fill the tile to M qubits (larger tiles cost nothing extra)
      for (int q = 0; q < n && popc(T) < M; q++) T |= 1ull << q;
    }
    std::vector<int> take;
    closure(recs, sub, done, T, &take, nullptr, cost_cap);
    if (take.empty()) {
      // cost cap smaller than one record: take the first pending record alone
      take.push_back(sub[0]);
    }
    SweepP sw;
    set_tile(sw, n, T, c, occ.data());
    plan_stages(recs, take, sw, tl.R, n, kron);
    for (int r : take) { done[r] = 1; left--; }
    if (remap) {
      std::vector<int> want = occ;
      if (!left) {
        for (int k = 0; k < sw.m; k++) {
          const int phys = k < sw.c ? k : sw.hb[k - sw.c];
          want[phys] = phys;
        }
        // a qubit whose home position is outside this tile cannot go home here
        bool ok = true;
        for (int k = 0; k < sw.m; k++) {
          const int phys = k < sw.c ? k : sw.hb[k - sw.c];
          if (tile_pos(sw, phys) < 0) ok = false;
        }
        if (!ok) want = occ;
      } else {
        // Layout invariant: a high position p holds qubit p or one of the
        // qubits 0..c-1, so at most c high positions are ever displaced and the
        // identity layout comes back within one tile.
        // Wanted low occupants: tile qubits of the earliest pending records.
        std::vector<int> pick;
        uint64_t seen = 0;
        for (size_t i = start; i < cand.size() && (int)pick.size() < c; i++) {
          const int r = cand[i];
          if (done[r]) continue;
          uint64_t q = recs[r].qmask & T & ~seen;
          while (q && (int)pick.size() < c) {
            const int b = __builtin_ctzll(q);
            q &= q - 1;
            pick.push_back(b);
            seen |= 1ull << b;
          }
        }
        uint64_t lowset = 0;
        for (int p = 0; p < c; p++) lowset |= 1ull << occ[p];
        std::vector<int> incoming;
        for (int q : pick)
          if (!(lowset & (1ull << q))) incoming.push_back(q);
        // low positions whose occupant is not wanted, evictable ones only: an
        // outgoing qubit >= c must go home, so its home position must be in the tile
        auto has_pos = [&](int phys) {
          if (phys < sw.c) return true;
          for (int k = 0; k < sw.nh; k++)
            if (sw.hb[k] == phys) return true;
          return false;
        };
        std::vector<int> freed;
        for (int p = 0; p < c; p++) {
          const int x = occ[p];
          if (seen & (1ull << x)) continue;
          if (x >= c && !has_pos(x)) continue;
          freed.push_back(p);
        }
        const size_t moves = std::min(freed.size(), incoming.size());
        std::vector<int> avail, place;
        for (size_t i = 0; i < moves; i++) {
          const int q = incoming[i];
          for (int k = 0; k < sw.m; k++) {
            const int phys = k < sw.c ? k : sw.hb[k - sw.c];
            if (occ[phys] == q) avail.push_back(phys);
          }
          want[freed[i]] = q;
        }
        for (size_t i = 0; i < moves; i++) {
          const int x = occ[freed[i]];
          if (x < c) {
            place.push_back(x);
            continue;
          }
          want[x] = x;   // back home
          auto it = std::find(avail.begin(), avail.end(), x);
          if (it != avail.end()) avail.erase(it);
          else place.push_back(occ[x]);   // the low qubit parked there moves on
        }
        for (size_t i = 0; i < avail.size(); i++) want[avail[i]] = place[i];
      }
      set_output_layout(sw, occ, want);
    }
    out.push_back(std::move(sw));
  }
  if (remap) {
    // restore the identity layout with one sweep that holds every displaced position
    uint64_t D = 0;
    for (int p = 0; p < n; p++)
      if (occ[p] != p) D |= 1ull << p;
    if (D) {
      uint64_t T = 0;
      for (int p = 0; p < c; p++) T |= 1ull << occ[p];
      for (int p = 0; p < n; p++)
        if (D & (1ull << p)) T |= 1ull << occ[p];
      for (int q = 0; q < n && popc(T) < M; q++) T |= 1ull << q;
      SweepP sw;
      set_tile(sw, n, T, c, occ.data());
      std::vector<int> want = occ;
      for (int k = 0; k < sw.m; k++) {
        const int phys = k < sw.c ? k : sw.hb[k - sw.c];
        want[phys] = phys;
      }
      set_output_layout(sw, occ, want);
      out.push_back(std::move(sw));
    }
  }
}

// Paper-style fusion: greedy in-order blocks of <= width qubits, one sweep per block.
static int fuse_greedy(const std::vector<GateRec> &recs, int width, std::vector<int> &block_of) {
  uint64_t open = 0;
  int nb = 0;
  block_of.resize(recs.size());
  for (size_t i = 0; i < recs.size(); i++) {
    const uint64_t q = recs[i].qmask;
    if (open && popc(open | q) > width) open = 0;
    if (!open) nb++;
    open |= q;
    block_of[i] = nb - 1;
  }
  return nb;
}

static void plan_fused(const std::vector<GateRec> &recs, int n, const Tiling &tl, int width,
                       std::vector<SweepP> &out, bool kron = false) {
  std::vector<int> block_of;
  int nb = fuse_greedy(recs, width, block_of);
  const int M = std::min(tl.M, n);
  const int c = std::min(tl.c, n);
  size_t i = 0;
  for (int b = 0; b < nb; b++) {
    std::vector<int> take;
    uint64_t Q = 0;
    while (i < recs.size() && block_of[i] == b) { take.push_back((int)i); Q |= recs[i].qmask; i++; }
    uint64_t T = (c >= 64 ? ~0ull : ((1ull << c) - 1)) | Q;
    for (int q = c; q < n && popc(T) < M; q++) T |= 1ull << q;
    SweepP sw;
    set_tile(sw, n, T, c);
    plan_stages(recs, take, sw, tl.R, n, kron);
    out.push_back(std::move(sw));
  }
}

// --------------------------------------------------------- plan material

struct Step {
  int kind = 0;              // 0 = tile sweep, 1 = single-gate kernel
  bool all_kron = false;     // every stage is a Kronecker stage (lean kernel)
  SweepArgs sa{};            // tile sweep (pointers patched at launch)
  GateArgsHost ga{};         // single gate
  int gate_coef = -1;
};

struct Plan {
  int n = 0;
  bool dbl = true;
  int M = 13, R = 5, NS = 1;
  std::vector<Step> steps;
  std::vector<StageDesc> stages;
  std::vector<MicroOp> ops;
  std::vector<CoefDesc> coefs;
  std::vector<TabFactor> factors;
  int ncoef = 0;
  std::vector<double> constants;     // appended after the user parameters
  int n_user_params = 0;
  int n_user_mats = 0;
  std::vector<int> mat_dim;          // per user matrix: doubles
  int nstatic = 0;
  // adjoint
  int n_gslots = 0;
  std::vector<int> slot_param;
  std::vector<int32_t> grad_rowptr, grad_slots;
  // device buffers
  void *d_buf = nullptr;
  size_t d_bytes = 0;
  StageDesc *d_stages = nullptr;
  MicroOp *d_ops = nullptr;
  CoefDesc *d_coefdesc = nullptr;
  TabFactor *d_factors = nullptr;
  double *d_coef = nullptr;
  double *d_params = nullptr;        // user params + constants
  double *d_statics = nullptr;
  int32_t *d_rowptr = nullptr, *d_gslots = nullptr;
  int n_sweeps = 0, n_blocks = 0;
  ~Plan() {
    if (d_buf) (void)hipFree(d_buf);
  }
};

static void add_coef(Plan &P, GateRec &g, int &coef_off) {
  coef_off = -1;
  if (g.ncoef == 0) return;
  CoefDesc cd{};
  cd.kind = g.coef_kind;
  cd.fmt = g.fmt | (g.dagger ? CF_DAGGER : 0);
  for (int k = 0; k < 3; k++) cd.pidx[k] = g.pidx[k];
  cd.dst = P.ncoef;
  if (g.fmt == CF_COPY) {
    int off = 0;
    for (int k = 0; k < g.user_mat; k++) off += P.mat_dim[k];
    cd.src = off;
    cd.len = g.ncoef;
  }
  P.coefs.push_back(cd);
  coef_off = P.ncoef;
  P.ncoef += g.ncoef;
}

static uint16_t spread_local(int j, const int *gq, int R) {
  int o = 0;
  for (int i = 0; i < R; i++)
    if ((j >> i) & 1) o |= 1 << gq[i];
  return (uint16_t)o;
}

static int perm_apply(const MicroOp &op, int j) {
  if (((uint32_t)j & op.cm) != op.cv) return j;
  if (op.type == MO_X) return j ^ (1 << op.t0);
  if (op.type == MO_SWAP) {
    int a = (j >> op.t0) & 1, b = (j >> op.t1) & 1;
    return a != b ? (j ^ (1 << op.t0) ^ (1 << op.t1)) : j;
  }
  return j;
}

// Thread maps of one sweep's stages (StageDesc::tpos): the lane bits take
// the stage's exchanged tile bits, the wave bits stay where the previous
// stage had them whenever that stage's group and exchanged bits allow it
// (then the transition is wave-local: SD_WLOCAL on the previous stage), and
// otherwise move to the non-group tile bits that the following stages leave
// free longest.  Tile bits at or above mm exist only past a small state's
// tile (m < M): they take the highest thread bits, so that the threads below
// 2^(mm - R) are exactly the ones holding the state (the gradient kernels
// count only those).
static void assign_thread_maps(Plan &P, int first, const std::vector<int> &gm,
                               const std::vector<int> &xb, int R, int mm) {
  const int M = P.M, ntb = M - R, nw = std::max(0, ntb - 6);
  const int ns = (int)gm.size();
  const int real = (1 << mm) - 1;
  std::vector<int> wprev;
  for (int s = 0; s < ns; s++) {
    StageDesc &sd = P.stages[first + s];
    const int ng = ((1 << M) - 1) & ~gm[s];
    const int ngr = ng & real, ngp = ng & ~real;
    std::vector<int> phant;
    for (int p = 0; p < M; p++)
      if ((ngp >> p) & 1) phant.push_back(p);
    int xs = xb[s] & ngr;
    if (__builtin_popcount((unsigned)xs) > 6) {   // cannot all be lane bits
      sd.dflags |= SD_XCHG;
      xs = 0;
    }
    std::vector<int> wr;   // wave bits on real tile bits
    const int nwr = nw - std::min(nw, (int)phant.size());
    const int avail = ngr & ~xs;
    bool keep = s > 0;
    int nprev_real = 0;
    for (int p : wprev)
      if ((real >> p) & 1) {
        nprev_real++;
        if (!((avail >> p) & 1)) keep = false;
      }
    if (nprev_real != nwr) keep = false;
    if (keep) {
      for (int p : wprev)
        if ((real >> p) & 1) wr.push_back(p);
    } else if (nwr > 0) {
      // free run of each candidate bit over the following stages
      std::vector<std::pair<int, int>> cand;
      for (int p = 0; p < M; p++) {
        if (!((avail >> p) & 1)) continue;
        int run = 0;
        for (int t = s + 1; t < ns && !(((gm[t] | xb[t]) >> p) & 1); t++) run++;
        cand.push_back({run, p});
      }
      std::sort(cand.begin(), cand.end(), [](const std::pair<int, int> &x, const std::pair<int, int> &y) {
        return x.first != y.first ? x.first > y.first : x.second > y.second;
      });
      for (int i = 0; i < nwr; i++) wr.push_back(cand[i].second);
      std::sort(wr.begin(), wr.end());
    }
    // wave bits: the real ones, then the highest phantom ones
    std::vector<int> w = wr;
    const int nwp = nw - nwr;
    for (int i = (int)phant.size() - nwp; i < (int)phant.size(); i++) w.push_back(phant[i]);
    if (keep || (s > 0 && w == wprev)) P.stages[first + s - 1].dflags |= SD_WLOCAL;
    int wmask = 0;
    for (int p : w) wmask |= 1 << p;
    // lane bits: the real ones first, then the remaining phantom ones
    std::vector<int> lanes, lanep;
    for (int p = 0; p < M; p++) {
      if (!((ng >> p) & 1) || ((wmask >> p) & 1)) continue;
      if ((real >> p) & 1) lanes.push_back(p);
      else lanep.push_back(p);
    }
    if ((int)(lanes.size() + lanep.size()) != ntb - nw) abort();   // planner invariant
    // An LDS access of one complex element serves 2^B consecutive lanes per
    // pass (B = 3 for 16-byte FP64 elements, 4 for 8-byte FP32 ones), and the
    // swizzle folds tile bit p onto element bit p mod B: the B lowest lane bits
    // go on tile bits of distinct p mod B where the real lane bits allow it.
    const int B = P.dbl ? 3 : 4;
    if ((int)lanes.size() >= B) {
      for (int i = 0; i < B; i++) {
        int used = 0;
        for (int j = 0; j < i; j++) used |= 1 << (lanes[j] % B);
        if (!((used >> (lanes[i] % B)) & 1)) continue;
        for (size_t j = i + 1; j < lanes.size(); j++)
          if (!((used >> (lanes[j] % B)) & 1)) { std::swap(lanes[i], lanes[j]); break; }
      }
    }
    int k = 0;
    for (int p : lanes) sd.tpos[k++] = (int8_t)p;
    for (int p : lanep) sd.tpos[k++] = (int8_t)p;
    for (int p : w) sd.tpos[k++] = (int8_t)p;
    for (; k < 16; k++) sd.tpos[k] = 0;
    wprev = w;
  }
}

// Emit the device descriptors of one tile sweep.
static void emit_sweep(Plan &P, std::vector<GateRec> &recs, const SweepP &sw, int n, int R,
                       int flags, int gslot_base, int &gslots_used) {
  const int SWB = P.dbl ? 3 : 4;
  const int EB = P.dbl ? 16 : 8;        // bytes per LDS complex element
  Step s;
  s.kind = 0;
  SweepArgs &a = s.sa;
  std::memset(&a, 0, sizeof a);
  a.n = n;
  a.m = sw.m;
  a.c = sw.c;
  a.nh = sw.nh;
  for (int k = 0; k < SVI_MMAX; k++) a.hb[k] = k < sw.nh ? sw.hb[k] : 0;
  a.flags = flags;
  if (sw.operm) {
    a.flags |= SW_OPERM;
    for (int k = 0; k < SVI_MMAX; k++) a.operm[k] = k < sw.m ? sw.perm[k] : 0;
  }
  a.ntiles = (int64_t)1 << (n - sw.m);
  a.stage_begin = (int)P.stages.size();
  a.gslot_begin = gslot_base;
  int gs = 0;
  std::vector<int> st_gmask, st_xbits;   // per stage: group bits, exchanged bits
  for (const StageP &st : sw.stages) {
    // group bits: qubit of tile position st.gq[i]
    auto local_of = [&](int q) {
      int p = tile_pos(sw, q);
      for (int i = 0; i < R; i++)
        if (st.gq[i] == p) return i;
      return -1;
    };
    std::vector<MicroOp> mops;                 // ST_OPS: gradient op, then gate op
    std::vector<MicroOp> gate_mop, grad_mop;   // per record of the stage (grad type -1: none)
    for (int r : st.recs) {
      GateRec &g = recs[r];
      MicroOp none{};
      none.type = -1;
      grad_mop.push_back(none);
      uint32_t cm = 0, cv = 0;
      for (int i = 0; i < g.nc; i++) {
        int l = local_of(g.c[i]);
        cm |= 1u << l;
        if ((g.cs >> i) & 1u) cv |= 1u << l;
      }
      if (g.grad && g.grad2l) {
        MicroOp go{};
        go.type = MO_GRAD2L;
        uint32_t tm = 0, pa, pb;
        for (int i = 0; i < g.nt; i++) tm |= 1u << local_of(g.t[i]);
        if (g.nt == 2) { pa = 1u << local_of(g.t[0]); pb = 1u << local_of(g.t[1]); }
        else {
          pa = (1u << local_of(g.t[0])) | (1u << local_of(g.t[1]));
          pb = (1u << local_of(g.t[2])) | (1u << local_of(g.t[3]));
        }
        go.mask = tm;
        go.gz = pa;
        go.t1 = (int)(pa ^ pb);
        go.cm = cm;
        go.cv = cv;
        go.coef = gs;
        P.slot_param.push_back(g.gparam);
        gs++;
        mops.push_back(go);
        grad_mop.back() = go;
      } else if (g.grad) {
        MicroOp go{};
        go.type = MO_GRAD;
        uint32_t xl = 0, zl = 0;
        for (int q = 0; q < n; q++) {
          if ((g.gx >> q) & 1) xl |= 1u << local_of(q);
          if ((g.gz >> q) & 1) zl |= 1u << local_of(q);
        }
        go.mask = xl;
        go.gz = zl;
        go.cm = cm;
        go.cv = cv;
        go.galpha = g.galpha;
        go.gbeta = g.gbeta;
        go.coef = gs;
        // per-slot table of the generator (sv_internal.h, MO_GRAD): plan
        // constants, copied into the coefficient buffer on every call
        {
          const int G = 1 << R;
          const int ny = __builtin_popcount(xl & zl) & 3;
          // beta multiplies the identity: the x = 0 form (phase gates only)
          if (g.gbeta != 0.0 && xl != 0) abort();   // planner invariant
          go.t1 = (ny & 1) ? GRAD_ODD : 0;
          const int base = P.n_user_params + (int)P.constants.size();
          for (int j = 0; j < G; j++) {
            double cj = 0.0;
            if (((uint32_t)j & cm) == cv) {
              const uint32_t k = (uint32_t)j ^ xl;
              cj = g.galpha * ((__builtin_popcount(k & zl) & 1) ? -1.0 : 1.0) * (ny >= 2 ? -1.0 : 1.0);
              cj += g.gbeta;
            }
            P.constants.push_back(cj);
          }
          CoefDesc cd{};
          cd.fmt = CF_CONSTS;
          cd.src = base;
          cd.len = G;
          cd.dst = P.ncoef;
          cd.pidx[0] = cd.pidx[1] = cd.pidx[2] = -1;
          P.coefs.push_back(cd);
          go.t0 = P.ncoef;
          P.ncoef += cd.len;
        }
        P.slot_param.push_back(g.gparam);
        gs++;
        mops.push_back(go);
        grad_mop.back() = go;
      }
      MicroOp op{};
      op.type = g.mo;
      op.cm = cm;
      op.cv = cv;
      int coff = -1;
      if (!st.kron) add_coef(P, g, coff);
      op.coef = coff < 0 ? 0 : coff;
      switch (g.mo) {
        case MO_U: case MO_R: case MO_X: op.t0 = local_of(g.t[0]); break;
        case MO_P: {
          uint32_t mk = 0;
          for (int i = 0; i < g.nt; i++) mk |= 1u << local_of(g.t[i]);
          op.mask = mk;
          break;
        }
        case MO_NEG: {
          int l = local_of(g.t[0]);
          op.cm |= 1u << l;
          op.cv |= 1u << l;
          break;
        }
        case MO_SWAP: case MO_Q: op.t0 = local_of(g.t[0]); op.t1 = local_of(g.t[1]); break;
        case MO_2L: {
          uint32_t tm = 0;
          for (int i = 0; i < g.nt; i++) tm |= 1u << local_of(g.t[i]);
          uint32_t pa, pb;
          if (g.nt == 2) { pa = 1u << local_of(g.t[0]); pb = 1u << local_of(g.t[1]); }
          else {
            pa = (1u << local_of(g.t[0])) | (1u << local_of(g.t[1]));
            pb = (1u << local_of(g.t[2])) | (1u << local_of(g.t[3]));
          }
          op.mask = tm;
          op.gz = pa;
          op.t1 = (int)(pa ^ pb);
          break;
        }
        case MO_DENSE: op.mask = g.nt; break;   // targets are group bits 0..k-1
        default: break;
      }
      mops.push_back(op);
      gate_mop.push_back(op);
    }
    StageDesc sd;
    std::memset(&sd, 0, sizeof sd);
    int sorted[SVI_RMAX];
    for (int i = 0; i < R; i++) sorted[i] = st.gq[i];
    std::sort(sorted, sorted + R);
    for (int i = 0; i < SVI_RMAX; i++) sd.sbits[i] = i < R ? sorted[i] : 0;
    std::vector<MicroOp> leadp, trailp, body;
    if (st.kron) {
      // mops holds every record's micro-op in stage order; split by role
      auto idx_of = [&](int r) {
        for (size_t k = 0; k < st.recs.size(); k++)
          if (st.recs[k] == r) return (int)k;
        return -1;
      };
      auto mop_of = [&](int r) { return gate_mop[idx_of(r)]; };
      for (int r : st.lead) leadp.push_back(mop_of(r));
      for (int r : st.trail) trailp.push_back(mop_of(r));
      sd.kind = ST_KRON;
      sd.kcoef = P.ncoef;
      const int G = 1 << R;
      P.ncoef += 4 * R + 4 * G + 2;
      uint32_t rmask = 0;
      for (int r : st.rops) {
        GateRec &g = recs[r];
        int t = local_of(g.t[0]);
        rmask |= 1u << t;
        CoefDesc cd{};
        cd.kind = g.coef_kind;
        cd.fmt = CF_FASTR | (g.dagger ? CF_DAGGER : 0) | (P.dbl ? CF_FORM0 : 0);
        for (int k = 0; k < 3; k++) cd.pidx[k] = g.pidx[k];
        cd.dst = sd.kcoef + 4 * t;
        P.coefs.push_back(cd);
      }
      sd.rmask = rmask;
      // fast-Givens scales of the stage's real gates (folded into D_after or a scalar)
      auto push_scales = [&]() {
        for (int r : st.rops) {
          TabFactor f{};
          f.kind = recs[r].coef_kind;
          f.pidx = recs[r].pidx[0];
          f.neg = 2;
          P.factors.push_back(f);
        }
      };
      bool dag = false;
      for (int r : st.recs) dag = dag || recs[r].dagger;
      auto table = [&](const std::vector<int> &rs, int dst, bool scales) {
        CoefDesc cd{};
        cd.fmt = CF_TABLE | (dag ? CF_DAGGER : 0) | (P.dbl ? CF_FORM0 : 0);
        cd.src = (int)P.factors.size();
        cd.len = R;
        cd.dst = dst;
        if (scales) push_scales();
        for (int r : rs) {
          GateRec &g = recs[r];
          MicroOp m = mop_of(r);
          TabFactor f{};
          f.kind = g.coef_kind;
          f.pidx = g.pidx[0];
          f.cm = m.cm;
          f.cv = m.cv;
          if (g.mo == MO_NEG) f.neg = 1;
          else f.mask = m.mask;
          P.factors.push_back(f);
        }
        cd.pidx[0] = (int)P.factors.size() - cd.src;
        P.coefs.push_back(cd);
      };
      if (!st.dbefore.empty()) { sd.dflags |= 1; table(st.dbefore, sd.kcoef + 4 * R, false); }
      if (!st.dafter.empty()) {
        sd.dflags |= 2;
        table(st.dafter, sd.kcoef + 4 * R + 2 * G, true);
      }
      // gradient ops at the three stage points (diagonal gates before any
      // rotation: stage input; rotations: after D_before; diagonal gates
      // after a rotation: after the rotations)
      sd.op_begin = (int)P.ops.size();
      for (int r : st.dbefore)
        if (grad_mop[idx_of(r)].type == MO_GRAD) P.ops.push_back(grad_mop[idx_of(r)]);
      sd.g1 = (int)P.ops.size();
      for (int r : st.rops)
        if (grad_mop[idx_of(r)].type == MO_GRAD) P.ops.push_back(grad_mop[idx_of(r)]);
      sd.g2 = (int)P.ops.size();
      for (int r : st.dafter)
        if (grad_mop[idx_of(r)].type == MO_GRAD) P.ops.push_back(grad_mop[idx_of(r)]);
      sd.op_end = (int)P.ops.size();
      // ranges whose generators are all diagonal (the kernel then makes one
      // product array for them instead of one per generator form)
      sd.gdiag = 0;
      const int gb[4] = {sd.op_begin, sd.g1, sd.g2, sd.op_end};
      for (int p = 0; p < 3; p++) {
        bool diag = true;
        for (int o = gb[p]; o < gb[p + 1]; o++) diag = diag && P.ops[o].mask == 0;
        if (diag) sd.gdiag |= 1u << p;
      }
      // the scalar slot holds the product of the fast-Givens scales: applied
      // to the state when there is no D_after to carry it, and used to rescale
      // gradients taken between the rotations and D_after
      const bool scalar = st.dafter.empty() && !st.rops.empty();
      if (scalar || sd.g2 < sd.op_end) {
        if (scalar) sd.dflags |= 4;
        CoefDesc cd{};
        cd.fmt = CF_SCALE | (dag ? CF_DAGGER : 0) | (P.dbl ? CF_FORM0 : 0);
        cd.src = (int)P.factors.size();
        push_scales();
        cd.pidx[0] = (int)P.factors.size() - cd.src;
        cd.dst = sd.kcoef + 4 * R + 4 * G;
        P.coefs.push_back(cd);
      }
    } else {
      // fold leading / trailing permutations into the LDS offsets
      size_t lead = 0;
      while (lead < mops.size() && (mops[lead].type == MO_X || mops[lead].type == MO_SWAP)) lead++;
      size_t trail = mops.size();
      if (lead < mops.size())
        while (trail > lead && (mops[trail - 1].type == MO_X || mops[trail - 1].type == MO_SWAP)) trail--;
      leadp.assign(mops.begin(), mops.begin() + lead);
      trailp.assign(mops.begin() + trail, mops.end());
      body.assign(mops.begin() + lead, mops.begin() + trail);
      sd.kind = ST_OPS;
      sd.op_begin = (int)P.ops.size();
      for (const MicroOp &m : body) P.ops.push_back(m);
      sd.op_end = (int)P.ops.size();
      sd.g1 = sd.g2 = sd.op_end;
    }
    // slot j's tile-local offsets: its group bits placed, then the leading
    // permutations undone (load) or the trailing ones applied (store), on tile
    // positions, since a Kronecker stage's X may target a non-group tile bit
    auto perm_tile = [&](int r, int x) {
      const GateRec &g = recs[r];
      for (int i = 0; i < g.nc; i++) {
        const int b = (x >> tile_pos(sw, g.c[i])) & 1;
        if (b != (int)((g.cs >> i) & 1u)) return x;
      }
      if (g.mo == MO_X) return x ^ (1 << tile_pos(sw, g.t[0]));
      const int a = tile_pos(sw, g.t[0]), b = tile_pos(sw, g.t[1]);
      return ((x >> a) & 1) != ((x >> b) & 1) ? x ^ (1 << a) ^ (1 << b) : x;
    };
    const int gmask = spread_local((1 << R) - 1, st.gq, R);
    int xbits = 0;   // tile bits outside the group that the slot offsets reach
    for (int j = 0; j < (1 << R); j++) {
      if (st.kron) {
        int xl = spread_local(j, st.gq, R);
        for (size_t k = st.lead.size(); k-- > 0;) xl = perm_tile(st.lead[k], xl);
        sd.ld_off[j] = svi_swz(xl, SWB) * EB;
        int xs = spread_local(j, st.gq, R);
        for (size_t k = 0; k < st.trail.size(); k++) xs = perm_tile(st.trail[k], xs);
        sd.st_off[j] = svi_swz(xs, SWB) * EB;
        xbits |= (xl | xs) & ~gmask;
        continue;
      }
      int jl = j;
      for (size_t k = leadp.size(); k-- > 0;) jl = perm_apply(leadp[k], jl);
      sd.ld_off[j] = svi_swz(spread_local(jl, st.gq, R), SWB) * EB;
      int js = j;
      for (size_t k = 0; k < trailp.size(); k++) js = perm_apply(trailp[k], js);
      sd.st_off[j] = svi_swz(spread_local(js, st.gq, R), SWB) * EB;
    }
    st_gmask.push_back(gmask);
    st_xbits.push_back(xbits);
    P.stages.push_back(sd);
    P.n_blocks++;
  }
  a.stage_end = (int)P.stages.size();
  assign_thread_maps(P, a.stage_begin, st_gmask, st_xbits, R, std::max(sw.m, R));
  a.n_gslots = gs;
  // the two-state Kronecker kernel takes at most SVI_GSLOTS_MAX gradient slots per sweep
  s.all_kron = gs <= SVI_GSLOTS_MAX;
  for (int k = a.stage_begin; k < a.stage_end; k++)
    if (P.stages[k].kind != ST_KRON) s.all_kron = false;
  gslots_used = gs;
  P.steps.push_back(s);
  P.n_sweeps++;
}

static void emit_gate(Plan &P, GateRec &g, int n) {
  Step s;
  s.kind = 1;
  GateArgsHost &a = s.ga;
  std::memset(&a, 0, sizeof a);
  a.type = g.mo;
  a.t0 = g.t[0];
  a.t1 = g.nt > 1 ? g.t[1] : 0;
  int pos[16], np = 0;
  uint64_t cval = 0;
  for (int i = 0; i < g.nc; i++) {
    pos[np++] = g.c[i];
    if ((g.cs >> i) & 1u) cval |= 1ull << g.c[i];
  }
  if (g.mo == MO_P) {
    for (int i = 0; i < g.nt; i++) a.pmask |= 1ull << g.t[i];
  } else if (g.mo == MO_NEG) {
    pos[np++] = g.t[0];
    cval |= 1ull << g.t[0];
  } else {
    for (int i = 0; i < g.nt; i++) pos[np++] = g.t[i];
  }
  std::sort(pos, pos + np);
  a.npos = np;
  for (int i = 0; i < np; i++) a.pos[i] = pos[i];
  a.cval = cval;
  a.nitems = (int64_t)1 << (n - np);
  int coff = -1;
  add_coef(P, g, coff);
  s.gate_coef = coff;
  P.steps.push_back(s);
  P.n_sweeps++;
  P.n_blocks++;
}

static sv_status upload_plan(Plan &P) {
  // layout: stages | ops | coefdesc | coef | params | statics | rowptr | gslots
  auto align = [](size_t v) { return (v + 255) & ~(size_t)255; };
  size_t o_st = 0;
  size_t o_ops = align(o_st + P.stages.size() * sizeof(StageDesc));
  size_t o_cd = align(o_ops + P.ops.size() * sizeof(MicroOp));
  size_t o_fa = align(o_cd + P.coefs.size() * sizeof(CoefDesc));
  size_t o_cf = align(o_fa + (P.factors.size() + 1) * sizeof(TabFactor));
  size_t o_pa = align(o_cf + (size_t)std::max(P.ncoef, 1) * 8);
  size_t npar = (size_t)P.n_user_params + P.constants.size();
  size_t o_stc = align(o_pa + std::max<size_t>(npar, 1) * 8);
  size_t o_rp = align(o_stc + (size_t)std::max(P.nstatic, 1) * 8);
  size_t o_gs = align(o_rp + (P.grad_rowptr.size() + 1) * 4);
  size_t total = align(o_gs + (P.grad_slots.size() + 1) * 4);
  HIPCHK(hipMalloc(&P.d_buf, total));
  P.d_bytes = total;
  char *b = (char *)P.d_buf;
  P.d_stages = (StageDesc *)(b + o_st);
  P.d_ops = (MicroOp *)(b + o_ops);
  P.d_coefdesc = (CoefDesc *)(b + o_cd);
  P.d_coef = (double *)(b + o_cf);
  P.d_factors = (TabFactor *)(b + o_fa);
  if (!P.factors.empty())
    HIPCHK(hipMemcpy(P.d_factors, P.factors.data(), P.factors.size() * sizeof(TabFactor), hipMemcpyHostToDevice));
  P.d_params = (double *)(b + o_pa);
  P.d_statics = (double *)(b + o_stc);
  P.d_rowptr = (int32_t *)(b + o_rp);
  P.d_gslots = (int32_t *)(b + o_gs);
  if (!P.stages.empty())
    HIPCHK(hipMemcpy(P.d_stages, P.stages.data(), P.stages.size() * sizeof(StageDesc), hipMemcpyHostToDevice));
  if (!P.ops.empty())
    HIPCHK(hipMemcpy(P.d_ops, P.ops.data(), P.ops.size() * sizeof(MicroOp), hipMemcpyHostToDevice));
  if (!P.coefs.empty())
    HIPCHK(hipMemcpy(P.d_coefdesc, P.coefs.data(), P.coefs.size() * sizeof(CoefDesc), hipMemcpyHostToDevice));
  if (!P.constants.empty())
    HIPCHK(hipMemcpy(P.d_params + P.n_user_params, P.constants.data(), P.constants.size() * 8, hipMemcpyHostToDevice));
  if (!P.grad_rowptr.empty())
    HIPCHK(hipMemcpy(P.d_rowptr, P.grad_rowptr.data(), P.grad_rowptr.size() * 4, hipMemcpyHostToDevice));
  if (!P.grad_slots.empty())
    HIPCHK(hipMemcpy(P.d_gslots, P.grad_slots.data(), P.grad_slots.size() * 4, hipMemcpyHostToDevice));
  return SV_OK;
}

// ---------------------------------------------------------------- handle

struct sv_state {
  int n = 0;
  sv_dtype dtype = SV_C128;
  void *re = nullptr, *im = nullptr;
  void *ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  Tiling tiling;
  int dev = 0;
  Tiling adj_tiling;                 // backward sweeps of the adjoint
  std::unordered_map<std::string, std::unique_ptr<Plan>> plans;
  // growable scratch (partials)
  void *scratch = nullptr;
  size_t scratch_bytes = 0;
  // |0..0> requested but not yet written: the next sweep synthesises it
  bool pending_zero = false;
  // kernel timing instrumentation
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<double> ev_bytes;      // algorithmic bytes of each timed launch
  // second pair of planes for the shot estimator's rotated copies (on demand)
  void *copy = nullptr;
  size_t copy_bytes = 0;
  ~sv_state() {
    if (scratch) (void)hipFree(scratch);
    if (copy) (void)hipFree(copy);
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
  }
};

static hipEvent_t next_event(sv_state *st) {
  if (st->ev_used == st->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    st->ev_pool.push_back(e);
  }
  return st->ev_pool[st->ev_used++];
}

static size_t elem_size(sv_dtype d) { return d == SV_C128 ? 8 : 4; }

static int sample_K(int n) { int cb = n < 10 ? n : 10; return (int)(((int64_t)1 << n) >> cb); }

extern "C" size_t sv_workspace_bytes(int32_t n, sv_dtype dtype, uint32_t flags) {
  if (n < 1 || n > SVI_NMAX || (dtype != SV_C128 && dtype != SV_C64)) return 0;
  size_t K = (size_t)sample_K(n);
  size_t b = ((2 * K + 1) * 8 + 255) & ~(size_t)255;
  if (flags & SV_WS_ADJOINT) b += 4 * ((size_t)1 << n) * elem_size(dtype);
  return b + 256;
}

static void ws_layout(const sv_state *st, double **S, double **P, void **lre, void **lim, void **wre,
                      void **wim) {
  size_t K = (size_t)sample_K(st->n);
  char *b = (char *)st->ws;
  *S = (double *)b;
  *P = (double *)(b + K * 8);
  size_t off = ((2 * K + 1) * 8 + 255) & ~(size_t)255;
  size_t plane = ((size_t)1 << st->n) * elem_size(st->dtype);
  *lre = b + off;
  *lim = b + off + plane;
  *wre = b + off + 2 * plane;
  *wim = b + off + 3 * plane;
}

static sv_status ensure_scratch(sv_state *st, size_t bytes) {
  if (st->scratch_bytes >= bytes) return SV_OK;
  if (st->scratch) {
    HIPCHK(hipStreamSynchronize(st->stream));
    HIPCHK(hipFree(st->scratch));
    st->scratch = nullptr;
  }
  size_t b = std::max(bytes, (size_t)1 << 20);
  HIPCHK(hipMalloc(&st->scratch, b));
  st->scratch_bytes = b;
  return SV_OK;
}

static Tiling default_tiling(int n, sv_dtype dt, int NS) {
  Tiling t;
  if (dt == SV_C128) {
    // forward: 13-qubit tiles, 256-byte rows, 8-amplitude register groups
    // (1024-thread workgroups); measured best on the 30-qubit layered
    // workload among the compiled tilings with 5 low qubits
    // adjoint backward: two 11-qubit tiles (psi, lambda), 8-amplitude groups
    if (NS == 2) { t.M = 11; t.R = 3; t.c = 3; }
    else { t.M = 13; t.R = 3; t.c = 5; }
  } else {
    if (NS == 2) { t.M = 13; t.R = 4; t.c = 3; }
    else { t.M = 14; t.R = 5; t.c = 3; }
  }
  (void)n;
  return t;
}

extern "C" sv_status sv_default_tiling(int32_t n, sv_dtype dtype, int32_t backward,
                                      int32_t *tile_bits, int32_t *low_bits, int32_t *group_bits) {
  if (dtype != SV_C128 && dtype != SV_C64) return fail(SV_EINVAL, "dtype %d", (int)dtype);
  if (!tile_bits || !low_bits || !group_bits) return fail(SV_EINVAL, "null output");
  const Tiling t = default_tiling(n, dtype, backward ? 2 : 1);
  *tile_bits = t.M;
  *low_bits = t.c;
  *group_bits = t.R;
  return SV_OK;
}

extern "C" sv_status sv_alloc(int32_t n, sv_dtype dtype, void *re, void *im, void *ws,
                              size_t ws_bytes, void *stream, sv_state **out) {
  if (!out) return fail(SV_EINVAL, "null output handle");
  *out = nullptr;
  if (dtype != SV_C128 && dtype != SV_C64) return fail(SV_EDTYPE, "unsupported dtype %d", (int)dtype);
  if (n < 1 || n > SVI_NMAX) return fail(SV_EINVAL, "n_qubits %d outside 1..%d", n, SVI_NMAX);
  if (!re || !im) return fail(SV_EINVAL, "null state plane");
  if (((uintptr_t)re & 15) || ((uintptr_t)im & 15)) return fail(SV_EINVAL, "state planes must be 16-byte aligned");
  size_t need = sv_workspace_bytes(n, dtype, 0);
  if (!ws || ws_bytes < need)
    return fail(SV_ENOMEM, "workspace %zu bytes < required %zu", ws_bytes, need);
  if ((uintptr_t)ws & 255) return fail(SV_EINVAL, "workspace must be 256-byte aligned");
  DevInfo di;
  sv_status s = device_info(di);
  if (s) return s;
  sv_state *st = new sv_state;
  st->n = n;
  st->dtype = dtype;
  st->re = re;
  st->im = im;
  st->ws = ws;
  st->ws_bytes = ws_bytes;
  st->stream = (hipStream_t)stream;
  st->tiling = default_tiling(n, dtype, 1);
  st->adj_tiling = default_tiling(n, dtype, 2);
  (void)hipGetDevice(&st->dev);
  st->pending_zero = true;
  *out = st;
  return SV_OK;
}

extern "C" sv_status sv_free(sv_state *st) {
  if (!st) return SV_OK;
  if (st->stream || true) (void)hipStreamSynchronize(st->stream);
  delete st;
  return SV_OK;
}

extern "C" sv_status sv_set_stream(sv_state *st, void *stream) {
  if (!st) return fail(SV_EINVAL, "null handle");
  st->stream = (hipStream_t)stream;
  return SV_OK;
}

extern "C" sv_status sv_set_tiling(sv_state *st, int32_t tile_bits, int32_t low_bits,
                                   int32_t group_bits) {
  if (!st) return fail(SV_EINVAL, "null handle");
  Tiling t = default_tiling(st->n, st->dtype, 1);
  if (tile_bits) t.M = tile_bits;
  if (low_bits) t.c = low_bits;
  if (group_bits) {
    if (!svk_has_sweep(st->dtype == SV_C128, t.M, group_bits, 1))
      return fail(SV_EINVAL, "no kernel for tile_bits=%d group_bits=%d", t.M, group_bits);
    t.R = group_bits;
  }
  if (!svk_has_sweep(st->dtype == SV_C128, t.M, t.R, 1)) {
    // try the other register width
    int altR = t.R == 5 ? 4 : 5;
    if (svk_has_sweep(st->dtype == SV_C128, t.M, altR, 1)) t.R = altR;
    else return fail(SV_EINVAL, "no kernel for tile_bits=%d", t.M);
  }
  if (t.c < 1 || t.c > t.M - t.R + 1) return fail(SV_EINVAL, "low_bits %d out of range", t.c);
  st->tiling = t;
  st->plans.clear();
  return SV_OK;
}

extern "C" sv_status sv_set_adjoint_tiling(sv_state *st, int32_t tile_bits, int32_t low_bits,
                                          int32_t group_bits) {
  if (!st) return fail(SV_EINVAL, "null handle");
  Tiling t = st->adj_tiling;
  if (tile_bits) t.M = tile_bits;
  if (group_bits) t.R = group_bits;
  if (low_bits) t.c = low_bits;
  if (!svk_has_sweep(st->dtype == SV_C128, t.M, t.R, 2))
    return fail(SV_EINVAL, "no adjoint sweep kernel for tile_bits %d, group_bits %d", t.M, t.R);
  if (t.c < 1 || t.c > t.M) return fail(SV_EINVAL, "low_bits %d outside 1..%d", t.c, t.M);
  st->adj_tiling = t;
  return SV_OK;
}

extern "C" sv_status sv_timing_enable(sv_state *st, int32_t on) {
  if (!st) return fail(SV_EINVAL, "null handle");
  HIPCHK(hipStreamSynchronize(st->stream));
  st->timing = on != 0;
  st->ev_used = 0;
  st->ev_bytes.clear();
  return SV_OK;
}

extern "C" sv_status sv_timing_read(sv_state *st, double *sweep_ms, int64_t *launches,
                                    double *bytes) {
  if (!st) return fail(SV_EINVAL, "null handle");
  HIPCHK(hipStreamSynchronize(st->stream));
  double ms = 0.0, by = 0.0;
  for (size_t k = 0; k + 1 < st->ev_used; k += 2) {
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, st->ev_pool[k], st->ev_pool[k + 1]));
    ms += t;
    by += st->ev_bytes[k / 2];
  }
  if (sweep_ms) *sweep_ms = ms;
  if (launches) *launches = (int64_t)(st->ev_used / 2);
  if (bytes) *bytes = by;
  st->ev_used = 0;
  st->ev_bytes.clear();
  return SV_OK;
}

// Write a pending |0..0> (when the next operation cannot absorb it).
static sv_status materialize_zero(sv_state *st) {
  if (!st->pending_zero) return SV_OK;
  hipError_t e = svk_launch_init_zero(st->dtype == SV_C128, st->re, st->im, (int64_t)1 << st->n, st->stream);
  if (e != hipSuccess) return fail(SV_EDEVICE, "init kernel: %s", hipGetErrorString(e));
  st->pending_zero = false;
  return SV_OK;
}

extern "C" sv_status sv_reset(sv_state *st) {
  if (!st) return fail(SV_EINVAL, "null handle");
  // Deferred: the first sweep of the next sv_apply_layer synthesises |0..0>
  // in LDS instead of reading the planes; other readers write it first.
  st->pending_zero = true;
  return SV_OK;
}

// --------------------------------------------------------- plan building

static sv_status validate_circuit(int n, const sv_op *ops, int n_ops, const double *params,
                                  int n_params) {
  if (n_ops < 0) return fail(SV_EINVAL, "negative n_ops");
  if (n_ops > 0 && !ops) return fail(SV_EINVAL, "null ops");
  if (n_params < 0) return fail(SV_EINVAL, "negative n_params");
  if (n_params > 0 && !params) return fail(SV_EUNBOUND, "null params with n_params=%d", n_params);
  for (int i = 0; i < n_ops; i++) {
    sv_status s = validate_op(ops[i], i, n, n_params);
    if (s) return s;
  }
  for (int p = 0; p < n_params; p++)
    if (!std::isfinite(params[p])) return fail(SV_EUNBOUND, "parameter %d is not finite", p);
  return SV_OK;
}

static std::string plan_key(int mode, int n, const Tiling &tl, bool dbl, const sv_op *ops, int n_ops,
                            int n_params) {
  std::string k;
  k.reserve(64 + (size_t)n_ops * 24);
  char buf[96];
  snprintf(buf, sizeof buf, "%d|%d|%d,%d,%d|%d|%d|", mode, n, tl.M, tl.c, tl.R, (int)dbl, n_params);
  k += buf;
  for (int i = 0; i < n_ops; i++) {
    const sv_op &o = ops[i];
    int v[16] = {o.kind, o.n_targets, o.targets[0], o.targets[1], o.targets[2], o.targets[3],
                 o.targets[4], o.n_controls, o.controls[0], o.controls[1], o.controls[2],
                 o.controls[3], o.controls[4], (int)o.control_states, o.param_index[0],
                 o.param_index[1]};
    for (int j = o.n_targets; j < 5; j++) v[2 + j] = 0;
    for (int j = o.n_controls; j < 5; j++) v[8 + j] = 0;
    int np = nparams_of(o.kind);
    if (np < 1) v[14] = 0;
    if (np < 2) v[15] = 0;
    k.append((const char *)v, sizeof v);
    int p2 = np >= 3 ? o.param_index[2] : 0;
    k.append((const char *)&p2, sizeof p2);
  }
  return k;
}

static void collect_user_mats(Plan &P, const sv_op *ops, int n_ops) {
  P.mat_dim.clear();
  for (int i = 0; i < n_ops; i++)
    if (ops[i].kind == SV_UNITARY) {
      int d = 1 << ops[i].n_targets;
      P.mat_dim.push_back(2 * d * d);
    }
  P.n_user_mats = (int)P.mat_dim.size();
  P.nstatic = 0;
  for (int v : P.mat_dim) P.nstatic += v;
}

// Modeled time of a tile-sweep plan, in units of one register stage of
// 3-qubit groups over the whole state.  A sweep streams the state through HBM
// while its tiles run their stages; measured on MI355X (FP64, 13-qubit
// tiles), a sweep takes about max(11, 5.3 + s) such units for s stages: the
// HBM copy of the state costs as much as 11 stages, and stages beyond about 5
// are not hidden under it.  Wider register groups cost more per stage.
static double plan_model(const std::vector<SweepP> &sweeps, int R) {
  const double w = R <= 3 ? 1.0 : R == 4 ? 1.2 : 1.6;
  double t = 0.0;
  for (const SweepP &sw : sweeps) t += std::max(11.0, 5.3 + w * (double)sw.stages.size());
  return t;
}

// AUTO plan: the greedy tile planner with and without qubit remapping; for
// large states also with per-sweep caps on the gates a sweep takes (which
// spread the register stages over the sweeps more evenly), keeping the plan
// of least modeled time.  The candidate list depends only on the circuit and
// the state size, so the choice is deterministic.
static void plan_auto_best(const std::vector<GateRec> &recs, int n, const Tiling &tl,
                           std::vector<SweepP> &out, bool allow_remap) {
  plan_auto(recs, n, tl, out, 1e300, true, false);
  double best = plan_model(out, tl.R);
  auto consider = [&](double cap, bool remap) {
    std::vector<SweepP> alt;
    plan_auto(recs, n, tl, alt, cap, true, remap);
    if (remap && !layout_consistent(alt, n)) return;
    const double m = plan_model(alt, tl.R);
    if (m < best) {
      best = m;
      out.swap(alt);
    }
  };
  if (allow_remap) consider(1e300, true);
  // Searching costs about a millisecond of host time per candidate at 30
  // qubits and is done once per circuit structure (plans are cached); the
  // number of candidates grows with the modeled sweep time of the state.
  if (n < 24) return;
  static const double caps[] = {500, 300, 400, 600, 350, 450, 250, 550, 700, 200, 480, 520,
                                280, 320, 380, 420, 460, 540, 580, 620, 660, 240, 260, 220,
                                180, 150, 510, 490, 310, 290, 470, 430, 390, 410, 370, 330};
  const int ncap = (int)(sizeof caps / sizeof caps[0]);
  const int budget = std::min(ncap, 4 << std::min(n - 24, 3));   // 4 at 24 qubits, 32 from 27
  for (int k = 0; k < budget; k++) {
    if (allow_remap) consider(caps[k], true);
    else consider(caps[k], false);
  }
}

// split1q: write uncontrolled H, RX, Y, U2, U3 as Kronecker-stage parts.  The
// batch planner keeps them whole: a batch launches its Kronecker-only kernel
// only when every circuit qualifies, and a circuit must round the same alone
// and in any mix.
static sv_status build_forward_plan(int mode, int n, bool dbl, const Tiling &tl, const sv_op *ops,
                                    int n_ops, int n_params, Plan &P, bool remap = true,
                                    bool split1q = true) {
  P.n = n;
  P.dbl = dbl;
  P.M = tl.M;
  P.R = tl.R;
  P.NS = 1;
  P.n_user_params = n_params;
  collect_user_mats(P, ops, n_ops);
  std::vector<GateRec> recs;
  int um = 0;
  int half_pi = -1;  // parameter slot of the constant pi/2, once needed
  auto const_half_pi = [&]() {
    if (half_pi < 0) {
      P.constants.push_back(1.57079632679489661923);
      half_pi = n_params + (int)P.constants.size() - 1;
    }
    return half_pi;
  };
  // one-qubit record of `kind` on qubit q, parameter slot p
  auto push1 = [&](int kind, int q, int p) {
    sv_op o{};
    o.kind = kind;
    o.n_targets = 1;
    o.targets[0] = q;
    o.param_index[0] = p;
    recs.push_back(lower_one(o, -1));
  };
  for (int i = 0; i < n_ops; i++) {
    const sv_op &op = ops[i];
    if (split1q && mode == SV_FUSE_AUTO && op.n_controls == 0) {
      // Uncontrolled one-qubit gates written as diagonals, RY rotations and
      // permutations, all Kronecker-stage parts (listed in the order applied):
      //   H = RY(pi/2) Z,  RX(t) = S^dag RY(t) S,  Y = S X S^dag,
      //   U3(t, f, l) = P(f) RY(t) P(l),  U2(f, l) = U3(pi/2, f, l)
      const int q = op.targets[0];
      bool split = true;
      switch (op.kind) {
        case SV_H: push1(SV_Z, q, 0); push1(SV_RY, q, const_half_pi()); break;
        case SV_RX: push1(SV_S, q, 0); push1(SV_RY, q, op.param_index[0]); push1(SV_SDG, q, 0); break;
        case SV_Y: push1(SV_SDG, q, 0); push1(SV_X, q, 0); push1(SV_S, q, 0); break;
        case SV_U3:
          push1(SV_P, q, op.param_index[2]);
          push1(SV_RY, q, op.param_index[0]);
          push1(SV_P, q, op.param_index[1]);
          break;
        case SV_U2:
          push1(SV_P, q, op.param_index[1]);
          push1(SV_RY, q, const_half_pi());
          push1(SV_P, q, op.param_index[0]);
          break;
        default: split = false;
      }
      if (split) continue;
    }
    GateRec g = lower_one(ops[i], ops[i].kind == SV_UNITARY ? um : -1);
    if (ops[i].kind == SV_UNITARY) um++;
    if (g.mo == MO_NOP) continue;
    recs.push_back(g);
  }
  if (mode == 0) {
    for (GateRec &g : recs) {
      if (g.mo == MO_2L || g.mo == MO_DENSE) {
        SweepP sw;
        const int M = std::min(tl.M, n), c = std::min(tl.c, n);
        uint64_t T = (c >= 64 ? ~0ull : ((1ull << c) - 1)) | g.qmask;
        for (int q = c; q < n && popc(T) < M; q++) T |= 1ull << q;
        set_tile(sw, n, T, c);
        std::vector<GateRec> one{g};
        plan_stages(one, std::vector<int>{0}, sw, tl.R, n);
        int used = 0;
        emit_sweep(P, one, sw, n, tl.R, 0, 0, used);
      } else {
        emit_gate(P, g, n);
      }
    }
  } else {
    std::vector<SweepP> sweeps;
    if (mode < 0) plan_auto_best(recs, n, tl, sweeps, remap);
    else plan_fused(recs, n, tl, mode, sweeps, true);
    for (const SweepP &sw : sweeps) {
      int used = 0;
      emit_sweep(P, recs, sw, n, tl.R, 0, 0, used);
    }
  }
  return SV_OK;
}

// Backward program of the adjoint: gates in reverse, each daggered, with a
// gradient micro-op before every parameterised rotation.
static sv_status build_adjoint_plan(int n, bool dbl, const Tiling &tl, const sv_op *ops, int n_ops,
                                    int n_params, Plan &P) {
  P.n = n;
  P.dbl = dbl;
  P.M = tl.M;
  P.R = tl.R;
  P.NS = 2;
  P.n_user_params = n_params;
  collect_user_mats(P, ops, n_ops);
  std::vector<GateRec> recs;
  int um_total = P.n_user_mats;
  int um = um_total;
  for (int i = n_ops - 1; i >= 0; i--) {
    const sv_op &op = ops[i];
    if (op.kind == SV_UNITARY) um--;
    GateRec g = lower_one(op, op.kind == SV_UNITARY ? um : -1);
    if (g.mo == MO_NOP) continue;
    if (op.kind == SV_U2 || op.kind == SV_U3) {
      // U3(t,f,l) = P(f) RY(t) P(l) exactly (no global phase), so a control
      // on U3 is the same control on each factor; reversed and daggered:
      // P(f)^dag, RY(t)^dag, P(l)^dag
      int pt, pf, pl;
      if (op.kind == SV_U3) { pt = op.param_index[0]; pf = op.param_index[1]; pl = op.param_index[2]; }
      else {
        P.constants.push_back(1.57079632679489661923);
        pt = n_params + (int)P.constants.size() - 1;
        pf = op.param_index[0];
        pl = op.param_index[1];
      }
      const int kinds[3] = {SV_P, SV_RY, SV_P};
      const int pids[3] = {pf, pt, pl};
      for (int k = 0; k < 3; k++) {
        sv_op sub = op;
        sub.kind = kinds[k];
        sub.param_index[0] = pids[k];
        sub.param_index[1] = sub.param_index[2] = -1;
        GateRec s = lower_one(sub, -1);
        s.dagger = true;
        bool trainable = !(op.kind == SV_U2 && k == 1);
        if (trainable) {
          s.grad = true;
          s.gparam = pids[k];
          generator_of(s, s.gx, s.gz, s.galpha, s.gbeta);
          s.cost += 8;
        }
        recs.push_back(s);
      }
      continue;
    }
    if (op.kind == SV_GIVENS || op.kind == SV_DEXC) {
      // generator: the Pauli-Y of the rotated pair of patterns, zero elsewhere
      g.dagger = true;
      g.grad = true;
      g.grad2l = true;
      g.gparam = op.param_index[0];
      g.cost += 4;
      recs.push_back(g);
      continue;
    }
    g.dagger = true;
    if (nparams_of(op.kind) > 0) {
      if (!generator_of(g, g.gx, g.gz, g.galpha, g.gbeta))
        return fail(SV_EUNSUPPORTED, "op %d: adjoint gradient of kind %d is not supported", i, op.kind);
      g.grad = true;
      g.gparam = op.param_index[0];
      g.cost += 8;
    }
    recs.push_back(g);
  }
  // the greedy planner without qubit remapping: remapping and the capped
  // plan search give the two-state sweeps no fewer sweeps here, and were
  // measured slower (26-qubit HEA adjoint 52.5 against 50.4 ms)
  std::vector<SweepP> sweeps;
  plan_auto(recs, n, tl, sweeps, 1e300, true);
  // cap gradient slots per sweep by splitting sweeps whose stages exceed the limit
  int gbase = 0;
  for (const SweepP &sw0 : sweeps) {
    // split the stage list into chunks of <= SVI_GSLOTS_MAX gradient slots;
    // the chunks run over the same tiles in the sweep's input layout, and only
    // the last one applies the sweep's output permutation (qubit remapping)
    std::vector<SweepP> chunks;
    SweepP cur = sw0;
    cur.stages.clear();
    cur.operm = false;
    int cnt = 0;
    for (const StageP &st : sw0.stages) {
      int g = 0;
      for (int r : st.recs) g += recs[r].grad ? 1 : 0;
      if (g > SVI_GSLOTS_HARD)
        return fail(SV_EUNSUPPORTED, "adjoint: %d parameterised gates in one register stage (max %d)",
                    g, SVI_GSLOTS_HARD);
      if (cnt + g > SVI_GSLOTS_MAX && !cur.stages.empty()) {
        chunks.push_back(cur);
        cur.stages.clear();
        cnt = 0;
      }
      cur.stages.push_back(st);
      cnt += g;
    }
    chunks.push_back(cur);
    chunks.back().operm = sw0.operm;
    for (const SweepP &ch : chunks) {
      if (ch.stages.empty() && !ch.operm) continue;
      int used = 0;
      emit_sweep(P, recs, ch, n, tl.R, 0, gbase, used);
      gbase += used;
    }
  }
  P.n_gslots = gbase;
  // CSR: parameter -> slots in ascending slot order
  int np = n_params + (int)P.constants.size();
  std::vector<std::vector<int>> rows(np);
  for (int s = 0; s < P.n_gslots; s++) rows[P.slot_param[s]].push_back(s);
  P.grad_rowptr.assign(n_params + 1, 0);
  P.grad_slots.clear();
  for (int p = 0; p < n_params; p++) {
    for (int s : rows[p]) P.grad_slots.push_back(s);
    P.grad_rowptr[p + 1] = (int32_t)P.grad_slots.size();
  }
  return SV_OK;
}

static sv_status get_plan(sv_state *st, int mode, const Tiling &tl, const sv_op *ops, int n_ops,
                          int n_params, bool adjoint, Plan **out) {
  std::string key = (adjoint ? "A" : "F") + plan_key(mode, st->n, tl, st->dtype == SV_C128, ops, n_ops, n_params);
  auto it = st->plans.find(key);
  if (it != st->plans.end()) {
    *out = it->second.get();
    return SV_OK;
  }
  std::unique_ptr<Plan> P(new Plan);
  sv_status s = adjoint ? build_adjoint_plan(st->n, st->dtype == SV_C128, tl, ops, n_ops, n_params, *P)
                        : build_forward_plan(mode, st->n, st->dtype == SV_C128, tl, ops, n_ops, n_params, *P);
  if (s) return s;
  s = upload_plan(*P);
  if (s) return s;
  if (st->plans.size() > 64) st->plans.clear();
  *out = P.get();
  st->plans.emplace(key, std::move(P));
  return SV_OK;
}

static sv_status upload_call_data(sv_state *st, Plan &P, const sv_op *ops, int n_ops,
                                  const double *params, int n_params) {
  if (n_params > 0)
    HIPCHK(hipMemcpyAsync(P.d_params, params, (size_t)n_params * 8, hipMemcpyHostToDevice, st->stream));
  if (P.nstatic > 0) {
    std::vector<double> stat(P.nstatic);
    int off = 0;
    for (int i = 0; i < n_ops; i++)
      if (ops[i].kind == SV_UNITARY) {
        int d = 1 << ops[i].n_targets;
        std::memcpy(&stat[off], ops[i].matrix, sizeof(double) * 2 * d * d);
        off += 2 * d * d;
      }
    HIPCHK(hipMemcpyAsync(P.d_statics, stat.data(), (size_t)P.nstatic * 8, hipMemcpyHostToDevice, st->stream));
    // the host vector dies at return: make the copy complete first
    HIPCHK(hipStreamSynchronize(st->stream));
  }
  hipError_t e = svk_launch_coefs(P.d_coefdesc, (int)P.coefs.size(), P.d_params, P.d_statics,
                                  P.d_factors, P.d_coef, st->stream);
  if (e != hipSuccess) return fail(SV_EDEVICE, "coefficient kernel: %s", hipGetErrorString(e));
  return SV_OK;
}

static sv_status materialize_zero(sv_state *st);

// A tile sweep of a state evolved from |0..0> by earlier sweeps only, whose
// tiles so far cover the qubits in *support: it runs only the tiles whose
// qubits off the support are 0 (SW_SPARSE, bases from bz), since the others
// hold zeros before and after (a sweep's gates, and a remapping sweep's
// output permutation, act within its tile).  Adds the sweep's tile to the
// support.  The first sweep (SW_INIT_ZERO) runs every tile.
static void restrict_to_support(SweepArgs &a, int n, uint64_t *support) {
  const uint64_t all = n >= 64 ? ~0ull : (1ull << n) - 1;
  uint64_t tile = (1ull << a.c) - 1;
  for (int k = 0; k < a.nh; k++) tile |= 1ull << a.hb[k];
  const uint64_t zero = all & ~tile & ~*support;
  if (!(a.flags & SW_INIT_ZERO) && zero) {
    // bases take zeros at the tile's high bits and at the qubits off the
    // support (ascending; the low bits are below the tile index)
    a.flags |= SW_SPARSE;
    a.nbz = 0;
    for (int q = a.c; q < n; q++)
      if (((tile | zero) >> q) & 1) a.bz[a.nbz++] = q;
    a.ntiles = (int64_t)1 << (n - a.m - __builtin_popcountll(zero));
  }
  *support |= tile;
}

static sv_status run_steps(sv_state *st, Plan &P, void *re, void *im, void *re2, void *im2,
                           double *gpart, int grid_override) {
  DevInfo di;
  sv_status s = device_info(di);
  if (s) return s;
  // a pending |0..0> on the handle's own planes: the first tile sweep builds it
  bool fuse_zero = false;
  if (re == st->re && st->pending_zero) {
    if (!P.steps.empty() && P.steps[0].kind == 0 && P.NS == 1) fuse_zero = true;
    else {
      s = materialize_zero(st);
      if (s) return s;
    }
  }
  const bool dbl = st->dtype == SV_C128;
  int occ = svk_sweep_occupancy(dbl, P.M, P.R, P.NS);
  int occk = svk_sweep_kron_occupancy(dbl, P.M, P.R, P.NS);
  // From |0..0>, the qubits that may be 1 in a nonzero amplitude, tracked
  // while every step is a sweep of the lean kernel.
  bool track = fuse_zero && P.NS == 1;
  uint64_t support = 0;
  for (Step &stp : P.steps) {
    if (stp.kind == 0) {
      SweepArgs a = stp.sa;
      a.re = re; a.im = im; a.re2 = re2; a.im2 = im2;
      if (fuse_zero && &stp == &P.steps[0]) a.flags |= SW_INIT_ZERO;
      a.stages = P.d_stages;
      a.ops = P.d_ops;
      a.coef = P.d_coef;
      a.gpart = gpart;
      // the two-state lean kernel takes gradient terms over whole register
      // groups, so it needs tiles at least one group wide
      const bool lean = stp.all_kron && occk > 0 && (P.NS == 1 || stp.sa.m >= P.R);
      if (track && !lean) track = false;
      if (track) restrict_to_support(a, st->n, &support);
      int64_t g = (int64_t)di.cus * (lean ? occk : occ);
      if (grid_override > 0) g = grid_override;
      if (g > a.ntiles) g = a.ntiles;
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (st->timing && P.NS == 1) {
        e0 = next_event(st);
        e1 = next_event(st);
        if (e0) (void)hipEventRecord(e0, st->stream);
      }
      hipError_t e = lean ? svk_launch_sweep_kron(dbl, P.M, P.R, P.NS, a, (int)g, st->stream)
                          : svk_launch_sweep(dbl, P.M, P.R, P.NS, a, (int)g, st->stream);
      if (e != hipSuccess) return fail(SV_EDEVICE, "sweep kernel: %s", hipGetErrorString(e));
      if (a.flags & SW_INIT_ZERO) st->pending_zero = false;
      if (e0 && e1) {
        (void)hipEventRecord(e1, st->stream);
        // read + write of both planes over the tiles run; a sweep that
        // synthesises |0..0> only writes
        const double planes_rw = (a.flags & SW_INIT_ZERO) ? 2.0 : 4.0;
        st->ev_bytes.push_back(planes_rw * (double)(a.ntiles << a.m) * (double)elem_size(st->dtype));
      }
    } else {
      track = false;
      GateArgsHost a = stp.ga;
      a.re = re; a.im = im;
      a.coef = P.d_coef + (stp.gate_coef < 0 ? 0 : stp.gate_coef);
      hipError_t e = svk_launch_gate(dbl, a, st->stream);
      if (e != hipSuccess) return fail(SV_EDEVICE, "gate kernel: %s", hipGetErrorString(e));
    }
  }
  return SV_OK;
}

// Smallest compiled register-group width >= need (same tile size if possible).
static sv_status widen_groups(bool dbl, int need, Tiling &tl) {
  if (need <= tl.R) return SV_OK;
  for (int R = need; R <= SVI_RMAX; R++)
    if (svk_has_sweep(dbl, tl.M, R, 1)) { tl.R = R; return SV_OK; }
  for (int M : {13, 12, 14}) for (int R = need; R <= SVI_RMAX; R++)
    if (svk_has_sweep(dbl, M, R, 1)) { tl.M = M; tl.R = R; tl.c = std::min(tl.c, M - R); return SV_OK; }
  return fail(SV_EUNSUPPORTED, "no kernel with %d-qubit register groups", need);
}

extern "C" sv_status sv_apply_layer(sv_state *st, const sv_op *ops, int32_t n_ops,
                                    const double *params, int32_t n_params, int32_t fuse_width) {
  if (!st) return fail(SV_EINVAL, "null handle");
  if (!(fuse_width == 0 || fuse_width == SV_FUSE_AUTO || (fuse_width >= 2 && fuse_width <= 5)))
    return fail(SV_EINVAL, "fuse_width %d: must be 0, 2..5 or SV_FUSE_AUTO", fuse_width);
  sv_status s = validate_circuit(st->n, ops, n_ops, params, n_params);
  if (s) return s;
  if (n_ops == 0) return SV_OK;
  Tiling tl = st->tiling;
  // register groups must be as wide as the widest op (and a fused block)
  int need = fuse_width >= 2 ? fuse_width : 1;
  for (int i = 0; i < n_ops; i++)
    need = std::max(need, ops[i].n_targets + ops[i].n_controls);
  s = widen_groups(st->dtype == SV_C128, need, tl);
  if (s) return s;
  Plan *P = nullptr;
  s = get_plan(st, fuse_width, tl, ops, n_ops, n_params, false, &P);
  if (s) return s;
  s = upload_call_data(st, *P, ops, n_ops, params, n_params);
  if (s) return s;
  return run_steps(st, *P, st->re, st->im, nullptr, nullptr, nullptr, 0);
}

// ------------------------------------------------------- Pauli reductions

struct PauliPlan {
  // reordered: streamed diagonal terms, then tiled passes, then wide terms
  std::vector<PauliTermDev> terms;
  struct Pass { int m, c, nh; int hb[SVI_MMAX]; int t0, t1; };
  std::vector<Pass> passes;
  int n_diag = 0;                     // terms[0..n_diag) run in k_zexp
  int wide_begin = 0;                 // terms[wide_begin..] run untiled (k_pauli_wide)
};

// Diagonal (Z-only) terms of an expectation-only call on a large state take
// the streaming kernel; with lambda output every term takes the tile passes.
static bool diag_stream(int n, bool lambda) { return !lambda && n >= 14; }

// Tile bits of the state-vector Pauli passes: 12-bit tiles, two workgroups
// per CU, so one workgroup's loads and stores overlap the other's term work
// (13-bit tiles, one per CU, serialised them); the batch kernel's passes run
// in its 13-bit tiles.
#define SVI_PAULI_M 12

static void plan_pauli(int n, const sv_pauli_term *terms, int nt, PauliPlan &pp,
                       bool stream_diag = false, int tile_bits = 13) {
  const int M = std::min(tile_bits, n);
  const int c = std::min(3, n);
  const uint64_t low = (1ull << c) - 1;
  struct Open { uint64_t U; std::vector<int> ids; };
  std::vector<Open> open;
  std::vector<int> wide;
  if (stream_diag)
    for (int j = 0; j < nt; j++)
      if (terms[j].x_mask == 0) {
        PauliTermDev d{};
        d.x = 0;
        d.z = terms[j].z_mask;
        d.c = terms[j].coeff;
        d.term = j;
        pp.terms.push_back(d);
        pp.n_diag++;
      }
  for (int j = 0; j < nt; j++) {
    if (stream_diag && terms[j].x_mask == 0) continue;
    uint64_t xh = terms[j].x_mask & ~low;
    if (popc(xh) > M - c) { wide.push_back(j); continue; }   // cannot fit in any tile
    bool placed = false;
    for (Open &o : open) {
      if ((int)o.ids.size() >= SVI_PTERMS_MAX) continue;
      if (popc(o.U | xh) <= M - c) { o.U |= xh; o.ids.push_back(j); placed = true; break; }
    }
    if (!placed) open.push_back(Open{xh, {j}});
  }
  for (Open &o : open) {
    PauliPlan::Pass ps{};
    uint64_t T = low | o.U;
    for (int q = c; q < n && popc(T) < M; q++) T |= 1ull << q;
    ps.c = c;
    ps.nh = 0;
    for (int q = c; q < n; q++)
      if (T & (1ull << q)) ps.hb[ps.nh++] = q;
    ps.m = c + ps.nh;
    ps.t0 = (int)pp.terms.size();
    for (int j : o.ids) {
      PauliTermDev d{};
      d.x = terms[j].x_mask;
      d.z = terms[j].z_mask;
      d.c = terms[j].coeff;
      d.term = j;
      pp.terms.push_back(d);
    }
    ps.t1 = (int)pp.terms.size();
    pp.passes.push_back(ps);
  }
  pp.wide_begin = (int)pp.terms.size();
  for (int j : wide) {
    PauliTermDev d{};
    d.x = terms[j].x_mask;
    d.z = terms[j].z_mask;
    d.c = terms[j].coeff;
    d.term = j;
    pp.terms.push_back(d);
  }
}

// Partial-sum rows of every Pauli kernel have this stride (the largest grid).
static int64_t pauli_grid_part(const DevInfo &di, bool dbl) {
  return (int64_t)di.cus * std::max(svk_pauli_occupancy(dbl), svk_zexp_occupancy(dbl));
}

// Scratch bytes of run_pauli: terms | partials | reduced values | spare.
static size_t pauli_scratch_bytes(size_t nterm, int64_t grid_part) {
  size_t b = 256 + nterm * sizeof(PauliTermDev) + nterm * (size_t)grid_part * 8 + 2 * (nterm + 1) * 8 + 1024;
  return (b + 255) & ~(size_t)255;
}

// Runs the Pauli passes; term values land in device array `d_terms` (original order).
// Scratch: the handle's growable buffer, or (ext != NULL) the caller's
// ext_bytes at ext, checked before any device work.
static sv_status run_pauli(sv_state *st, const sv_pauli_term *terms, int nt, void *re, void *im,
                           void *lre, void *lim, double **d_terms_out, void *ext = nullptr,
                           size_t ext_bytes = 0) {
  PauliPlan pp;
  plan_pauli(st->n, terms, nt, pp, diag_stream(st->n, lre != nullptr), SVI_PAULI_M);
  DevInfo di;
  sv_status s = device_info(di);
  if (s) return s;
  const bool dbl = st->dtype == SV_C128;
  int occ = svk_pauli_occupancy(dbl);
  int64_t grid_max = (int64_t)di.cus * occ;
  const int64_t grid_z = (int64_t)di.cus * svk_zexp_occupancy(dbl);
  const int64_t grid_part = pauli_grid_part(di, dbl);
  // scratch: terms | partials | reduced (by pass order) | reduced (original order)
  size_t nterm = pp.terms.size();
  size_t need = pauli_scratch_bytes(nterm, grid_part);
  if (ext && need > ext_bytes)
    return fail(SV_ENOMEM, "%zu terms need %zu bytes of scratch; the fixed scratch holds %zu",
                nterm, need, ext_bytes);
  if (re == st->re) {
    sv_status z = materialize_zero(st);
    if (z) return z;
  }
  if (!ext) {
    s = ensure_scratch(st, need);
    if (s) return s;
  }
  char *b = ext ? (char *)ext : (char *)st->scratch;
  PauliTermDev *d_terms = (PauliTermDev *)b;
  double *d_part = (double *)(b + ((nterm * sizeof(PauliTermDev) + 255) & ~(size_t)255));
  double *d_red = d_part + nterm * grid_part;
  double *d_vals = d_red + nterm + 1;
  if (nterm)
    HIPCHK(hipMemcpyAsync(d_terms, pp.terms.data(), nterm * sizeof(PauliTermDev), hipMemcpyHostToDevice, st->stream));
  if (lre && nterm == 0) {
    size_t bytes = ((size_t)1 << st->n) * elem_size(st->dtype);
    HIPCHK(hipMemsetAsync(lre, 0, bytes, st->stream));
    HIPCHK(hipMemsetAsync(lim, 0, bytes, st->stream));
  }
  // streamed diagonal terms, SVI_ZTERMS_HOST per read of the state
  for (int g0 = 0; g0 < pp.n_diag; g0 += SVI_ZTERMS_HOST) {
    const int cnt = std::min(SVI_ZTERMS_HOST, pp.n_diag - g0);
    double *part = d_part + (size_t)g0 * grid_part;
    hipError_t e = svk_launch_zexp(dbl, re, im, st->n, d_terms + g0, cnt, part, (int)grid_z, st->stream);
    if (e != hipSuccess) return fail(SV_EDEVICE, "diagonal Pauli kernel: %s", hipGetErrorString(e));
    e = svk_launch_reduce_rows(part, cnt, (int)grid_z, d_red + g0, st->stream);
    if (e != hipSuccess) return fail(SV_EDEVICE, "reduce kernel: %s", hipGetErrorString(e));
  }
  for (size_t p = 0; p < pp.passes.size(); p++) {
    const PauliPlan::Pass &ps = pp.passes[p];
    PauliPassArgs a{};
    a.re = re; a.im = im; a.lre = lre; a.lim = lim;
    a.terms = d_terms;
    a.n = st->n; a.m = ps.m; a.c = ps.c; a.nh = ps.nh;
    for (int k = 0; k < SVI_MMAX; k++) a.hb[k] = k < ps.nh ? ps.hb[k] : 0;
    a.t_begin = ps.t0; a.t_end = ps.t1;
    a.accumulate = p > 0;
    a.ntiles = (int64_t)1 << (st->n - ps.m);
    if (ps.m > SVI_PAULI_M || ps.m > st->n) return fail(SV_EINVAL, "internal: Pauli tile of %d bits", ps.m);
    int64_t g = std::min<int64_t>(grid_max, a.ntiles);
    a.part = d_part + (size_t)ps.t0 * grid_part;
    hipError_t e = svk_launch_pauli(dbl, SVI_PAULI_M, a, (int)g, st->stream);
    if (e != hipSuccess) return fail(SV_EDEVICE, "pauli kernel: %s", hipGetErrorString(e));
    e = svk_launch_reduce_rows(a.part, ps.t1 - ps.t0, (int)g, d_red + ps.t0, st->stream);
    if (e != hipSuccess) return fail(SV_EDEVICE, "reduce kernel: %s", hipGetErrorString(e));
  }
  // wide terms: one untiled pass each, after the tiled passes
  {
    const int64_t N = (int64_t)1 << st->n;
    const int gw = (int)std::min<int64_t>(grid_max, (N + 255) / 256);
    for (size_t k = (size_t)pp.wide_begin; k < nterm; k++) {
      const PauliTermDev &d = pp.terms[k];
      double *part = d_part + k * (size_t)grid_part;
      const bool acc = !pp.passes.empty() || k > (size_t)pp.wide_begin;
      hipError_t e = svk_launch_pauli_wide(dbl, re, im, lre, lim, d.x, d.z, d.c, N, acc ? 1 : 0,
                                           part, gw, st->stream);
      if (e != hipSuccess) return fail(SV_EDEVICE, "pauli wide kernel: %s", hipGetErrorString(e));
      e = svk_launch_reduce_rows(part, 1, gw, d_red + k, st->stream);
      if (e != hipSuccess) return fail(SV_EDEVICE, "reduce kernel: %s", hipGetErrorString(e));
    }
  }
  // d_red is in pass order; return it with the permutation on the host side
  *d_terms_out = d_red;
  (void)d_vals;
  return SV_OK;
}

static void pauli_order(int n, const sv_pauli_term *terms, int nt, std::vector<int> &order,
                        bool lambda) {
  PauliPlan pp;
  plan_pauli(n, terms, nt, pp, diag_stream(n, lambda), SVI_PAULI_M);
  order.clear();
  for (auto &t : pp.terms) order.push_back(t.term);
}

static sv_status validate_terms(int n, const sv_pauli_term *terms, int nt) {
  if (nt < 0) return fail(SV_EINVAL, "negative n_terms");
  if (nt > 0 && !terms) return fail(SV_EINVAL, "null terms");
  for (int j = 0; j < nt; j++) {
    if (n < 64 && ((terms[j].x_mask | terms[j].z_mask) >> n))
      return fail(SV_EINVAL, "term %d: mask beyond %d qubits", j, n);
    if (!std::isfinite(terms[j].coeff)) return fail(SV_EINVAL, "term %d: non-finite coefficient", j);
  }
  return SV_OK;
}

static sv_status expect_pauli(sv_state *st, const sv_pauli_term *terms, int32_t n_terms,
                              double *out_terms, double *out_sum, void *ext, size_t ext_bytes) {
  if (!st) return fail(SV_EINVAL, "null handle");
  sv_status s = validate_terms(st->n, terms, n_terms);
  if (s) return s;
  if (n_terms == 0) {
    if (out_sum) *out_sum = 0.0;
    return SV_OK;
  }
  double *d_red = nullptr;
  s = run_pauli(st, terms, n_terms, st->re, st->im, nullptr, nullptr, &d_red, ext, ext_bytes);
  if (s) return s;
  std::vector<double> red(n_terms);
  HIPCHK(hipMemcpyAsync(red.data(), d_red, n_terms * 8, hipMemcpyDeviceToHost, st->stream));
  HIPCHK(hipStreamSynchronize(st->stream));
  std::vector<int> order;
  pauli_order(st->n, terms, n_terms, order, false);
  std::vector<double> vals(n_terms);
  for (int k = 0; k < n_terms; k++) vals[order[k]] = red[k];
  if (out_terms)
    for (int j = 0; j < n_terms; j++) out_terms[j] = vals[j];
  if (out_sum) {
    double e = 0.0;
    for (int j = 0; j < n_terms; j++) e += terms[j].coeff * vals[j];
    *out_sum = e;
  }
  return SV_OK;
}

extern "C" sv_status sv_expect_pauli(sv_state *st, const sv_pauli_term *terms, int32_t n_terms,
                                     double *out_terms, double *out_sum) {
  return expect_pauli(st, terms, n_terms, out_terms, out_sum, nullptr, 0);
}

// ------------------------------------------------- allocation-free <P>
// The Pauli kernels' partial sums, term descriptors and reduced values live in
// a file-scope device array of fixed size, one copy per GPU (each GPU holds
// it until the process ends).  Its host-side name stands in for a device
// address only inside device code: host code takes the address from
// hipGetSymbolAddress once per device, with that device current, and passes
// that pointer to the kernels.  Every call on one GPU shares the array (calls
// that overlap on one GPU race); every byte a call reads is written by the
// same call's kernels first, so nothing needs clearing.
static __device__ __align__(256) char scratch[SV_NOALLOC_SCRATCH_BYTES];

static std::mutex g_noalloc_mu;
static std::unordered_map<int, void *> g_noalloc;   // device -> address of `scratch`

static sv_status noalloc_scratch(void **out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  auto it = g_noalloc.find(dev);
  if (it == g_noalloc.end()) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(SV_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                  hipGetErrorString(e));
    it = g_noalloc.emplace(dev, p).first;
  }
  *out = it->second;
  return SV_OK;
}

extern "C" sv_status sv_expect_pauli_noalloc(sv_state *st, const sv_pauli_term *terms,
                                             int32_t n_terms, double *out_terms, double *out_sum) {
  if (!st) return fail(SV_EINVAL, "null handle");
  void *p = nullptr;
  sv_status s = noalloc_scratch(&p);
  if (s) return s;
  return expect_pauli(st, terms, n_terms, out_terms, out_sum, p, SV_NOALLOC_SCRATCH_BYTES);
}

// -------------------------------------------------------- density matrices
// rho of n qubits is held as a vector of 2n qubits, rho_{rc} at r 2^n + c (row
// bits are qubits n..2n-1).  U rho U^dagger = (U (x) conj U) vec rho: U on the
// row qubits, conj(U) on the column qubits; a channel sum_k K rho K^dagger is
// the 4x4 matrix sum_k K (x) conj K on (column qubit, row qubit).

static sv_status dm_check(const sv_state *st, int n) {
  if (!st) return fail(SV_EINVAL, "null handle");
  if (n < 1 || 2 * n != st->n)
    return fail(SV_EINVAL, "a density matrix of %d qubits needs a handle of %d qubits (got %d)", n,
                2 * n, st->n);
  return SV_OK;
}

extern "C" sv_status sv_dm_apply(sv_state *st, int32_t n, const sv_op *ops, int32_t n_ops,
                                 const double *params, int32_t n_params) {
  sv_status s = dm_check(st, n);
  if (s) return s;
  s = validate_circuit(n, ops, n_ops, params, n_params);
  if (s) return s;
  if (n_ops == 0) return SV_OK;
  // parameters, then their negations (angles of the conjugated gates)
  std::vector<double> p2(2 * (size_t)n_params);
  for (int i = 0; i < n_params; i++) {
    p2[i] = params[i];
    p2[n_params + i] = -params[i];
  }
  std::vector<std::vector<double>> mats;  // conjugated matrices, alive until the call returns
  mats.reserve(n_ops);
  std::vector<sv_op> out;
  out.reserve(2 * (size_t)n_ops);
  for (int i = 0; i < n_ops; i++) {
    const sv_op &op = ops[i];
    sv_op row = op;
    for (int k = 0; k < op.n_targets; k++) row.targets[k] += n;
    for (int k = 0; k < op.n_controls; k++) row.controls[k] += n;
    out.push_back(row);
    sv_op col = op;
    switch (op.kind) {
      case SV_S: col.kind = SV_SDG; break;
      case SV_SDG: col.kind = SV_S; break;
      case SV_T: col.kind = SV_TDG; break;
      case SV_TDG: col.kind = SV_T; break;
      case SV_RX: case SV_RZ: case SV_P: case SV_RXX: case SV_RYY: case SV_RZZ:
        col.param_index[0] += n_params;   // conj exp(-i t P / 2) = exp(+i t P / 2) for real P
        break;
      case SV_U2:
        col.param_index[0] += n_params;
        col.param_index[1] += n_params;
        break;
      case SV_U3:                          // conj U3(t, f, l) = U3(t, -f, -l)
        col.param_index[1] += n_params;
        col.param_index[2] += n_params;
        break;
      case SV_Y: case SV_SX: case SV_UNITARY: {
        const int d = 1 << op.n_targets;
        std::vector<double> m(2 * (size_t)d * d);
        if (op.kind == SV_Y) m = {0, 0, 0, 1, 0, -1, 0, 0};                 // [[0, i], [-i, 0]]
        else if (op.kind == SV_SX) m = {0.5, -0.5, 0.5, 0.5, 0.5, 0.5, 0.5, -0.5};
        else
          for (int e = 0; e < d * d; e++) {
            m[2 * e] = op.matrix[2 * e];
            m[2 * e + 1] = -op.matrix[2 * e + 1];
          }
        mats.push_back(std::move(m));
        col.kind = SV_UNITARY;
        col.matrix = mats.back().data();
        break;
      }
      default: break;                      // real matrices: X, Z, H, RY, SWAP, GIVENS, DEXC, I
    }
    out.push_back(col);
  }
  return sv_apply_layer(st, out.data(), (int32_t)out.size(), p2.empty() ? nullptr : p2.data(),
                        2 * n_params, SV_FUSE_AUTO);
}

extern "C" sv_status sv_dm_apply_kraus(sv_state *st, int32_t n, const int32_t *qubits,
                                       int32_t n_qubits, const double *kraus, int32_t n_kraus) {
  sv_status s = dm_check(st, n);
  if (s) return s;
  if (n_qubits < 0 || (n_qubits > 0 && !qubits)) return fail(SV_EINVAL, "bad qubit list");
  uint64_t seen = 0;
  for (int i = 0; i < n_qubits; i++) {
    if (qubits[i] < 0 || qubits[i] >= n) return fail(SV_EINVAL, "qubit %d out of range [0,%d)", qubits[i], n);
    if (seen >> qubits[i] & 1) return fail(SV_EINVAL, "qubit %d repeated", qubits[i]);
    seen |= 1ull << qubits[i];
  }
  if (n_kraus < 1 || !kraus) return fail(SV_EINVAL, "no Kraus operators");
  for (int i = 0; i < 8 * n_kraus; i++)
    if (!std::isfinite(kraus[i])) return fail(SV_EINVAL, "non-finite Kraus entry");
  // local index l = c + 2 r (first target: the column qubit)
  double m[32] = {0};
  for (int k = 0; k < n_kraus; k++) {
    const double *K = kraus + 8 * k;
    for (int r1 = 0; r1 < 2; r1++)
      for (int c1 = 0; c1 < 2; c1++)
        for (int r0 = 0; r0 < 2; r0++)
          for (int c0 = 0; c0 < 2; c0++) {
            // K[r1][r0] * conj(K[c1][c0])
            const double ar = K[2 * (2 * r1 + r0)], ai = K[2 * (2 * r1 + r0) + 1];
            const double br = K[2 * (2 * c1 + c0)], bi = -K[2 * (2 * c1 + c0) + 1];
            const int row = c1 + 2 * r1, colx = c0 + 2 * r0;
            m[2 * (4 * row + colx)] += ar * br - ai * bi;
            m[2 * (4 * row + colx) + 1] += ar * bi + ai * br;
          }
  }
  // one streaming pass per qubit (channels on different qubits commute)
  if (n_qubits == 0) return SV_OK;
  s = materialize_zero(st);
  if (s) return s;
  // On vectors of 12 or more qubits the channels go through LDS-tile passes
  // of up to five channels (13-bit tiles, vectors of 13 or more qubits) or
  // four (12-bit tiles), as few passes as that allows; the sorted qubits are
  // dealt round-robin over the passes, so every pass holds some of the lowest
  // qubits and its loads run over long consecutive stretches (a pass of two
  // or three channels measured faster than the two- and one-channel
  // streaming passes).  A pass left with one channel, and every channel of a
  // smaller vector, takes the streaming passes: two per pass, then one.
  std::vector<int> rest;
  if (st->n >= 12 && n_qubits >= 2) {
    const int kmax = st->n >= 13 ? 5 : 4;
    const int npass = (n_qubits + kmax - 1) / kmax;
    std::vector<int> sq(qubits, qubits + n_qubits);
    std::sort(sq.begin(), sq.end());
    for (int p = 0; p < npass; p++) {
      int grp[5], k = 0;
      for (int i = p; i < n_qubits; i += npass) grp[k++] = sq[i];
      if (k == 1) {
        rest.push_back(grp[0]);
        continue;
      }
      hipError_t e = svk_launch_dm_channel_tile(st->dtype == SV_C128, st->re, st->im, st->n, n,
                                                grp, k, m, st->stream);
      if (e != hipSuccess) return fail(SV_EDEVICE, "channel kernel: %s", hipGetErrorString(e));
    }
  } else {
    rest.assign(qubits, qubits + n_qubits);
  }
  for (size_t i = 0; i < rest.size(); i += 2) {
    hipError_t e = i + 1 < rest.size()
        ? svk_launch_dm_channel2(st->dtype == SV_C128, st->re, st->im, st->n, rest[i],
                                 rest[i + 1], n, m, m, st->stream)
        : svk_launch_dm_channel(st->dtype == SV_C128, st->re, st->im, st->n, rest[i],
                                rest[i] + n, m, st->stream);
    if (e != hipSuccess) return fail(SV_EDEVICE, "channel kernel: %s", hipGetErrorString(e));
  }
  HIPCHK(hipStreamSynchronize(st->stream));
  return SV_OK;
}

extern "C" sv_status sv_dm_apply_kraus2(sv_state *st, int32_t n, int32_t q0, int32_t q1,
                                        const double *kraus, int32_t n_kraus) {
  sv_status s = dm_check(st, n);
  if (s) return s;
  if (q0 < 0 || q0 >= n || q1 < 0 || q1 >= n || q0 == q1)
    return fail(SV_EINVAL, "qubits %d, %d: distinct and in [0,%d)", q0, q1, n);
  if (n_kraus < 1 || !kraus) return fail(SV_EINVAL, "no Kraus operators");
  for (int i = 0; i < 32 * n_kraus; i++)
    if (!std::isfinite(kraus[i])) return fail(SV_EINVAL, "non-finite Kraus entry");
  // S[(ur', uc'), (ur, uc)] = sum_k K[ur'][ur] conj(K[uc'][uc]); entry e = uc + 4 ur
  std::vector<double> S(2 * 256, 0.0);
  for (int k = 0; k < n_kraus; k++) {
    const double *K = kraus + 32 * k;
    for (int r1 = 0; r1 < 4; r1++)
      for (int c1 = 0; c1 < 4; c1++)
        for (int r0 = 0; r0 < 4; r0++)
          for (int c0 = 0; c0 < 4; c0++) {
            const double ar = K[2 * (4 * r1 + r0)], ai = K[2 * (4 * r1 + r0) + 1];
            const double br = K[2 * (4 * c1 + c0)], bi = -K[2 * (4 * c1 + c0) + 1];
            const int o = c1 + 4 * r1, l = c0 + 4 * r0;
            S[2 * (16 * o + l)] += ar * br - ai * bi;
            S[2 * (16 * o + l) + 1] += ar * bi + ai * br;
          }
  }
  s = materialize_zero(st);
  if (s) return s;
  s = ensure_scratch(st, S.size() * 8 + 256);
  if (s) return s;
  double *d_S = (double *)st->scratch;
  HIPCHK(hipMemcpyAsync(d_S, S.data(), S.size() * 8, hipMemcpyHostToDevice, st->stream));
  hipError_t e = svk_launch_dm_channel16(st->dtype == SV_C128, st->re, st->im, st->n, q0, q1, n, d_S,
                                         st->stream);
  if (e != hipSuccess) return fail(SV_EDEVICE, "channel kernel: %s", hipGetErrorString(e));
  HIPCHK(hipStreamSynchronize(st->stream));
  return SV_OK;
}

extern "C" sv_status sv_dm_expect_pauli(sv_state *st, int32_t n, const sv_pauli_term *terms,
                                        int32_t n_terms, double *out_terms, double *out_sum) {
  sv_status s = dm_check(st, n);
  if (s) return s;
  s = validate_terms(n, terms, n_terms);
  if (s) return s;
  if (n_terms == 0) {
    if (out_sum) *out_sum = 0.0;
    return SV_OK;
  }
  s = materialize_zero(st);
  if (s) return s;
  const int nb = (int)std::min<int64_t>(std::max<int64_t>(1, ((int64_t)1 << n) / 256), 1024);
  const size_t tb = ((size_t)n_terms * sizeof(PauliTermDev) + 255) & ~(size_t)255;
  const size_t pb = ((size_t)n_terms * nb * 8 + 255) & ~(size_t)255;
  s = ensure_scratch(st, tb + pb + (size_t)n_terms * 8 + 256);
  if (s) return s;
  PauliTermDev *d_terms = (PauliTermDev *)st->scratch;
  double *d_part = (double *)((char *)st->scratch + tb);
  double *d_out = (double *)((char *)st->scratch + tb + pb);
  std::vector<PauliTermDev> td(n_terms);
  for (int j = 0; j < n_terms; j++) {
    td[j] = PauliTermDev{};
    td[j].x = terms[j].x_mask;
    td[j].z = terms[j].z_mask;
    td[j].c = terms[j].coeff;
    td[j].term = j;
  }
  HIPCHK(hipMemcpyAsync(d_terms, td.data(), td.size() * sizeof(PauliTermDev), hipMemcpyHostToDevice,
                        st->stream));
  hipError_t e = svk_launch_dm_pauli(st->dtype == SV_C128, st->re, st->im, n, d_terms, n_terms, nb,
                                     d_part, st->stream);
  if (e == hipSuccess) e = svk_launch_reduce_rows(d_part, n_terms, nb, d_out, st->stream);
  if (e != hipSuccess) return fail(SV_EDEVICE, "density-matrix trace: %s", hipGetErrorString(e));
  std::vector<double> vals(n_terms);
  HIPCHK(hipMemcpyAsync(vals.data(), d_out, (size_t)n_terms * 8, hipMemcpyDeviceToHost, st->stream));
  HIPCHK(hipStreamSynchronize(st->stream));
  if (out_terms)
    for (int j = 0; j < n_terms; j++) out_terms[j] = vals[j];
  if (out_sum) {
    double acc = 0.0;
    for (int j = 0; j < n_terms; j++) acc += terms[j].coeff * vals[j];
    *out_sum = acc;
  }
  return SV_OK;
}

// ----------------------------------------------------------------- adjoint

static sv_status adjoint_enqueue(sv_state *st, const sv_op *ops, int n_ops, const double *params,
                                 int n_params, const sv_pauli_term *terms, int n_terms,
                                 double **d_terms, double **d_grad, Plan **bwd_out) {
  if (!st) return fail(SV_EINVAL, "null handle");
  sv_status s = validate_circuit(st->n, ops, n_ops, params, n_params);
  if (s) return s;
  s = validate_terms(st->n, terms, n_terms);
  if (s) return s;
  if (st->ws_bytes < sv_workspace_bytes(st->n, st->dtype, SV_WS_ADJOINT))
    return fail(SV_ENOMEM, "workspace too small for the adjoint (%zu < %zu)", st->ws_bytes,
                sv_workspace_bytes(st->n, st->dtype, SV_WS_ADJOINT));
  Tiling tf = st->tiling;
  Tiling tb = st->adj_tiling;
  int width = 1;
  for (int i = 0; i < n_ops; i++) width = std::max(width, ops[i].n_targets + ops[i].n_controls);
  s = widen_groups(st->dtype == SV_C128, width, tf);
  if (s) return s;
  if (width > tb.R) {
    // wider ops need wider backward register groups (same tile if compiled)
    bool found = false;
    for (int R = width; R <= SVI_RMAX && !found; R++)
      for (int M : {tb.M, 12, 11, 13})
        if (svk_has_sweep(st->dtype == SV_C128, M, R, 2)) {
          tb.M = M;
          tb.R = R;
          tb.c = std::min(tb.c, M - R);
          found = true;
          break;
        }
    if (!found)
      return fail(SV_EUNSUPPORTED,
                  "adjoint: an op on %d qubits (targets and controls); the backward sweeps take "
                  "ops on at most 4", width);
  }
  Plan *F = nullptr, *B = nullptr;
  if (n_ops > 0) {
    s = get_plan(st, SV_FUSE_AUTO, tf, ops, n_ops, n_params, false, &F);
    if (s) return s;
  }
  s = get_plan(st, SV_FUSE_AUTO, tb, ops, n_ops, n_params, true, &B);
  if (s) return s;
  double *S, *Pp;
  void *lre, *lim, *wre, *wim;
  ws_layout(st, &S, &Pp, &lre, &lim, &wre, &wim);
  // forward on the caller's planes
  if (F) {
    s = upload_call_data(st, *F, ops, n_ops, params, n_params);
    if (s) return s;
    s = run_steps(st, *F, st->re, st->im, nullptr, nullptr, nullptr, 0);
    if (s) return s;
  }
  // lambda = H psi and <P_j> on the final state
  double *d_red = nullptr;
  s = run_pauli(st, terms, n_terms, st->re, st->im, lre, lim, &d_red);
  if (s) return s;
  // working copy of psi for the backward sweep
  size_t plane = ((size_t)1 << st->n) * elem_size(st->dtype);
  HIPCHK(hipMemcpyAsync(wre, st->re, plane, hipMemcpyDeviceToDevice, st->stream));
  HIPCHK(hipMemcpyAsync(wim, st->im, plane, hipMemcpyDeviceToDevice, st->stream));
  // backward sweeps
  DevInfo di;
  s = device_info(di);
  if (s) return s;
  int occ = std::max(svk_sweep_occupancy(st->dtype == SV_C128, B->M, B->R, 2),
                     svk_sweep_kron_occupancy(st->dtype == SV_C128, B->M, B->R, 2));
  int64_t grid = (int64_t)di.cus * occ;
  int64_t maxtiles = (int64_t)1 << (st->n - std::min(B->M, st->n));
  if (grid > maxtiles) grid = maxtiles;
  // scratch after the Pauli area: partials [slots][grid] | slot sums | grad
  const size_t pauli_bytes = pauli_scratch_bytes((size_t)n_terms, pauli_grid_part(di, st->dtype == SV_C128));
  size_t need = pauli_bytes + (size_t)B->n_gslots * grid * 8 + (size_t)B->n_gslots * 8 +
                ((size_t)n_params + 1) * 8 + 1024;
  if (need > st->scratch_bytes) {
    // growing would free the Pauli results: re-run them after growing
    s = ensure_scratch(st, need);
    if (s) return s;
    s = run_pauli(st, terms, n_terms, st->re, st->im, lre, lim, &d_red);
    if (s) return s;
  }
  char *b = (char *)st->scratch + pauli_bytes;
  double *gpart = (double *)b;
  double *slot_sum = gpart + (size_t)B->n_gslots * grid;
  double *grad = slot_sum + B->n_gslots;
  s = upload_call_data(st, *B, ops, n_ops, params, n_params);
  if (s) return s;
  s = run_steps(st, *B, wre, wim, lre, lim, gpart, (int)grid);
  if (s) return s;
  hipError_t e = svk_launch_reduce_rows(gpart, B->n_gslots, (int)grid, slot_sum, st->stream);
  if (e != hipSuccess) return fail(SV_EDEVICE, "reduce: %s", hipGetErrorString(e));
  e = svk_launch_gather_grad(slot_sum, B->d_rowptr, B->d_gslots, n_params, grad, st->stream);
  if (e != hipSuccess) return fail(SV_EDEVICE, "gather: %s", hipGetErrorString(e));
  *d_terms = d_red;
  *d_grad = grad;
  *bwd_out = B;
  return SV_OK;
}

extern "C" sv_status sv_adjoint_grad(sv_state *st, const sv_op *ops, int32_t n_ops,
                                     const double *params, int32_t n_params,
                                     const sv_pauli_term *terms, int32_t n_terms, double *energy,
                                     double *grad, int32_t *n_evals) {
  double *d_terms = nullptr, *d_grad = nullptr;
  Plan *B = nullptr;
  sv_status s = adjoint_enqueue(st, ops, n_ops, params, n_params, terms, n_terms, &d_terms, &d_grad, &B);
  if (s) return s;
  std::vector<double> red(std::max(n_terms, 1));
  if (n_terms)
    HIPCHK(hipMemcpyAsync(red.data(), d_terms, n_terms * 8, hipMemcpyDeviceToHost, st->stream));
  if (grad && n_params)
    HIPCHK(hipMemcpyAsync(grad, d_grad, n_params * 8, hipMemcpyDeviceToHost, st->stream));
  HIPCHK(hipStreamSynchronize(st->stream));
  std::vector<int> order;
  pauli_order(st->n, terms, n_terms, order, true);
  std::vector<double> vals(std::max(n_terms, 1));
  for (int k = 0; k < n_terms; k++) vals[order[k]] = red[k];
  double e = 0.0;
  for (int j = 0; j < n_terms; j++) e += terms[j].coeff * vals[j];
  if (energy) *energy = e;
  if (n_evals) *n_evals = 1;
  return SV_OK;
}

extern "C" sv_status sv_adjoint_grad_device(sv_state *st, const sv_op *ops, int32_t n_ops,
                                            const double *params, int32_t n_params,
                                            const sv_pauli_term *terms, int32_t n_terms,
                                            double *d_out) {
  if (!d_out) return fail(SV_EINVAL, "null output");
  double *d_terms = nullptr, *d_grad = nullptr;
  Plan *B = nullptr;
  sv_status s = adjoint_enqueue(st, ops, n_ops, params, n_params, terms, n_terms, &d_terms, &d_grad, &B);
  if (s) return s;
  // energy from the device term list (pass order): no host data, no synchronisation
  hipError_t e = svk_launch_energy_terms(d_terms, (const PauliTermDev *)st->scratch, n_terms, d_out,
                                         st->stream);
  if (e != hipSuccess) return fail(SV_EDEVICE, "energy: %s", hipGetErrorString(e));
  if (n_params)
    HIPCHK(hipMemcpyAsync(d_out + 1, d_grad, n_params * 8, hipMemcpyDeviceToDevice, st->stream));
  return SV_OK;
}

// ---------------------------------------------------------------- sampling

// Scratch of one sampling call: block totals and offsets of the blocked
// prefix, the samples, then `extra_bytes` for the caller.
struct SampleScratch {
  double *QE = nullptr;
  uint64_t *samples = nullptr;
  void *extra = nullptr;
};

static sv_status sample_scratch(sv_state *st, int64_t shots, size_t extra_bytes, SampleScratch &sc) {
  const int64_t K = sample_K(st->n), J = K / (K < 1024 ? K : 1024);
  const size_t qe_bytes = (((size_t)(2 * J + 1) * 8) + 255) & ~(size_t)255;
  const size_t smp_bytes = ((size_t)shots * 8 + 255) & ~(size_t)255;
  sv_status s = ensure_scratch(st, qe_bytes + smp_bytes + extra_bytes + 1024);
  if (s) return s;
  sc.QE = (double *)st->scratch;
  sc.samples = (uint64_t *)((char *)st->scratch + qe_bytes);
  sc.extra = (char *)st->scratch + qe_bytes + smp_bytes;
  return SV_OK;
}

static sv_status sample_on_device(sv_state *st, const void *re, const void *im, uint64_t seed,
                                  int64_t shots, const int32_t *qubits, int nq, const SampleScratch &sc) {
  double *S, *P;
  void *a, *b, *c, *d;
  ws_layout(st, &S, &P, &a, &b, &c, &d);
  hipError_t e = svk_launch_sampling(st->dtype == SV_C128, re, im, st->n, S, P, sc.QE, seed, shots,
                                     qubits, nq, sc.samples, st->stream);
  if (e != hipSuccess) return fail(SV_EDEVICE, "sampling: %s", hipGetErrorString(e));
  return SV_OK;
}

extern "C" sv_status sv_sample(sv_state *st, uint64_t seed, int64_t shots, const int32_t *qubits,
                               int32_t n_measured, uint64_t *out) {
  if (!st) return fail(SV_EINVAL, "null handle");
  if (shots < 0) return fail(SV_EINVAL, "negative shots");
  if (n_measured < 0 || n_measured > 64) return fail(SV_EINVAL, "n_measured %d outside 0..64", n_measured);
  if (n_measured > 0 && !qubits) return fail(SV_EINVAL, "null qubits");
  for (int i = 0; i < n_measured; i++)
    if (qubits[i] < 0 || qubits[i] >= st->n) return fail(SV_EINVAL, "measured qubit %d out of range", qubits[i]);
  if (shots > 0 && !out) return fail(SV_EINVAL, "null output");
  if (shots == 0) return SV_OK;
  sv_status s = materialize_zero(st);
  if (s) return s;
  SampleScratch sc;
  s = sample_scratch(st, shots, 0, sc);
  if (s) return s;
  s = sample_on_device(st, st->re, st->im, seed, shots, qubits, n_measured, sc);
  if (s) return s;
  HIPCHK(hipMemcpyAsync(out, sc.samples, (size_t)shots * 8, hipMemcpyDeviceToHost, st->stream));
  HIPCHK(hipStreamSynchronize(st->stream));
  return SV_OK;
}

extern "C" sv_status sv_sample_counts(sv_state *st, uint64_t seed, int64_t shots,
                                      const int32_t *qubits, int32_t n_measured, uint64_t *counts) {
  if (!st) return fail(SV_EINVAL, "null handle");
  if (shots < 0) return fail(SV_EINVAL, "negative shots");
  if (n_measured < 0 || n_measured > SV_COUNTS_MAX_QUBITS)
    return fail(SV_EINVAL, "n_measured %d outside 0..%d", n_measured, SV_COUNTS_MAX_QUBITS);
  if (n_measured > 0 && !qubits) return fail(SV_EINVAL, "null qubits");
  for (int i = 0; i < n_measured; i++)
    if (qubits[i] < 0 || qubits[i] >= st->n) return fail(SV_EINVAL, "measured qubit %d out of range", qubits[i]);
  if (!counts) return fail(SV_EINVAL, "null counts");
  const size_t nb = (size_t)1 << n_measured;
  if (shots == 0) {
    std::memset(counts, 0, nb * 8);
    return SV_OK;
  }
  sv_status s = materialize_zero(st);
  if (s) return s;
  SampleScratch sc;
  s = sample_scratch(st, shots, nb * 8, sc);
  if (s) return s;
  s = sample_on_device(st, st->re, st->im, seed, shots, qubits, n_measured, sc);
  if (s) return s;
  uint64_t *d_counts = (uint64_t *)sc.extra;
  hipError_t e = svk_launch_histogram(sc.samples, shots, n_measured, d_counts, st->stream);
  if (e != hipSuccess) return fail(SV_EDEVICE, "histogram: %s", hipGetErrorString(e));
  HIPCHK(hipMemcpyAsync(counts, d_counts, nb * 8, hipMemcpyDeviceToHost, st->stream));
  HIPCHK(hipStreamSynchronize(st->stream));
  return SV_OK;
}

// Greedy qubit-wise-commuting groups in term order; identity terms join none.
struct ShotGroup {
  std::vector<int> terms;
  uint64_t xs = 0, zs = 0;  // measurement basis: X on xs & ~zs, Y on xs & zs, Z on zs & ~xs
  uint64_t support() const { return xs | zs; }
};

static std::vector<ShotGroup> qwc_group(const sv_pauli_term *terms, int nt) {
  std::vector<ShotGroup> groups;
  for (int j = 0; j < nt; j++) {
    const uint64_t x = terms[j].x_mask, z = terms[j].z_mask, u = x | z;
    if (!u) continue;
    bool placed = false;
    for (ShotGroup &g : groups) {
      const uint64_t both = g.support() & u;
      if (((g.xs ^ x) & both) || ((g.zs ^ z) & both)) continue;  // a letter differs on a shared qubit
      g.terms.push_back(j);
      g.xs |= x;
      g.zs |= z;
      placed = true;
      break;
    }
    if (!placed) {
      ShotGroup g;
      g.terms.push_back(j);
      g.xs = x;
      g.zs = z;
      groups.push_back(g);
    }
  }
  return groups;
}

static uint64_t pack_bits(uint64_t mask, uint64_t support) {
  uint64_t out = 0;
  int pos = 0;
  for (int q = 0; q < 64; q++)
    if (support >> q & 1) {
      if (mask >> q & 1) out |= 1ull << pos;
      pos++;
    }
  return out;
}

extern "C" sv_status sv_shot_estimate(sv_state *st, uint64_t seed, int64_t shots,
                                      const sv_pauli_term *terms, int32_t n_terms, double *values,
                                      double *energy, double *variance, int32_t *n_groups) {
  if (!st) return fail(SV_EINVAL, "null handle");
  sv_status s = validate_terms(st->n, terms, n_terms);
  if (s) return s;
  if (shots < 0) return fail(SV_EINVAL, "negative shots");
  if ((n_terms > 0 && !values) || !energy || !variance) return fail(SV_EINVAL, "null output");
  std::vector<ShotGroup> groups = qwc_group(terms, n_terms);
  const int G = (int)groups.size();
  if (G > 0 && shots < G) return fail(SV_EINVAL, "%lld shots for %d measurement groups", (long long)shots, G);
  for (const ShotGroup &g : groups)
    if (g.terms.size() > (size_t)SV_SHOT_GROUP_MAX_TERMS)
      return fail(SV_EUNSUPPORTED, "a measurement group of %zu terms (at most %d)", g.terms.size(),
                  SV_SHOT_GROUP_MAX_TERMS);
  for (int j = 0; j < n_terms; j++) values[j] = 1.0;
  double var_total = 0.0;
  if (G > 0) {
    s = materialize_zero(st);
    if (s) return s;
    const size_t plane = ((size_t)1 << st->n) * elem_size(st->dtype);
    if (st->copy_bytes < 2 * plane) {
      HIPCHK(hipStreamSynchronize(st->stream));
      if (st->copy) (void)hipFree(st->copy);
      st->copy = nullptr;
      st->copy_bytes = 0;
      if (hipMalloc(&st->copy, 2 * plane) != hipSuccess) {
        (void)hipGetLastError();
        return fail(SV_ENOMEM, "no device memory for the rotated copy (%zu bytes)", 2 * plane);
      }
      st->copy_bytes = 2 * plane;
    }
    void *cre = st->copy, *cim = (char *)st->copy + plane;
    size_t max_masks = 0;
    for (const ShotGroup &g : groups) max_masks = std::max(max_masks, g.terms.size() * (g.terms.size() + 1) / 2);
    const int64_t max_n = shots / G + 1;
    SampleScratch sc;
    s = sample_scratch(st, max_n, 16 * max_masks + 256, sc);
    if (s) return s;
    uint64_t *d_masks = (uint64_t *)sc.extra;
    uint64_t *d_odd = d_masks + max_masks;
    const bool dbl = st->dtype == SV_C128;
    for (int gi = 0; gi < G; gi++) {
      const ShotGroup &g = groups[gi];
      const int64_t N = shots / G + (gi < shots % G ? 1 : 0);
      HIPCHK(hipMemcpyAsync(cre, st->re, plane, hipMemcpyDeviceToDevice, st->stream));
      HIPCHK(hipMemcpyAsync(cim, st->im, plane, hipMemcpyDeviceToDevice, st->stream));
      // rotate the copy into the Z basis: H on X qubits, H S^dagger on Y
      // qubits, written as H = RY(pi/2) Z and H S^dagger = RY(pi/2) S so the
      // plan takes Kronecker stages (diagonal tables and rotations)
      std::vector<sv_op> rot;
      for (int q = 0; q < st->n; q++) {
        if (!(g.xs >> q & 1)) continue;
        sv_op o{};
        o.n_targets = 1;
        o.targets[0] = q;
        o.kind = (g.zs >> q & 1) ? SV_S : SV_Z;
        rot.push_back(o);
      }
      for (int q = 0; q < st->n; q++) {
        if (!(g.xs >> q & 1)) continue;
        sv_op o{};
        o.n_targets = 1;
        o.targets[0] = q;
        o.kind = SV_RY;
        o.param_index[0] = 0;
        rot.push_back(o);
      }
      const double half_pi = 1.5707963267948966;
      if (!rot.empty()) {
        Tiling tl = st->tiling;
        s = widen_groups(dbl, 1, tl);
        if (s) return s;
        Plan *P = nullptr;
        s = get_plan(st, SV_FUSE_AUTO, tl, rot.data(), (int)rot.size(), 1, false, &P);
        if (s) return s;
        s = upload_call_data(st, *P, rot.data(), (int)rot.size(), &half_pi, 1);
        if (s) return s;
        s = run_steps(st, *P, cre, cim, nullptr, nullptr, nullptr, 0);
        if (s) return s;
      }
      int32_t q_list[64];
      int nq = 0;
      for (int q = 0; q < st->n; q++)
        if (g.support() >> q & 1) q_list[nq++] = q;
      s = sample_on_device(st, cre, cim, seed + (uint64_t)gi, N, q_list, nq, sc);
      if (s) return s;
      // masks: each term, then each pair j < k (symmetric difference)
      const int T = (int)g.terms.size();
      std::vector<uint64_t> masks;
      for (int a = 0; a < T; a++)
        masks.push_back(pack_bits(terms[g.terms[a]].x_mask | terms[g.terms[a]].z_mask, g.support()));
      for (int a = 0; a < T; a++)
        for (int b = a + 1; b < T; b++) masks.push_back(masks[a] ^ masks[b]);
      const int nm = (int)masks.size();
      HIPCHK(hipMemcpyAsync(d_masks, masks.data(), (size_t)nm * 8, hipMemcpyHostToDevice, st->stream));
      hipError_t e = svk_launch_parity_counts(sc.samples, N, d_masks, nm, d_odd, st->stream);
      if (e != hipSuccess) return fail(SV_EDEVICE, "parity counts: %s", hipGetErrorString(e));
      std::vector<uint64_t> odd(nm);
      HIPCHK(hipMemcpyAsync(odd.data(), d_odd, (size_t)nm * 8, hipMemcpyDeviceToHost, st->stream));
      HIPCHK(hipStreamSynchronize(st->stream));
      auto val = [&](uint64_t o) { return (double)(N - 2 * (int64_t)o) / (double)N; };
      std::vector<double> v(T);
      for (int a = 0; a < T; a++) {
        v[a] = val(odd[a]);
        values[g.terms[a]] = v[a];
      }
      // pair index of (a, b), a < b, after the T single-term masks
      auto pair = [&](int a, int b) { return T + a * (2 * T - a - 1) / 2 + (b - a - 1); };
      double var = 0.0;
      for (int a = 0; a < T; a++)
        for (int b = 0; b < T; b++) {
          const double vab = a == b ? 1.0 : val(odd[a < b ? pair(a, b) : pair(b, a)]);
          var += terms[g.terms[a]].coeff * terms[g.terms[b]].coeff * (vab - v[a] * v[b]);
        }
      var_total += var / (double)N;
    }
  }
  double e = 0.0;
  for (int j = 0; j < n_terms; j++) e += terms[j].coeff * values[j];
  *energy = e;
  *variance = var_total;
  if (n_groups) *n_groups = G;
  return SV_OK;
}

// ------------------------------------------------------------ host copies

extern "C" sv_status sv_copy_to_host(const sv_state *st, void *re, void *im, uint64_t offset,
                                     uint64_t count) {
  if (!st) return fail(SV_EINVAL, "null handle");
  uint64_t N = 1ull << st->n;
  if (offset > N || count > N - offset) return fail(SV_EINVAL, "range [%llu,+%llu) beyond 2^n",
                                                   (unsigned long long)offset, (unsigned long long)count);
  size_t es = elem_size(st->dtype);
  sv_status z = materialize_zero(const_cast<sv_state *>(st));
  if (z) return z;
  if (re) HIPCHK(hipMemcpyAsync(re, (char *)st->re + offset * es, count * es, hipMemcpyDeviceToHost, st->stream));
  if (im) HIPCHK(hipMemcpyAsync(im, (char *)st->im + offset * es, count * es, hipMemcpyDeviceToHost, st->stream));
  HIPCHK(hipStreamSynchronize(st->stream));
  return SV_OK;
}

extern "C" sv_status sv_copy_from_host(sv_state *st, const void *re, const void *im, uint64_t offset,
                                       uint64_t count) {
  if (!st) return fail(SV_EINVAL, "null handle");
  uint64_t N = 1ull << st->n;
  if (offset > N || count > N - offset) return fail(SV_EINVAL, "range beyond 2^n");
  if (!re || !im) return fail(SV_EINVAL, "null host plane");
  size_t es = elem_size(st->dtype);
  sv_status z = materialize_zero(st);
  if (z) return z;
  HIPCHK(hipMemcpyAsync((char *)st->re + offset * es, re, count * es, hipMemcpyHostToDevice, st->stream));
  HIPCHK(hipMemcpyAsync((char *)st->im + offset * es, im, count * es, hipMemcpyHostToDevice, st->stream));
  HIPCHK(hipStreamSynchronize(st->stream));
  return SV_OK;
}

// ------------------------------------------------------- host-only helpers

static sv_status lower_all(int n, const sv_op *ops, int n_ops, std::vector<GateRec> &recs) {
  int np = 0;
  for (int i = 0; i < n_ops; i++)
    for (int k = 0; k < nparams_of(ops[i].kind); k++) np = std::max(np, ops[i].param_index[k] + 1);
  sv_status s = validate_circuit(n, ops, n_ops, nullptr, 0);
  if (s && s != SV_EUNBOUND) return s;
  for (int i = 0; i < n_ops; i++) {
    sv_status v = validate_op(ops[i], i, n, np);
    if (v) return v;
  }
  int um = 0;
  for (int i = 0; i < n_ops; i++) {
    GateRec g = lower_one(ops[i], ops[i].kind == SV_UNITARY ? um : -1);
    if (ops[i].kind == SV_UNITARY) um++;
    recs.push_back(g);
  }
  return SV_OK;
}

extern "C" sv_status sv_fuse_blocks(const sv_op *ops, int32_t n_ops, int32_t width, int32_t *block_of,
                                    int32_t *n_blocks) {
  if (width < 2 || width > 64) return fail(SV_EINVAL, "width %d", width);
  if (n_ops < 0 || (n_ops && (!ops || !block_of)) || !n_blocks) return fail(SV_EINVAL, "bad arguments");
  std::vector<GateRec> recs;
  sv_status s = lower_all(64, ops, n_ops, recs);
  if (s) return s;
  std::vector<int> bo;
  *n_blocks = fuse_greedy(recs, width, bo);
  for (int i = 0; i < n_ops; i++) block_of[i] = bo[i];
  return SV_OK;
}

extern "C" sv_status sv_plan_stats(int32_t n, const sv_op *ops, int32_t n_ops, int32_t fuse_width,
                                   int32_t tile_bits, int32_t low_bits, int32_t group_bits,
                                   int32_t *n_sweeps, int32_t *n_blocks) {
  if (n < 1 || n > SVI_NMAX) return fail(SV_EINVAL, "n %d outside 1..%d", n, SVI_NMAX);
  if (!(fuse_width == 0 || fuse_width == SV_FUSE_AUTO || (fuse_width >= 2 && fuse_width <= 5)))
    return fail(SV_EINVAL, "fuse_width %d", fuse_width);
  std::vector<GateRec> recs;
  sv_status s = lower_all(n, ops, n_ops, recs);
  if (s) return s;
  Tiling tl = default_tiling(n, SV_C128, 1);
  if (tile_bits) tl.M = tile_bits;
  if (low_bits) tl.c = low_bits;
  if (group_bits) tl.R = group_bits;
  if (fuse_width > tl.R) tl.R = 5;
  std::vector<GateRec> live;
  for (auto &g : recs)
    if (g.mo != MO_NOP) live.push_back(g);
  std::vector<SweepP> sweeps;
  int blocks = 0;
  if (fuse_width == 0) {
    if (n_sweeps) *n_sweeps = (int)live.size();
    if (n_blocks) *n_blocks = (int)live.size();
    return SV_OK;
  } else if (fuse_width < 0) {
    plan_auto_best(live, n, tl, sweeps, true);
  } else {
    plan_fused(live, n, tl, fuse_width, sweeps, true);
  }
  if (!layout_consistent(sweeps, n)) return fail(SV_EINVAL, "internal: inconsistent qubit layout in plan");
  for (auto &sw : sweeps) blocks += (int)sw.stages.size();
  if (n_sweeps) *n_sweeps = (int)sweeps.size();
  if (n_blocks) *n_blocks = blocks;
  return SV_OK;
}

extern "C" sv_status sv_adjoint_plan_stats(int32_t n, const sv_op *ops, int32_t n_ops, int32_t n_params,
                                           int32_t tile_bits, int32_t low_bits, int32_t group_bits,
                                           int32_t *n_sweeps, int32_t *n_stages, int32_t *n_gslots) {
  if (n < 1 || n > SVI_NMAX) return fail(SV_EINVAL, "n %d outside 1..%d", n, SVI_NMAX);
  for (int i = 0; i < n_ops; i++) {
    sv_status s = validate_op(ops[i], i, n, n_params);
    if (s) return s;
  }
  Tiling tl = default_tiling(n, SV_C128, 2);
  if (tile_bits) tl.M = tile_bits;
  if (low_bits) tl.c = low_bits;
  if (group_bits) tl.R = group_bits;
  Plan P;
  sv_status s = build_adjoint_plan(n, true, tl, ops, n_ops, n_params, P);
  if (s) return s;
  if (n_sweeps) *n_sweeps = (int)P.steps.size();
  if (n_stages) *n_stages = (int)P.stages.size();
  if (n_gslots) *n_gslots = P.n_gslots;
  return SV_OK;
}

// ------------------------------------------------------------ ragged batch
// Host side of the persistent batch launch: every circuit gets its own tile
// plan (the same planner as sv_apply_layer), the plans are concatenated into
// one set of device arrays, and the work units of all circuits are queued
// level by level (sweep 0 of every circuit, then sweep 1, ..., then the Pauli
// passes), so each unit depends only on units queued before it.

struct sv_batch {
  int nc = 0;
  sv_dtype dtype = SV_C128;
  bool dbl = true;
  int M = 13, R = 3, c = 5;
  bool kron_only = true;             // every stage of every sweep is a Kronecker stage
  int grid = 1;
  int32_t spin_limit = 1 << 20;   // ~1-2 s of polls
  int ncoefdesc = 0;
  int nunits = 0;
  int64_t total_sweeps = 0;
  double updates = 0.0;
  double bytes = 0.0;                // algorithmic HBM bytes of one run
  std::vector<int> nq;
  std::vector<int64_t> param_off;    // per circuit; [nc] = total
  std::vector<int64_t> n_user_params;
  std::vector<size_t> state_off;     // byte offset of circuit c's re plane (im follows)
  void *d_state = nullptr;
  void *d_meta = nullptr;
  double *d_params = nullptr, *d_coef = nullptr, *d_statics = nullptr, *d_part = nullptr;
  double *d_results = nullptr, *d_redcoef = nullptr;
  CoefDesc *d_coefdesc = nullptr;
  TabFactor *d_factors = nullptr;
  BatchUnit *d_units = nullptr;
  SweepArgs *d_sweeps = nullptr;
  PauliPassArgs *d_passes = nullptr;
  PauliTermDev *d_terms = nullptr;
  StageDesc *d_stages = nullptr;
  MicroOp *d_ops = nullptr;
  int32_t *d_ctl = nullptr;          // [0] head, [1] err, [2..2+nc) done
  int32_t *d_redrow = nullptr, *d_redslot = nullptr;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  ~sv_batch() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (d_state) (void)hipFree(d_state);
    if (d_meta) (void)hipFree(d_meta);
  }
};

static sv_status batch_validate(const sv_circuit_desc *cs, int nc, int &need) {
  if (nc < 1) return fail(SV_EINVAL, "a batch needs at least one circuit (got %d)", nc);
  if (!cs) return fail(SV_EINVAL, "null circuit array");
  need = 1;
  for (int k = 0; k < nc; k++) {
    const sv_circuit_desc &d = cs[k];
    if (d.n_qubits < 1 || d.n_qubits > 30)
      return fail(SV_EINVAL, "circuit %d: n_qubits %d outside 1..30", k, d.n_qubits);
    if (d.n_ops < 0 || (d.n_ops > 0 && !d.ops)) return fail(SV_EINVAL, "circuit %d: bad op list", k);
    if (d.n_params < 0) return fail(SV_EINVAL, "circuit %d: negative n_params", k);
    for (int i = 0; i < d.n_ops; i++) {
      sv_status s = validate_op(d.ops[i], i, d.n_qubits, d.n_params);
      if (s) return fail(s, "circuit %d: %s", k, std::string(g_err).c_str());
      need = std::max(need, d.ops[i].n_targets + d.ops[i].n_controls);
    }
    sv_status s = validate_terms(d.n_qubits, d.terms, d.n_terms);
    if (s) return fail(s, "circuit %d: %s", k, std::string(g_err).c_str());
  }
  return SV_OK;
}

extern "C" sv_status sv_batch_plan(const sv_circuit_desc *circuits, int32_t n_circuits,
                                   sv_dtype dtype, int32_t tile_bits, int32_t low_bits,
                                   int32_t group_bits, sv_batch **out) {
  if (!out) return fail(SV_EINVAL, "null output handle");
  *out = nullptr;
  if (dtype != SV_C128 && dtype != SV_C64) return fail(SV_EDTYPE, "unsupported dtype %d", (int)dtype);
  int need = 1;
  sv_status s = batch_validate(circuits, n_circuits, need);
  if (s) return s;
  const bool dbl = dtype == SV_C128;
  const int M = tile_bits ? tile_bits : 13;
  int R = group_bits;
  if (!R) {
    R = std::max(3, need);
    while (R <= SVI_RMAX && !svk_has_batch(dbl, M, R)) R++;
  }
  if (R < need) return fail(SV_EINVAL, "group_bits %d narrower than the widest op (%d qubits)", R, need);
  if (R > SVI_RMAX || !svk_has_batch(dbl, M, R))
    return fail(SV_EINVAL, "no batch kernel for tile_bits %d, group_bits %d, dtype %d", M, R, (int)dtype);
  const int c = low_bits ? low_bits : 5;
  if (c < 1 || c > M) return fail(SV_EINVAL, "low_bits %d outside 1..%d", c, M);

  std::unique_ptr<sv_batch> b(new sv_batch);
  b->nc = n_circuits;
  b->dtype = dtype;
  b->dbl = dbl;
  b->M = M;
  b->R = R;
  b->c = c;
  const size_t es = elem_size(dtype);
  const Tiling tl{M, c, R};

  // ---- per-circuit plans, merged
  std::vector<StageDesc> stages;
  std::vector<MicroOp> ops;
  std::vector<CoefDesc> coefs;
  std::vector<TabFactor> factors;
  std::vector<double> statics, constants_init;
  std::vector<SweepArgs> sweeps;
  std::vector<PauliPassArgs> passes;
  std::vector<PauliTermDev> terms;
  std::vector<std::vector<std::vector<BatchUnit>>> levels(n_circuits);  // [circ][level] units
  std::vector<std::vector<std::pair<double, int>>> red(n_circuits);     // (coef, part slot)
  int64_t ncoef = 0, nparam = 0, npart = 0;
  size_t state_bytes = 0;
  b->nq.resize(n_circuits);
  b->param_off.resize(n_circuits + 1);
  b->n_user_params.resize(n_circuits);
  b->state_off.resize(n_circuits);
  std::vector<std::pair<int, double>> const_init;   // (param slot, value)

  auto tiles_per_unit = [](int64_t ntiles) -> int64_t {
    return std::max<int64_t>(1, std::min<int64_t>(8, ntiles / 32));
  };

  for (int k = 0; k < n_circuits; k++) {
    const sv_circuit_desc &d = circuits[k];
    const int n = d.n_qubits;
    b->nq[k] = n;
    b->state_off[k] = state_bytes;
    const size_t plane = (((size_t)1 << n) * es + 255) & ~(size_t)255;
    state_bytes += 2 * plane;
    Plan P;
    s = build_forward_plan(-1, n, dbl, tl, d.ops, d.n_ops, d.n_params, P, false, false);
    if (s) return s;
    if (P.M != M || P.R != R) return fail(SV_EINVAL, "internal: plan tiling mismatch");
    for (const Step &st : P.steps) {
      if (st.kind != 0) return fail(SV_EUNSUPPORTED, "circuit %d: plan needs a single-gate kernel", k);
      if (!st.all_kron) b->kron_only = false;
    }
    const int64_t stage_off = (int64_t)stages.size(), op_off = (int64_t)ops.size();
    const int64_t factor_off = (int64_t)factors.size(), static_off = (int64_t)statics.size();
    const int64_t coef_off = ncoef;
    b->param_off[k] = nparam;
    b->n_user_params[k] = d.n_params;
    for (size_t j = 0; j < P.constants.size(); j++)
      const_init.push_back({(int)(nparam + d.n_params + (int64_t)j), P.constants[j]});
    nparam += d.n_params + (int64_t)P.constants.size();
    stages.insert(stages.end(), P.stages.begin(), P.stages.end());
    ops.insert(ops.end(), P.ops.begin(), P.ops.end());
    for (CoefDesc cd : P.coefs) {
      const int fmt = cd.fmt & 0xff;
      cd.dst += (int32_t)coef_off;
      if (fmt == CF_TABLE || fmt == CF_SCALE) cd.src += (int32_t)factor_off;
      else if (fmt == CF_COPY) cd.src += (int32_t)static_off;
      else if (fmt != CF_IDENT2)
        for (int q = 0; q < 3; q++)
          if (cd.pidx[q] >= 0) cd.pidx[q] += (int32_t)b->param_off[k];
      coefs.push_back(cd);
    }
    for (TabFactor f : P.factors) {
      if (f.pidx >= 0) f.pidx += (int32_t)b->param_off[k];
      factors.push_back(f);
    }
    for (int i = 0; i < d.n_ops; i++)
      if (d.ops[i].kind == SV_UNITARY) {
        const int dd = 1 << d.ops[i].n_targets;
        statics.insert(statics.end(), d.ops[i].matrix, d.ops[i].matrix + 2 * dd * dd);
      }
    ncoef += P.ncoef;

    // sweeps (an empty circuit still needs one sweep that writes |0..0>)
    std::vector<SweepArgs> csw;
    for (const Step &st : P.steps) csw.push_back(st.sa);
    if (csw.empty()) {
      SweepArgs z;
      std::memset(&z, 0, sizeof z);
      const int m = std::min(M, n), cc = std::min(c, n);
      z.n = n;
      z.m = m;
      z.c = cc;
      z.nh = m - cc;
      for (int q = 0; q < z.nh; q++) z.hb[q] = cc + q;
      z.ntiles = (int64_t)1 << (n - m);
      csw.push_back(z);
    }
    csw[0].flags |= SW_INIT_ZERO;
    uint64_t support = 0;
    double cbytes = 0.0;   // every tile a sweep runs is read and written (the first only written)
    for (SweepArgs &a : csw) {
      restrict_to_support(a, n, &support);
      cbytes += ((a.flags & SW_INIT_ZERO) ? 2.0 : 4.0) * (double)es * (double)(a.ntiles << a.m);
    }
    int64_t before = 0;   // units of this circuit in earlier levels
    for (SweepArgs &a : csw) {
      a.re = nullptr;     // patched after the device allocation
      a.im = nullptr;
      a.stages = (const StageDesc *)(intptr_t)stage_off;   // offsets, patched later
      a.ops = (const MicroOp *)(intptr_t)op_off;
      a.coef = (const double *)(intptr_t)coef_off;
      a.re2 = (void *)(intptr_t)k;                          // circuit id until patched
      const int idx = (int)sweeps.size();
      sweeps.push_back(a);
      std::vector<BatchUnit> lu;
      const int64_t tpu = tiles_per_unit(a.ntiles);
      for (int64_t t = 0; t < a.ntiles; t += tpu) {
        BatchUnit u{};
        u.kind = UK_SWEEP;
        u.circ = k;
        u.arg = idx;
        u.wait = (int32_t)before;
        u.t0 = t;
        u.t1 = std::min(a.ntiles, t + tpu);
        lu.push_back(u);
      }
      before += (int64_t)lu.size();
      levels[k].push_back(std::move(lu));
    }
    b->total_sweeps += (int64_t)csw.size();
    b->updates += (double)d.n_ops * (double)((int64_t)1 << n);
    b->bytes += cbytes;

    // Pauli passes: one level after the last sweep
    if (d.n_terms > 0) {
      PauliPlan pp;
      plan_pauli(n, d.terms, d.n_terms, pp);
      if (pp.wide_begin != (int)pp.terms.size())
        return fail(SV_EUNSUPPORTED, "circuit %d: a term's X/Y support does not fit in one %d-qubit tile",
                    k, std::min(13, n));
      const int term_off = (int)terms.size();
      terms.insert(terms.end(), pp.terms.begin(), pp.terms.end());
      std::vector<BatchUnit> lu;
      for (const PauliPlan::Pass &ps : pp.passes) {
        PauliPassArgs pa;
        std::memset(&pa, 0, sizeof pa);
        pa.terms = (const PauliTermDev *)nullptr;
        pa.n = n;
        pa.m = ps.m;
        pa.c = ps.c;
        pa.nh = ps.nh;
        for (int q = 0; q < SVI_MMAX; q++) pa.hb[q] = q < ps.nh ? ps.hb[q] : 0;
        pa.t_begin = term_off + ps.t0;
        pa.t_end = term_off + ps.t1;
        pa.ntiles = (int64_t)1 << (n - ps.m);
        pa.lre = (void *)(intptr_t)k;   // circuit id until patched
        const int idx = (int)passes.size();
        passes.push_back(pa);
        const int64_t tpu = tiles_per_unit(pa.ntiles);
        for (int64_t t = 0; t < pa.ntiles; t += tpu) {
          BatchUnit u{};
          u.kind = UK_PAULI;
          u.circ = k;
          u.arg = idx;
          u.wait = (int32_t)before;
          u.t0 = t;
          u.t1 = std::min(pa.ntiles, t + tpu);
          u.part = (int32_t)npart;
          for (int j = ps.t0; j < ps.t1; j++) red[k].push_back({pp.terms[j].c, (int)(npart + j - ps.t0)});
          npart += ps.t1 - ps.t0;
          lu.push_back(u);
        }
      }
      levels[k].push_back(std::move(lu));
      b->bytes += 2.0 * (double)pp.passes.size() * (double)es * (double)((int64_t)1 << n);
    }
  }
  b->param_off[n_circuits] = nparam;

  // ---- queue: level by level; within a level, circuits with more levels first
  std::vector<int> order(n_circuits);
  for (int k = 0; k < n_circuits; k++) order[k] = k;
  std::stable_sort(order.begin(), order.end(), [&](int a, int c2) {
    return levels[a].size() > levels[c2].size();
  });
  size_t maxlev = 0;
  for (int k = 0; k < n_circuits; k++) maxlev = std::max(maxlev, levels[k].size());
  std::vector<BatchUnit> units;
  for (size_t l = 0; l < maxlev; l++)
    for (int k : order)
      if (l < levels[k].size())
        units.insert(units.end(), levels[k][l].begin(), levels[k][l].end());
  if (units.size() > (size_t)INT32_MAX) return fail(SV_ENOMEM, "batch too large");
  b->nunits = (int)units.size();

  // ---- reduction rows
  std::vector<int32_t> redrow(n_circuits + 1, 0), redslot;
  std::vector<double> redcoef;
  for (int k = 0; k < n_circuits; k++) {
    for (auto &e : red[k]) { redcoef.push_back(e.first); redslot.push_back(e.second); }
    redrow[k + 1] = (int32_t)redslot.size();
  }

  // ---- device memory (everything above is host-only planning)
  DevInfo di;
  s = device_info(di);
  if (s) return s;
  HIPCHK(hipMalloc(&b->d_state, std::max<size_t>(state_bytes, 256)));
  auto align = [](size_t v) { return (v + 255) & ~(size_t)255; };
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align(off + std::max<size_t>(bytes, 8)); return o; };
  const size_t o_params = take((size_t)nparam * 8);
  const size_t o_coef = take((size_t)ncoef * 8);
  const size_t o_statics = take(statics.size() * 8);
  const size_t o_part = take((size_t)npart * 8);
  const size_t o_results = take((size_t)n_circuits * 8);
  const size_t o_redcoef = take(redcoef.size() * 8);
  const size_t o_coefdesc = take(coefs.size() * sizeof(CoefDesc));
  const size_t o_factors = take(factors.size() * sizeof(TabFactor));
  const size_t o_units = take(units.size() * sizeof(BatchUnit));
  const size_t o_sweeps = take(sweeps.size() * sizeof(SweepArgs));
  const size_t o_passes = take(passes.size() * sizeof(PauliPassArgs));
  const size_t o_terms = take(terms.size() * sizeof(PauliTermDev));
  const size_t o_stages = take(stages.size() * sizeof(StageDesc));
  const size_t o_ops = take(ops.size() * sizeof(MicroOp));
  const size_t o_ctl = take((size_t)(n_circuits + 2) * 4);
  const size_t o_redrow = take(redrow.size() * 4);
  const size_t o_redslot = take(redslot.size() * 4);
  HIPCHK(hipMalloc(&b->d_meta, off));
  char *mb = (char *)b->d_meta;
  b->d_params = (double *)(mb + o_params);
  b->d_coef = (double *)(mb + o_coef);
  b->d_statics = (double *)(mb + o_statics);
  b->d_part = (double *)(mb + o_part);
  b->d_results = (double *)(mb + o_results);
  b->d_redcoef = (double *)(mb + o_redcoef);
  b->d_coefdesc = (CoefDesc *)(mb + o_coefdesc);
  b->d_factors = (TabFactor *)(mb + o_factors);
  b->d_units = (BatchUnit *)(mb + o_units);
  b->d_sweeps = (SweepArgs *)(mb + o_sweeps);
  b->d_passes = (PauliPassArgs *)(mb + o_passes);
  b->d_terms = (PauliTermDev *)(mb + o_terms);
  b->d_stages = (StageDesc *)(mb + o_stages);
  b->d_ops = (MicroOp *)(mb + o_ops);
  b->d_ctl = (int32_t *)(mb + o_ctl);
  b->d_redrow = (int32_t *)(mb + o_redrow);
  b->d_redslot = (int32_t *)(mb + o_redslot);
  b->ncoefdesc = (int)coefs.size();

  // patch pointers
  char *sb = (char *)b->d_state;
  for (SweepArgs &a : sweeps) {
    const int k = (int)(intptr_t)a.re2;
    const size_t plane = (((size_t)1 << b->nq[k]) * es + 255) & ~(size_t)255;
    a.re = sb + b->state_off[k];
    a.im = sb + b->state_off[k] + plane;
    a.re2 = a.im2 = nullptr;
    a.gpart = nullptr;
    a.stages = b->d_stages + (intptr_t)a.stages;
    a.ops = b->d_ops + (intptr_t)a.ops;
    a.coef = b->d_coef + (intptr_t)a.coef;
  }
  for (PauliPassArgs &pa : passes) {
    const int k = (int)(intptr_t)pa.lre;
    const size_t plane = (((size_t)1 << b->nq[k]) * es + 255) & ~(size_t)255;
    pa.re = sb + b->state_off[k];
    pa.im = sb + b->state_off[k] + plane;
    pa.lre = pa.lim = nullptr;
    pa.terms = b->d_terms;
    pa.part = nullptr;
  }
  std::vector<double> params_init((size_t)std::max<int64_t>(nparam, 1), 0.0);
  for (auto &ci : const_init) params_init[ci.first] = ci.second;
  auto up = [&](void *dst, const void *src, size_t bytes) -> sv_status {
    if (bytes) HIPCHK(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
    return SV_OK;
  };
  if ((s = up(b->d_params, params_init.data(), (size_t)nparam * 8))) return s;
  if ((s = up(b->d_statics, statics.data(), statics.size() * 8))) return s;
  if ((s = up(b->d_redcoef, redcoef.data(), redcoef.size() * 8))) return s;
  if ((s = up(b->d_coefdesc, coefs.data(), coefs.size() * sizeof(CoefDesc)))) return s;
  if ((s = up(b->d_factors, factors.data(), factors.size() * sizeof(TabFactor)))) return s;
  if ((s = up(b->d_units, units.data(), units.size() * sizeof(BatchUnit)))) return s;
  if ((s = up(b->d_sweeps, sweeps.data(), sweeps.size() * sizeof(SweepArgs)))) return s;
  if ((s = up(b->d_passes, passes.data(), passes.size() * sizeof(PauliPassArgs)))) return s;
  if ((s = up(b->d_terms, terms.data(), terms.size() * sizeof(PauliTermDev)))) return s;
  if ((s = up(b->d_stages, stages.data(), stages.size() * sizeof(StageDesc)))) return s;
  if ((s = up(b->d_ops, ops.data(), ops.size() * sizeof(MicroOp)))) return s;
  if ((s = up(b->d_redrow, redrow.data(), redrow.size() * 4))) return s;
  if ((s = up(b->d_redslot, redslot.data(), redslot.size() * 4))) return s;
  HIPCHK(hipMemset(b->d_results, 0, (size_t)n_circuits * 8));

  const int occ = svk_batch_occupancy(dbl, M, R, b->kron_only ? 1 : 0);
  b->grid = std::max(1, std::min(b->nunits, di.cus * std::max(1, occ)));
  *out = b.release();
  return SV_OK;
}

static sv_status batch_enqueue(sv_batch *b, hipStream_t s) {
  hipError_t e = svk_launch_batch_reset(b->d_ctl, b->d_ctl + 2, b->d_ctl + 1, b->nc, s);
  if (e == hipSuccess)
    e = svk_launch_coefs(b->d_coefdesc, b->ncoefdesc, b->d_params, b->d_statics, b->d_factors,
                         b->d_coef, s);
  if (e == hipSuccess) {
    BatchKernelArgs a{};
    a.units = b->d_units;
    a.sweeps = b->d_sweeps;
    a.passes = b->d_passes;
    a.part = b->d_part;
    a.head = b->d_ctl;
    a.err = b->d_ctl + 1;
    a.done = b->d_ctl + 2;
    a.nunits = b->nunits;
    a.spin_limit = b->spin_limit;
    e = svk_launch_batch(b->dbl, b->M, b->R, b->kron_only ? 1 : 0, a, b->grid, s);
  }
  if (e == hipSuccess)
    e = svk_launch_batch_reduce(b->d_redrow, b->d_redslot, b->d_redcoef, b->d_part, b->d_results,
                                b->nc, s);
  if (e != hipSuccess) return fail(SV_EDEVICE, "batch launch: %s", hipGetErrorString(e));
  return SV_OK;
}

extern "C" sv_status sv_batch_run(sv_batch *b, void *stream) {
  if (!b) return fail(SV_EINVAL, "null batch");
  return batch_enqueue(b, (hipStream_t)stream);
}

extern "C" sv_status sv_batch_graph_launch(sv_batch *b, void *stream) {
  if (!b) return fail(SV_EINVAL, "null batch");
  if (!b->gexec) {
    if (!b->cap_stream) HIPCHK(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    sv_status s = batch_enqueue(b, b->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
    if (s) {
      if (g) (void)hipGraphDestroy(g);
      return s;
    }
    if (e != hipSuccess) return fail(SV_EDEVICE, "graph capture: %s", hipGetErrorString(e));
    b->graph = g;
    HIPCHK(hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0));
  }
  HIPCHK(hipGraphLaunch(b->gexec, (hipStream_t)stream));
  return SV_OK;
}

extern "C" sv_status sv_batch_upload_params(sv_batch *b, const double *params, int64_t count) {
  if (!b) return fail(SV_EINVAL, "null batch");
  if (count != b->param_off[b->nc]) {
    int64_t users = 0;
    for (int k = 0; k < b->nc; k++) users += b->n_user_params[k];
    if (count != users)
      return fail(SV_EINVAL, "expected %lld parameters, got %lld", (long long)users, (long long)count);
  }
  if (count > 0 && !params) return fail(SV_EUNBOUND, "null params");
  for (int64_t i = 0; i < count; i++)
    if (!std::isfinite(params[i])) return fail(SV_EUNBOUND, "parameter %lld is not finite", (long long)i);
  // concatenated user parameters, circuit by circuit, into each circuit's block
  int64_t src = 0;
  for (int k = 0; k < b->nc; k++) {
    const int64_t np = b->n_user_params[k];
    if (np) HIPCHK(hipMemcpy(b->d_params + b->param_off[k], params + src, (size_t)np * 8, hipMemcpyHostToDevice));
    src += np;
  }
  return SV_OK;
}

extern "C" double *sv_batch_params_device(sv_batch *b) { return b ? b->d_params : nullptr; }

extern "C" int64_t sv_batch_param_offset(const sv_batch *b, int32_t circuit) {
  if (!b || circuit < 0 || circuit > b->nc) return -1;
  return b->param_off[circuit];
}

extern "C" double *sv_batch_results_device(sv_batch *b) { return b ? b->d_results : nullptr; }

extern "C" sv_status sv_batch_check(sv_batch *b, void *stream) {
  if (!b) return fail(SV_EINVAL, "null batch");
  int32_t err = 0;
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  HIPCHK(hipMemcpy(&err, b->d_ctl + 1, 4, hipMemcpyDeviceToHost));
  if (err) return fail(SV_EDEVICE, "batch: a work unit's dependency wait expired; results are invalid");
  return SV_OK;
}

extern "C" sv_status sv_batch_set_spin_limit(sv_batch *b, int32_t polls) {
  if (!b) return fail(SV_EINVAL, "null batch");
  b->spin_limit = polls;
  if (b->gexec) {   // the limit is a kernel argument: capture again on next use
    (void)hipGraphExecDestroy(b->gexec);
    (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
  }
  return SV_OK;
}

extern "C" sv_status sv_batch_state(sv_batch *b, int32_t circuit, void **re, void **im) {
  if (!b || circuit < 0 || circuit >= b->nc || !re || !im) return fail(SV_EINVAL, "bad batch state query");
  const size_t plane = (((size_t)1 << b->nq[circuit]) * elem_size(b->dtype) + 255) & ~(size_t)255;
  *re = (char *)b->d_state + b->state_off[circuit];
  *im = (char *)b->d_state + b->state_off[circuit] + plane;
  return SV_OK;
}

extern "C" sv_status sv_batch_copy_results(sv_batch *b, double *out, void *stream) {
  if (!b || !out) return fail(SV_EINVAL, "bad batch result query");
  HIPCHK(hipMemcpyAsync(out, b->d_results, (size_t)b->nc * 8, hipMemcpyDeviceToHost, (hipStream_t)stream));
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  return SV_OK;
}

extern "C" sv_status sv_batch_copy_state(sv_batch *b, int32_t circuit, void *re, void *im,
                                         void *stream) {
  void *dre = nullptr, *dim = nullptr;
  sv_status s = sv_batch_state(b, circuit, &dre, &dim);
  if (s) return s;
  if (!re || !im) return fail(SV_EINVAL, "null host plane");
  const size_t bytes = ((size_t)1 << b->nq[circuit]) * elem_size(b->dtype);
  HIPCHK(hipMemcpyAsync(re, dre, bytes, hipMemcpyDeviceToHost, (hipStream_t)stream));
  HIPCHK(hipMemcpyAsync(im, dim, bytes, hipMemcpyDeviceToHost, (hipStream_t)stream));
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  return SV_OK;
}

extern "C" sv_status sv_batch_stats(const sv_batch *b, int64_t *units, int64_t *sweeps,
                                    double *updates, double *bytes) {
  if (!b) return fail(SV_EINVAL, "null batch");
  if (units) *units = b->nunits;
  if (sweeps) *sweeps = b->total_sweeps;
  if (updates) *updates = b->updates;
  if (bytes) *bytes = b->bytes;
  return SV_OK;
}

extern "C" sv_status sv_batch_free(sv_batch *b) {
  if (!b) return SV_OK;
  (void)hipDeviceSynchronize();
  delete b;
  return SV_OK;
}

// Empirical choice of the batch tiling: plan every compiled candidate
// (register-group width x contiguous low bits), time `reps` runs of each with
// HIP events on `stream`, keep the fastest.
extern "C" sv_status sv_batch_autotune(const sv_circuit_desc *circuits, int32_t n_circuits,
                                       sv_dtype dtype, const double *params, int32_t reps,
                                       void *stream, int32_t *tile_bits, int32_t *low_bits,
                                       int32_t *group_bits, double *best_ms) {
  if (!tile_bits || !low_bits || !group_bits) return fail(SV_EINVAL, "null output");
  if (reps < 1) return fail(SV_EINVAL, "reps %d < 1", reps);
  int need = 1;
  sv_status s = batch_validate(circuits, n_circuits, need);
  if (s) return s;
  hipStream_t hs = (hipStream_t)stream;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  double best = 1e300;
  int bR = 0, bc = 0;
  const bool dbl = dtype == SV_C128;
  for (int R = std::max(3, need); R <= SVI_RMAX; R++) {
    if (!svk_has_batch(dbl, 13, R)) continue;
    for (int c : {2, 3, 4, 5}) {
      sv_batch *b = nullptr;
      s = sv_batch_plan(circuits, n_circuits, dtype, 13, c, R, &b);
      if (s) break;
      if (params) {
        int64_t users = 0;
        for (int k = 0; k < n_circuits; k++) users += circuits[k].n_params;
        s = sv_batch_upload_params(b, params, users);
      }
      if (!s) s = sv_batch_run(b, hs);                 // warm-up
      float ms = 0.f;
      if (!s) {
        (void)hipEventRecord(e0, hs);
        for (int r = 0; r < reps && !s; r++) s = sv_batch_run(b, hs);
        (void)hipEventRecord(e1, hs);
        if (!s) s = sv_batch_check(b, hs);
        if (!s && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) s = fail(SV_EDEVICE, "event timing failed");
      }
      sv_batch_free(b);
      if (s) break;
      const double t = ms / reps;
      if (t < best) { best = t; bR = R; bc = c; }
    }
    if (s) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s) return s;
  if (!bR) return fail(SV_EUNSUPPORTED, "no compiled batch kernel holds %d-qubit ops", need);
  *tile_bits = 13;
  *low_bits = bc;
  *group_bits = bR;
  if (best_ms) *best_ms = best;
  return SV_OK;
}

// ---------------------------------------------------------------- serving
// Small adjoint requests run whole inside one workgroup each (k_serve): the
// forward and backward plans are built for 12-qubit tiles and cached per
// request structure; a submission copies one staging block (request
// descriptors, sweep arguments, observables, parameters) to the device and
// launches two kernels.  A ring of staging slots lets submissions queue on the
// stream while earlier ones run.

struct ServePlan {
  Plan F, B;
  bool general = false;        // some stage is a micro-op (interpreter) stage
  sv_status status = SV_OK;
  std::string why;
};

struct ServeSlot {
  void *d_buf = nullptr;
  size_t d_bytes = 0;
  void *h_buf = nullptr;       // pinned staging
  size_t h_bytes = 0;
  hipEvent_t done = nullptr;
  bool busy = false;
  std::vector<std::shared_ptr<ServePlan>> held;   // plans the queued run reads
};

#define SVS_SLOTS 4

struct sv_serve {
  int dev = 0;
  std::unordered_map<std::string, std::shared_ptr<ServePlan>> plans;
  ServeSlot slot[SVS_SLOTS];
  int next = 0;
};

static const Tiling kServeFwd{12, 5, 3}, kServeBwd{12, 3, 3};

static sv_status serve_wait(ServeSlot &sl) {
  if (sl.busy) {
    HIPCHK(hipEventSynchronize(sl.done));
    sl.busy = false;
    sl.held.clear();
  }
  return SV_OK;
}

// Plan pair of one request (cached by structure); its status says whether the
// serving kernel can run it.
static sv_status serve_plan(sv_serve *sv, const sv_circuit_desc &d, std::shared_ptr<ServePlan> &out) {
  int Ms = 0, Rs = 0;
  (void)svk_serve_tiling(&Ms, &Rs);
  const std::string key = plan_key(-2, d.n_qubits, kServeFwd, true, d.ops, d.n_ops, d.n_params);
  auto it = sv->plans.find(key);
  if (it != sv->plans.end()) {
    out = it->second;
    return out->status ? fail(out->status, "%s", out->why.c_str()) : SV_OK;
  }
  std::shared_ptr<ServePlan> sp(new ServePlan);
  auto refuse = [&](const char *fmt, int a, int b) {
    char buf[160];
    snprintf(buf, sizeof buf, fmt, a, b);
    sp->status = SV_EUNSUPPORTED;
    sp->why = buf;
  };
  const int n = d.n_qubits;
  int width = 1;
  bool user_mat = false;
  for (int i = 0; i < d.n_ops; i++) {
    width = std::max(width, d.ops[i].n_targets + d.ops[i].n_controls);
    if (d.ops[i].kind == SV_UNITARY) user_mat = true;
  }
  if (n < Rs || n > svk_serve_max_qubits())
    refuse("serving kernel: %d qubits outside 3..%d", n, svk_serve_max_qubits());
  else if (width > Rs)
    refuse("serving kernel: an op on %d qubits (at most %d)", width, Rs);
  else if (user_mat)
    refuse("serving kernel: user matrices are not taken (%d, %d)", 0, 0);
  if (!sp->status) {
    sv_status s = build_forward_plan(-1, n, true, kServeFwd, d.ops, d.n_ops, d.n_params, sp->F, false, false);
    if (s) return s;
    s = build_adjoint_plan(n, true, kServeBwd, d.ops, d.n_ops, d.n_params, sp->B);
    if (s) return s;
    for (const Step &st : sp->F.steps)
      if (st.kind != 0 || sp->F.M != Ms || sp->F.R != Rs) refuse("serving kernel: forward plan step %d of kind %d", 0, st.kind);
    for (const Step &st : sp->B.steps)
      if (st.kind != 0 || st.sa.m < Rs || st.sa.n_gslots > SVI_GSLOTS_MAX)
        refuse("serving kernel: backward step of kind %d is not a tile sweep (m=%d)", st.kind, st.sa.m);
    for (const Plan *P : {&sp->F, &sp->B})
      for (const Step &st : P->steps) sp->general = sp->general || !st.all_kron;
  }
  if (sv->plans.size() >= 256) sv->plans.clear();   // queued runs keep their plans alive
  sv->plans.emplace(key, sp);
  out = sp;
  return sp->status ? fail(sp->status, "%s", sp->why.c_str()) : SV_OK;
}

extern "C" sv_status sv_serve_create(sv_serve **out) {
  if (!out) return fail(SV_EINVAL, "null output handle");
  *out = nullptr;
  std::unique_ptr<sv_serve> sv(new sv_serve);
  sv->dev = -1;   // bound to the current device at the first submission
  *out = sv.release();
  return SV_OK;
}

extern "C" int32_t sv_serve_max_qubits(void) { return svk_serve_max_qubits(); }

static sv_status serve_check_plan(sv_serve *sv, const sv_circuit_desc *request,
                                  std::shared_ptr<ServePlan> &sp) {
  if (!sv || !request) return fail(SV_EINVAL, "null argument");
  const sv_circuit_desc &d = *request;
  if (d.n_qubits < 1 || d.n_qubits > SVI_NMAX)
    return fail(SV_EINVAL, "n_qubits %d outside 1..%d", d.n_qubits, SVI_NMAX);
  if (d.n_ops < 0 || (d.n_ops > 0 && !d.ops)) return fail(SV_EINVAL, "bad op list");
  if (d.n_params < 0) return fail(SV_EINVAL, "negative n_params");
  for (int i = 0; i < d.n_ops; i++) {
    sv_status s = validate_op(d.ops[i], i, d.n_qubits, d.n_params);
    if (s) return s;
  }
  sv_status s = validate_terms(d.n_qubits, d.terms, d.n_terms);
  if (s) return s;
  return serve_plan(sv, d, sp);
}

extern "C" sv_status sv_serve_check(sv_serve *sv, const sv_circuit_desc *request) {
  std::shared_ptr<ServePlan> sp;
  return serve_check_plan(sv, request, sp);
}

extern "C" sv_status sv_serve_submit(sv_serve *sv, const sv_circuit_desc *requests, int32_t n_requests,
                                     const double *params, double *d_out, void *hip_stream) {
  if (!sv) return fail(SV_EINVAL, "null handle");
  if (n_requests < 1 || n_requests > 65535)
    return fail(SV_EINVAL, "n_requests %d outside 1..65535", n_requests);
  if (!requests || !d_out) return fail(SV_EINVAL, "null requests or output");
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (sv->dev < 0) {
    for (ServeSlot &sl : sv->slot) HIPCHK(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
    sv->dev = dev;
  }
  if (dev != sv->dev) return fail(SV_EINVAL, "handle used on device %d, current device %d", sv->dev, dev);
  // ---- validate everything and get the plans before touching the device
  std::vector<std::shared_ptr<ServePlan>> plans(n_requests);
  int64_t pofs = 0;
  for (int r = 0; r < n_requests; r++) {
    const sv_circuit_desc &d = requests[r];
    if (d.n_params > 0 && !params) return fail(SV_EUNBOUND, "null params");
    sv_status s = serve_check_plan(sv, &d, plans[r]);
    if (!s) s = validate_circuit(d.n_qubits, d.ops, d.n_ops, params + pofs, d.n_params);
    if (s) return fail(s, "request %d: %s", r, std::string(g_err).c_str());
    pofs += d.n_params;
  }
  for (auto &sp : plans)
    if (!sp->F.d_buf) {
      sv_status s = upload_plan(sp->F);
      if (!s) s = upload_plan(sp->B);
      if (s) return s;
    }
  // ---- layout: staged part (copied from host) | device-only part
  auto align = [](size_t v) { return (v + 255) & ~(size_t)255; };
  size_t off = 256;   // [0], [1]: queue heads of the lean and the general kernel
  const size_t o_reqs = off;
  off = align(off + (size_t)n_requests * sizeof(ServeReq));
  int nsw = 0, max_desc = 0;
  size_t nterm = 0;
  for (int r = 0; r < n_requests; r++) {
    nsw += (int)std::max<size_t>(plans[r]->F.steps.size(), 1) + (int)plans[r]->B.steps.size();
    nterm += (size_t)requests[r].n_terms;
    max_desc = std::max(max_desc, (int)(plans[r]->F.coefs.size() + plans[r]->B.coefs.size()));
  }
  const size_t o_sweeps = off;
  off = align(off + (size_t)nsw * sizeof(SweepArgs));
  const size_t o_terms = off;
  off = align(off + std::max<size_t>(nterm, 1) * sizeof(PauliTermDev));
  std::vector<size_t> o_fp(n_requests), o_bp(n_requests);
  for (int r = 0; r < n_requests; r++) {
    const int nu = requests[r].n_params;
    o_fp[r] = off;
    off = align(off + (size_t)(nu + plans[r]->F.constants.size() + 1) * 8);
    o_bp[r] = off;
    off = align(off + (size_t)(nu + plans[r]->B.constants.size() + 1) * 8);
  }
  const size_t staged = off;
  std::vector<size_t> o_fc(n_requests), o_bc(n_requests), o_st(n_requests), o_sl(n_requests);
  for (int r = 0; r < n_requests; r++) {
    const size_t plane = align(((size_t)1 << requests[r].n_qubits) * 8);
    o_fc[r] = off;
    off = align(off + (size_t)(plans[r]->F.ncoef + 1) * 8);
    o_bc[r] = off;
    off = align(off + (size_t)(plans[r]->B.ncoef + 1) * 8);
    o_st[r] = off;
    off += 4 * plane;
    o_sl[r] = off;
    off = align(off + (size_t)(plans[r]->B.n_gslots + 1) * 8);
  }
  const size_t total = off;
  // queue order: requests of the lean kernel first, then those of the general
  // one (each request always runs in the same kernel, whatever the mix)
  std::vector<int> pos(n_requests);
  int n_lean = 0;
  for (int r = 0; r < n_requests; r++)
    if (!plans[r]->general) pos[r] = n_lean++;
  for (int r = 0, g = n_lean; r < n_requests; r++)
    if (plans[r]->general) pos[r] = g++;

  // ---- a free staging slot (waits for the run that used it last)
  ServeSlot &sl = sv->slot[sv->next];
  sv->next = (sv->next + 1) % SVS_SLOTS;
  sv_status s = serve_wait(sl);
  if (s) return s;
  if (sl.d_bytes < total) {
    if (sl.d_buf) HIPCHK(hipFree(sl.d_buf));
    sl.d_buf = nullptr;
    sl.d_bytes = 0;
    HIPCHK(hipMalloc(&sl.d_buf, total));
    sl.d_bytes = total;
  }
  if (sl.h_bytes < staged) {
    if (sl.h_buf) HIPCHK(hipHostFree(sl.h_buf));
    sl.h_buf = nullptr;
    sl.h_bytes = 0;
    HIPCHK(hipHostMalloc(&sl.h_buf, staged, hipHostMallocDefault));
    sl.h_bytes = staged;
  }
  char *h = (char *)sl.h_buf;
  char *d = (char *)sl.d_buf;
  std::memset(h, 0, 256);
  ServeReq *hq = (ServeReq *)(h + o_reqs);
  SweepArgs *hs = (SweepArgs *)(h + o_sweeps);
  PauliTermDev *ht = (PauliTermDev *)(h + o_terms);
  int isw = 0;
  size_t it = 0;
  int64_t out_off = 0;
  pofs = 0;
  for (int r = 0; r < n_requests; r++) {
    const sv_circuit_desc &dc = requests[r];
    const Plan &F = plans[r]->F, &B = plans[r]->B;
    const int n = dc.n_qubits, nu = dc.n_params;
    const size_t plane = align(((size_t)1 << n) * 8);
    ServeReq q;
    std::memset(&q, 0, sizeof q);
    q.n = n;
    q.n_params = nu;
    q.f_ndesc = (int)F.coefs.size();
    q.b_ndesc = (int)B.coefs.size();
    q.n_terms = dc.n_terms;
    q.f_desc = F.d_coefdesc;
    q.b_desc = B.d_coefdesc;
    q.f_fac = F.d_factors;
    q.b_fac = B.d_factors;
    q.f_params = (const double *)(d + o_fp[r]);
    q.b_params = (const double *)(d + o_bp[r]);
    q.f_coef = (double *)(d + o_fc[r]);
    q.b_coef = (double *)(d + o_bc[r]);
    q.re = d + o_st[r];
    q.im = d + o_st[r] + plane;
    q.lre = d + o_st[r] + 2 * plane;
    q.lim = d + o_st[r] + 3 * plane;
    q.terms = (const PauliTermDev *)(d + o_terms) + it;
    q.slots = (double *)(d + o_sl[r]);
    q.rowptr = B.d_rowptr;
    q.gslots = B.d_gslots;
    q.out = d_out + out_off;
    out_off += 1 + nu;
    // parameters: the user's, then each plan's constants
    double *fp = (double *)(h + o_fp[r]), *bp = (double *)(h + o_bp[r]);
    if (nu) {
      std::memcpy(fp, params + pofs, (size_t)nu * 8);
      std::memcpy(bp, params + pofs, (size_t)nu * 8);
    }
    if (!F.constants.empty()) std::memcpy(fp + nu, F.constants.data(), F.constants.size() * 8);
    if (!B.constants.empty()) std::memcpy(bp + nu, B.constants.data(), B.constants.size() * 8);
    pofs += nu;
    for (int j = 0; j < dc.n_terms; j++) {
      PauliTermDev t{};
      t.x = dc.terms[j].x_mask;
      t.z = dc.terms[j].z_mask;
      t.c = dc.terms[j].coeff;
      t.term = j;
      ht[it++] = t;
    }
    // forward sweeps (an empty circuit still gets one sweep that writes |0..0>)
    q.f_sweep = isw;
    if (F.steps.empty()) {
      SweepArgs z;
      std::memset(&z, 0, sizeof z);
      const int m = std::min(kServeFwd.M, n), cc = std::min(kServeFwd.c, n);
      z.n = n;
      z.m = m;
      z.c = cc;
      z.nh = m - cc;
      for (int k = 0; k < z.nh; k++) z.hb[k] = cc + k;
      z.ntiles = (int64_t)1 << (n - m);
      z.stages = F.d_stages;
      z.ops = F.d_ops;
      z.coef = q.f_coef;
      z.re = q.re;
      z.im = q.im;
      z.flags = SW_INIT_ZERO;
      hs[isw++] = z;
    } else {
      for (size_t k = 0; k < F.steps.size(); k++) {
        SweepArgs a = F.steps[k].sa;
        a.re = q.re; a.im = q.im; a.re2 = a.im2 = nullptr;
        a.stages = F.d_stages; a.ops = F.d_ops; a.coef = q.f_coef; a.gpart = nullptr;
        if (k == 0) a.flags |= SW_INIT_ZERO;
        hs[isw++] = a;
      }
    }
    q.f_nsweeps = isw - q.f_sweep;
    q.b_sweep = isw;
    for (const Step &st : B.steps) {
      SweepArgs a = st.sa;
      a.re = q.re; a.im = q.im; a.re2 = q.lre; a.im2 = q.lim;
      a.stages = B.d_stages; a.ops = B.d_ops; a.coef = q.b_coef; a.gpart = nullptr;
      hs[isw++] = a;
    }
    q.b_nsweeps = isw - q.b_sweep;
    hq[pos[r]] = q;
  }
  hipStream_t stream = (hipStream_t)hip_stream;
  HIPCHK(hipMemcpyAsync(d, h, staged, hipMemcpyHostToDevice, stream));
  DevInfo di;
  s = device_info(di);
  if (s) return s;
  const ServeReq *d_reqs = (const ServeReq *)(d + o_reqs);
  const SweepArgs *d_sweeps = (const SweepArgs *)(d + o_sweeps);
  hipError_t e = svk_launch_serve_coefs(d_reqs, n_requests, max_desc, stream);
  const int n_gen = n_requests - n_lean;
  if (e == hipSuccess && n_lean)
    e = svk_launch_serve(d_reqs, d_sweeps, (int32_t *)d, n_lean, 0,
                         std::min(n_lean, std::max(1, di.cus)), stream);
  if (e == hipSuccess && n_gen)
    e = svk_launch_serve(d_reqs + n_lean, d_sweeps, (int32_t *)d + 1, n_gen, 1,
                         std::min(n_gen, std::max(1, di.cus)), stream);
  if (e != hipSuccess) return fail(SV_EDEVICE, "serving kernels: %s", hipGetErrorString(e));
  HIPCHK(hipEventRecord(sl.done, stream));
  sl.busy = true;
  sl.held = std::move(plans);
  return SV_OK;
}

extern "C" sv_status sv_serve_free(sv_serve *sv) {
  if (!sv) return SV_OK;
  for (ServeSlot &sl : sv->slot) {
    if (sl.busy) (void)hipEventSynchronize(sl.done);
    if (sl.d_buf) (void)hipFree(sl.d_buf);
    if (sl.h_buf) (void)hipHostFree(sl.h_buf);
    if (sl.done) (void)hipEventDestroy(sl.done);
  }
  delete sv;
  return SV_OK;
}
