// Persistent ragged-batch kernel (one instantiation per translation unit,
// selected with -DSVB_VT=double -DSVB_VM=13 -DSVB_VR=3; one entry of
// SVB_VARIANTS).
//
// The paper evolves a batch of equally sized states together (Section 4.1,
// batched state vector).  Here the circuits of a batch may differ in qubit
// count and depth, so instead of one tensor the batch is a device queue of
// work units -- a range of tiles of one sweep, or of one Pauli pass, of one
// circuit -- drained by a single persistent launch.  Each workgroup takes the
// next unit with an atomic counter, waits (bounded) until the circuit's
// earlier units are complete, runs it, and publishes its completion.  Small
// circuits (n <= tile bits) are one unit each: the whole circuit runs in LDS.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "sv_device.h"
#include "sv_variants.h"

#if !defined(SVB_VT) || !defined(SVB_VM) || !defined(SVB_VR)
#error "compile with -DSVB_VT= -DSVB_VM= -DSVB_VR="
#endif

#define SVB_PTERMS 64   // terms per Pauli pass (the host planner's limit)

namespace svk {
namespace {

template <typename T, int M, int R>
struct BatchLds {
  typename C2T<T>::type tile[1 << M];
  double wsum[(1 << (M - R)) / 64][SVB_PTERMS];
  double tacc[SVB_PTERMS];
  uint32_t xl[SVB_PTERMS], zl[SVB_PTERMS];
  int32_t hb[SVI_MMAX];
  int32_t unit;
};

// Tiles [t0, t1) of one Pauli pass: per-term sums of
// Re conj(psi_{b^x}) i^{nY} (-1)^{popcount(b & z)} psi_b over the tiles' b
// (paper Section 4.4), written to out[term of the pass].
template <typename T, int M, int R>
__device__ void pauli_tiles(const SVI_CONST PauliPassArgs &p, int64_t t0, int64_t t1, double *out,
                            BatchLds<T, M, R> &L) {
  constexpr int NT = 1 << (M - R);
  constexpr int EPT = (1 << M) / NT;
  constexpr int NWAVE = NT / 64;
  using C2 = typename C2T<T>::type;
  const int tid = threadIdx.x;
  const int m = p.m, c = p.c, nh = p.nh;
  const int nel = 1 << m;
  const int nterm = p.t_end - p.t_begin;
  const SVI_CONST PauliTermDev *terms = cptr(p.terms) + p.t_begin;
  const T *pre = (const T *)p.re, *pim = (const T *)p.im;

  if (tid < SVI_MMAX) L.hb[tid] = p.hb[tid < nh ? tid : 0];
  for (int t = tid; t < nterm; t += NT) {
    const uint64_t x = p.terms[p.t_begin + t].x, z = p.terms[p.t_begin + t].z;
    uint32_t xl = 0, zl = 0;
    for (int b = 0; b < c; b++) {
      xl |= (uint32_t)((x >> b) & 1) << b;
      zl |= (uint32_t)((z >> b) & 1) << b;
    }
    for (int k = 0; k < nh; k++) {
      xl |= (uint32_t)((x >> p.hb[k]) & 1) << (c + k);
      zl |= (uint32_t)((z >> p.hb[k]) & 1) << (c + k);
    }
    L.xl[t] = xl;
    L.zl[t] = zl;
    L.tacc[t] = 0.0;
  }
  __syncthreads();

  for (int64_t tile = t0; tile < t1; tile++) {
    const uint64_t base = tile_base(tile, c, L.hb, nh);
    for (int i = tid; i < nel; i += NT) {
      const uint64_t g = base + spread_row(i >> c, L.hb, nh) + (uint64_t)(i & ((1 << c) - 1));
      L.tile[swz<T>(i)] = C2{pre[g], pim[g]};
    }
    __syncthreads();
    for (int t = 0; t < nterm; t++) {
      const uint64_t x = terms[t].x, z = terms[t].z;
      const uint32_t xl = L.xl[t], zl = L.zl[t];
      const int ny = __builtin_popcountll(x & z) & 3;
      const bool bneg = __builtin_popcountll(base & z) & 1;
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < EPT; k++) {
        const int i = tid + k * NT;
        if (i < nel) {
          const C2 pb = L.tile[swz<T>(i)];
          const C2 pp = L.tile[swz<T>(i ^ (int)xl)];
          const double wr = (double)pb.x, wi = (double)pb.y;
          double tr, ti;
          switch (ny) {
            case 0: tr = wr; ti = wi; break;
            case 1: tr = -wi; ti = wr; break;
            case 2: tr = -wr; ti = -wi; break;
            default: tr = wi; ti = -wr; break;
          }
          const bool neg = bneg ^ (bool)(__builtin_popcount((uint32_t)i & zl) & 1);
          const double v = (double)pp.x * tr + (double)pp.y * ti;
          acc = neg ? acc - v : acc + v;
        }
      }
      acc = wave_sum(acc);
      if ((tid & 63) == 0) L.wsum[tid >> 6][t] = acc;
    }
    __syncthreads();
    for (int t = tid; t < nterm; t += NT) {
      double v = 0.0;
      for (int w = 0; w < NWAVE; w++) v += L.wsum[w][t];
      L.tacc[t] += v;
    }
    __syncthreads();
  }
  for (int t = tid; t < nterm; t += NT) out[t] = L.tacc[t];
}

template <typename T, int M, int R, bool KO>
__global__ void __launch_bounds__(1 << (M - R)) k_batch(BatchKernelArgs b) {
  static_assert(M - R >= 6, "workgroups of whole waves");
  __shared__ BatchLds<T, M, R> L;
  const int tid = threadIdx.x;
  // Queue and counter traffic is done by wave 0 as a whole wave (one lane
  // contributes, the others add 0), never under a lane-divergent branch: every
  // branch in this loop is uniform within each wave, so however the compiler
  // lays out the loop, each wave meets each barrier once per unit.
  const bool wave0 = __builtin_amdgcn_readfirstlane(tid) == 0;
  const int one = tid == 0 ? 1 : 0;
  for (;;) {
    if (wave0) {
      const int v = __hip_atomic_fetch_add(b.head, one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      L.unit = __builtin_amdgcn_readfirstlane(v);
    }
    __syncthreads();
    const int u = __builtin_amdgcn_readfirstlane(L.unit);
    if (u >= b.nunits) break;
    const SVI_CONST BatchUnit &un = cptr(b.units)[u];
    const int need = un.wait, circ = un.circ;
    if (wave0 && need > 0) {
      // Bounded wait for the circuit's earlier units.  Every unit this one
      // depends on precedes it in the queue and was taken by a running
      // workgroup, so the wait ends; the bound turns a broken plan into an
      // error flag instead of a hang.  The polls are relaxed agent-scope loads
      // (coherent across XCDs, no cache maintenance per poll); the acquire
      // fence below runs once, after the wait.
      bool expired = b.spin_limit < 0;
      for (int32_t spins = 0; !expired; spins++) {
        const int d = __builtin_amdgcn_readfirstlane(
            __hip_atomic_load(b.done + circ, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (d >= need) break;
        if (spins >= b.spin_limit) expired = true;
        else __builtin_amdgcn_s_sleep(32);
      }
      if (expired) __hip_atomic_fetch_or(b.err, one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    // acquire: the producers' state writes are visible to this wave's loads
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (un.kind == UK_SWEEP)
      sweep_tiles<T, M, R, KO>(cptr(b.sweeps)[un.arg], un.t0, un.t1, L.tile, L.hb);
    else
      pauli_tiles<T, M, R>(cptr(b.passes)[un.arg], un.t0, un.t1, b.part + un.part, L);
    // release: this wave's writes are visible device-wide before the count
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (wave0) __hip_atomic_fetch_add(b.done + circ, one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

}  // namespace
}  // namespace svk

hipError_t SVB_VNAME(launch, SVB_VT, SVB_VM, SVB_VR)(const BatchKernelArgs &a, int grid,
                                                    int kron_only, hipStream_t s) {
  if (kron_only)
    hipLaunchKernelGGL((svk::k_batch<SVB_VT, SVB_VM, SVB_VR, true>), dim3(grid),
                       dim3(1 << (SVB_VM - SVB_VR)), 0, s, a);
  else
    hipLaunchKernelGGL((svk::k_batch<SVB_VT, SVB_VM, SVB_VR, false>), dim3(grid),
                       dim3(1 << (SVB_VM - SVB_VR)), 0, s, a);
  return hipGetLastError();
}

int SVB_VNAME(occ, SVB_VT, SVB_VM, SVB_VR)(int kron_only) {
  int nb = 0;
  const hipError_t e =
      kron_only ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                      &nb, svk::k_batch<SVB_VT, SVB_VM, SVB_VR, true>, 1 << (SVB_VM - SVB_VR), 0)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                      &nb, svk::k_batch<SVB_VT, SVB_VM, SVB_VR, false>, 1 << (SVB_VM - SVB_VR), 0);
  if (e != hipSuccess) return 1;
  return nb > 0 ? nb : 1;
}
