// One tile-sweep instantiation per translation unit, selected on the command
// line (-DSVI_VT=double -DSVI_VM=13 -DSVI_VR=5 -DSVI_VNS=1; one entry of
// SVI_VARIANTS), so the variants compile in parallel.
#include <hip/hip_runtime.h>

#include "sv_device.h"
#include "sv_variants.h"

#if !defined(SVI_VT) || !defined(SVI_VM) || !defined(SVI_VR) || !defined(SVI_VNS)
#error "compile with -DSVI_VT= -DSVI_VM= -DSVI_VR= -DSVI_VNS="
#endif

hipError_t SVI_VNAME(launch, SVI_VT, SVI_VM, SVI_VR, SVI_VNS)(const SweepArgs &a, int grid,
                                                              hipStream_t s) {
  hipLaunchKernelGGL((svk::k_sweep<SVI_VT, SVI_VM, SVI_VR, SVI_VNS>), dim3(grid),
                     dim3(1 << (SVI_VM - SVI_VR)), 0, s, a);
  return hipGetLastError();
}

int SVI_VNAME(occ, SVI_VT, SVI_VM, SVI_VR, SVI_VNS)() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &nb, svk::k_sweep<SVI_VT, SVI_VM, SVI_VR, SVI_VNS>, 1 << (SVI_VM - SVI_VR), 0) !=
      hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

#if SVI_VNS != 1
hipError_t SVI_VNAME(launchk, SVI_VT, SVI_VM, SVI_VR, SVI_VNS)(const SweepArgs &a, int grid,
                                                               hipStream_t s) {
  hipLaunchKernelGGL((svk::k_sweep_kron2<SVI_VT, SVI_VM, SVI_VR>), dim3(grid),
                     dim3(1 << (SVI_VM - SVI_VR)), 0, s, a);
  return hipGetLastError();
}

int SVI_VNAME(occk, SVI_VT, SVI_VM, SVI_VR, SVI_VNS)() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &nb, svk::k_sweep_kron2<SVI_VT, SVI_VM, SVI_VR>, 1 << (SVI_VM - SVI_VR), 0) != hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}
#else
hipError_t SVI_VNAME(launchk, SVI_VT, SVI_VM, SVI_VR, SVI_VNS)(const SweepArgs &a, int grid,
                                                               hipStream_t s) {
  hipLaunchKernelGGL((svk::k_sweep_kron<SVI_VT, SVI_VM, SVI_VR>), dim3(grid),
                     dim3(1 << (SVI_VM - SVI_VR)), 0, s, a);
  return hipGetLastError();
}

int SVI_VNAME(occk, SVI_VT, SVI_VM, SVI_VR, SVI_VNS)() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &nb, svk::k_sweep_kron<SVI_VT, SVI_VM, SVI_VR>, 1 << (SVI_VM - SVI_VR), 0) != hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}
#endif
