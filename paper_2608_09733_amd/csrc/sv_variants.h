// The tile-sweep kernel instantiations: (element type, tile bits M, register
// group bits R, number of states NS).  Each is compiled in its own translation
// unit (sv_sweep_variant.hip with -DSVI_V=<index>).
#pragma once

#define SVI_VARIANTS(X)      \
  X(double, 13, 5, 1)        \
  X(double, 12, 5, 1)        \
  X(double, 13, 4, 1)        \
  X(double, 12, 4, 1)        \
  X(double, 12, 3, 1)        \
  X(double, 13, 3, 1)        \
  X(double, 11, 4, 1)        \
  X(double, 11, 3, 1)        \
  X(double, 11, 5, 1)        \
  X(double, 12, 4, 2)        \
  X(double, 11, 4, 2)        \
  X(double, 12, 3, 2)        \
  X(double, 11, 3, 2)        \
  X(float, 14, 5, 1)         \
  X(float, 13, 5, 1)         \
  X(float, 13, 4, 2)

#define SVI_NVARIANTS 16
#define SVI_VCAT(a, b, c, d, e, f) svk_##a##_##b##_##c##_##d##_##e##f
#define SVI_VNAME(what, T, M, R, NS) SVI_VCAT(what, T, M, R, NS, _v)

// The persistent ragged-batch kernel instantiations: (element type, tile bits
// M, register group bits R), one translation unit each
// (sv_batch_variant.hip with -DSVB_VT= -DSVB_VM= -DSVB_VR=).
#define SVB_VARIANTS(X) \
  X(double, 13, 3)      \
  X(double, 13, 5)      \
  X(float, 13, 3)       \
  X(float, 13, 5)

#define SVB_VCAT(a, b, c, d, e) svb_##a##_##b##_##c##_##d##e
#define SVB_VNAME(what, T, M, R) SVB_VCAT(what, T, M, R, _v)
