// FP32 instantiation of the patch kernels: state and fluxes in float, wet/dry
// decisions, the wall test and step control in double.
#define REAL float
#define SFX f32
#define KNS k32
#ifndef GF_RIEMANN_FP64
#define GF_RIEMANN_FP64 1
#endif
#include "gf_kernels.inc"
