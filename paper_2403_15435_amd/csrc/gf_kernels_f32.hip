// FP32 instantiation of the patch kernels: state and fluxes in float, wet/dry
// decisions, the wall test and step control in double.
#define REAL float
#define SFX f32
#define KNS k32
#include "gf_kernels.inc"
