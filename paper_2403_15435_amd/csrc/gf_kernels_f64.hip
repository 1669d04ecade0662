// FP64 instantiation of the patch kernels (the plain comparator path).
#define REAL double
#define SFX f64
#define KNS k64
#define GF_RIEMANN_FP64 0
#include "gf_kernels.inc"
