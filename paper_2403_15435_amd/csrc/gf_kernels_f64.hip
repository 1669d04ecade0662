// FP64 instantiation of the patch kernels (the plain comparator path).
#define REAL double
#define SFX f64
#define KNS k64
#include "gf_kernels.inc"
