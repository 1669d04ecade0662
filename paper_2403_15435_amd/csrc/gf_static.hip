// Device scratch of the entry point that allocates nothing (gf_mass_static):
// a file-scope array in device memory, one copy per GPU, whose address each
// context takes once at creation on its own device.  Host code uses only that
// address (the array's name is a host-side stand-in, not a device address).
#include "gf_internal.h"


namespace gf {

// per-patch partial volumes, then the three results of the last call
static __device__ __align__(256) double scratch[kStaticMassPatches + 64];

// The scenario's volume, clamp volume and boundary volume from the per-patch
// partials: a Neumaier sum over its patches in leaf order (the work list is
// in scenario, then leaf order) and plain sums of the per-slot accumulators
// from the scenario's running totals, the same operations in the same order
// as gf_mass does them on the host.  One workgroup: 256 entries at a time are
// staged in LDS, then one thread adds them in order.
__global__ void __launch_bounds__(256) mass_ordered_kernel(const double *part, const PatchDesc *d, int nw, int scen,
                                                           const double *ca, const double *ba, double clamp_base,
                                                           double bnd_base, double *res)
{
    __shared__ double sv[256], sc_[256], sb[256];
    __shared__ int use[256];
    double S = 0.0, C = 0.0, cl = clamp_base, bd = bnd_base;
    for (int base = 0; base < nw; base += 256) {
        const int k = base + (int)threadIdx.x;
        if (k < nw) {
            const PatchDesc &P = d[k];
            use[threadIdx.x] = P.scen == scen;
            sv[threadIdx.x] = part[k];
            sc_[threadIdx.x] = ca[P.slot];
            sb[threadIdx.x] = ba[P.slot];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            const int n = min(256, nw - base);
            for (int i = 0; i < n; ++i) {
                if (!use[i]) continue;
                const double v = sv[i], t = S + v;
                if (fabs(S) >= fabs(v)) C += (S - t) + v; else C += (v - t) + S;
                S = t;
                cl += sc_[i];
                bd += sb[i];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        res[0] = S + C;
        res[1] = cl;
        res[2] = bd;
    }
}

}  // namespace gf

using namespace gf;

hipError_t gf_static_scratch(double **ptr)
{
    // the address of this device's copy; asked once per context at creation,
    // with the context's device current
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    *ptr = (double *)p;
    return hipSuccess;
}

hipError_t gf_launch_mass_ordered(const double *part, const PatchDesc *d, int nw, int scen, const double *ca,
                                  const double *ba, double clamp_base, double bnd_base, double *res, hipStream_t s)
{
    hipLaunchKernelGGL(mass_ordered_kernel, dim3(1), dim3(256), 0, s, part, d, nw, scen, ca, ba, clamp_base, bnd_base,
                       res);
    return hipGetLastError();
}
