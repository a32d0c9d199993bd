// Float32 sampler instances with 32 lanes per chain (components per lane, residual
// entries per lane, prefetch words per thread as listed).
#include "sample32.h"

namespace asmk {

hipError_t launch_sample32_l32(const SampleArgs &a, int ept, int rpt, int threads, int grid, size_t lds,
                               hipStream_t s) {
    if (ept == 1 && rpt == 2) return launch_sample32_t<32, 1, 2, 0>(a, threads, grid, lds, s);
    if (ept == 4 && rpt == 7) return launch_sample32_t<32, 4, 7, 0>(a, threads, grid, lds, s);
    if (ept == 4 && rpt == 13) return launch_sample32_t<32, 4, 13, 0>(a, threads, grid, lds, s);
    if (ept == 4 && rpt == 2) return launch_sample32_t<32, 4, 2, 0>(a, threads, grid, lds, s);
    return hipErrorInvalidValue;
}

hipError_t allow_lds_sample32_l32(int bytes) {
    hipError_t e = hipSuccess, e1;
    if ((e1 = allow_lds_sample32_t<32, 1, 2, 0>(bytes)) != hipSuccess) e = e1;
    if ((e1 = allow_lds_sample32_t<32, 4, 7, 0>(bytes)) != hipSuccess) e = e1;
    if ((e1 = allow_lds_sample32_t<32, 4, 13, 0>(bytes)) != hipSuccess) e = e1;
    if ((e1 = allow_lds_sample32_t<32, 4, 2, 0>(bytes)) != hipSuccess) e = e1;
    return e;
}

}  // namespace asmk
