// Float32 sampler instances with 4 lanes per chain (components per lane, residual
// entries per lane, prefetch words per thread as listed).
#include "sample32.h"

namespace asmk {

hipError_t launch_sample32_l4(const SampleArgs &a, int ept, int rpt, int threads, int grid, size_t lds,
                               hipStream_t s) {
    if (ept == 8 && rpt == 16) return launch_sample32_t<4, 8, 16, 0>(a, threads, grid, lds, s);
    if (ept == 32 && rpt == 52) return launch_sample32_t<4, 32, 52, 0>(a, threads, grid, lds, s);
    if (ept == 32 && rpt == 16) return launch_sample32_t<4, 32, 16, 0>(a, threads, grid, lds, s);
    return hipErrorInvalidValue;
}

hipError_t allow_lds_sample32_l4(int bytes) {
    hipError_t e = hipSuccess, e1;
    if ((e1 = allow_lds_sample32_t<4, 8, 16, 0>(bytes)) != hipSuccess) e = e1;
    if ((e1 = allow_lds_sample32_t<4, 32, 52, 0>(bytes)) != hipSuccess) e = e1;
    if ((e1 = allow_lds_sample32_t<4, 32, 16, 0>(bytes)) != hipSuccess) e = e1;
    return e;
}

}  // namespace asmk
