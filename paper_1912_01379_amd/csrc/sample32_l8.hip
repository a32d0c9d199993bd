// Float32 sampler instances with 8 lanes per chain (components per lane, residual
// entries per lane, prefetch words per thread as listed).
#include "sample32.h"

namespace asmk {

hipError_t launch_sample32_l8(const SampleArgs &a, int ept, int rpt, int threads, int grid, size_t lds,
                               hipStream_t s) {
    if (ept == 4 && rpt == 8) return launch_sample32_t<8, 4, 8, 0>(a, threads, grid, lds, s);
    if (ept == 13 && rpt == 26) return launch_sample32_t<8, 13, 26, 0>(a, threads, grid, lds, s);
    if (ept == 16 && rpt == 52) return launch_sample32_t<8, 16, 52, 0>(a, threads, grid, lds, s);
    if (ept == 16 && rpt == 8) return launch_sample32_t<8, 16, 8, 0>(a, threads, grid, lds, s);
    return hipErrorInvalidValue;
}

hipError_t allow_lds_sample32_l8(int bytes) {
    hipError_t e = hipSuccess, e1;
    if ((e1 = allow_lds_sample32_t<8, 4, 8, 0>(bytes)) != hipSuccess) e = e1;
    if ((e1 = allow_lds_sample32_t<8, 13, 26, 0>(bytes)) != hipSuccess) e = e1;
    if ((e1 = allow_lds_sample32_t<8, 16, 52, 0>(bytes)) != hipSuccess) e = e1;
    if ((e1 = allow_lds_sample32_t<8, 16, 8, 0>(bytes)) != hipSuccess) e = e1;
    return e;
}

}  // namespace asmk
