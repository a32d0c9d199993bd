// Float32 sampler instances with 16 lanes per chain (components per lane, residual
// entries per lane, prefetch words per thread as listed).
#include "sample32.h"

namespace asmk {

hipError_t launch_sample32_l16(const SampleArgs &a, int ept, int rpt, int threads, int grid, size_t lds,
                               hipStream_t s) {
    if (ept == 2 && rpt == 4) return launch_sample32_t<16, 2, 4, 0>(a, threads, grid, lds, s);
    if (ept == 7 && rpt == 13) return launch_sample32_t<16, 7, 13, 26>(a, threads, grid, lds, s);
    if (ept == 8 && rpt == 13) return launch_sample32_t<16, 8, 13, 0>(a, threads, grid, lds, s);
    if (ept == 8 && rpt == 26) return launch_sample32_t<16, 8, 26, 0>(a, threads, grid, lds, s);
    if (ept == 8 && rpt == 32) return launch_sample32_t<16, 8, 32, 0>(a, threads, grid, lds, s);
    if (ept == 8 && rpt == 4) return launch_sample32_t<16, 8, 4, 0>(a, threads, grid, lds, s);
    return hipErrorInvalidValue;
}

hipError_t allow_lds_sample32_l16(int bytes) {
    hipError_t e = hipSuccess, e1;
    if ((e1 = allow_lds_sample32_t<16, 2, 4, 0>(bytes)) != hipSuccess) e = e1;
    if ((e1 = allow_lds_sample32_t<16, 7, 13, 26>(bytes)) != hipSuccess) e = e1;
    if ((e1 = allow_lds_sample32_t<16, 8, 13, 0>(bytes)) != hipSuccess) e = e1;
    if ((e1 = allow_lds_sample32_t<16, 8, 26, 0>(bytes)) != hipSuccess) e = e1;
    if ((e1 = allow_lds_sample32_t<16, 8, 32, 0>(bytes)) != hipSuccess) e = e1;
    if ((e1 = allow_lds_sample32_t<16, 8, 4, 0>(bytes)) != hipSuccess) e = e1;
    return e;
}

}  // namespace asmk
