// Float32 sampler instances with 64 lanes per chain, one chain per wavefront (components per
// lane, residual entries per lane, prefetch words per thread as listed): for batches of few
// chains, where narrower chains would leave most SIMDs idle.
#include "sample32.h"

namespace asmk {

hipError_t launch_sample32_l64(const SampleArgs &a, int ept, int rpt, int threads, int grid, size_t lds,
                               hipStream_t s) {
    if (ept == 1 && rpt == 4) return launch_sample32_t<64, 1, 4, 0>(a, threads, grid, lds, s);
    if (ept == 2 && rpt == 7) return launch_sample32_t<64, 2, 7, 0>(a, threads, grid, lds, s);
    return hipErrorInvalidValue;
}

hipError_t allow_lds_sample32_l64(int bytes) {
    hipError_t e = hipSuccess, e1;
    if ((e1 = allow_lds_sample32_t<64, 1, 4, 0>(bytes)) != hipSuccess) e = e1;
    if ((e1 = allow_lds_sample32_t<64, 2, 7, 0>(bytes)) != hipSuccess) e = e1;
    return e;
}

}  // namespace asmk
