// The eight-lane float32 sampler (sample32w.h): instances and their choice.
#include "sample32w.h"

namespace asmk {

// (EPT, RPT): components and residual entries per lane; blocks of up to 8 EPT points and up
// to 8 RPT data points
hipError_t launch_sample32w(const SampleArgs &a, int ept, int rpt, int grid, size_t lds, hipStream_t s) {
    if (ept == 16 && rpt == 28) return launch_sample32w_t<8, 16, 28>(a, grid, lds, s);
    if (ept == 16 && rpt == 52) return launch_sample32w_t<8, 16, 52>(a, grid, lds, s);
    return hipErrorInvalidValue;
}

// the smallest instance for the sizes; data modes per block at most 32 (the uniforms of the
// data moves come from one Philox call per lane)
int sample32w_pick(int64_t max_nb, int64_t max_m, int64_t max_kb, int *ept, int *rpt) {
    if (max_nb > 16 * 8 || max_kb > 32) return -1;
    if (max_m <= 28 * 8) {
        *ept = 16;
        *rpt = 28;
        return 0;
    }
    if (max_m <= 52 * 8) {
        *ept = 16;
        *rpt = 52;
        return 0;
    }
    return -1;
}

hipError_t allow_lds_sample32w(int bytes) {
    hipError_t e = allow_lds_sample32w_t<8, 16, 28>(bytes);
    const hipError_t e1 = allow_lds_sample32w_t<8, 16, 52>(bytes);
    return e != hipSuccess ? e : e1;
}

}  // namespace asmk
