// Two-role float32 sampler instances with 16 lanes per chain (512 threads): problems of up to
// 208 data points with blocks of up to 112 points and the U rows staged in LDS (prefetch words
// per thread 9 for the data rows, 5 for the singular values and U rows, 26 for the zero rows);
// blocks of up to 128 points with the U rows read from global memory, for problems of up to 208
// data points (13, 1 and 24) and of up to 416 (14, 1 and 24).
#include "sample32p.h"

namespace asmk {

hipError_t launch_sample32p(const SampleArgs &a, int ept, int rpt, int grid, size_t lds, hipStream_t s) {
    if (ept == 7 && rpt == 13 && a.u_lds) return launch_sample32p_t<16, 7, 13, 9, 5, 26, true>(a, grid, lds, s);
    if (ept == 8 && rpt == 13 && !a.u_lds) return launch_sample32p_t<16, 8, 13, 13, 1, 24, false>(a, grid, lds, s);
    if (ept == 8 && rpt == 26 && !a.u_lds) return launch_sample32p_t<16, 8, 26, 14, 1, 24, false>(a, grid, lds, s);
    return hipErrorInvalidValue;
}

int sample32p_pick(int64_t max_nb, int64_t max_m, int u_lds, int *ept, int *rpt, int *pfr, int *pfu, int *pfz) {
    if (max_m > 26 * 16) return -1;
    if (u_lds && max_nb <= 7 * 16 && max_m <= 13 * 16) {
        *ept = 7;
        *rpt = 13;
        *pfr = 9;
        *pfu = 5;
        *pfz = 26;
        return 0;
    }
    if (!u_lds && max_nb <= 8 * 16) {
        *ept = 8;
        *rpt = max_m <= 13 * 16 ? 13 : 26;
        *pfr = max_m <= 13 * 16 ? 13 : 14;
        *pfu = 1;
        *pfz = 24;
        return 0;
    }
    return -1;
}

hipError_t allow_lds_sample32p(int bytes) {
    hipError_t e = allow_lds_sample32p_t<16, 7, 13, 9, 5, 26, true>(bytes);
    const hipError_t e1 = allow_lds_sample32p_t<16, 8, 13, 13, 1, 24, false>(bytes);
    const hipError_t e2 = allow_lds_sample32p_t<16, 8, 26, 14, 1, 24, false>(bytes);
    return e != hipSuccess ? e : e1 != hipSuccess ? e1 : e2;
}

}  // namespace asmk
