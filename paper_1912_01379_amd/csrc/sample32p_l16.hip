// Two-role float32 sampler instance with 16 lanes per chain (512 threads): blocks of up to
// 112 points, problems of up to 208 data points, U rows staged in LDS; prefetch words per
// thread 9 (data rows), 5 (singular values and U rows), 26 (zero rows).
#include "sample32p.h"

namespace asmk {

hipError_t launch_sample32p(const SampleArgs &a, int ept, int rpt, int grid, size_t lds, hipStream_t s) {
    if (ept == 7 && rpt == 13 && a.u_lds) return launch_sample32p_t<16, 7, 13, 9, 5, 26, true>(a, grid, lds, s);
    return hipErrorInvalidValue;
}

int sample32p_pick(int64_t max_nb, int64_t max_m, int u_lds, int *ept, int *rpt, int *pfr, int *pfu, int *pfz) {
    if (!u_lds || max_nb > 7 * 16 || max_m > 13 * 16) return -1;
    *ept = 7;
    *rpt = 13;
    *pfr = 9;
    *pfu = 5;
    *pfz = 26;
    return 0;
}

hipError_t allow_lds_sample32p(int bytes) { return allow_lds_sample32p_t<16, 7, 13, 9, 5, 26, true>(bytes); }

}  // namespace asmk
