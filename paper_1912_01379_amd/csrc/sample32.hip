// The compiled float32 sampler instances and their selection.
#include "internal.h"

namespace asmk {

namespace {
struct Inst32 {
    int L, EPT, RPT, PF;
};
// (lanes per chain, components per lane, residual entries per lane, prefetch words per
// thread): a block of up to EPT L grid points and a problem of up to RPT L data points
const Inst32 kInst32[] = {
    {4, 8, 16, 0}, {4, 32, 16, 0}, {4, 32, 52, 0}, {8, 4, 8, 0}, {8, 13, 26, 0}, {8, 16, 8, 0}, {8, 16, 52, 0},
    {16, 2, 4, 0}, {16, 7, 13, 26}, {16, 8, 4, 0}, {16, 8, 13, 0}, {16, 8, 26, 0}, {16, 8, 32, 0}, {32, 1, 2, 0},
    {32, 4, 2, 0}, {32, 4, 7, 0}, {32, 4, 13, 0}, {64, 1, 4, 0}, {64, 2, 7, 0}};
}  // namespace

int sample32_pick(int lanes, int64_t max_nb, int64_t max_m, int hier, int *ept, int *rpt, int *pf) {
    int best = -1;
    for (int k = 0; k < (int)(sizeof kInst32 / sizeof kInst32[0]); ++k) {
        const Inst32 &c = kInst32[k];
        if (c.L != lanes || (int64_t)c.EPT * c.L < max_nb || (int64_t)c.RPT * c.L < max_m) continue;
        if (hier && c.PF > 0) continue;   // hierarchies: non-prefetching instances only
        // the least per-lane work: 4 operations per component, 2 per residual entry
        if (best < 0 || 2 * c.EPT + c.RPT < 2 * kInst32[best].EPT + kInst32[best].RPT) best = k;
    }
    if (best < 0) return -1;
    *ept = kInst32[best].EPT;
    *rpt = kInst32[best].RPT;
    *pf = kInst32[best].PF;
    return 0;
}

hipError_t launch_sample32_inst(const SampleArgs &a, int lanes, int ept, int rpt, int chains_per_wg,
                                int grid, size_t lds_bytes, hipStream_t s) {
    const int threads = lanes * chains_per_wg;
    if (threads % 64 != 0 || threads > 512) return hipErrorInvalidValue;
    // prefetching instances are compiled for at most 256 threads
    for (const Inst32 &c : kInst32)
        if (c.L == lanes && c.EPT == ept && c.RPT == rpt && c.PF > 0 && threads > 256) return hipErrorInvalidValue;
    switch (lanes) {
    case 4: return launch_sample32_l4(a, ept, rpt, threads, grid, lds_bytes, s);
    case 8: return launch_sample32_l8(a, ept, rpt, threads, grid, lds_bytes, s);
    case 16: return launch_sample32_l16(a, ept, rpt, threads, grid, lds_bytes, s);
    case 32: return launch_sample32_l32(a, ept, rpt, threads, grid, lds_bytes, s);
    case 64: return launch_sample32_l64(a, ept, rpt, threads, grid, lds_bytes, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t set_sample32_lds_limit(int bytes) {
    hipError_t e = hipSuccess, e1;
    if ((e1 = allow_lds_sample32_l4(bytes)) != hipSuccess) e = e1;
    if ((e1 = allow_lds_sample32_l8(bytes)) != hipSuccess) e = e1;
    if ((e1 = allow_lds_sample32_l16(bytes)) != hipSuccess) e = e1;
    if ((e1 = allow_lds_sample32_l32(bytes)) != hipSuccess) e = e1;
    if ((e1 = allow_lds_sample32_l64(bytes)) != hipSuccess) e = e1;
    return e;
}

}  // namespace asmk
