// Sweep instantiations of the MIXED path (BF16 Gram, FP32 storage, FP64
// aggregates; messages in FP64 with exact reciprocals, in FP32 with series
// reciprocals): stored pair records, or stateless with 1..8 levels (1..6
// with series reciprocals), over the materialised or recomputed K'.
#include "gabp_device.h"

namespace gabp {

hipError_t launch_sweep_mixed(int ksrc, int gram, int levels, bool first, int ser, const SweepArgs& a,
                              hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (ksrc == KSRC_PLANE) return sweep_depth<float, double, double, KSRC_PLANE, GRAM_F32>(levels, first, ser, a, s, e0, e1);
    switch (gram) {
        case GRAM_BF16: return sweep_depth<float, double, double, KSRC_RECOMPUTE, GRAM_BF16>(levels, first, ser, a, s, e0, e1);
        case GRAM_BF16X3: return sweep_depth<float, double, double, KSRC_RECOMPUTE, GRAM_BF16X3>(levels, first, ser, a, s, e0, e1);
        case GRAM_BF16X6: return sweep_depth<float, double, double, KSRC_RECOMPUTE, GRAM_BF16X6>(levels, first, ser, a, s, e0, e1);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_served_sweep_mixed(int levels, int ser, bool grouped, const ReqDesc* reqs, const uint2* items,
                                     int n, hipStream_t s) {
    return served_sweep<float, double, double>(levels, ser, grouped, reqs, items, n, s);
}

hipError_t launch_sweep_grouped_mixed(int ksrc, int gram, int levels, int ser, const SweepArgs& a,
                                   const uint32_t* within, int nwithin, const uint32_t* dir, int ndir, int t,
                                   hipStream_t s) {
    if (ksrc == KSRC_PLANE)
        return sweep_grouped<float, double, double, KSRC_PLANE, GRAM_F32>(levels, ser, a, within, nwithin, dir, ndir, t, s);
    switch (gram) {
        case GRAM_BF16: return sweep_grouped<float, double, double, KSRC_RECOMPUTE, GRAM_BF16>(levels, ser, a, within, nwithin, dir, ndir, t, s);
        case GRAM_BF16X3: return sweep_grouped<float, double, double, KSRC_RECOMPUTE, GRAM_BF16X3>(levels, ser, a, within, nwithin, dir, ndir, t, s);
        case GRAM_BF16X6: return sweep_grouped<float, double, double, KSRC_RECOMPUTE, GRAM_BF16X6>(levels, ser, a, within, nwithin, dir, ndir, t, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace gabp
