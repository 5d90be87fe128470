// Sweep instantiations of the FP64 path: stored pair records, or
// stateless with 1..8 levels (1..6 with series reciprocals), over the
// materialised or recomputed K'.
#include "gabp_device.h"

namespace gabp {

hipError_t launch_sweep_f64(int ksrc, int gram, int levels, bool first, int ser, const SweepArgs& a,
                              hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (ksrc == KSRC_PLANE) return sweep_depth<double, double, double, KSRC_PLANE, GRAM_F64>(levels, first, ser, a, s, e0, e1);
    (void)gram;
    return hipErrorInvalidValue;   // FP64 K' is always materialised
}

hipError_t launch_served_sweep_f64(int levels, int ser, bool grouped, const ReqDesc* reqs, const uint2* items,
                                     int n, hipStream_t s) {
    return served_sweep<double, double, double>(levels, ser, grouped, reqs, items, n, s);
}

hipError_t launch_sweep_grouped_f64(int ksrc, int gram, int levels, int ser, const SweepArgs& a,
                                   const uint32_t* within, int nwithin, const uint32_t* dir, int ndir, int t,
                                   hipStream_t s) {
    if (ksrc == KSRC_PLANE)
        return sweep_grouped<double, double, double, KSRC_PLANE, GRAM_F64>(levels, ser, a, within, nwithin, dir, ndir, t, s);
    return hipErrorInvalidValue;
}

}  // namespace gabp
