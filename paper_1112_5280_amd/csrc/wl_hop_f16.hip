// wl_hop_f16.hip -- the hopping-term kernels for FP16 storage (one translation unit
// per precision so the kernel variants compile in parallel).
#include "wl_hop.h"

namespace wl {

hipError_t launch_storage_f16(const Geom &g, int prec, bool link12, const Phases &ph,
                              const HopCall &call, int red, hipStream_t s) {
    return launch_storage<Half>(g, prec, link12, ph, call, red, s);
}

}  // namespace wl
