// phase_n2.hip -- the sweep's phase kernel for PCPD (n = 2). One translation unit
// per model, so that the models' kernel copies compile in parallel.

#include "brs_phase.h"

namespace pcpd {

hipError_t launch_phase_model2(const uint64_t *src, uint64_t *dst, const LatDesc *lats,
                                const TileDesc *tiles, uint32_t ntiles, const uint64_t *clock,
                                uint64_t s_off, uint32_t S, uint32_t B, const PhaseShape &shape,
                                hipStream_t stream) {
    return launch_phase_n<2>(src, dst, lats, tiles, ntiles, clock, s_off, S, B, shape, stream);
}

}  // namespace pcpd
