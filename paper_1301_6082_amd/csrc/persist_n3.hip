// persist_n3.hip -- the persistent sweep kernel for TCPD (n = 3), in a
// translation unit of its own so that it compiles in parallel with the
// per-phase kernel of the model (phase_n3.hip).

#include "brs_phase.h"

namespace pcpd {

hipError_t launch_persist_model3(const PersistLaunch &a, const PhaseShape &shape,
                                  hipStream_t stream) {
    return launch_persist_n<3>(a, shape, stream);
}

}  // namespace pcpd
