// MTTKRP kernel instantiations: factors uint16_t, entry values float, accumulation float.
#include "mttkrp_kernels.h"

namespace spt {

int launch_mttkrp_bf16(const MttkrpArgs &a, int d, const void *const *factors, int G, int CPL) {
    return launch_typed<uint16_t, float, float>(a, d, factors, G, CPL);
}

}  // namespace spt
