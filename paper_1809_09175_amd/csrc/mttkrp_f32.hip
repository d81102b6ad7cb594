// MTTKRP kernel instantiations: factors float, entry values float, accumulation float.
#include "mttkrp_kernels.h"

namespace spt {

int launch_mttkrp_f32(const MttkrpArgs &a, int d, const void *const *factors, int G, int CPL) {
    return launch_typed<float, float, float>(a, d, factors, G, CPL);
}

}  // namespace spt
