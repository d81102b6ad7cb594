// MTTKRP kernel instantiations: factors double, entry values double, accumulation double.
#include "mttkrp_kernels.h"

namespace spt {

int launch_mttkrp_f64(const MttkrpArgs &a, int d, const void *const *factors, int G, int CPL) {
    return launch_typed<double, double, double>(a, d, factors, G, CPL);
}

}  // namespace spt
