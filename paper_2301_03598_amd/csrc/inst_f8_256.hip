// Kernel instances: F8 inputs, 256x256 output tiles.
#include "sk_dispatch.hpp"

namespace sk {
KernelEntry pick_f8_256(const KernelKey &k) { return pick<Dt::F8, 256, 256>(k); }
}  // namespace sk
