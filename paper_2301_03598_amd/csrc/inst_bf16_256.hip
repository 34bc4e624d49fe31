// Kernel instances: BF16 inputs, 256x256 output tiles.
#include "sk_dispatch.hpp"

namespace sk {
KernelEntry pick_bf16_256(const KernelKey &k) { return pick<Dt::BF16, 256, 256>(k); }
}  // namespace sk
