// Kernel instances: BF16 inputs, 128x128 output tiles.
#include "sk_dispatch.hpp"

namespace sk {
KernelEntry pick_bf16_128(const KernelKey &k) { return pick<Dt::BF16, 128, 128>(k); }
}  // namespace sk
