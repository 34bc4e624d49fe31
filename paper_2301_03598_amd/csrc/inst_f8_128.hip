// Kernel instances: F8 inputs, 128x128 output tiles.
#include "sk_dispatch.hpp"

namespace sk {
KernelEntry pick_f8_128(const KernelKey &k) { return pick<Dt::F8, 128, 128>(k); }
}  // namespace sk
