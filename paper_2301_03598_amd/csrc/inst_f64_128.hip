// Kernel instances: F64 inputs, 128x128 output tiles.
#include "sk_dispatch.hpp"

namespace sk {
KernelEntry pick_f64_128(const KernelKey &k) { return pick<Dt::F64, 128, 128>(k); }
}  // namespace sk
