// Kernel instances: F64 inputs, 64x64 output tiles.
#include "sk_dispatch.hpp"

namespace sk {
KernelEntry pick_f64_64(const KernelKey &k) { return pick<Dt::F64, 64, 64>(k); }
}  // namespace sk
