// Kernel entry points for one configuration; the generated inst_*.hip units
// (one per dtype x tile x operand contiguity) instantiate them so hipcc can
// compile them in parallel, and sk_table.cpp selects among them.
#pragma once
#include "sk_kernel.hpp"

namespace sk {

template <Dt D, int BM, int BN, bool A, bool B, bool G, int NW = 4>
KernelEntry entry(bool dp_only) {
    using C = Cfg<D, BM, BN, A, B, G, NW>;
    return dp_only ? KernelEntry{launch_dp<C>, occupancy_sk<C>}
                   : KernelEntry{launch_sk<C>, occupancy_sk<C>};
}

}  // namespace sk
