// Instance tables: one translation unit per (dtype, tile) so the kernels
// compile in parallel.  Each unit builds the sk_kernel / dp_kernel pairs for
// both operand contiguities and for single and grouped launches.
#pragma once
#include "sk_kernel.hpp"

namespace sk {

template <Dt D, int BM, int BN, bool A, bool B, bool G>
KernelEntry entry(bool dp_only) {
    using C = Cfg<D, BM, BN, A, B, G>;
    return dp_only ? KernelEntry{launch_dp<C>, occupancy_sk<C>}
                   : KernelEntry{launch_sk<C>, occupancy_sk<C>};
}

template <Dt D, int BM, int BN>
KernelEntry pick(const KernelKey &k) {
    if (k.bm != BM || k.bn != BN) return KernelEntry{nullptr, nullptr};
    if (k.grouped) {
        if (k.a_kc) return k.b_kc ? entry<D, BM, BN, true, true, true>(k.dp_only)
                                  : entry<D, BM, BN, true, false, true>(k.dp_only);
        return k.b_kc ? entry<D, BM, BN, false, true, true>(k.dp_only)
                      : entry<D, BM, BN, false, false, true>(k.dp_only);
    }
    if (k.a_kc) return k.b_kc ? entry<D, BM, BN, true, true, false>(k.dp_only)
                              : entry<D, BM, BN, true, false, false>(k.dp_only);
    return k.b_kc ? entry<D, BM, BN, false, true, false>(k.dp_only)
                  : entry<D, BM, BN, false, false, false>(k.dp_only);
}

}  // namespace sk
