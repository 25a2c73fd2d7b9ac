// Instantiations of the fused join kernel for d in {11, 12, 13}.
#include "join_kernel.cuh"

namespace snaps {

JoinFn join_pick_group2(int D, int kc, int xf) {
    switch (D) {
        case 11: return join_pick_d<11>(kc, xf);
        case 12: return join_pick_d<12>(kc, xf);
        case 13: return join_pick_d<13>(kc, xf);
    }
    return nullptr;
}

}  // namespace snaps
