// Instantiations of the fused join kernel for d in {2, 3, 4, 5, 6}.
#include "join_kernel.cuh"

namespace snaps {

JoinFn join_pick_group0(int D, int kc, int xf) {
    switch (D) {
        case 2: return join_pick_d<2>(kc, xf);
        case 3: return join_pick_d<3>(kc, xf);
        case 4: return join_pick_d<4>(kc, xf);
        case 5: return join_pick_d<5>(kc, xf);
        case 6: return join_pick_d<6>(kc, xf);
    }
    return nullptr;
}

}  // namespace snaps
