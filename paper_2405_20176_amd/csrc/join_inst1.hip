// Instantiations of the fused join kernel for d in {7, 8, 9, 10}.
#include "join_kernel.cuh"

namespace snaps {

JoinFn join_pick_group1(int D, int kc, int xf) {
    switch (D) {
        case 7: return join_pick_d<7>(kc, xf);
        case 8: return join_pick_d<8>(kc, xf);
        case 9: return join_pick_d<9>(kc, xf);
        case 10: return join_pick_d<10>(kc, xf);
    }
    return nullptr;
}

}  // namespace snaps
