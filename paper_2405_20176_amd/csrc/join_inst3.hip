// Instantiations of the fused join kernel for d in {14, 15, 16}.
#include "join_kernel.cuh"

namespace snaps {

JoinFn join_pick_group3(int D, int kc, int xf) {
    switch (D) {
        case 14: return join_pick_d<14>(kc, xf);
        case 15: return join_pick_d<15>(kc, xf);
        case 16: return join_pick_d<16>(kc, xf);
    }
    return nullptr;
}

}  // namespace snaps
