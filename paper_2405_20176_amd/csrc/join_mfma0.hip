// Instantiations of the matrix-core join kernel for d in {2, ..., 8}, the leaner walk (H = 0).
#include "join_mfma.cuh"

namespace snaps {

JoinFn join_mfma_pick_group0(int D, int kc) {
    switch (D) {
        case 2: return join_mfma_pick_kc<2, 0>(kc);
        case 3: return join_mfma_pick_kc<3, 0>(kc);
        case 4: return join_mfma_pick_kc<4, 0>(kc);
        case 5: return join_mfma_pick_kc<5, 0>(kc);
        case 6: return join_mfma_pick_kc<6, 0>(kc);
        case 7: return join_mfma_pick_kc<7, 0>(kc);
        case 8: return join_mfma_pick_kc<8, 0>(kc);
    }
    return nullptr;
}

}  // namespace snaps
