// Instantiations of the matrix-core join kernel for d in {2, ..., 8},
// the walk with super-tile and candidate-half culls (H = 1).
#include "join_mfma.cuh"

namespace snaps {

JoinFn join_mfma_pick_group2(int D, int kc) {
    switch (D) {
        case 2: return join_mfma_pick_kc<2, 1>(kc);
        case 3: return join_mfma_pick_kc<3, 1>(kc);
        case 4: return join_mfma_pick_kc<4, 1>(kc);
        case 5: return join_mfma_pick_kc<5, 1>(kc);
        case 6: return join_mfma_pick_kc<6, 1>(kc);
        case 7: return join_mfma_pick_kc<7, 1>(kc);
        case 8: return join_mfma_pick_kc<8, 1>(kc);
    }
    return nullptr;
}

}  // namespace snaps
