// Instantiations of the matrix-core join kernel for d in {9, ..., 16},
// the walk with super-tile and candidate-half culls (H = 1).
#include "join_mfma.cuh"

namespace snaps {

JoinFn join_mfma_pick_group3(int D, int kc) {
    switch (D) {
        case 9: return join_mfma_pick_kc<9, 1>(kc);
        case 10: return join_mfma_pick_kc<10, 1>(kc);
        case 11: return join_mfma_pick_kc<11, 1>(kc);
        case 12: return join_mfma_pick_kc<12, 1>(kc);
        case 13: return join_mfma_pick_kc<13, 1>(kc);
        case 14: return join_mfma_pick_kc<14, 1>(kc);
        case 15: return join_mfma_pick_kc<15, 1>(kc);
        case 16: return join_mfma_pick_kc<16, 1>(kc);
    }
    return nullptr;
}

}  // namespace snaps
