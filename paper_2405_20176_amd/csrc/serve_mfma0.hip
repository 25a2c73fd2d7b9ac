// Instantiations of the matrix-core alert kernel for d in {2, ..., 8}.
#include "serve_mfma.cuh"

namespace snaps {

AlertKernel alert_mfma_pick_group0(int D, int kc) {
    switch (D) {
        case 2: return alert_mfma_kc<2>(kc);
        case 3: return alert_mfma_kc<3>(kc);
        case 4: return alert_mfma_kc<4>(kc);
        case 5: return alert_mfma_kc<5>(kc);
        case 6: return alert_mfma_kc<6>(kc);
        case 7: return alert_mfma_kc<7>(kc);
        case 8: return alert_mfma_kc<8>(kc);
    }
    return nullptr;
}

}  // namespace snaps
