// stage_march.hip -- the row-marching stage kernel (stage_march.h) for the default scheme:
// Osher-Dumbser-Toro flux, the new pressure gradient, walls and periodic sides, local
// pseudo-time steps; FP64 and mixed precision, BDF orders 1-3, one launch for all tanks.
#include "stage_march.h"

namespace vdac {

int march_strips(int nx) { return (nx + march::kOut - 1) / march::kOut; }

int launch_stage_march(const TankDev *tanks_dev, const MarchUnit *units, int n_entries,
                       int waves_per_block, const Scheme &sc, int stage, const IterArgs &ia,
                       int waves_simd, void *stream)
{
    if (sc.general)
        return launch_stage_march_general(tanks_dev, units, n_entries, waves_per_block, sc, stage, ia,
                                          stream);
    return march::launch<false>(tanks_dev, units, n_entries, waves_per_block, sc, stage, ia,
                                waves_simd, stream);
}

}  // namespace vdac
