// stage_march_gen.hip -- the row-marching stage kernel (stage_march.h) with the general options
// chosen at run time: Roe or exact (Bassi) flux (Sec. 2.4.1-2.4.2), the k-limiter or the split
// limiter on p (Sec. 2.3.2), zero-gradient sides, and the global pseudo-time step (Sec. 2.2.3:
// the minimum local step, which the final stage of each pseudo-iteration reduces for the next).
#include "stage_march.h"

namespace vdac {

int launch_stage_march_general(const TankDev *tanks_dev, const MarchUnit *units, int n_entries,
                               int waves_per_block, const Scheme &sc, int stage, const IterArgs &ia,
                               void *stream)
{
    return march::launch<true>(tanks_dev, units, n_entries, waves_per_block, sc, stage, ia, 2, stream);
}

}  // namespace vdac
