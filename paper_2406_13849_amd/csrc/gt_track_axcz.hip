// The persistent single-geometry tracker built for geometries of axis planes
// and z-cylinders only (SF_AXCZ); see gt_persistent.h.
#pragma clang fp contract(off)

#include "gt_persistent.h"

namespace gt {

int launch_persistent_axcz(const gt_geometry *g, const LaunchRec *lr, int prec, int w, int kind, uint64_t n,
                          unsigned block, bool tail, bool cache, uint32_t regroup, bool mesh, hipStream_t st) {
    return launch_persistent_set<SF_AXCZ>(g, lr, prec, w, kind, n, block, tail, cache, regroup, mesh, st);
}

}  // namespace gt
