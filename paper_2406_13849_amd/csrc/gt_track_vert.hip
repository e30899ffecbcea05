// The persistent single-geometry tracker built for geometries of axis planes,
// planes parallel to the z axis and z-cylinders (SF_VERT); see gt_persistent.h.
#pragma clang fp contract(off)

#include "gt_persistent.h"

namespace gt {

int launch_persistent_vert(const gt_geometry *g, const LaunchRec *lr, int prec, int w, int kind, uint64_t n,
                          unsigned block, bool tail, bool cache, uint32_t regroup, bool mesh, hipStream_t st) {
    return launch_persistent_set<SF_VERT>(g, lr, prec, w, kind, n, block, tail, cache, regroup, mesh, st);
}

}  // namespace gt
