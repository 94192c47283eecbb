// Quadtree builds of several matrices at once (defined in matrix.hip).
#pragma once

#include "common.h"

namespace qbsm {

// Builds the depth-D trees of the listed matrices that hold none yet, with
// one host read for all of their level sizes (null entries and repeats are
// skipped); matrix_tree then finds them cached.
void matrix_trees(Matrix *const *ms, int nm, int D, hipStream_t s);

}  // namespace qbsm
