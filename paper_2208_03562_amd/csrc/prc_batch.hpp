// Internal interface between the batch (prc_batch.hip) and the request
// server (prc_serve.hip): one interval of a batched solve.
#pragma once

#include <cstdint>
#include <vector>

#include "prc.h"

namespace prc {

struct BatchChecked {
    int32_t id;
    double R;  // relative residual of this check
};

struct BatchLeft {
    int32_t id;
    int32_t status;  // prc_member_status
    int64_t steps;   // steps taken since the member joined
    double R;        // relative residual of its last check
};

// One interval of a batched solve: velocity snapshots of members that have
// none yet, check_every (even) steps of every active member, their check,
// then CONVERGED / DIVERGED / MAX_STEPS members leave the batch.  The
// members checked are appended to *checked and those that left to *left
// (either may be null).  Members that had already reached max_steps leave
// without stepping.
prc_status batch_interval(prc_batch *b, double tol, int64_t check_every, int64_t max_steps,
                          std::vector<BatchChecked> *checked, std::vector<BatchLeft> *left,
                          hipStream_t s);

}  // namespace prc
