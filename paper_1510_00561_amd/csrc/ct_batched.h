// Batched form: stage descriptors shared by the plan builder (host) and the
// persistent work-queue kernel (device).
//
// A plan holds, for every stream, the chain of stages of one pass of the hot
// path (forward CT, quantise, dequantise, inverse CT). Each stage is a set of
// independent tiles; a stage may start once its predecessor in the chain has
// finished all its tiles. Work items (stage, tile) are ordered wave by wave:
// the first stage of every stream, then the second, ..., each wave largest
// stream first, so a stage's predecessor is always earlier in the order.
#pragma once

#include "ct_stages.h"

namespace ct {

enum StageType : int {
    kStLevelAna = 0,     // LP level + DFB tree levels 1-2, analysis
    kStSplit1Ana = 1,    // one DFB tree level, analysis
    kStSplit2Ana = 2,    // two DFB tree levels, analysis
    kStPartial = 3,      // lowpass min/max partials
    kStQuantize = 4,
    kStDequantize = 5,
    kStSplit1Syn = 6,
    kStSplit2Syn = 7,
    kStLevelSyn = 8,     // DFB tree levels 1-2 + LP level, synthesis
};

struct StageDesc {
    int type;
    int ntiles;
    int dep;             // stage index of the predecessor, or -1
    int batch;
    int lo_r;            // reach of the LP `lo` filter: 4 (hbar) or 3 (gbar, transposes)
    double bytes;        // compulsory bytes (profiling)
    Lift lift;
    union {
        stage::LevelAnaArgs la;
        stage::LevelSynArgs ls;
        SplitArgs sp;
        QuantArgs q;
    } u;
};

constexpr int kBatchedThreads = 512;

// Launches the counter reset and the persistent kernel for `nstages` stages
// with `total_items` work items. `counters` holds nstages + 1 ints.
hipError_t launch_batched(const StageDesc* stages, const int* first_item, int nstages,
                          int total_items, int* counters, int grid, hipStream_t s);
// Workgroups of the persistent kernel that can be resident at once.
int batched_capacity();

}  // namespace ct
