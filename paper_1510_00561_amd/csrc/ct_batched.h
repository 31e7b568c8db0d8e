// Batched form: stage descriptors shared by the plan builder (host) and the
// group kernels (device).
//
// A plan holds, for every stream, the chain of stages of one pass of the hot
// path (forward CT, quantise, dequantise, inverse CT). Each stage is a set of
// independent tiles and may start once its predecessor in the chain has
// finished. The plan runs the chains position by position: the stages at
// one chain position of all streams are independent of each other, so those
// of one type are laid end to end and run as one launch (a group), and the
// launches follow in chain order on one stream, so that stream order carries
// every dependency.
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
    // the same stages with quantised final subbands (fused encoder / decoder)
    kStLevelAnaQ = 9,
    kStSplit1AnaQ = 10,
    kStSplit2AnaQ = 11,
    kStSplit1SynQ = 12,
    kStSplit2SynQ = 13,
    kStLevelSynQ = 14,
    // three DFB tree levels per pass, plain and with quantised final subbands
    kStSplit3Ana = 15,
    kStSplit3Syn = 16,
    kStSplit3AnaQ = 17,
    kStSplit3SynQ = 18,
    kStNumTypes = 19,
};

struct StageDesc {
    int type;
    int ntiles;
    int batch;
    int lo_r;            // reach of the LP `lo` filter: 4 (hbar) or 3 (gbar, transposes)
    double bytes;        // compulsory bytes (profiling): every array read once, written once
    double alg;          // of these, the codec's own inputs and outputs (frames, float
                         // coefficients, indices): the algorithmic bytes
    Lift lift;
    union {
        stage::LevelAnaArgs la;
        stage::LevelSynArgs ls;
        SplitArgs sp;
        QuantArgs q;
    } u;
};

constexpr int kBatchedThreads = 256;

// Launches one group: `n` stages of type `type` whose tiles are laid end to
// end (stage i owns tiles [first[i], first[i+1]), `tiles` in total), one
// workgroup of kBatchedThreads per tile. `stages` and `first` are device
// arrays.
hipError_t launch_group(int type, const StageDesc* stages, const int* first, int n, int tiles,
                        hipStream_t s);

}  // namespace ct
