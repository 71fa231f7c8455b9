// Parameters of the team (panel) solver: several workgroups share one panel
// of right-hand sides, splitting its rows among them.
#pragma once
#include <stdint.h>

#include "scocg_params.hpp"

namespace scocg {

struct TParams {
    KParams k;               // matrices, maps, shifts, outputs (as for the one-workgroup solvers)
    int32_t G;               // workgroups per team (rows of the system split among them)
    int32_t W;               // right-hand sides per panel (columns solved together)
    int32_t nteams;
    int32_t npanels;         // ceil(nrhs / W)
    int32_t pairs_max;       // per workgroup: ceil(W K / G) (RHS, shift) pairs at most
    int32_t rows_max;        // per workgroup: block rows of its share, at most (LDS direction sizing)
    int64_t team_bytes;      // global working memory of one team
    int64_t vec_stride;      // doubles between two panel vectors ([Mp][W] each)
    char* tws;               // teams' working memory (nteams * team_bytes)
    int32_t* sync;           // per team: [0] arrival counter, [1] current job; 32 ints per team
    double* part;            // per team: [2][G][pstride] reduction partials
    int32_t pstride;
    int32_t* abort_flag;     // set when a team wait exceeds its bound (every workgroup then leaves)
    int64_t spin_ticks;      // bound of one wait, in wall-clock ticks
};

}  // namespace scocg
