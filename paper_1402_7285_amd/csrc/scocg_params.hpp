// Parameter block shared by the host library and the solver kernel.
#pragma once
#include <stdint.h>

namespace scocg {

// One local system: block rows [0, nrows) with CSR rows at rowptr[row_base..]
// whose values index entries [ent_base + rowptr[a], ent_base + rowptr[a+1]).
struct SysInfo {
    int64_t row_base;
    int64_t ent_base;
    int32_t nrows;
    int32_t pad;
};

// One right-hand side: its system, the local index of e_j, and where its
// requested rows (local indices) start in out_local.
struct RhsInfo {
    int32_t sys;
    int32_t b_local;
    int64_t out_base;
    int32_t nout;
    int32_t full_x;
};

enum { NSTAT = 8 };

struct KParams {
    // matrix values on the merged block pattern (entry g -> block g)
    const void* Hv;            // FP64 / FP32 / BF16 per kernel variant
    const void* Sv;            // same; nullptr when S = I
    const double* Hv64;        // FP64 copies (FP32 forms: replacement and audit)
    const double* Sv64;
    // local block maps
    const int64_t* rowptr_l;
    const int32_t* ecol;       // local block column of an entry
    const int32_t* egid;       // global block index of an entry
    const SysInfo* sys;
    const RhsInfo* rhs;
    const int32_t* out_local;
    const int64_t* out_off;    // output rows offset per RHS (values at K*out_off[r])
    const int32_t* order;      // work-queue order of RHS
    const double* z;           // shifts, interleaved (re, im), K entries
    int32_t nrhs;
    int32_t K;
    int32_t seed0;
    int32_t maxiter;           // 0 = max(1000, 4 M_j)
    double tol;
    double inner_tol;          // FP64 inner CG
    double inner_tol_lo;       // FP32 inner CG
    int32_t inner_maxiter;
    int32_t replace_every;     // FP32 forms
    int32_t audit;             // FP32 forms
    int32_t s_unit_diag;       // S's diagonal blocks are exactly I
    int32_t ent_direct;        // egid is the identity: entry e holds block e
    // S = I + off-diagonal blocks (global system, identity diagonal blocks):
    // the off-diagonal blocks alone in their own CSR, entry e holding block e
    const int64_t* s_rowptr;
    const int32_t* s_ecol;
    const double* s_vals;
    // the same blocks in ELL form, s_ell_w entries per block row (0: none):
    // columns [nbrows][s_ell_w], blocks in that order; a row shorter than
    // s_ell_w is padded with its own column and a zero block
    const int32_t* s_ell_col;
    const double* s_ell_val;
    int32_t s_ell_w;
    // work queue and per-workgroup memory
    int32_t* queue;            // next RHS to hand out
    char* ws;
    int64_t slot_bytes;
    int64_t Mp;                // padded max cluster dimension (elements)
    int64_t nIp;               // projected mode: padded max requested rows
    // outputs (device)
    double* out;               // interleaved complex
    int32_t* iters;
    int8_t* status;
    double* resid;
    int64_t* stats;            // [nrhs][NSTAT]
};

}  // namespace scocg
