// Host-callable launchers of the solver kernels (defined in scocg_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "scocg_params.hpp"
#include "team_params.hpp"

namespace scocg {

// The allocation-free entry point's fixed device working memory (per device).
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
// Device address of that memory on `device` (fetched once per device, then cached).
hipError_t noalloc_scratch(int device, void** ptr);

bool supported_bdim(int bd);
size_t solver_lds_bytes(int K, int nt);
// Working memory of one resident workgroup (bytes) for K shifts and Mp rows.
int64_t solver_slot_bytes(int K, int64_t Mp, int prec);
// Same for the projected (requested-rows-only) FP64 solve with nIp padded rows.
int64_t solver_slot_bytes_proj(int K, int64_t Mp, int64_t nIp);
// prec: 0 FP64, 1 FP32, 2 FP32 compute with bfloat16 blocks, 3 projected FP64; sid: S = I.
hipError_t launch_solver(const KParams& P, int bd, int prec, bool sid, int nt, int slots, hipStream_t st);
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st);
// Private (scratch) bytes per lane of the instance the one-workgroup launchers would run
// ((size_t)-1 if it cannot be queried); instances with spills are not launched.
size_t solver_private_bytes(int bd, int prec, bool sid, int nt);
size_t qmr_private_bytes(int bd, bool sid, bool gal, bool dl, int unit, int nt);
// Shifted QMR over the real S-Lanczos basis (qmr_kernels.hip).
size_t qmr_lds_bytes(int K, int nt, int64_t Mp, bool dl);
int64_t qmr_slot_bytes(int K, int64_t Mp, int64_t nIp);
// gal: the COCG (Galerkin) iterates on the same basis instead of the QMR ones.
hipError_t launch_qmr(const KParams& P, int bd, bool sid, bool gal, bool dl, int unit, int nt, int slots,
                      hipStream_t st);
// Energy integration of a plan's output (integrate_kernels.hip).
hipError_t launch_integrate(const double* G, const double* z, const double* w, const RhsInfo* rhs,
                            const int64_t* out_off, const int32_t* out_local, int nrhs, int K, double mu, double kT,
                            double* rho, double* ldos, hipStream_t st);
hipError_t launch_cohp(const double* h, const double* rho, double* cohp, int64_t n, hipStream_t st);
// Team (panel) solver on the real S-Lanczos basis (team_kernels.hip): G workgroups per panel of W RHS.
size_t team_lds_bytes(int nt, int W, int pairs, int rows_max, bool dl, bool rv = false);
int64_t team_ws_bytes(int W, int K, int64_t Mp, int64_t nIp, bool qmr);
// variant: 0 S = I, 1 inner CG direction in LDS, 2 the same with S = I + off-diagonal blocks, 3 direction in
// HBM, 4 / 5 the inner CG's vectors in registers (ri block-row quads per wave) with S = I + off-diagonal
// blocks / S as stored
hipError_t launch_team(const TParams& T, int bd, bool gal, int variant, int ri, int nt, int grid, size_t lds,
                       hipStream_t st);
// resident workgroups of that kernel per compute unit, and its private (scratch) bytes per lane
hipError_t team_occupancy(int bd, bool gal, int variant, int ri, int nt, int W, size_t lds, int* per_cu,
                          size_t* private_bytes);
// whether the register-resident form is compiled for (threads, panel width, block-row quads per wave)
bool team_rv_ok(int nt, int W, int ri);

}  // namespace scocg
