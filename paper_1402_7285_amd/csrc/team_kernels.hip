// Team (panel) solver for the shifted Krylov methods on the real S-Lanczos
// basis (gfx950): the shifted COCG iterates of every shift (Galerkin form)
// and the generalized shifted QMR iterates (Sec. 3, items (i)-(ii)), for
// (z_k S - H) x = b with real symmetric H, real SPD S and b = e_j (Sec. 3,
// Eq. 2).
//
// Why a team.  The one-workgroup solver gives each right-hand side (RHS)
// its own compute unit, so every RHS streams all of H's and S's blocks
// through its CU in every sparse product: the block traffic is paid once per
// RHS, and one large order-N cluster bounds the launch by its own latency.
// Here G workgroups (a team) solve a panel of W RHS together:
//   * rows: the system's block rows are split among the G workgroups; each
//     applies H and S to its own rows only, so a team covers a sparse
//     product in 1/G of the time one workgroup would need;
//   * panel: the W RHS share one system (the global system), so every block
//     read serves W columns; for 4x4 blocks and W a multiple of 4 the block
//     products run on FP64 matrix cores (v_mfma_f64_4x4x4_4b: four block
//     rows times four RHS per instruction, the 4x4 orbital block being the
//     dense operand the panel creates).
// The method's global reductions (alpha_n, ||t||^2, the inner CG's two dots,
// q^T t) are summed per workgroup (DPP row operations inside each wavefront,
// then a fixed-order sum over the waves), exchanged through the team's
// partial-sum buffer and summed again in rank order, so every workgroup
// gets bitwise the same totals and takes the same branches.  The waits are
// bounded: a wait that exceeds its bound sets an abort flag that every
// workgroup honours at its next wait, so a launch always ends.
//
// Data a workgroup publishes for others (vectors that products gather, the
// partial sums, the job number) is written with device-coherent stores and
// read with device-coherent loads; everything private to a workgroup uses
// ordinary accesses.
//
// One outer iteration n of a panel column (the S-Lanczos process on
// S^{-1}H, with q = beta_n v_n kept unnormalised and t_{n-1} = beta_n w_n):
//   u   = H q_n / beta_n;                alpha_n = v_n^T u
//   t_n = u - alpha_n w_n - beta_n w_{n-1}
//   q_{n+1} = S^{-1} t_n                 inner CG (two team reductions per step)
//   beta_{n+1} = sqrt(q_{n+1}^T t_n)
//   every shift: one LDL^T pivot (COCG iterates) or one Givens rotation
//   (QMR) and the requested rows of its direction and x.
// The inner CG updates the search-direction product as w <- S r + beta w, so
// each step gathers only the residual, which is complete after the step's
// second reduction: two waits per CG step.
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "scocg_device.hpp"
#include "scocg_params.hpp"
#include "team_params.hpp"

namespace scocg {
namespace team {

enum { ST_CONVERGED = 0, ST_MAXITER = 1, ST_BREAKDOWN = 2, ST_NONFINITE = 3, ST_ABORTED = 4 };

// ---------------------------------------------------------------------------
// accesses to data other workgroups of the team read or wrote
// ---------------------------------------------------------------------------
__device__ __forceinline__ void st_pub(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_pub(const double* p) {
    return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_pub_i(int* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_pub_i(const int* p) {
    return __hip_atomic_load(const_cast<int*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// column sums of a matrix-core tile (the wave reductions themselves are in
// scocg_device.hpp)
// ---------------------------------------------------------------------------
// Sum over the lanes that share (lane & 3) (the four columns of a matrix-core
// output tile): within each row by rotations of 4 and 8, across the four rows
// by two exchanges.  Lanes 0..3 (and every lane) end with their column's sum.
__device__ __forceinline__ double col4_sum(double v) {
    v += dpp64<0x124, 0xF>(v);
    v += dpp64<0x128, 0xF>(v);
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    return v;
}

// ---------------------------------------------------------------------------
// team context: rank, barrier, reductions
// ---------------------------------------------------------------------------
struct Team {
    int G, rank, id;
    int* ctr;          // arrival counter (monotonic within a launch)
    int* job;          // current job of the team
    double* part;      // [2][G][pstride]
    int pstride;
    int* abort_flag;
    long long spin_ticks;
    int epoch;
};

// Wait until every member of the team has arrived here as often as this
// workgroup (thread 0 waits, the workgroup then proceeds together).  Returns
// false in every thread if the wait was abandoned (bound exceeded, or another
// workgroup abandoned one): the caller leaves.
__device__ bool team_wait(Team& tm, int* s_flag) {
    __builtin_amdgcn_s_waitcnt(0);   // this thread's published stores have completed
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        if (tm.G > 1) {
            const int target = tm.G * (tm.epoch + 1);
            __hip_atomic_fetch_add(tm.ctr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const long long t0 = wall_clock64();
            while (ld_pub_i(tm.ctr) < target) {
                if (ld_pub_i(tm.abort_flag)) { ok = 0; break; }
                if (wall_clock64() - t0 > tm.spin_ticks) {
                    st_pub_i(tm.abort_flag, 1);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        } else if (ld_pub_i(tm.abort_flag)) {
            ok = 0;
        }
        *s_flag = ok;
    }
    __syncthreads();
    const bool ok = *s_flag != 0;
    tm.epoch += 1;
    return ok;
}

// Per-wave partials are in red[w * NV + n] (n < NV); sums them over the
// workgroup (fixed wave order) and then over the team (rank order) into
// out[0..NV) in LDS, visible to every thread on return.
template <int NT, int NV>
__device__ bool team_sum(double* red, double* out, Team& tm, int* s_flag) {
    constexpr int NW = NT / 64;
    __syncthreads();
    const int tid = threadIdx.x;
    const int buf = tm.epoch & 1;
    if (tid < NV) {
        double s = 0.0;
        for (int w = 0; w < NW; ++w) s += red[w * NV + tid];
        if (tm.G > 1) st_pub(tm.part + ((int64_t)buf * tm.G + tm.rank) * tm.pstride + tid, s);
        else out[tid] = s;
    }
    if (tm.G == 1) {
        const bool ok = team_wait(tm, s_flag);
        return ok;
    }
    if (!team_wait(tm, s_flag)) return false;
    if (tid < NV) {
        double s = 0.0;
        for (int r = 0; r < tm.G; ++r) s += ld_pub(tm.part + ((int64_t)buf * tm.G + r) * tm.pstride + tid);
        out[tid] = s;
    }
    __syncthreads();
    return true;
}

// ---------------------------------------------------------------------------
// element ownership inside a workgroup
// ---------------------------------------------------------------------------
// MF (4x4 blocks, W a multiple of 4): the layout of the matrix-core tile.
// Lane l of wave w handles, for block-row quad qd = w, w + NW, ..., the block
// row a = a0 + 4 qd + ((l >> 2) & 3), row i = l >> 4 of it, and columns
// 4 s + (l & 3), s < W / 4 (slots).  Otherwise one thread per row, all W
// columns (slot s = column s).
template <int BD, int NT, int W>
struct Lay {
    static constexpr bool MF = (BD == 4) && (W % 4 == 0);
    static constexpr int NS = MF ? W / 4 : W;
    static constexpr int NW = NT / 64;
};

// Calls f(row, slot, col, ldsidx) for every element this thread owns in
// block rows [a0, a1); ldsidx is the element's index in a workgroup-local
// [rows][W] array.
template <int BD, int NT, int W, class F>
__device__ __forceinline__ void for_elems(int a0, int a1, F f) {
    using L = Lay<BD, NT, W>;
    const int tid = threadIdx.x;
    if constexpr (L::MF) {
        const int lane = tid & 63, w = tid >> 6;
        const int beta = (lane >> 2) & 3, ii = lane >> 4, jj = lane & 3;
        const int nbl = a1 - a0;
        for (int qd = w; 4 * qd < nbl; qd += L::NW) {
            const int a = a0 + 4 * qd + beta;
            if (a >= a1) continue;
            const int row = 4 * a + ii;
            const int li = (4 * (a - a0) + ii) * W;
#pragma unroll
            for (int s = 0; s < L::NS; ++s) f(row, s, 4 * s + jj, li + 4 * s + jj);
        }
    } else {
        const int i0 = a0 * BD, i1 = a1 * BD;
        for (int i = i0 + tid; i < i1; i += NT) {
#pragma unroll
            for (int s = 0; s < W; ++s) f(i, s, s, (i - i0) * W + s);
        }
    }
}

// Per-thread partials acc[NS] -> per-wave column partials red[w * NV + off + col].
template <int BD, int NT, int W, int NV>
__device__ __forceinline__ void wave_put(const double (&acc)[Lay<BD, NT, W>::NS], double* red, int off) {
    using L = Lay<BD, NT, W>;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if constexpr (L::MF) {
#pragma unroll
        for (int s = 0; s < L::NS; ++s) {
            const double t = col4_sum(acc[s]);
            if (lane < 4) red[w * NV + off + 4 * s + lane] = t;
        }
    } else {
#pragma unroll
        for (int s = 0; s < W; ++s) {
            const double t = wave_total(acc[s]);
            if (lane == 0) red[w * NV + off + s] = t;
        }
    }
}

// ---------------------------------------------------------------------------
// block-sparse products over a workgroup's rows
// ---------------------------------------------------------------------------
struct Sys {
    const int64_t* rowptr;
    const int32_t* ecol;
    const int32_t* egid;   // nullptr: entry e holds block gbase + e
    int64_t gbase;
    int nrows;
    int M;
};

// y = A x (+ x if UNIT) on the owned elements of block rows [a0, a1);
// ep(row, slot, col, ldsidx, y) receives each result.  x is [M][W] and was
// published by the team (device-coherent loads).  LX (matrix-core layout
// only): the workgroup's own rows of x are read from LDS instead (xl,
// [rows][W] in the workgroup's local order).
template <int BD, int NT, int W, bool UNIT, class EP, bool LX = false>
__device__ __forceinline__ void spmm(const double* __restrict__ A, const Sys& sy, int a0, int a1,
                                     const double* __restrict__ x, EP ep, const double* xl = nullptr) {
    static_assert(!LX || Lay<BD, NT, W>::MF, "LDS rows in the matrix-core layout only");
    using L = Lay<BD, NT, W>;
    const int tid = threadIdx.x;
    const bool direct = sy.egid == nullptr;
    if constexpr (L::MF) {
        constexpr int CH = 4;
        const int lane = tid & 63, w = tid >> 6;
        const int beta = (lane >> 2) & 3, lo2 = lane & 3, hi2 = lane >> 4;
        const int nbl = a1 - a0;
        for (int qd = w; 4 * qd < nbl; qd += L::NW) {
            const int a = a0 + 4 * qd + beta;
            const bool va = a < a1;
            const int64_t e0 = va ? sy.rowptr[a] : 0;
            const int ne = va ? (int)(sy.rowptr[a + 1] - e0) : 0;
            // the wave's longest row among its four block rows
            int nemax = max(max(__builtin_amdgcn_readlane(ne, 0), __builtin_amdgcn_readlane(ne, 4)),
                            max(__builtin_amdgcn_readlane(ne, 8), __builtin_amdgcn_readlane(ne, 12)));
            double acc[L::NS];
#pragma unroll
            for (int s = 0; s < L::NS; ++s) acc[s] = 0.0;
            for (int eb = 0; eb < nemax; eb += CH) {
                int col[CH];
                double av[CH];
                double bv[CH][L::NS];
#pragma unroll
                for (int u = 0; u < CH; ++u) {
                    const bool ok = eb + u < ne;
                    // a padded slot re-reads entry 0 of the system (always present) and multiplies by zero
                    const int64_t e = ok ? e0 + eb + u : 0;
                    col[u] = sy.ecol[e];
                    const int64_t g = direct ? sy.gbase + e : (int64_t)sy.egid[e];
                    const double v = A[g * 16 + lo2 * 4 + hi2];     // A operand: row lo2, k = hi2
                    av[u] = ok ? v : 0.0;
                }
#pragma unroll
                for (int u = 0; u < CH; ++u) {
                    const double* xb = x + ((int64_t)col[u] * 4 + hi2) * W + lo2;   // B operand: k = hi2, col lo2
                    const bool own = LX && col[u] >= a0 && col[u] < a1;
#pragma unroll
                    for (int s = 0; s < L::NS; ++s) {
                        if (own) bv[u][s] = xl[((col[u] - a0) * 4 + hi2) * W + 4 * s + lo2];
                        else bv[u][s] = ld_pub(xb + 4 * s);
                    }
                }
#pragma unroll
                for (int u = 0; u < CH; ++u) {
#pragma unroll
                    for (int s = 0; s < L::NS; ++s)
                        acc[s] = __builtin_amdgcn_mfma_f64_4x4x4f64(av[u], bv[u][s], acc[s], 0, 0, 0);
                }
            }
            if (va) {
                const int row = 4 * a + hi2;                           // D: row hi2, column lo2
                const int li = (4 * (a - a0) + hi2) * W;
#pragma unroll
                for (int s = 0; s < L::NS; ++s) {
                    const int col = 4 * s + lo2;
                    double y = acc[s];
                    if constexpr (UNIT) y += LX ? xl[li + col] : ld_pub(x + (int64_t)row * W + col);
                    ep(row, s, col, li + col, y);
                }
            }
        }
    } else {
        constexpr int CH0 = BD == 1 ? 8 : (BD <= 4 ? 4 : 2);
        constexpr int CH = NT >= 1024 && CH0 > 1 ? CH0 / 2 : CH0;
        constexpr bool QUAD = BD == 4 && W == 1;
        const int i0 = a0 * BD, i1 = a1 * BD;
        // One loop per block-address form (entry number or map), chosen once per product, so that a
        // chunk's index loads, and then all its block and vector loads, go out together: no branch
        // between entries, and a padded slot re-reads the row's last entry and masks its value.
        auto rows = [&](auto dir) __attribute__((always_inline)) {
            constexpr bool DIRECT = decltype(dir)::value;
            for (int i = i0 + tid; i < i1; i += NT) {
                const int a = i / BD, r = i - a * BD;
                const int64_t e0 = sy.rowptr[a], e1 = sy.rowptr[a + 1];
                double acc[W];
#pragma unroll
                for (int c = 0; c < W; ++c) acc[c] = 0.0;
                // a chunk's column and block indices (padded slots: the row's last entry)
                int32_t bn[CH], gn[CH];
                auto load_idx = [&](int64_t eb) __attribute__((always_inline)) {
#pragma unroll
                    for (int u = 0; u < CH; ++u) {
                        const int64_t e = eb + u < e1 ? eb + u : e1 - 1;
                        bn[u] = sy.ecol[e];
                        gn[u] = DIRECT ? (int32_t)(eb + u) : sy.egid[e];
                    }
                };
                if (e0 < e1) load_idx(e0);
                for (int64_t eb = e0; eb < e1; eb += CH) {
                    int32_t b[CH];
                    int64_t g[CH];
                    bool ok[CH];
#pragma unroll
                    for (int u = 0; u < CH; ++u) {
                        ok[u] = eb + u < e1;
                        b[u] = bn[u];
                        g[u] = DIRECT ? sy.gbase + (ok[u] ? eb + u : e1 - 1) : (int64_t)gn[u];
                    }
                    double av[CH][BD];
                    double own[QUAD ? CH : 1];
                    double xv[QUAD ? 1 : CH][QUAD ? 1 : BD * W];
#pragma unroll
                    for (int u = 0; u < CH; ++u) {
                        const int64_t off = (g[u] * BD + r) * BD;
#pragma unroll
                        for (int c = 0; c < BD; ++c) {
                            const double v = A[off + c];
                            av[u][c] = ok[u] ? v : 0.0;
                        }
                        if constexpr (QUAD) {
                            own[u] = ld_pub(x + (int64_t)b[u] * 4 + r);
                        } else {
                            const double* xb = x + (int64_t)b[u] * BD * W;
#pragma unroll
                            for (int k = 0; k < BD * W; ++k) xv[u][k] = ld_pub(xb + k);
                        }
                    }
                    // the next chunk's indices go out behind this chunk's loads (unconditionally: past
                    // the row's end they re-read its last entry), so they arrive while it is summed
                    load_idx(eb + CH);
#pragma unroll
                    for (int u = 0; u < CH; ++u) {
                        if constexpr (QUAD) {
                            acc[0] += av[u][0] * quad_bcast<0>(own[u]) + av[u][1] * quad_bcast<1>(own[u]) +
                                      av[u][2] * quad_bcast<2>(own[u]) + av[u][3] * quad_bcast<3>(own[u]);
                        } else {
#pragma unroll
                            for (int c = 0; c < BD; ++c)
#pragma unroll
                                for (int s = 0; s < W; ++s) acc[s] += av[u][c] * xv[u][c * W + s];
                        }
                    }
                }
#pragma unroll
                for (int s = 0; s < W; ++s) {
                    double y = acc[s];
                    if constexpr (UNIT) y += ld_pub(x + (int64_t)i * W + s);
                    ep(i, s, s, (i - i0) * W + s, y);
                }
            }
        };
        if (direct) rows(std::true_type{});
        else rows(std::false_type{});
    }
}

// ---------------------------------------------------------------------------
// register-resident form (4x4 blocks, W a multiple of 4): the matrix-core
// layout with the block-row quads of each wave unrolled (RI of them at most),
// so that per-thread vectors can live in registers indexed [k][slot].
// ---------------------------------------------------------------------------
// f(integral_constant<0>), ..., f(integral_constant<N - 1>): indices known when the body is generated,
// so that per-thread arrays indexed by them stay in registers
template <class F, int... I>
__device__ __forceinline__ void sfor_impl(F& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void sfor(F&& f) {
    sfor_impl(f, std::make_integer_sequence<int, N>{});
}

// f(K, S, row, col, ldsidx) for every owned element; K and S are integral constants.
template <int NT, int W, int RI, class F>
__device__ __forceinline__ void for_elems_r(int a0, int a1, F f) {
    constexpr int NW = NT / 64, NS = W / 4;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int beta = (lane >> 2) & 3, ii = lane >> 4, jj = lane & 3;
    sfor<RI>([&](auto K) __attribute__((always_inline)) {
        const int a = a0 + 4 * (w + NW * (int)K) + beta;
        if (a < a1) {
            const int row = 4 * a + ii;
            const int li = (4 * (a - a0) + ii) * W;
            sfor<NS>([&](auto S) __attribute__((always_inline)) { f(K, S, row, 4 * (int)S + jj, li + 4 * (int)S + jj); });
        }
    });
}

// ---------------------------------------------------------------------------
// Complex Givens rotation [[c, s], [-conj(s), c]], c >= 0 real, mapping (a, b) to (r, 0).
__device__ __forceinline__ void givens(zc a, zc b, double& c, zc& s, zc& r) {
    const double aa = zabs(a), ab = zabs(b);
    if (ab == 0.0) {
        c = 1.0;
        s = zmk(0.0, 0.0);
        r = a;
    } else if (aa == 0.0) {
        c = 0.0;
        s = zmk(b.re / ab, -b.im / ab);
        r = zmk(ab, 0.0);
    } else {
        const double nrm = hypot(aa, ab);
        const zc ph = zmk(a.re / aa, a.im / aa);
        c = aa / nrm;
        s = zmul(ph, zmk(b.re / nrm, -b.im / nrm));
        r = zmk(ph.re * nrm, ph.im * nrm);
    }
}

// ---------------------------------------------------------------------------
// LDS of one workgroup
// ---------------------------------------------------------------------------
enum { NCOL = 24 };   // per-column scalar slots (below)
enum {
    C_BCUR = 0,       // normalisation of q_n (v_n = q_n / bcur, w_n = t_{n-1} / bcur)
    C_BPREV,          // normalisation one step back (w_{n-1} = t_{n-2} / bprev)
    C_BLAN,           // Lanczos beta_n (0 at n = 0)
    C_ALPHA, C_TT, C_QT, C_BNEXT, C_SUMW2, C_BETA0,
    C_RR, C_A, C_BCG, C_STOP,
    C_ACT,            // 1: the column's Lanczos process runs
    C_CGACT,          // 1: the column's inner CG runs
    C_CGIT,           // inner CG steps of the current solve
    C_NOUT, C_INNER, C_SUMUPD, C_BAD,   // outer iterations, inner total, shift updates, 1 NaN / 2 breakdown
    C_BLOC,           // local row of e_j (-1 if the column is empty)
    C_NPAIR,          // unfinished pairs (from the last reduction)
    C_RHS             // RHS number (queue position resolved), -1 empty
};

struct Lds {
    double* red;     // NW * NVMAX partials
    double* rres;    // NVMAX reduced values
    double* col;     // [NCOL][W] per-column scalars
    // owned (RHS column, shift) pairs, local index m
    zc* p_g;
    zc* p_tau;
    zc* p_e;
    zc* p_f;
    zc* p_irnn;
    zc* p_s1;
    zc* p_s2;
    double* p_c1;
    double* p_c2;
    double* p_res;
    int* p_it;
    int* upd;
    unsigned char* p_done;
    unsigned char* p_stat;
    int* ctl;        // [0] pairs to update, [1] flag, [2] cg-any, [3] act-any
    double* d;       // DL: the CG search direction on the workgroup's rows, [rows][W]
};

__host__ __device__ inline size_t lds_fixed_bytes(int NT, int W, int pairs) {
    const int NW = NT / 64, NV = 2 * W;
    size_t b = sizeof(double) * ((size_t)NW * NV + NV + (size_t)NCOL * W);
    b += (size_t)pairs * (7 * sizeof(zc) + 3 * sizeof(double) + 2 * sizeof(int) + 2);
    b += 16 + 8 * sizeof(int);   // alignment of the control words, and the words
    return (b + 255) & ~(size_t)255;
}
// dl: one region of rows_max x W doubles (the CG direction, or in the register-resident form the
// residual); rv: a second one (the register-resident form's staging of product results)
__host__ __device__ inline size_t lds_bytes(int NT, int W, int pairs, int rows_max, bool dl, bool rv = false) {
    return lds_fixed_bytes(NT, W, pairs) + ((dl ? 1 : 0) + (rv ? 1 : 0)) * sizeof(double) * (size_t)rows_max * W;
}

__device__ inline Lds carve(unsigned char* q, int NT, int W, int pairs) {
    const int NW = NT / 64, NV = 2 * W;
    Lds L;
    L.red = (double*)q; q += sizeof(double) * NW * NV;
    L.rres = (double*)q; q += sizeof(double) * NV;
    L.col = (double*)q; q += sizeof(double) * NCOL * W;
    L.p_g = (zc*)q; q += sizeof(zc) * pairs;
    L.p_tau = (zc*)q; q += sizeof(zc) * pairs;
    L.p_e = (zc*)q; q += sizeof(zc) * pairs;
    L.p_f = (zc*)q; q += sizeof(zc) * pairs;
    L.p_irnn = (zc*)q; q += sizeof(zc) * pairs;
    L.p_s1 = (zc*)q; q += sizeof(zc) * pairs;
    L.p_s2 = (zc*)q; q += sizeof(zc) * pairs;
    L.p_c1 = (double*)q; q += sizeof(double) * pairs;
    L.p_c2 = (double*)q; q += sizeof(double) * pairs;
    L.p_res = (double*)q; q += sizeof(double) * pairs;
    L.p_it = (int*)q; q += sizeof(int) * pairs;
    L.upd = (int*)q; q += sizeof(int) * pairs;
    L.p_done = q; q += pairs;
    L.p_stat = q; q += pairs;
    q = (unsigned char*)(((uintptr_t)q + 15) & ~(uintptr_t)15);
    L.ctl = (int*)q;
    return L;
}

#define COLV(L, slot, c) ((L).col[(slot) * W + (c)])

// Working memory of one team: [0..5] panel vectors of [Mp][W] doubles (q A/B,
// t A/B, u/residual, CG product), [6] the CG direction when it is not in LDS,
// then per (RHS column, shift) pair its requested rows of x and of the one
// (COCG iterates) or two (QMR) direction vectors, complex, nIp each.
__host__ __device__ inline int64_t team_bytes(int W, int K, int64_t Mp, int64_t nIp, bool qmr) {
    const int64_t vec = Mp * W;
    return (7 * vec * 8 + (int64_t)W * K * nIp * 16 * (qmr ? 3 : 2) + 255) / 256 * 256;
}

// ---------------------------------------------------------------------------
// one panel
// ---------------------------------------------------------------------------
// The owned pairs of column c are the local indices m in [lo, hi) with
// p = rank + G m in [c K, (c + 1) K).
__device__ __forceinline__ void col_range(int c, int K, int G, int rank, int npairs, int& lo, int& hi) {
    const int p0 = c * K - rank, p1 = (c + 1) * K - rank;
    lo = p0 <= 0 ? 0 : (p0 + G - 1) / G;
    hi = p1 <= 0 ? 0 : (p1 + G - 1) / G;
    lo = min(lo, npairs);
    hi = min(hi, npairs);
}

// RI > 0: the register-resident form (4x4 blocks, W a multiple of 4, S != I): the inner CG's
// direction, solution and S-product live in registers, its residual on the workgroup's rows in LDS
// (the LDS region DL would give the direction), published for the other workgroups' halo reads.
template <int BD, int NT, int W, bool SID, bool GAL, bool DL, bool UNIT, int RI>
__device__ bool solve_panel(const TParams& T, int panel, Team& tm, const Lds& L, int* s_flag) {
    static_assert(RI == 0 || (BD == 4 && W % 4 == 0 && !SID && DL), "register-resident form");
    constexpr bool RV = RI > 0;
    constexpr int RK = RV ? RI : 1;
    using LY = Lay<BD, NT, W>;
    constexpr int NS = LY::NS;
    constexpr int NV = 2 * W;
    constexpr int NW = NT / 64;
    const KParams& P = T.k;
    const int tid = threadIdx.x;
    const int K = P.K;
    const int G = tm.G, rank = tm.rank;

    // ---- the panel's columns (RHS) and their common system
    if (tid < W) {
        const int q = panel * W + tid;
        const int rj = q < P.nrhs ? P.order[q] : -1;
        COLV(L, C_RHS, tid) = rj;
        COLV(L, C_BLOC, tid) = rj >= 0 ? P.rhs[rj].b_local : -1;
    }
    const int sysid = P.rhs[P.order[panel * W]].sys;   // W = 1 for order-N clusters
    const SysInfo si = P.sys[sysid];
    Sys sy;
    sy.rowptr = P.rowptr_l + si.row_base;
    sy.ecol = P.ecol + si.ent_base;
    sy.egid = P.ent_direct ? nullptr : P.egid + si.ent_base;
    sy.gbase = si.ent_base;
    sy.nrows = si.nrows;
    sy.M = si.nrows * BD;
    Sys syS = sy;
    if constexpr (UNIT) {
        syS.rowptr = P.s_rowptr;
        syS.ecol = P.s_ecol;
        syS.egid = nullptr;
        syS.gbase = 0;
    }
    const double* Hb = P.Hv64;
    const double* Sb = UNIT ? P.s_vals : P.Sv64;
    const int M = sy.M;
    const int a0 = (int)((int64_t)sy.nrows * rank / G), a1 = (int)((int64_t)sy.nrows * (rank + 1) / G);
    const int maxiter = P.maxiter > 0 ? P.maxiter : max(1000, 4 * M);
    const int nIpi = (int)P.nIp;
    const int nrow_arr = GAL ? 2 : 3;

    char* tb = T.tws + (int64_t)tm.id * T.team_bytes;
    const int64_t vs = T.vec_stride;
    double* ures = (double*)tb + 4 * vs;      // u, then the CG residual
    double* wcg = (double*)tb + 5 * vs;       // S d
    double* dd = DL ? L.d : (double*)tb + 6 * vs + (int64_t)a0 * BD * W;   // CG direction, local index
    double2* pairmem = (double2*)((double*)tb + 7 * vs);
    // register-resident form: the CG's direction, solution and S-product (also u = H q / beta) per element
    double rd[RK][NS], rq[RK][NS], rw[RK][NS];
    double* resl = L.d;                       // register-resident form: the CG residual on this workgroup's rows
    double* ystg = L.d + (int64_t)T.rows_max * W;   // and the products' results, staged per element

    // ---- owned pairs: p = rank + G m < W K; column p / K, shift p % K
    const int npairs = (W * K - rank + G - 1) / G;
    for (int m = tid; m < npairs; m += NT) {
        L.p_done[m] = 0;
        L.p_stat[m] = ST_MAXITER;
        L.p_it[m] = -1;
        L.p_res[m] = INFINITY;
        L.p_g[m] = zmk(0.0, 0.0);
        L.p_c1[m] = 1.0;
        L.p_c2[m] = 1.0;
        L.p_s1[m] = GAL ? zmk(1.0, 0.0) : zmk(0.0, 0.0);
        L.p_s2[m] = zmk(0.0, 0.0);
    }
    for (int idx = tid; idx < npairs * nIpi; idx += NT) {
        const int m = idx / nIpi, o = idx - m * nIpi;
        double2* base = pairmem + (int64_t)(rank + G * m) * nIpi * nrow_arr;
        for (int r = 0; r < nrow_arr; ++r) base[(int64_t)r * nIpi + o] = make_double2(0.0, 0.0);
    }
    __syncthreads();
    if (tid < W) {
        const int c = tid;
        const bool valid = COLV(L, C_RHS, c) >= 0;
        COLV(L, C_ACT, c) = valid ? 1.0 : 0.0;
        COLV(L, C_NOUT, c) = 0.0;
        COLV(L, C_INNER, c) = 0.0;
        COLV(L, C_SUMUPD, c) = 0.0;
        COLV(L, C_BAD, c) = 0.0;
        COLV(L, C_TT, c) = valid ? 1.0 : 0.0;       // ||e_j||^2
        COLV(L, C_BLAN, c) = 0.0;
        COLV(L, C_BPREV, c) = 1.0;
        COLV(L, C_BNEXT, c) = 0.0;
        COLV(L, C_CGIT, c) = 0.0;
    }
    __syncthreads();

    // ---- buffers: q_n / q_{n+1} and t_{n-1} / t_n (S = I: q_{n+1} is t_n itself)
    double* qA = (double*)tb;
    double* qB = (double*)tb + vs;
    double* tprev = (double*)tb + 2 * vs;     // t_{-1} = b
    double* tcur = (double*)tb + 3 * vs;
    for_elems<BD, NT, W>(a0, a1, [&](int row, int s, int c, int li) __attribute__((always_inline)) {
        st_pub(tprev + (int64_t)row * W + c, row == (int)COLV(L, C_BLOC, c) ? 1.0 : 0.0);
    });
    // every member's rows of b are written before any product reads them (the first S product of
    // q_0's CG reads the neighbours' rows; without this wait it can see the previous panel's vector)
    if (!team_wait(tm, s_flag)) return false;
    double* qcur = SID ? tprev : qA;
    double* qnew = qB;

    // S q = rhs by CG for the active columns (rhs published, [M][W]); q left in
    // qout with ordinary stores on the workgroup's rows; C_CGIT = steps taken.
    auto inner_cg = [&](const double* rhs, double* qout) __attribute__((always_inline)) -> bool {
        for_elems<BD, NT, W>(a0, a1, [&](int row, int s, int c, int li) __attribute__((always_inline)) {
            const double v = ld_pub(rhs + (int64_t)row * W + c);
            ures[(int64_t)row * W + c] = v;
            dd[li] = v;
        });
        if (tid < W) {
            const int c = tid;
            const double tt = COLV(L, C_TT, c);
            COLV(L, C_RR, c) = tt;
            COLV(L, C_STOP, c) = P.inner_tol * sqrt(tt);
            const bool run = COLV(L, C_ACT, c) != 0.0 && tt > 0.0 && !(sqrt(tt) <= P.inner_tol * sqrt(tt));
            COLV(L, C_CGACT, c) = run ? 1.0 : 0.0;
            COLV(L, C_CGIT, c) = 0.0;
            COLV(L, C_BCG, c) = 0.0;
        }
        __syncthreads();
        for (int m = 0; m < P.inner_maxiter; ++m) {
            int any = 0;
            for (int c = 0; c < W; ++c) any |= COLV(L, C_CGACT, c) != 0.0;
            if (!any) break;
            // (a) d = r + bcg d and w = S r + bcg w (first step: d = rhs, w = S rhs); d^T w
            double acc[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s) acc[s] = 0.0;
            spmm<BD, NT, W, UNIT>(Sb, syS, a0, a1, m == 0 ? rhs : ures,
                                  [&](int row, int s, int c, int li, double y) __attribute__((always_inline)) {
                if (COLV(L, C_CGACT, c) == 0.0) return;
                const int64_t gi = (int64_t)row * W + c;
                double dv, wv;
                if (m == 0) {
                    dv = dd[li];
                    wv = y;
                } else {
                    const double bc = COLV(L, C_BCG, c);
                    dv = ures[gi] + bc * dd[li];
                    wv = y + bc * wcg[gi];
                    dd[li] = dv;
                }
                wcg[gi] = wv;
                acc[s] += dv * wv;
            });
            wave_put<BD, NT, W, NV>(acc, L.red, 0);
            if (!team_sum<NT, NV>(L.red, L.rres, tm, s_flag)) return false;
            if (tid < W) {
                const int c = tid;
                COLV(L, C_A, c) = COLV(L, C_CGACT, c) != 0.0 ? COLV(L, C_RR, c) / L.rres[c] : 0.0;
            }
            __syncthreads();
            // (b) q += a d, r -= a w (published), ||r||^2
#pragma unroll
            for (int s = 0; s < NS; ++s) acc[s] = 0.0;
            for_elems<BD, NT, W>(a0, a1, [&](int row, int s, int c, int li) __attribute__((always_inline)) {
                if (COLV(L, C_CGACT, c) == 0.0) return;
                const double a = COLV(L, C_A, c);
                const int64_t gi = (int64_t)row * W + c;
                const double dv = dd[li];
                qout[gi] = (m == 0 ? 0.0 : qout[gi]) + a * dv;
                const double rv = ures[gi] - a * wcg[gi];
                st_pub(ures + gi, rv);
                acc[s] += rv * rv;
            });
            wave_put<BD, NT, W, NV>(acc, L.red, 0);
            if (!team_sum<NT, NV>(L.red, L.rres, tm, s_flag)) return false;
            if (tid < W) {
                const int c = tid;
                if (COLV(L, C_CGACT, c) != 0.0) {
                    const double rn = L.rres[c];
                    COLV(L, C_BCG, c) = rn / COLV(L, C_RR, c);
                    COLV(L, C_RR, c) = rn;
                    COLV(L, C_CGIT, c) += 1.0;
                    if (sqrt(rn) <= COLV(L, C_STOP, c) || m + 1 >= P.inner_maxiter) COLV(L, C_CGACT, c) = 0.0;
                }
            }
            __syncthreads();
        }
        return true;
    };

    // The same CG with its vectors in registers and its residual in LDS (resl, published in ures for
    // the other workgroups); the solution is left in rq.
    // the products' results go to LDS (the same thread reads each back in the register pass)
    auto stage = [&](int row, int s, int c, int li, double y) __attribute__((always_inline)) { ystg[li] = y; };
    auto inner_cg_r = [&](const double* rhs) __attribute__((always_inline)) -> bool {
        if constexpr (RV) {
            // every register element starts defined (also those a thread does not own), so that none is
            // live from one inner solve into the next
#pragma unroll
            for (int k = 0; k < RK; ++k)
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    rd[k][s] = 0.0;
                    rq[k][s] = 0.0;
                    rw[k][s] = 0.0;
                }
            for_elems_r<NT, W, RI>(a0, a1, [&](auto k, auto s, int row, int c, int li) __attribute__((always_inline)) {
                const double v = ld_pub(rhs + (int64_t)row * W + c);
                resl[li] = v;
                rd[k][s] = v;
            });
            if (tid < W) {
                const int c = tid;
                const double tt = COLV(L, C_TT, c);
                COLV(L, C_RR, c) = tt;
                COLV(L, C_STOP, c) = P.inner_tol * sqrt(tt);
                const bool run = COLV(L, C_ACT, c) != 0.0 && tt > 0.0 && !(sqrt(tt) <= P.inner_tol * sqrt(tt));
                COLV(L, C_CGACT, c) = run ? 1.0 : 0.0;
                COLV(L, C_CGIT, c) = 0.0;
                COLV(L, C_BCG, c) = 0.0;
            }
            __syncthreads();
            for (int m = 0; m < P.inner_maxiter; ++m) {
                int any = 0;
                for (int c = 0; c < W; ++c) any |= COLV(L, C_CGACT, c) != 0.0;
                if (!any) break;
                // (a) d = r + bcg d, w = S r + bcg w (first step: d = rhs, w = S rhs); d^T w
                double acc[NS];
#pragma unroll
                for (int s = 0; s < NS; ++s) acc[s] = 0.0;
                spmm<BD, NT, W, UNIT, decltype(stage), true>(Sb, syS, a0, a1, m == 0 ? rhs : ures, stage, resl);
                for_elems_r<NT, W, RI>(a0, a1, [&](auto k, auto s, int row, int c, int li) __attribute__((always_inline)) {
                    if (COLV(L, C_CGACT, c) == 0.0) return;
                    const double y = ystg[li];
                    if (m == 0) {
                        rw[k][s] = y;
                    } else {
                        const double bc = COLV(L, C_BCG, c);
                        rd[k][s] = resl[li] + bc * rd[k][s];
                        rw[k][s] = y + bc * rw[k][s];
                    }
                    acc[s] += rd[k][s] * rw[k][s];
                });
                wave_put<BD, NT, W, NV>(acc, L.red, 0);
                if (!team_sum<NT, NV>(L.red, L.rres, tm, s_flag)) return false;
                if (tid < W) {
                    const int c = tid;
                    COLV(L, C_A, c) = COLV(L, C_CGACT, c) != 0.0 ? COLV(L, C_RR, c) / L.rres[c] : 0.0;
                }
                __syncthreads();
                // (b) q += a d, r -= a w (LDS, and published), ||r||^2
#pragma unroll
                for (int s = 0; s < NS; ++s) acc[s] = 0.0;
                for_elems_r<NT, W, RI>(a0, a1, [&](auto k, auto s, int row, int c, int li) __attribute__((always_inline)) {
                    if (COLV(L, C_CGACT, c) == 0.0) return;
                    const double a = COLV(L, C_A, c);
                    rq[k][s] += a * rd[k][s];
                    const double rv = resl[li] - a * rw[k][s];
                    resl[li] = rv;
                    st_pub(ures + (int64_t)row * W + c, rv);
                    acc[s] += rv * rv;
                });
                wave_put<BD, NT, W, NV>(acc, L.red, 0);
                if (!team_sum<NT, NV>(L.red, L.rres, tm, s_flag)) return false;
                if (tid < W) {
                    const int c = tid;
                    if (COLV(L, C_CGACT, c) != 0.0) {
                        const double rn = L.rres[c];
                        COLV(L, C_BCG, c) = rn / COLV(L, C_RR, c);
                        COLV(L, C_RR, c) = rn;
                        COLV(L, C_CGIT, c) += 1.0;
                        if (sqrt(rn) <= COLV(L, C_STOP, c) || m + 1 >= P.inner_maxiter) COLV(L, C_CGACT, c) = 0.0;
                    }
                }
                __syncthreads();
            }
        }
        return true;
    };

    // ---- q_0 = S^{-1} b (published); beta_0 = sqrt(b^T q_0) = sqrt(q_0[j])
    if constexpr (RV) {
        if (!inner_cg_r(tprev)) return false;
        for_elems_r<NT, W, RI>(a0, a1, [&](auto k, auto s, int row, int c, int li) __attribute__((always_inline)) {
            st_pub(qcur + (int64_t)row * W + c, COLV(L, C_CGIT, c) > 0.0 ? rq[k][s] : 0.0);
        });
        if (tid < W) COLV(L, C_INNER, tid) += COLV(L, C_CGIT, tid);
    } else if constexpr (!SID) {
        if (!inner_cg(tprev, qcur)) return false;
        for_elems<BD, NT, W>(a0, a1, [&](int row, int s, int c, int li) __attribute__((always_inline)) {
            const int64_t gi = (int64_t)row * W + c;
            st_pub(qcur + gi, COLV(L, C_CGIT, c) > 0.0 ? qcur[gi] : 0.0);
        });
        if (tid < W) COLV(L, C_INNER, tid) += COLV(L, C_CGIT, tid);
    }
    {
        double acc[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) acc[s] = 0.0;
        for_elems<BD, NT, W>(a0, a1, [&](int row, int s, int c, int li) __attribute__((always_inline)) {
            if (row == (int)COLV(L, C_BLOC, c)) acc[s] += ld_pub(qcur + (int64_t)row * W + c);
        });
        wave_put<BD, NT, W, NV>(acc, L.red, 0);
        if (!team_sum<NT, NV>(L.red, L.rres, tm, s_flag)) return false;
        if (tid < W) {
            const int c = tid;
            const double bb = L.rres[c];
            const double b0 = bb > 0.0 ? sqrt(bb) : 0.0;
            COLV(L, C_BETA0, c) = b0;
            COLV(L, C_BCUR, c) = b0;
            COLV(L, C_SUMW2, c) = b0 > 0.0 ? 1.0 / (b0 * b0) : 0.0;
            if (COLV(L, C_ACT, c) != 0.0 && !(b0 > 0.0 && isfinite(b0))) {
                COLV(L, C_BAD, c) = isfinite(bb) ? 2.0 : 1.0;
                COLV(L, C_ACT, c) = 0.0;
            }
        }
        __syncthreads();
        for (int m = tid; m < npairs; m += NT) {
            const int c = (rank + G * m) / K;
            L.p_g[m] = zmk(COLV(L, C_BETA0, c), 0.0);
            if (COLV(L, C_RHS, c) < 0) {
                L.p_done[m] = 2;
            } else if (COLV(L, C_BAD, c) != 0.0) {
                L.p_done[m] = 2;
                L.p_stat[m] = COLV(L, C_BAD, c) == 1.0 ? ST_NONFINITE : ST_BREAKDOWN;
            }
        }
        __syncthreads();
    }

    // ---- outer iterations
    for (int n = 0; n < maxiter; ++n) {
        int any = 0;
        for (int c = 0; c < W; ++c) any |= COLV(L, C_ACT, c) != 0.0;
        if (!any) break;
        // (1) u = H q_n / bcur into ures; alpha partial sum v_i u_i; and the unfinished owned pairs
        {
            double acc[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s) acc[s] = 0.0;
            if constexpr (RV) {
                spmm<BD, NT, W, false>(Hb, sy, a0, a1, qcur, [&](int row, int s, int c, int li, double y) __attribute__((always_inline)) {
                    if (COLV(L, C_ACT, c) == 0.0) return;
                    const double ib = 1.0 / COLV(L, C_BCUR, c);
                    const double u = y * ib;
                    ystg[li] = u;
                    acc[s] += ld_pub(qcur + (int64_t)row * W + c) * ib * u;
                });
            } else {
                spmm<BD, NT, W, false>(Hb, sy, a0, a1, qcur, [&](int row, int s, int c, int li, double y) __attribute__((always_inline)) {
                    if (COLV(L, C_ACT, c) == 0.0) return;
                    const double ib = 1.0 / COLV(L, C_BCUR, c);
                    const double u = y * ib;
                    ures[(int64_t)row * W + c] = u;
                    acc[s] += ld_pub(qcur + (int64_t)row * W + c) * ib * u;
                });
            }
            wave_put<BD, NT, W, NV>(acc, L.red, 0);
            if (tid < W) {
                int lo, hi, cnt = 0;
                col_range(tid, K, G, rank, npairs, lo, hi);
                for (int m = lo; m < hi; ++m) cnt += L.p_done[m] == 0;
                L.red[W + tid] = (double)cnt;
                for (int w = 1; w < NW; ++w) L.red[w * NV + W + tid] = 0.0;
            }
            if (!team_sum<NT, NV>(L.red, L.rres, tm, s_flag)) return false;
            if (tid < W) {
                const int c = tid;
                COLV(L, C_ALPHA, c) = L.rres[c];
                if (COLV(L, C_ACT, c) != 0.0 && L.rres[W + c] == 0.0) COLV(L, C_ACT, c) = 0.0;
            }
            __syncthreads();
        }
        any = 0;
        for (int c = 0; c < W; ++c) any |= COLV(L, C_ACT, c) != 0.0;
        if (!any) break;
        // (2) t_n = u - (alpha / bcur) t_{n-1} - (blan / bprev) t_{n-2} into tcur (published); ||t_n||^2
        {
            double acc[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s) acc[s] = 0.0;
            auto tstep = [&](int row, int c, double u) __attribute__((always_inline)) -> double {
                const int64_t gi = (int64_t)row * W + c;
                const double bl = COLV(L, C_BLAN, c);
                double tv = u - COLV(L, C_ALPHA, c) / COLV(L, C_BCUR, c) * ld_pub(tprev + gi);
                if (bl != 0.0) tv -= bl / COLV(L, C_BPREV, c) * ld_pub(tcur + gi);
                st_pub(tcur + gi, tv);
                return tv * tv;
            };
            if constexpr (RV) {
                for_elems<BD, NT, W>(a0, a1, [&](int row, int s, int c, int li) __attribute__((always_inline)) {
                    if (COLV(L, C_ACT, c) != 0.0) acc[s] += tstep(row, c, ystg[li]);
                });
            } else {
                for_elems<BD, NT, W>(a0, a1, [&](int row, int s, int c, int li) __attribute__((always_inline)) {
                    if (COLV(L, C_ACT, c) != 0.0) acc[s] += tstep(row, c, ures[(int64_t)row * W + c]);
                });
            }
            wave_put<BD, NT, W, NV>(acc, L.red, 0);
            if (!team_sum<NT, NV>(L.red, L.rres, tm, s_flag)) return false;
            if (tid < W) COLV(L, C_TT, tid) = COLV(L, C_ACT, tid) != 0.0 ? L.rres[tid] : 0.0;
            __syncthreads();
        }
        // (3) q_{n+1} = S^{-1} t_n, published;  (4) q^T t
        if constexpr (SID) {
            if (tid < W) COLV(L, C_QT, tid) = COLV(L, C_TT, tid);
            __syncthreads();
        } else {
            double acc[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s) acc[s] = 0.0;
            if constexpr (RV) {
                if (!inner_cg_r(tcur)) return false;
                for_elems_r<NT, W, RI>(a0, a1, [&](auto k, auto s, int row, int c, int li) __attribute__((always_inline)) {
                    if (COLV(L, C_ACT, c) == 0.0) return;
                    const int64_t gi = (int64_t)row * W + c;
                    const double v = COLV(L, C_CGIT, c) > 0.0 ? rq[k][s] : 0.0;
                    st_pub(qnew + gi, v);
                    acc[s] += v * ld_pub(tcur + gi);
                });
            } else {
                if (!inner_cg(tcur, qnew)) return false;
                for_elems<BD, NT, W>(a0, a1, [&](int row, int s, int c, int li) __attribute__((always_inline)) {
                    if (COLV(L, C_ACT, c) == 0.0) return;
                    const int64_t gi = (int64_t)row * W + c;
                    const double v = COLV(L, C_CGIT, c) > 0.0 ? qnew[gi] : 0.0;
                    st_pub(qnew + gi, v);
                    acc[s] += v * ld_pub(tcur + gi);
                });
            }
            wave_put<BD, NT, W, NV>(acc, L.red, 0);
            if (!team_sum<NT, NV>(L.red, L.rres, tm, s_flag)) return false;
            if (tid < W) {
                const bool act = COLV(L, C_ACT, tid) != 0.0;
                COLV(L, C_QT, tid) = act ? L.rres[tid] : 0.0;
                if (act) COLV(L, C_INNER, tid) += COLV(L, C_CGIT, tid);
            }
            __syncthreads();
        }
        if (tid < W) {
            const int c = tid;
            if (COLV(L, C_ACT, c) != 0.0) {
                const double qt = COLV(L, C_QT, c), al = COLV(L, C_ALPHA, c);
                const bool bad = !isfinite(qt) || !isfinite(al);
                COLV(L, C_BNEXT, c) = qt > 0.0 ? sqrt(qt) : 0.0;
                COLV(L, C_BAD, c) = bad ? 1.0 : (qt < 0.0 ? 2.0 : 0.0);
                if (!bad && qt > 0.0) COLV(L, C_SUMW2, c) += COLV(L, C_TT, c) / qt;
                COLV(L, C_NOUT, c) = n + 1;
            }
        }
        __syncthreads();
        // (5) shift step of the owned pairs: FP64 complex scalars, one thread per pair
        for (int m = tid; m < npairs; m += NT) {
            const int p = rank + G * m, c = p / K, k = p - c * K;
            if (L.p_done[m] || COLV(L, C_ACT, c) == 0.0) continue;
            if (COLV(L, C_BAD, c) != 0.0) {
                L.p_stat[m] = COLV(L, C_BAD, c) == 1.0 ? ST_NONFINITE : ST_BREAKDOWN;
                L.p_done[m] = 2;
                continue;
            }
            const zc zk = zmk(P.z[2 * k], P.z[2 * k + 1]);
            const double alpha = COLV(L, C_ALPHA, c), beta = COLV(L, C_BLAN, c), bnext = COLV(L, C_BNEXT, c);
            if constexpr (GAL) {
                const zc dprev = L.p_s1[m];
                zc cc = zmk(0.0, 0.0), dn = zmk(zk.re - alpha, zk.im), gk = zmk(COLV(L, C_BETA0, c), 0.0);
                if (n > 0) {
                    cc = zdiv(zmk(beta, 0.0), dprev);
                    dn = zsub(dn, zmul(zmk(beta, 0.0), cc));
                    gk = zmul(cc, L.p_g[m]);
                }
                if (zzero(dn) || !zfinite(dn)) {
                    L.p_stat[m] = zfinite(dn) ? ST_BREAKDOWN : ST_NONFINITE;
                    L.p_done[m] = 2;
                    continue;
                }
                L.p_g[m] = gk;
                L.p_tau[m] = zdiv(gk, dn);
                L.p_e[m] = cc;
                L.p_s1[m] = dn;
            } else {
                const zc a_prev = zmk(-beta, 0.0);
                const zc a_diag = zmk(zk.re - alpha, zk.im);
                const zc a_next = zmk(-bnext, 0.0);
                const zc e = zmul(L.p_s2[m], a_prev);
                const zc f0 = zmk(L.p_c2[m] * a_prev.re, L.p_c2[m] * a_prev.im);
                const zc s1 = L.p_s1[m];
                const double c1 = L.p_c1[m];
                const zc f = zadd(zmk(c1 * f0.re, c1 * f0.im), zmul(s1, a_diag));
                const zc gam = zadd(zmul(zmk(-s1.re, s1.im), f0), zmk(c1 * a_diag.re, c1 * a_diag.im));
                double cr;
                zc sr, rnn;
                givens(gam, a_next, cr, sr, rnn);
                if (zzero(rnn)) {
                    L.p_stat[m] = ST_BREAKDOWN;
                    L.p_done[m] = 2;
                    continue;
                }
                const zc gk = L.p_g[m];
                L.p_tau[m] = zmk(cr * gk.re, cr * gk.im);
                L.p_g[m] = zmul(zmk(-sr.re, sr.im), gk);
                L.p_e[m] = e;
                L.p_f[m] = f;
                L.p_irnn[m] = zdiv(zmk(1.0, 0.0), rnn);
                L.p_c2[m] = c1;
                L.p_s2[m] = s1;
                L.p_c1[m] = cr;
                L.p_s1[m] = sr;
            }
        }
        __syncthreads();
        // the pairs updated this iteration (wave 0 builds the list in ascending m), and their count per column
        if (tid < 64) {
            int cnt = 0;
            for (int base = 0; base < npairs; base += 64) {
                const int m = base + tid;
                bool fl = false;
                if (m < npairs) fl = !L.p_done[m] && COLV(L, C_ACT, (rank + G * m) / K) != 0.0;
                const uint64_t mk = __ballot(fl);
                const int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(mk >> 32),
                                                            __builtin_amdgcn_mbcnt_lo((uint32_t)mk, 0));
                if (fl) L.upd[cnt + below] = m;
                cnt += __popcll(mk);
            }
            if (tid == 0) L.ctl[0] = cnt;
            if (tid < W) {
                int lo, hi, cu = 0;
                col_range(tid, K, G, rank, npairs, lo, hi);
                if (COLV(L, C_ACT, tid) != 0.0)
                    for (int m = lo; m < hi; ++m) cu += L.p_done[m] == 0;
                COLV(L, C_SUMUPD, tid) += (double)cu;
            }
        }
        __syncthreads();
        const int nupd = L.ctl[0];
        // requested rows: v_n = q_n / bcur at each row; the direction(s) and x of every updated pair
        for (int idx = tid; idx < nupd * nIpi; idx += NT) {
            const int mm = idx / nIpi, o = idx - mm * nIpi;
            const int m = L.upd[mm];
            const int p = rank + G * m, c = p / K;
            const RhsInfo ri = P.rhs[(int)COLV(L, C_RHS, c)];
            if (o >= ri.nout) continue;
            const int row = P.out_local[ri.out_base + o];
            const double vv = ld_pub(qcur + (int64_t)row * W + c) / COLV(L, C_BCUR, c);
            double2* base = pairmem + (int64_t)p * nIpi * nrow_arr;
            double2* xI = base;
            const zc tk = L.p_tau[m];
            zc dn;
            if constexpr (GAL) {
                double2* D0 = base + nIpi;
                const double2 pv = D0[o];
                const zc cc = L.p_e[m];
                dn = zmk(vv + cc.re * pv.x - cc.im * pv.y, cc.re * pv.y + cc.im * pv.x);
                D0[o] = make_double2(dn.re, dn.im);
            } else {
                double2* Da = base + nIpi;
                double2* Db = base + 2 * nIpi;
                double2* Dn2 = (n & 1) ? Db : Da;     // holds d_{n-2}; receives d_n
                double2* Dn1 = (n & 1) ? Da : Db;     // holds d_{n-1}
                const double2 d2 = Dn2[o], d1 = Dn1[o];
                const zc num = zsub(zsub(zmk(vv, 0.0), zmul(L.p_e[m], zmk(d2.x, d2.y))),
                                    zmul(L.p_f[m], zmk(d1.x, d1.y)));
                dn = zmul(num, L.p_irnn[m]);
                Dn2[o] = make_double2(dn.re, dn.im);
            }
            const double2 xv = xI[o];
            xI[o] = make_double2(xv.x + tk.re * dn.re - tk.im * dn.im, xv.y + tk.re * dn.im + tk.im * dn.re);
        }
        // convergence of the updated pairs (||b|| = 1): COCG iterates |zeta_n| ||t_n||, QMR its bound
        for (int mm = tid; mm < nupd; mm += NT) {
            const int m = L.upd[mm];
            const int c = (rank + G * m) / K;
            const double bnext = COLV(L, C_BNEXT, c);
            const double est = GAL ? zabs(L.p_tau[m]) * sqrt(COLV(L, C_TT, c))
                                   : zabs(L.p_g[m]) * sqrt(COLV(L, C_SUMW2, c));
            L.p_res[m] = est;
            if (est < P.tol || bnext == 0.0) {
                L.p_done[m] = 1;
                L.p_stat[m] = ST_CONVERGED;
                L.p_it[m] = n + 1;
                if (bnext == 0.0) L.p_res[m] = 0.0;
            }
        }
        // (6) the next step's normalisations (after every thread has read this step's); a column whose
        // recurrence broke down or closed stops
        __syncthreads();
        if (tid < W) {
            const int c = tid;
            if (COLV(L, C_ACT, c) != 0.0) {
                if (COLV(L, C_BAD, c) != 0.0 || COLV(L, C_BNEXT, c) == 0.0) {
                    COLV(L, C_ACT, c) = 0.0;
                } else {
                    COLV(L, C_BPREV, c) = COLV(L, C_BCUR, c);
                    COLV(L, C_BCUR, c) = COLV(L, C_BNEXT, c);
                    COLV(L, C_BLAN, c) = COLV(L, C_BNEXT, c);
                }
            }
        }
        __syncthreads();
        if constexpr (SID) {
            double* t_ = tprev;      // t_{n-1} (= q_n): receives t_{n+1} next
            tprev = tcur;            // t_n
            tcur = t_;
            qcur = tprev;            // q_{n+1} = t_n
        } else {
            double* t_ = tprev;
            tprev = tcur;
            tcur = t_;
            double* q_ = qcur;
            qcur = qnew;
            qnew = q_;
        }
    }

    // ---- outputs of the owned pairs
    for (int idx = tid; idx < npairs * nIpi; idx += NT) {
        const int m = idx / nIpi, o = idx - m * nIpi;
        const int p = rank + G * m, c = p / K, k = p - c * K;
        const int rj = (int)COLV(L, C_RHS, c);
        if (rj < 0) continue;
        const RhsInfo ri = P.rhs[rj];
        if (o >= ri.nout) continue;
        const double2 xv = pairmem[(int64_t)p * nIpi * nrow_arr + o];
        const int64_t ob = (P.out_off[rj] * (int64_t)K + (int64_t)k * ri.nout + o) * 2;
        P.out[ob] = xv.x;
        P.out[ob + 1] = xv.y;
    }
    for (int m = tid; m < npairs; m += NT) {
        const int p = rank + G * m, c = p / K, k = p - c * K;
        const int rj = (int)COLV(L, C_RHS, c);
        if (rj < 0) continue;
        const int64_t o = (int64_t)rj * K + k;
        if (P.iters) P.iters[o] = L.p_it[m];
        if (P.status) P.status[o] = (int8_t)L.p_stat[m];
        if (P.resid) P.resid[o] = L.p_res[m];
    }
    if (tid < W && P.stats) {
        const int c = tid;
        const int rj = (int)COLV(L, C_RHS, c);
        if (rj >= 0) {
            int64_t* st_ = P.stats + (int64_t)rj * NSTAT;
            // the shift updates of every workgroup's pairs add up in [1] (zeroed before the launch)
            atomicAdd((unsigned long long*)(st_ + 1), (unsigned long long)COLV(L, C_SUMUPD, c));
            if (rank == 0) {
                st_[0] = (int64_t)COLV(L, C_NOUT, c);
                st_[2] = (int64_t)COLV(L, C_INNER, c);
                st_[3] = 0;
                st_[4] = M;
                st_[5] = sy.rowptr[sy.nrows] - sy.rowptr[0];
                st_[6] = 0;
                st_[7] = 0;
            }
        }
    }
    __syncthreads();
    return true;
}

// Persistent team kernel: the team's rank-0 workgroup takes the next panel
// from the work queue and publishes it; the team solves it together.
template <int BD, int NT, int W, bool SID, bool GAL, bool DL, bool UNIT, int RI>
__global__ __launch_bounds__(NT) void k_team(TParams T) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_flag, s_job;
    const int G = T.G;
    const int b = blockIdx.x;
    Team tm;
    tm.G = G;
    if (gridDim.x % (8 * G) == 0) {
        // workgroups are dealt to the eight XCDs in turn: keep a team on one XCD (one L2)
        const int x = b & 7, y = b >> 3;
        tm.id = (y / G) * 8 + x;
        tm.rank = y % G;
    } else {
        tm.id = b / G;
        tm.rank = b % G;
    }
    tm.ctr = T.sync + (int64_t)tm.id * 32;
    tm.job = tm.ctr + 1;
    tm.pstride = T.pstride;
    tm.part = T.part + (int64_t)tm.id * 2 * G * T.pstride;
    tm.abort_flag = T.abort_flag;
    tm.spin_ticks = T.spin_ticks;
    tm.epoch = 0;
    Lds L = carve(smem, NT, W, T.pairs_max);
    L.d = DL ? (double*)(smem + lds_fixed_bytes(NT, W, T.pairs_max)) : nullptr;
    const KParams& P = T.k;
    for (;;) {
        // Between panels the rows change owners (each panel splits its own system's rows), and the
        // ordinary stores of the last panel may still sit in another XCD's L2: every member writes its
        // L2 back before it arrives and drops stale lines after the wait (agent-scope release and
        // acquire, once per panel; the waits inside a panel order only the device-coherent accesses)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (tm.rank == 0 && threadIdx.x == 0) st_pub_i(tm.job, atomicAdd(P.queue, 1));
        if (!team_wait(tm, &s_flag)) break;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (threadIdx.x == 0) s_job = ld_pub_i(tm.job);
        __syncthreads();
        const int job = __builtin_amdgcn_readfirstlane(s_job);   // uniform: its loads are scalar
        __syncthreads();
        if (job >= T.npanels) break;
        if (!solve_panel<BD, NT, W, SID, GAL, DL, UNIT, RI>(T, job, tm, L, &s_flag)) {
            // a wait was abandoned: this panel's pairs owned here are reported as such
            const int npairs = (W * P.K - tm.rank + G - 1) / G;
            for (int m = threadIdx.x; m < npairs; m += NT) {
                const int p = tm.rank + G * m, c = p / P.K, k = p - c * P.K;
                const int q = job * W + c;
                if (q < P.nrhs && P.status) P.status[(int64_t)P.order[q] * P.K + k] = (int8_t)ST_ABORTED;
            }
            break;
        }
    }
}

// Register-resident instances compiled: (threads, panel width, block-row quads per wave).
// (the one shape whose instances keep every value in registers)
__host__ __device__ constexpr bool rv_ok(int NT, int W, int RI) { return NT == 512 && W == 4 && RI == 8; }

// Calls f.template run<BD, NT, W, SID, GAL, DL, UNIT, RI>() for the compiled instance.
// variant: 0 S = I, 1 S with the CG direction in LDS, 2 the same with S = I + off-diagonal blocks,
// 3 S with the direction in HBM, 4 register-resident CG with S = I + off-diagonal blocks,
// 5 register-resident CG with S as stored
template <int BD, int NT, int W, bool GAL, int RI, bool UN, class F>
static hipError_t rv_run(F& f) {
    if constexpr (BD == 4 && W % 4 == 0 && rv_ok(NT, W, RI)) return f.template run<BD, NT, W, false, GAL, true, UN, RI>();
    else return hipErrorInvalidValue;
}
template <int BD, int NT, int W, bool GAL, bool UN, class F>
static hipError_t rv_by_ri(int ri, F& f) {
    if (ri == 8) return rv_run<BD, NT, W, GAL, 8, UN>(f);
    return hipErrorInvalidValue;
}
template <int BD, int NT, int W, bool GAL, class F>
static hipError_t by_variant(int variant, int ri, F& f) {
    switch (variant) {
        case 0: return f.template run<BD, NT, W, true, GAL, false, false, 0>();
        case 1: return f.template run<BD, NT, W, false, GAL, true, false, 0>();
        case 2: return f.template run<BD, NT, W, false, GAL, true, true, 0>();
        case 3: return f.template run<BD, NT, W, false, GAL, false, false, 0>();
        case 4: return rv_by_ri<BD, NT, W, GAL, true>(ri, f);
        case 5: return rv_by_ri<BD, NT, W, GAL, false>(ri, f);
        default: return hipErrorInvalidValue;
    }
}
template <int BD, int NT, int W, class F>
static hipError_t by_gal(bool gal, int variant, int ri, F& f) {
    return gal ? by_variant<BD, NT, W, true>(variant, ri, f) : by_variant<BD, NT, W, false>(variant, ri, f);
}
template <int BD, int NT, class F>
static hipError_t by_w(int W, bool gal, int variant, int ri, F& f) {
    if constexpr (BD == 4) {
        if (W == 8) return by_gal<BD, NT, 8>(gal, variant, ri, f);
        if (W == 4) return by_gal<BD, NT, 4>(gal, variant, ri, f);
    }
    if (W != 1 || variant >= 4) return hipErrorInvalidValue;
    return by_gal<BD, NT, 1>(gal, variant, ri, f);
}
template <int BD, class F>
static hipError_t by_nt(int nt, int W, bool gal, int variant, int ri, F& f) {
    if (nt == 1024) return by_w<BD, 1024>(W, gal, variant, ri, f);
    if (nt == 512) return by_w<BD, 512>(W, gal, variant, ri, f);
    return hipErrorInvalidValue;
}
template <class F>
static hipError_t dispatch(int bd, int nt, int W, bool gal, int variant, int ri, F& f) {
    switch (bd) {
        case 1: return by_nt<1>(nt, W, gal, variant, ri, f);
        case 4: return by_nt<4>(nt, W, gal, variant, ri, f);
        case 9: return by_nt<9>(nt, W, gal, variant, ri, f);
        default: return hipErrorInvalidValue;
    }
}

struct Launch {
    const TParams* T;
    int grid, nt;
    size_t lds;
    hipStream_t st;
    template <int BD, int NT, int W, bool SID, bool GAL, bool DL, bool UNIT, int RI>
    hipError_t run() {
        hipLaunchKernelGGL((k_team<BD, NT, W, SID, GAL, DL, UNIT, RI>), dim3(grid), dim3(NT), lds, st, *T);
        return hipGetLastError();
    }
};

struct Occupancy {
    size_t lds;
    int* out;
    size_t* priv;
    template <int BD, int NT, int W, bool SID, bool GAL, bool DL, bool UNIT, int RI>
    hipError_t run() {
        hipFuncAttributes fa{};
        hipError_t e = hipFuncGetAttributes(&fa, (const void*)k_team<BD, NT, W, SID, GAL, DL, UNIT, RI>);
        if (e != hipSuccess) return e;
        *priv = fa.localSizeBytes;
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, k_team<BD, NT, W, SID, GAL, DL, UNIT, RI>, NT, lds);
    }
};

}  // namespace team

size_t team_lds_bytes(int nt, int W, int pairs, int rows_max, bool dl, bool rv) {
    return team::lds_bytes(nt, W, pairs, rows_max, dl, rv);
}

int64_t team_ws_bytes(int W, int K, int64_t Mp, int64_t nIp, bool qmr) { return team::team_bytes(W, K, Mp, nIp, qmr); }

hipError_t launch_team(const TParams& T, int bd, bool gal, int variant, int ri, int nt, int grid, size_t lds,
                       hipStream_t st) {
    team::Launch f{&T, grid, nt, lds, st};
    return team::dispatch(bd, nt, T.W, gal, variant, ri, f);
}

hipError_t team_occupancy(int bd, bool gal, int variant, int ri, int nt, int W, size_t lds, int* per_cu,
                          size_t* private_bytes) {
    *per_cu = 0;
    *private_bytes = 0;
    team::Occupancy f{lds, per_cu, private_bytes};
    return team::dispatch(bd, nt, W, gal, variant, ri, f);
}

bool team_rv_ok(int nt, int W, int ri) { return team::rv_ok(nt, W, ri); }

}  // namespace scocg
