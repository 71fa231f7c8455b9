// Generalized shifted QMR (gfx950): the paper's second Krylov solver for
// (z_k S - H) x = b (Sec. 3, item (ii)), here for real symmetric H, real SPD
// S and b = e_j, where the Krylov space shared by all shifts is real.
//
// One workgroup per RHS (persistent, atomic queue, as the COCG solver).  Per
// iteration n the workgroup runs one step of the S-Lanczos process on
// S^{-1}H in REAL arithmetic:
//   u = H v_n;  alpha_n = v_n^T u;  t = u - alpha_n w_n - beta_n w_{n-1}
//   q = S^{-1} t (inner CG on real vectors);  beta_{n+1} = sqrt(q^T t)
//   v_{n+1} = q / beta_{n+1};  w_{n+1} = t / beta_{n+1}        (w = S v)
// and every unconverged shift k (one thread each, FP64 complex scalars) adds
// the new column (-beta_n, z_k - alpha_n, -beta_{n+1}) of Hbar(z_k) = z_k I -
// Tbar to its QR factorisation with complex Givens rotations; the requested
// rows of the direction d and of x_k follow from the three-term recurrence
// d_n = (v_n - e d_{n-2} - f d_{n-1}) / R_nn, x_k += tau_n d_n.  Shift k stops
// when its quasi-residual |g_{n+1}| times (sum_{i<=n+1} ||w_i||^2)^{1/2}, an
// upper bound of ||b - (z_k S - H) x_k||, is below tol ||b||.  No seed shift
// and no seed switching: the Lanczos process does not depend on the shifts.
// All long-vector traffic is real (8 bytes per element), half that of the
// complex COCG seed process.
//
// The same basis also gives the shifted COCG iterates themselves (GAL): with
// a real basis COCG's unconjugated form u^T S v is the S-inner product, so
// COCG's Galerkin condition makes x_k = V_n y_k with (z_k I - T_n) y_k =
// beta_0 e_1.  Each shift factors z_k I - T_n as L D L^T, one pivot per
// iteration, delta_n = z_k - alpha_n - beta_n^2 / delta_{n-1}, and updates
// p_n = v_n + (beta_n / delta_{n-1}) p_{n-1}, x_k += zeta_n p_n with
// zeta_n = g_n / delta_n, g_n = (beta_n / delta_{n-1}) g_{n-1}; its residual
// is zeta_n t (t = beta_{n+1} w_{n+1}), whose norm |zeta_n| ||t|| is the
// stopping test.  Same iterates as the seed-switching COCG in exact
// arithmetic, without a seed.
#include <hip/hip_runtime.h>

#include "scocg_device.hpp"
#include "scocg_params.hpp"

namespace scocg {

namespace qmr {

enum { ST_CONVERGED = 0, ST_MAXITER = 1, ST_BREAKDOWN = 2, ST_NONFINITE = 3 };

struct Sys {
    const int64_t* rowptr;
    const int32_t* ecol;
    const int32_t* egid;   // nullptr: entry e holds block gbase + e (the global system)
    int64_t gbase;
    int nrows;
    int M;
    int ew;                // > 0: ELL form, ew entries per block row (rowptr unused)
};

// LDS: per shift the two previous rotations (c real, s complex), the running
// right-hand side g, and this iteration's update coefficients.
struct Lds {
    double* c1;
    double* c2;
    zc* s1;
    zc* s2;
    zc* g;
    zc* tau;
    zc* e;
    zc* f;
    zc* irnn;
    double* resid;
    int* iters;
    int* upd;
    unsigned char* done;
    unsigned char* stat;
    double* red;
    int* ctl;    // [0] shifts updated this iteration, [1] shifts done
};

__host__ __device__ inline size_t lds_bytes(int K, int NT) {
    size_t b = 2 * sizeof(double) * (size_t)K + 7 * sizeof(zc) * (size_t)K + sizeof(double) * (size_t)K +
               2 * sizeof(int) * (size_t)K + 2 * (size_t)K;
    b = (b + 15) & ~(size_t)15;
    b += sizeof(double) * (NT / 64) * 4 + 4 * sizeof(int);
    return b;
}

// Offset of the inner CG's search direction when it is kept in LDS (DL):
// after the per-shift arrays, M_j doubles.
__host__ __device__ inline size_t lds_dir_offset(int K, int NT) { return (lds_bytes(K, NT) + 15) & ~(size_t)15; }

__device__ inline Lds carve(unsigned char* q, int K, int NT) {
    Lds L;
    L.s1 = (zc*)q; q += sizeof(zc) * K;
    L.s2 = (zc*)q; q += sizeof(zc) * K;
    L.g = (zc*)q; q += sizeof(zc) * K;
    L.tau = (zc*)q; q += sizeof(zc) * K;
    L.e = (zc*)q; q += sizeof(zc) * K;
    L.f = (zc*)q; q += sizeof(zc) * K;
    L.irnn = (zc*)q; q += sizeof(zc) * K;
    L.c1 = (double*)q; q += sizeof(double) * K;
    L.c2 = (double*)q; q += sizeof(double) * K;
    L.resid = (double*)q; q += sizeof(double) * K;
    L.iters = (int*)q; q += sizeof(int) * K;
    L.upd = (int*)q; q += sizeof(int) * K;
    L.done = q; q += K;
    L.stat = q; q += K;
    q = (unsigned char*)(((uintptr_t)q + 15) & ~(uintptr_t)15);
    L.red = (double*)q; q += sizeof(double) * (NT / 64) * 4;
    L.ctl = (int*)q;
    return L;
}

// Real row sum over one row's block entries (row r of block row a): the
// entries in chunks whose index loads go together, then all block and
// vector loads of the chunk, then the arithmetic; a chunk's slots past the
// row's end re-read its last entry and add zero (every block row holds its
// diagonal block).  4x4 blocks: the quad of lanes of one block row shares
// the vector block by DPP.  DIRECT (the global system, entry e holds block
// e): the block loads need no block index, so they go out with the column
// index loads and a chunk waits on one dependent load instead of two.
template <int BD, int NT>
struct Chunk {
    static constexpr int v = (BD == 1 ? 8 : (BD <= 4 ? 4 : 2)) / (NT >= 1024 ? 2 : 1);
    static constexpr int value = v < 1 ? 1 : v;
};

template <int BD, int NT, bool DIRECT, int CH = Chunk<BD, NT>::value>
__device__ __forceinline__ double row_dot(const double* __restrict__ A, const Sys& sy, int a, int r,
                                          const double* __restrict__ p) {
    constexpr bool QUAD = BD == 4 && NT % 64 == 0;
    const int64_t e0 = sy.rowptr[a], e1 = sy.rowptr[a + 1];
    double acc = 0.0;
    for (int64_t eb = e0; eb < e1; eb += CH) {
        int32_t b[CH];
        int64_t g[CH];
        bool ok[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            ok[u] = eb + u < e1;
            const int64_t e = ok[u] ? eb + u : e1 - 1;
            b[u] = sy.ecol[e];
            g[u] = DIRECT ? sy.gbase + e : (int64_t)sy.egid[e];
        }
        double own[QUAD ? CH : 1];
        double av[CH][BD];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int64_t off = (g[u] * BD + r) * BD;
            if constexpr (QUAD) own[u] = p[(int64_t)b[u] * BD + r];
#pragma unroll
            for (int c = 0; c < BD; ++c) av[u][c] = A[off + c];
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const double* pb = p + (int64_t)b[u] * BD;
#pragma unroll
            for (int c = 0; c < BD; ++c) {
                double pv;
                if constexpr (QUAD) {
                    if (c == 0) pv = quad_bcast<0>(own[u]);
                    else if (c == 1) pv = quad_bcast<1>(own[u]);
                    else if (c == 2) pv = quad_bcast<2>(own[u]);
                    else pv = quad_bcast<3>(own[u]);
                } else {
                    pv = pb[c];
                }
                acc += (ok[u] ? av[u][c] : 0.0) * pv;
            }
        }
    }
    return acc;
}

// The same row product on the ELL form (every block row has sy.ew entries,
// at a * ew + u): no row-pointer load, and a chunk of CH entries (column
// indices and blocks together) goes out at once, so a row costs ceil(ew / CH)
// memory latencies instead of one for its extent plus one per chunk.
template <int BD, int NT>
struct ChunkEll {
    static constexpr int v = (BD <= 4 ? 8 : 4) / (NT >= 1024 ? 2 : 1);
    static constexpr int value = v < 1 ? 1 : v;
};

template <int BD, int NT, int CH>
__device__ __forceinline__ double row_dot_ell(const double* __restrict__ A, const Sys& sy, int a, int r,
                                              const double* __restrict__ p) {
    constexpr bool QUAD = BD == 4 && NT % 64 == 0;
    const int ew = sy.ew;
    const int64_t e0 = (int64_t)a * ew;
    double acc = 0.0;
    for (int u0 = 0; u0 < ew; u0 += CH) {
        int32_t b[CH];
        double av[CH][BD];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            if (u0 + u < ew) {      // the same in every lane
                const int64_t e = e0 + u0 + u;
                b[u] = sy.ecol[e];
#pragma unroll
                for (int c = 0; c < BD; ++c) av[u][c] = A[(e * BD + r) * BD + c];
            } else {
                b[u] = a;
#pragma unroll
                for (int c = 0; c < BD; ++c) av[u][c] = 0.0;
            }
        }
        double own[QUAD ? CH : 1];
#pragma unroll
        for (int u = 0; u < CH; ++u)
            if constexpr (QUAD) own[u] = p[(int64_t)b[u] * BD + r];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const double* pb = p + (int64_t)b[u] * BD;
#pragma unroll
            for (int c = 0; c < BD; ++c) {
                double pv;
                if constexpr (QUAD) {
                    if (c == 0) pv = quad_bcast<0>(own[u]);
                    else if (c == 1) pv = quad_bcast<1>(own[u]);
                    else if (c == 2) pv = quad_bcast<2>(own[u]);
                    else pv = quad_bcast<3>(own[u]);
                } else {
                    pv = pb[c];
                }
                acc += av[u][c] * pv;
            }
        }
    }
    return acc;
}

// y = A x over this thread's rows; returns the partial x^T y.  UNIT: A is
// I plus the blocks of sy (S with exactly-identity diagonal blocks, its
// off-diagonal blocks alone in sy), so the identity part is x_i itself.
template <int BD, int NT, bool DIRECT, bool UNIT, int CH = Chunk<BD, NT>::value>
__device__ __forceinline__ double spmv_rows(const double* __restrict__ A, const Sys& sy,
                                            const double* __restrict__ x, double* __restrict__ y) {
    double part = 0.0;
    for (int i = threadIdx.x; i < sy.M; i += NT) {
        const int a = i / BD, r = i - a * BD;
        const double xi = x[i];
        const double v = row_dot<BD, NT, DIRECT, CH>(A, sy, a, r, x) + (UNIT ? xi : 0.0);
        y[i] = v;
        part += xi * v;
    }
    return part;
}

// UNIT on the ELL form: y = x + (off-diagonal blocks) x, CH entries per chunk.
template <int BD, int NT, int CH = ChunkEll<BD, NT>::value>
__device__ __forceinline__ double spmv_rows_ell(const double* __restrict__ A, const Sys& sy,
                                                const double* __restrict__ x, double* __restrict__ y) {
    double part = 0.0;
    for (int i = threadIdx.x; i < sy.M; i += NT) {
        const int a = i / BD, r = i - a * BD;
        const double xi = x[i];
        const double v = row_dot_ell<BD, NT, CH>(A, sy, a, r, x) + xi;
        y[i] = v;
        part += xi * v;
    }
    return part;
}

// The Lanczos step's product with H, outside the inner CG: with the CG's register arrays
// dead there, 4x4 blocks at 512 threads take whole chunks of 8 entries (a row of an
// order-one neighbour shell in one load latency after its extent).
template <int BD, int NT>
__device__ __forceinline__ double spmv_h(const double* __restrict__ A, const Sys& sy, const double* __restrict__ x,
                                         double* __restrict__ y) {
    constexpr int CH = BD == 4 && NT <= 512 ? 8 : Chunk<BD, NT>::value;
    if (sy.egid == nullptr) return spmv_rows<BD, NT, true, false, CH>(A, sy, x, y);
    return spmv_rows<BD, NT, false, false, CH>(A, sy, x, y);
}

template <int BD, int NT, bool UNIT = false>
__device__ __forceinline__ double spmv(const double* __restrict__ A, const Sys& sy, const double* __restrict__ x,
                                       double* __restrict__ y) {
    if constexpr (UNIT) {
        if (sy.ew > 0) return spmv_rows_ell<BD, NT>(A, sy, x, y);
        return spmv_rows<BD, NT, true, true>(A, sy, x, y);        // off-diagonal copy: entry e is block e
    } else {
        if (sy.egid == nullptr) return spmv_rows<BD, NT, true, false>(A, sy, x, y);
        return spmv_rows<BD, NT, false, false>(A, sy, x, y);
    }
}

// Solve S q = t (real SPD S, real vectors) by CG from 0 to ||res|| <= tol ||t||;
// tt = ||t||^2 (already reduced).  Returns the iteration count.
template <int BD, int NT, bool UNIT>
__device__ int inner_cg(const double* __restrict__ S, const Sys& sy, const double* __restrict__ t,
                        double* __restrict__ q, double* __restrict__ res, double* __restrict__ d,
                        double* __restrict__ w, double tt, double tol, int maxit, double* red) {
    for (int i = threadIdx.x; i < sy.M; i += NT) {
        const double v = t[i];
        q[i] = 0.0;
        res[i] = v;
        d[i] = v;
    }
    if (tt == 0.0) return 0;
    __syncthreads();
    const double stop = tol * sqrt(tt);
    double rr = tt;
    int it = 0;
    while (it < maxit && !(sqrt(rr) <= stop)) {
        double dw[1] = {spmv<BD, NT, UNIT>(S, sy, d, w)};
        block_sum<NT, 1>(dw, red);
        const double a = rr / dw[0];
        double rn[1] = {0.0};
        for (int i = threadIdx.x; i < sy.M; i += NT) {
            q[i] += a * d[i];
            const double s = res[i] - a * w[i];
            res[i] = s;
            rn[0] += s * s;
        }
        block_sum<NT, 1>(rn, red);
        const double bt = rn[0] / rr;
        for (int i = threadIdx.x; i < sy.M; i += NT) d[i] = res[i] + bt * d[i];
        __syncthreads();
        rr = rn[0];
        ++it;
    }
    return it;
}

// The same CG with this thread's rows of the residual and of the solution in
// registers (rows i = tid + m NT, m < R; the search direction d stays in LDS,
// the product S d in the workgroup's slot): per step the vector passes read
// and write only S d in memory.  The arithmetic, and its order, is that of
// inner_cg, so the results are bitwise the same.  The S product takes its
// row's entries in chunks of 6 here (a row of six blocks in one load
// latency), which still leaves the registers the two arrays need.  The row
// index is passed through an empty asm statement where a pass (or a group
// of rows) begins, so the compiler forms each row's address where it is
// used instead of computing all R of them once and holding (or spilling)
// them across the solve.
template <int NT>
struct RegRows {
    static constexpr int value = 16384 / NT;     // rows per thread held in registers
};

template <int BD, int NT, int R, int RG = 8>
__device__ int inner_cg_reg(const double* __restrict__ S, const Sys& sy, const double* __restrict__ t,
                            double* __restrict__ q, double* __restrict__ d, double* __restrict__ w, double tt,
                            double tol, int maxit, double* red) {
    const int M = sy.M;
    double rr_[R], qq_[R];
    int tb0 = threadIdx.x;
    asm volatile("" : "+v"(tb0));
    const int mfull = M / NT;       // rows m < mfull exist in every thread
    // r = d = t, q = 0: a whole group's loads of t go out before its stores (as in the passes below)
#pragma unroll
    for (int m0 = 0; m0 < R; m0 += RG) {
        if (m0 + RG <= mfull) {
            int tg = tb0 + m0 * NT;
            asm volatile("" : "+v"(tg));
            double tv[RG];
#pragma unroll
            for (int u = 0; u < RG; ++u) tv[u] = t[tg + u * NT];
#pragma unroll
            for (int u = 0; u < RG; ++u) {
                rr_[m0 + u] = tv[u];
                qq_[m0 + u] = 0.0;
                d[tg + u * NT] = tv[u];
            }
        } else {
#pragma unroll
            for (int u = 0; u < RG; ++u) {
                const int i = tb0 + (m0 + u) * NT;
                const double v = i < M ? t[i] : 0.0;
                rr_[m0 + u] = v;
                qq_[m0 + u] = 0.0;
                if (i < M) d[i] = v;
            }
        }
    }
    int it = 0;
    if (tt != 0.0) {
        __syncthreads();
        const double stop = tol * sqrt(tt);
        double rr = tt;
        while (it < maxit && !(sqrt(rr) <= stop)) {
            double dw[1] = {spmv_rows_ell<BD, NT, 6>(S, sy, d, w)};
            block_sum<NT, 1>(dw, red);
            const double a = rr / dw[0];
            double rn[1] = {0.0};
            int tb = threadIdx.x;
            asm volatile("" : "+v"(tb));
            // Both passes take their rows in groups of RG: a group whose rows exist in every thread
            // (m < M / NT) issues all its loads before any arithmetic, so a pass waits R / RG times
            // for memory instead of R times; a group at the ragged end goes row by row.  The
            // arithmetic is inner_cg's, fused the same way.
#pragma unroll
            for (int m0 = 0; m0 < R; m0 += RG) {
                if (m0 + RG <= mfull) {
                    int tg = tb + m0 * NT;
                    asm volatile("" : "+v"(tg));
                    double wv[RG], dv[RG];
#pragma unroll
                    for (int u = 0; u < RG; ++u) {
                        wv[u] = w[tg + u * NT];
                        dv[u] = d[tg + u * NT];
                    }
#pragma unroll
                    for (int u = 0; u < RG; ++u) {
                        qq_[m0 + u] = __builtin_fma(a, dv[u], qq_[m0 + u]);
                        const double s = __builtin_fma(-a, wv[u], rr_[m0 + u]);
                        rr_[m0 + u] = s;
                        rn[0] = __builtin_fma(s, s, rn[0]);
                    }
                } else {
#pragma unroll
                    for (int u = 0; u < RG; ++u) {
                        const int i = tb + (m0 + u) * NT;
                        if (i < M) {
                            qq_[m0 + u] = __builtin_fma(a, d[i], qq_[m0 + u]);
                            const double s = __builtin_fma(-a, w[i], rr_[m0 + u]);
                            rr_[m0 + u] = s;
                            rn[0] = __builtin_fma(s, s, rn[0]);
                        }
                    }
                }
            }
            block_sum<NT, 1>(rn, red);
            const double bt = rn[0] / rr;
#pragma unroll
            for (int m0 = 0; m0 < R; m0 += RG) {
                if (m0 + RG <= mfull) {
                    int tg = tb + m0 * NT;
                    asm volatile("" : "+v"(tg));
                    double dv[RG];
#pragma unroll
                    for (int u = 0; u < RG; ++u) dv[u] = d[tg + u * NT];
#pragma unroll
                    for (int u = 0; u < RG; ++u) d[tg + u * NT] = __builtin_fma(bt, dv[u], rr_[m0 + u]);
                } else {
#pragma unroll
                    for (int u = 0; u < RG; ++u) {
                        const int i = tb + (m0 + u) * NT;
                        if (i < M) d[i] = __builtin_fma(bt, d[i], rr_[m0 + u]);
                    }
                }
            }
            __syncthreads();
            rr = rn[0];
            ++it;
        }
    }
    asm volatile("" : "+v"(tb0));
#pragma unroll
    for (int m = 0; m < R; ++m) {
        const int i = tb0 + m * NT;
        if (i < M) q[i] = qq_[m];
    }
    return it;
}

// UNIT 0: S as stored; 1: S = I + its off-diagonal blocks; 2: as 1, on the ELL
// form, with the CG's residual and solution in registers.
template <int BD, int NT, int UNIT>
__device__ __forceinline__ int inner_solve(const double* __restrict__ S, const Sys& sy, const double* __restrict__ t,
                                           double* __restrict__ q, double* __restrict__ res, double* __restrict__ d,
                                           double* __restrict__ w, double tt, double tol, int maxit, double* red) {
    if constexpr (UNIT == 2) return inner_cg_reg<BD, NT, RegRows<NT>::value>(S, sy, t, q, d, w, tt, tol, maxit, red);
    else return inner_cg<BD, NT, UNIT != 0>(S, sy, t, q, res, d, w, tt, tol, maxit, red);
}

// Complex Givens rotation [[c, s], [-conj(s), c]] with c >= 0 real that maps
// (a, b) to (r, 0).
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

__host__ __device__ inline int64_t slot_bytes(int K, int64_t Mp, int64_t nIp) {
    return ((8 * Mp) * 8 + 3 * (int64_t)K * nIp * 16 + 255) / 256 * 256;
}

// DL: the inner CG's search direction d lives in LDS (ldsd, M_j doubles)
// instead of the workgroup's HBM slot, so the sparse product on S gathers it
// from LDS and the CG's vector passes touch one vector fewer in HBM.
// UNIT: S has exactly-identity diagonal blocks and the plan holds a copy of
// its off-diagonal blocks alone (global system): the inner CG applies
// S = I + (those blocks) and never reads the identity blocks.
template <int BD, int NT, bool SID, bool GAL, bool DL, int UNIT>
__device__ void solve_one(const KParams& P, int rj, char* ws, const Lds& L, double* ldsd) {
    const int tid = threadIdx.x;
    const int K = P.K;
    const RhsInfo ri = P.rhs[rj];
    const SysInfo si = P.sys[ri.sys];
    Sys sy;
    sy.rowptr = P.rowptr_l + si.row_base;
    sy.ecol = P.ecol + si.ent_base;
    sy.egid = P.ent_direct ? nullptr : P.egid + si.ent_base;
    sy.gbase = si.ent_base;
    sy.nrows = si.nrows;
    sy.M = si.nrows * BD;
    sy.ew = 0;
    const int M = sy.M;
    const int64_t Mp = P.Mp, nIp = P.nIp;
    const double* Hb = (const double*)P.Hv64;
    const double* Sb = UNIT ? (P.s_ell_w > 0 ? P.s_ell_val : P.s_vals) : (const double*)P.Sv64;
    Sys syS = sy;
    if constexpr (UNIT) {
        syS.rowptr = P.s_rowptr;
        syS.ecol = P.s_ell_w > 0 ? P.s_ell_col : P.s_ecol;
        syS.egid = nullptr;
        syS.gbase = 0;
        syS.ew = P.s_ell_w;
    }
    const int nI = ri.nout;
    const int32_t* rows = P.out_local + ri.out_base;

    double* v = (double*)ws;
    double* wA = v + Mp;
    double* wB = wA + Mp;
    double* tA = wB + Mp;
    double* q = tA + Mp;
    double* res = q + Mp;
    double* d = DL ? ldsd : res + Mp;
    double* wcg = res + 2 * Mp;
    double2* xI = (double2*)(wcg + Mp);
    double2* D0 = xI + (int64_t)K * nIp;
    double2* D1 = D0 + (int64_t)K * nIp;
    double* w = wA;        // w_n
    double* wp = wB;       // w_{n-1}
    double* t = tA;        // u, then t

    const int maxiter = P.maxiter > 0 ? P.maxiter : max(1000, 4 * M);
    constexpr int RG = 4;                  // rows per thread per group in the Lanczos step's vector passes
    int64_t inner_total = 0, sum_upd = 0;

    // ---- v_0 = S^{-1} b / beta_0, w_0 = b / beta_0  (b = e_j)
    for (int i = tid; i < M; i += NT) {
        t[i] = i == ri.b_local ? 1.0 : 0.0;
        wp[i] = 0.0;
    }
    __syncthreads();
    double* q0 = SID ? t : q;
    if constexpr (!SID) inner_total += inner_solve<BD, NT, UNIT>(Sb, syS, t, q, res, d, wcg, 1.0, P.inner_tol,
                                                                 P.inner_maxiter, L.red);
    __syncthreads();
    const double beta0 = sqrt(q0[ri.b_local]);
    for (int i = tid; i < M; i += NT) {
        v[i] = q0[i] / beta0;
        w[i] = (i == ri.b_local ? 1.0 : 0.0) / beta0;
    }
    double sum_w2 = 1.0 / (beta0 * beta0);
    for (int k = tid; k < K; k += NT) {
        L.c1[k] = 1.0;
        L.c2[k] = 1.0;
        L.s1[k] = GAL ? zmk(1.0, 0.0) : zmk(0.0, 0.0);    // GAL: previous pivot
        L.s2[k] = zmk(0.0, 0.0);
        L.g[k] = zmk(beta0, 0.0);
        L.done[k] = 0;
        L.stat[k] = ST_MAXITER;
        L.iters[k] = -1;
        L.resid[k] = INFINITY;
    }
    for (int idx = tid; idx < K * nI; idx += NT) {
        const int k = idx / nI, o = idx - k * nI;
        const int64_t a = (int64_t)k * nIp + o;
        xI[a] = make_double2(0.0, 0.0);
        D0[a] = make_double2(0.0, 0.0);
        D1[a] = make_double2(0.0, 0.0);
    }
    __syncthreads();
    if (!(beta0 > 0.0) || !isfinite(beta0)) {
        for (int k = tid; k < K; k += NT) {
            L.stat[k] = isfinite(beta0) ? ST_BREAKDOWN : ST_NONFINITE;
            L.done[k] = 1;
        }
    }
    __syncthreads();

    double beta = 0.0;
    int n_outer = 0;
    for (int n = 0; n < maxiter && L.ctl[1] < K && beta0 > 0.0 && isfinite(beta0); ++n) {
        n_outer = n + 1;
        // ---- u = H v, alpha = v^T u
        double al[1] = {spmv_h<BD, NT>(Hb, sy, v, t)};
        block_sum<NT, 1>(al, L.red);
        const double alpha = al[0];
        // ---- t = u - alpha w - beta w_prev, ||t||^2
        double tt[1] = {0.0};
        // (this pass and the two below take RG rows per thread at a time, every load of the
        // group before its stores, rows past M clamped and masked; the sums in row order)
        for (int i0 = tid; i0 < M; i0 += RG * NT) {
            double tv[RG], wv[RG], pv[RG];
#pragma unroll
            for (int u = 0; u < RG; ++u) {
                const int ic = i0 + u * NT < M ? i0 + u * NT : i0;
                tv[u] = t[ic];
                wv[u] = w[ic];
                pv[u] = wp[ic];
            }
#pragma unroll
            for (int u = 0; u < RG; ++u) {
                if (i0 + u * NT < M) {
                    const double x_ = tv[u] - alpha * wv[u] - beta * pv[u];
                    t[i0 + u * NT] = x_;
                    tt[0] += x_ * x_;
                }
            }
        }
        block_sum<NT, 1>(tt, L.red);
        // ---- q = S^{-1} t, beta_{n+1} = sqrt(q^T t)
        double* qq = SID ? t : q;
        if constexpr (!SID) inner_total += inner_solve<BD, NT, UNIT>(Sb, syS, t, q, res, d, wcg, tt[0], P.inner_tol,
                                                                     P.inner_maxiter, L.red);
        double qt[1] = {0.0};
        if constexpr (SID) {
            qt[0] = tt[0];
        } else {
            for (int i0 = tid; i0 < M; i0 += RG * NT) {
                double qv[RG], tv[RG];
#pragma unroll
                for (int u = 0; u < RG; ++u) {
                    const int ic = i0 + u * NT < M ? i0 + u * NT : i0;
                    qv[u] = q[ic];
                    tv[u] = t[ic];
                }
#pragma unroll
                for (int u = 0; u < RG; ++u)
                    if (i0 + u * NT < M) qt[0] += qv[u] * tv[u];
            }
            block_sum<NT, 1>(qt, L.red);
        }
        const bool bad = !isfinite(qt[0]) || !isfinite(alpha);
        const double beta_next = qt[0] > 0.0 ? sqrt(qt[0]) : 0.0;
        if (bad || qt[0] < 0.0) {
            for (int k = tid; k < K; k += NT)
                if (!L.done[k]) { L.stat[k] = bad ? ST_NONFINITE : ST_BREAKDOWN; L.done[k] = 1; }
            __syncthreads();
            break;
        }
        if (beta_next > 0.0) sum_w2 += tt[0] / qt[0];
        const double bscale = sqrt(sum_w2);
        // ---- per-shift scalars (FP64), one thread per shift
        if constexpr (GAL) {
            for (int k = tid; k < K; k += NT) {
                if (L.done[k]) continue;
                const zc zk = zmk(P.z[2 * k], P.z[2 * k + 1]);
                const zc dprev = L.s1[k];
                zc c = zmk(0.0, 0.0), dn = zmk(zk.re - alpha, zk.im), gk = zmk(beta0, 0.0);
                if (n > 0) {
                    c = zdiv(zmk(beta, 0.0), dprev);
                    dn = zsub(dn, zmul(zmk(beta, 0.0), c));
                    gk = zmul(c, L.g[k]);
                }
                if (zzero(dn) || !zfinite(dn)) {
                    L.stat[k] = zfinite(dn) ? ST_BREAKDOWN : ST_NONFINITE;
                    L.done[k] = 1;
                    continue;
                }
                L.g[k] = gk;
                L.tau[k] = zdiv(gk, dn);
                L.e[k] = c;
                L.s1[k] = dn;
            }
        }
        for (int k = tid; k < K && !GAL; k += NT) {
            if (L.done[k]) continue;
            const zc zk = zmk(P.z[2 * k], P.z[2 * k + 1]);
            const zc a_prev = zmk(-beta, 0.0);
            const zc a_diag = zmk(zk.re - alpha, zk.im);
            const zc a_next = zmk(-beta_next, 0.0);
            const zc e = zmul(L.s2[k], a_prev);
            const zc f0 = zmk(L.c2[k] * a_prev.re, L.c2[k] * a_prev.im);
            const zc s1 = L.s1[k];
            const double c1 = L.c1[k];
            const zc f = zadd(zmk(c1 * f0.re, c1 * f0.im), zmul(s1, a_diag));
            const zc gam = zadd(zmul(zmk(-s1.re, s1.im), f0), zmk(c1 * a_diag.re, c1 * a_diag.im));
            double c;
            zc s, rnn;
            givens(gam, a_next, c, s, rnn);
            if (zzero(rnn)) {
                L.stat[k] = ST_BREAKDOWN;
                L.done[k] = 1;
                continue;
            }
            const zc gk = L.g[k];
            L.tau[k] = zmk(c * gk.re, c * gk.im);
            L.g[k] = zmul(zmk(-s.re, s.im), gk);
            L.e[k] = e;
            L.f[k] = f;
            L.irnn[k] = zdiv(zmk(1.0, 0.0), rnn);
            L.c2[k] = c1;
            L.s2[k] = s1;
            L.c1[k] = c;
            L.s1[k] = s;
        }
        __syncthreads();
        // list of shifts to update: the ones not done before this iteration's test
        if (tid < 64) {
            int cnt = 0;
            for (int base = 0; base < K; base += 64) {
                const int k = base + tid;
                const bool fl = k < K && !L.done[k];
                const uint64_t m = __ballot(fl);
                const int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                             __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
                if (fl) L.upd[cnt + below] = k;
                cnt += __popcll(m);
            }
            if (tid == 0) L.ctl[0] = cnt;
        }
        __syncthreads();
        const int nupd = L.ctl[0];
        sum_upd += nupd;
        // ---- d_n = (v_n - e d_{n-2} - f d_{n-1}) / R_nn; x += tau d_n on the requested rows
        double2* Dn2 = (n & 1) ? D1 : D0;      // holds d_{n-2}; receives d_n
        double2* Dn1 = (n & 1) ? D0 : D1;      // holds d_{n-1}
        for (int idx = tid; idx < nupd * nI && GAL; idx += NT) {
            const int kk = idx / nI, o = idx - kk * nI;
            const int k = L.upd[kk];
            const int64_t a = (int64_t)k * nIp + o;
            const double2 pv = D0[a];
            const zc c = L.e[k];
            const zc pn = zmk(v[rows[o]] + c.re * pv.x - c.im * pv.y, c.re * pv.y + c.im * pv.x);
            D0[a] = make_double2(pn.re, pn.im);
            const zc tk = L.tau[k];
            const double2 xv = xI[a];
            xI[a] = make_double2(xv.x + tk.re * pn.re - tk.im * pn.im, xv.y + tk.re * pn.im + tk.im * pn.re);
        }
        for (int idx = tid; idx < nupd * nI && !GAL; idx += NT) {
            const int kk = idx / nI, o = idx - kk * nI;
            const int k = L.upd[kk];
            const int64_t a = (int64_t)k * nIp + o;
            const double2 d2 = Dn2[a], d1 = Dn1[a];
            const zc num = zsub(zsub(zmk(v[rows[o]], 0.0), zmul(L.e[k], zmk(d2.x, d2.y))),
                                zmul(L.f[k], zmk(d1.x, d1.y)));
            const zc dn = zmul(num, L.irnn[k]);
            Dn2[a] = make_double2(dn.re, dn.im);
            const zc tk = L.tau[k];
            const double2 xv = xI[a];
            xI[a] = make_double2(xv.x + tk.re * dn.re - tk.im * dn.im, xv.y + tk.re * dn.im + tk.im * dn.re);
        }
        // ---- convergence (bound on the true residual; ||b|| = 1)
        const double tnorm = sqrt(tt[0]);
        for (int k = tid; k < K; k += NT) {
            if (L.done[k]) continue;
            const double est = GAL ? zabs(L.tau[k]) * tnorm : zabs(L.g[k]) * bscale;
            L.resid[k] = est;
            if (est < P.tol || beta_next == 0.0) {
                L.done[k] = 1;
                L.stat[k] = ST_CONVERGED;
                L.iters[k] = n + 1;
                if (beta_next == 0.0) L.resid[k] = 0.0;
            }
        }
        __syncthreads();
        if (tid < 64) {
            int nd = 0;
            for (int base = 0; base < K; base += 64) {
                const int k = base + tid;
                nd += __popcll(__ballot(k < K && L.done[k]));
            }
            if (tid == 0) L.ctl[1] = nd;
        }
        // ---- next Lanczos vectors: v = q / beta_{n+1}, w_prev = w, w = t / beta_{n+1}
        if (beta_next > 0.0) {
            const double ib = 1.0 / beta_next;
            for (int i0 = tid; i0 < M; i0 += RG * NT) {
                double qv[RG], tv[RG];
#pragma unroll
                for (int u = 0; u < RG; ++u) {
                    const int ic = i0 + u * NT < M ? i0 + u * NT : i0;
                    qv[u] = qq[ic];
                    tv[u] = t[ic];
                }
#pragma unroll
                for (int u = 0; u < RG; ++u) {
                    if (i0 + u * NT < M) {
                        v[i0 + u * NT] = qv[u] * ib;
                        t[i0 + u * NT] = tv[u] * ib;
                    }
                }
            }
        }
        __syncthreads();
        double* tmp = wp;
        wp = w;
        w = t;
        t = tmp;
        beta = beta_next;
        if (beta_next == 0.0) break;
    }
    __syncthreads();

    const int64_t obase = P.out_off[rj] * (int64_t)K;
    for (int idx = tid; idx < K * nI; idx += NT) {
        const int k = idx / nI, o = idx - k * nI;
        const double2 xv = xI[(int64_t)k * nIp + o];
        P.out[2 * (obase + idx)] = xv.x;
        P.out[2 * (obase + idx) + 1] = xv.y;
    }
    for (int k = tid; k < K; k += NT) {
        const int64_t o = (int64_t)rj * K + k;
        if (P.iters) P.iters[o] = L.iters[k];
        if (P.status) P.status[o] = (int8_t)L.stat[k];
        if (P.resid) P.resid[o] = L.resid[k];
    }
    if (tid == 0 && P.stats) {
        int64_t* st_ = P.stats + (int64_t)rj * NSTAT;
        st_[0] = n_outer;
        st_[1] = sum_upd;
        st_[2] = inner_total;
        st_[3] = 0;
        st_[4] = M;
        st_[5] = sy.rowptr[sy.nrows] - sy.rowptr[0];
        st_[6] = 0;
        st_[7] = 0;
    }
    __syncthreads();
}

template <int BD, int NT, bool SID, bool GAL, bool DL, int UNIT>
__global__ __launch_bounds__(NT) void k_sqmr(KParams P) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_job;
    const Lds L = carve(smem, P.K, NT);
    double* ldsd = DL ? (double*)(smem + lds_dir_offset(P.K, NT)) : nullptr;
    char* ws = P.ws + (int64_t)blockIdx.x * P.slot_bytes;
    for (;;) {
        if (threadIdx.x == 0) {
            s_job = atomicAdd(P.queue, 1);
            L.ctl[1] = 0;
        }
        __syncthreads();
        const int job = __builtin_amdgcn_readfirstlane(s_job);   // uniform: its loads are scalar
        __syncthreads();
        if (job >= P.nrhs) break;
        solve_one<BD, NT, SID, GAL, DL, UNIT>(P, P.order[job], ws, L, ldsd);
    }
}

// The register-resident form (UNIT 2) is built for 4x4 blocks at 512 threads.
template <int BD, int NT>
constexpr bool reg_form() { return BD == 4 && NT == 512; }

template <int BD, int NT, bool GAL>
static hipError_t launch_dl(const KParams& P, int unit, int slots, hipStream_t st) {
    const size_t lds = lds_dir_offset(P.K, NT) + sizeof(double) * (size_t)P.Mp;
    if (unit == 2) {
        if constexpr (reg_form<BD, NT>())
            hipLaunchKernelGGL((k_sqmr<BD, NT, false, GAL, true, 2>), dim3(slots), dim3(NT), lds, st, P);
        else
            return hipErrorInvalidValue;
    } else if (unit) {
        hipLaunchKernelGGL((k_sqmr<BD, NT, false, GAL, true, 1>), dim3(slots), dim3(NT), lds, st, P);
    } else {
        hipLaunchKernelGGL((k_sqmr<BD, NT, false, GAL, true, 0>), dim3(slots), dim3(NT), lds, st, P);
    }
    return hipSuccess;
}

template <int BD, int NT>
static hipError_t launch_nt(const KParams& P, bool sid, bool gal, bool dl, int unit, int slots, hipStream_t st) {
    const size_t lds = lds_bytes(P.K, NT);
    hipError_t e = hipSuccess;
    if (gal) {
        if (sid) hipLaunchKernelGGL((k_sqmr<BD, NT, true, true, false, 0>), dim3(slots), dim3(NT), lds, st, P);
        else if (dl) e = launch_dl<BD, NT, true>(P, unit, slots, st);
        else hipLaunchKernelGGL((k_sqmr<BD, NT, false, true, false, 0>), dim3(slots), dim3(NT), lds, st, P);
    } else {
        if (sid) hipLaunchKernelGGL((k_sqmr<BD, NT, true, false, false, 0>), dim3(slots), dim3(NT), lds, st, P);
        else if (dl) e = launch_dl<BD, NT, false>(P, unit, slots, st);
        else hipLaunchKernelGGL((k_sqmr<BD, NT, false, false, false, 0>), dim3(slots), dim3(NT), lds, st, P);
    }
    return e != hipSuccess ? e : hipGetLastError();
}

template <int BD>
static hipError_t launch_bd(const KParams& P, bool sid, bool gal, bool dl, int unit, int nt, int slots,
                            hipStream_t st) {
    if (nt == 256) return launch_nt<BD, 256>(P, sid, gal, dl, unit, slots, st);
    if (nt == 1024) return launch_nt<BD, 1024>(P, sid, gal, dl, unit, slots, st);
    return launch_nt<BD, 512>(P, sid, gal, dl, unit, slots, st);
}

template <int BD, int NT, bool SID, bool GAL, bool DL, int UNIT>
static size_t priv_one() {
    hipFuncAttributes fa{};
    if (hipFuncGetAttributes(&fa, (const void*)k_sqmr<BD, NT, SID, GAL, DL, UNIT>) != hipSuccess) return (size_t)-1;
    return fa.localSizeBytes;
}
template <int BD, int NT, bool GAL>
static size_t priv_var(bool sid, bool dl, int unit) {
    if (sid) return priv_one<BD, NT, true, GAL, false, 0>();
    if (dl) {
        if (unit == 2) {
            if constexpr (reg_form<BD, NT>()) return priv_one<BD, NT, false, GAL, true, 2>();
            else return (size_t)-1;
        }
        return unit ? priv_one<BD, NT, false, GAL, true, 1>() : priv_one<BD, NT, false, GAL, true, 0>();
    }
    return priv_one<BD, NT, false, GAL, false, 0>();
}
template <int BD>
static size_t priv_bd(bool sid, bool gal, bool dl, int unit, int nt) {
    if (nt == 256) return gal ? priv_var<BD, 256, true>(sid, dl, unit) : priv_var<BD, 256, false>(sid, dl, unit);
    if (nt == 1024) return gal ? priv_var<BD, 1024, true>(sid, dl, unit) : priv_var<BD, 1024, false>(sid, dl, unit);
    return gal ? priv_var<BD, 512, true>(sid, dl, unit) : priv_var<BD, 512, false>(sid, dl, unit);
}

}  // namespace qmr

size_t qmr_private_bytes(int bd, bool sid, bool gal, bool dl, int unit, int nt) {
    switch (bd) {
        case 1: return qmr::priv_bd<1>(sid, gal, dl, unit, nt);
        case 4: return qmr::priv_bd<4>(sid, gal, dl, unit, nt);
        case 9: return qmr::priv_bd<9>(sid, gal, dl, unit, nt);
        default: return (size_t)-1;
    }
}

size_t qmr_lds_bytes(int K, int nt, int64_t Mp, bool dl) {
    return dl ? qmr::lds_dir_offset(K, nt) + sizeof(double) * (size_t)Mp : qmr::lds_bytes(K, nt);
}

int64_t qmr_slot_bytes(int K, int64_t Mp, int64_t nIp) { return qmr::slot_bytes(K, Mp, nIp); }

hipError_t launch_qmr(const KParams& P, int bd, bool sid, bool gal, bool dl, int unit, int nt, int slots,
                      hipStream_t st) {
    if (dl && sid) return hipErrorInvalidValue;      // no inner CG when S = I
    if (unit && (!dl || (P.s_ell_w > 0 ? (!P.s_ell_col || !P.s_ell_val) : (!P.s_rowptr || !P.s_ecol || !P.s_vals))))
        return hipErrorInvalidValue;
    // the register-resident form needs the ELL blocks and at most its rows per thread
    if (unit == 2 && (bd != 4 || nt != 512 || P.s_ell_w <= 0 || P.Mp > (int64_t)qmr::RegRows<512>::value * 512))
        return hipErrorInvalidValue;
    switch (bd) {
        case 1: return qmr::launch_bd<1>(P, sid, gal, dl, unit, nt, slots, st);
        case 4: return qmr::launch_bd<4>(P, sid, gal, dl, unit, nt, slots, st);
        case 9: return qmr::launch_bd<9>(P, sid, gal, dl, unit, nt, slots, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace scocg
