// Persistent shifted-COCG solver kernel for gfx950.
//
// One workgroup owns one right-hand side b = e_j at a time and runs the
// whole method for it (the generalized shifted COCG of Sec. 3, item (i), for
// (z_k S - H) x = b, Sec. 3 Eq. 2), then pops the next RHS from an atomic
// work queue.  Per outer iteration n, for seed shift s:
//
//   q      = (z_s S - H) p_s          fused H and S pass over the local BSR
//   mu     = p_s^T q                  unconjugated (complex-symmetric form)
//   alpha  = gamma / mu;  rho -= alpha q
//   r      = S^{-1} rho               Hermitian CG on the real SPD S (S = I: r = rho)
//   gamma' = rho^T r, nu = ||rho||_2, beta = gamma'/gamma
//   for every unconverged shift k (FP64 scalars, one thread per shift):
//     pi_{n+1} = (1 + alpha (z_k - z_s)) pi_n + (beta_{n-1} alpha / alpha_{n-1}) (pi_n - pi_{n-1})
//     alpha_k = (pi_n/pi_{n+1}) alpha,  beta_k = (pi_n/pi_{n+1})^2 beta
//     converged when nu / |pi_{n+1}| < tol ||b||
//   x_k += alpha_k p_k;  p_k = r / pi_{n+1} + beta_k p_k      (the HBM-bound sweep)
//   if the seed converged: switch to the unconverged shift with the smallest
//   |pi| and rescale rho, r, gamma, alpha, beta and every pi by its pi.
//
// The recurrences follow from the collinearity of the shifted residuals in
// the common Krylov space (r_k = r / pi_k with pi_k = R_n(z_s - z_k) for the
// seed's residual polynomial R_n); they are written out in the library's
// design notes.  No grid-wide synchronisation is used anywhere.
#include <hip/hip_runtime.h>

#include "scocg_device.hpp"
#include "scocg_params.hpp"

namespace scocg {

enum { ST_CONVERGED = 0, ST_MAXITER = 1, ST_BREAKDOWN = 2, ST_NONFINITE = 3 };

// Seed residual replacement is taken only while ||true - recursive|| <= 0.1 ||recursive||.
constexpr double REPLACE_GAP2 = 1e-2;

// A local system seen from one workgroup.
struct Sys {
    const int64_t* rowptr;
    const int32_t* ecol;
    const int32_t* egid;
    int nrows;
    int M;
};

// LDS layout for K shifts (dynamic shared memory).
struct Lds {
    zc* pi;
    zc* piold;
    zc* ca;
    zc* cb;
    zc* cr;
    double* resid;
    int* iters;
    int* upd;
    unsigned char* done;
    unsigned char* stat;
    unsigned char* updf;
    unsigned char* dirty;   // FP32 forms: x_lo holds unflushed updates
    double* red;
    int* ctl;   // [0] nupd, [1] ndone, [2] new seed, [3] flush count
};

__host__ __device__ inline size_t lds_bytes(int K, int NT) {
    size_t b = 5 * sizeof(zc) * (size_t)K + sizeof(double) * (size_t)K + 2 * sizeof(int) * (size_t)K;
    b += 4 * (size_t)K;
    b = (b + 15) & ~(size_t)15;
    b += sizeof(double) * (NT / 64) * 4 + 4 * sizeof(int);
    return b;
}

__device__ inline Lds lds_carve(unsigned char* base, int K, int NT) {
    Lds L;
    unsigned char* q = base;
    L.pi = (zc*)q; q += sizeof(zc) * K;
    L.piold = (zc*)q; q += sizeof(zc) * K;
    L.ca = (zc*)q; q += sizeof(zc) * K;
    L.cb = (zc*)q; q += sizeof(zc) * K;
    L.cr = (zc*)q; q += sizeof(zc) * K;
    L.resid = (double*)q; q += sizeof(double) * K;
    L.iters = (int*)q; q += sizeof(int) * K;
    L.upd = (int*)q; q += sizeof(int) * K;
    L.done = q; q += K;
    L.stat = q; q += K;
    L.updf = q; q += K;
    L.dirty = q; q += K;
    q = base + (((size_t)(q - base) + 15) & ~(size_t)15);
    L.red = (double*)q; q += sizeof(double) * (NT / 64) * 4;
    L.ctl = (int*)q;
    return L;
}

// Row sums over the block entries of one row (row r of block row a):
// h += H_row . p and s += S_row . p, entries in CSR order.  The entries are
// visited in chunks of CH whose column and block indices are loaded together
// and whose block and vector loads are then all in flight at once, so a row
// costs a couple of memory latencies instead of one dependent chain per
// entry.  A chunk's slots past the end of the row re-read the row's last
// entry and contribute zero (so the sums equal the plain entry-by-entry ones).
// For 4x4 blocks the four rows of a block row are the four lanes of a quad
// (rows are dealt to threads in order and NT is a multiple of 64): each lane
// loads one entry of the vector block and the quad shares them by DPP, which
// quarters the vector loads and their registers.
template <int BD, int NT, int NMAT>
struct RowChunk {
    static constexpr int base = BD == 1 ? 8 : (BD <= 4 ? 4 : 2);
    static constexpr int v = base / (NT >= 1024 ? 2 : 1) / NMAT;
    static constexpr int value = v < 1 ? 1 : v;
};

template <int BD, int NT, class TV, class TB, bool WITH_H, bool WITH_S>
__device__ __forceinline__ void row_sums(const TB* __restrict__ H, const TB* __restrict__ S, const Sys& sy, int a,
                                         int r, const v2<TV>* __restrict__ p, TV& hr, TV& hi, TV& sr, TV& si) {
    constexpr int CH = RowChunk<BD, NT, (WITH_H ? 1 : 0) + (WITH_S ? 1 : 0)>::value;
    constexpr bool QUAD = BD == 4 && NT % 64 == 0;
    const int64_t e0 = sy.rowptr[a], e1 = sy.rowptr[a + 1];
    for (int64_t eb = e0; eb < e1; eb += CH) {
        int32_t b[CH], g[CH];
        bool ok[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            ok[u] = eb + u < e1;
            const int64_t e = ok[u] ? eb + u : e1 - 1;
            b[u] = sy.ecol[e];
            g[u] = sy.egid[e];
        }
        // all loads of the chunk first, then the arithmetic
        v2<TV> own[QUAD ? CH : 1];
        TV hv[WITH_H ? CH : 1][BD], sv[WITH_S ? CH : 1][BD];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int64_t off = ((int64_t)g[u] * BD + r) * BD;
            if constexpr (QUAD) own[u] = p[(int64_t)b[u] * BD + r];
#pragma unroll
            for (int c = 0; c < BD; ++c) {
                if constexpr (WITH_H) hv[u][c] = (TV)bval(H + off, c);
                if constexpr (WITH_S) sv[u][c] = (TV)bval(S + off, c);
            }
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const v2<TV>* pb = p + (int64_t)b[u] * BD;
#pragma unroll
            for (int c = 0; c < BD; ++c) {
                v2<TV> pv;
                if constexpr (QUAD) {
                    if (c == 0) pv = quad_bcast2<0>(own[u]);
                    else if (c == 1) pv = quad_bcast2<1>(own[u]);
                    else if (c == 2) pv = quad_bcast2<2>(own[u]);
                    else pv = quad_bcast2<3>(own[u]);
                } else {
                    pv = pb[c];
                }
                if constexpr (WITH_H) {
                    const TV h = ok[u] ? hv[u][c] : (TV)0;
                    hr += h * pv.x;
                    hi += h * pv.y;
                }
                if constexpr (WITH_S) {
                    const TV sc = ok[u] ? sv[u][c] : (TV)0;
                    sr += sc * pv.x;
                    si += sc * pv.y;
                }
            }
        }
    }
}

// q = (z S - H) p over this thread's rows; returns the partial p^T q.
template <int BD, int NT, class TV, class TB, bool SID>
__device__ __forceinline__ zc op_apply(const TB* __restrict__ H, const TB* __restrict__ S, const Sys& sy, zc z,
                                       const v2<TV>* __restrict__ p, v2<TV>* __restrict__ q) {
    zc mu = zmk(0.0, 0.0);
    for (int i = threadIdx.x; i < sy.M; i += NT) {
        const int a = i / BD, r = i - a * BD;
        TV hr = 0, hi = 0, sr = 0, si = 0;
        row_sums<BD, NT, TV, TB, true, !SID>(H, S, sy, a, r, p, hr, hi, sr, si);
        const zc pi_ = ld<TV>(p, i);
        const zc sp = SID ? pi_ : zmk((double)sr, (double)si);
        const zc qv = rnd<TV>(zsub(zmul(z, sp), zmk((double)hr, (double)hi)));
        st<TV>(q, i, qv);    // the stored (possibly rounded) value enters p^T q
        mu = zadd(mu, zmul(pi_, qv));
    }
    return mu;
}

// w = S d over this thread's rows; returns the partial Re(d^H w).
template <int BD, int NT, class TV, class TB>
__device__ __forceinline__ double spmv_S(const TB* __restrict__ S, const Sys& sy, const v2<TV>* __restrict__ d,
                                         v2<TV>* __restrict__ w) {
    double part = 0.0;
    for (int i = threadIdx.x; i < sy.M; i += NT) {
        const int a = i / BD, r = i - a * BD;
        TV hr = 0, hi = 0, sr = 0, si = 0;
        row_sums<BD, NT, TV, TB, false, true>(S, S, sy, a, r, d, hr, hi, sr, si);
        const zc ws = rnd<TV>(zmk((double)sr, (double)si));
        st<TV>(w, i, ws);
        const zc dv = ld<TV>(d, i);
        part += dv.re * ws.re + dv.im * ws.im;
    }
    return part;
}

// Solve S r = rho (Hermitian CG from r = 0) to ||res|| <= tol ||rho||.
// nr2 = ||rho||^2 (already reduced).  Returns the iteration count.
template <int BD, int NT, class TV, class TB>
__device__ int inner_cg(const TB* S, const Sys& sy, const v2<TV>* rho, v2<TV>* r, v2<TV>* res,
                        v2<TV>* d, v2<TV>* w, double nr2, double tol, int maxit, double* red) {
#pragma unroll 4
    for (int i = threadIdx.x; i < sy.M; i += NT) {
        const zc v = ld<TV>(rho, i);
        st<TV>(r, i, zmk(0.0, 0.0));
        st<TV>(res, i, v);
        st<TV>(d, i, v);
    }
    if (nr2 == 0.0) return 0;
    __syncthreads();
    const double stop = tol * sqrt(nr2);
    double rr = nr2;
    int it = 0;
    while (it < maxit && !(sqrt(rr) <= stop)) {
        double dw[1] = {spmv_S<BD, NT, TV, TB>(S, sy, d, w)};
        block_sum<NT, 1>(dw, red);
        const double a = rr / dw[0];
        double rn[1] = {0.0};
#pragma unroll 4
        for (int i = threadIdx.x; i < sy.M; i += NT) {
            const zc dv = ld<TV>(d, i), wv = ld<TV>(w, i);
            zc rv = ld<TV>(r, i), sv = ld<TV>(res, i);
            rv = zmk(rv.re + a * dv.re, rv.im + a * dv.im);
            sv = rnd<TV>(zmk(sv.re - a * wv.re, sv.im - a * wv.im));
            st<TV>(r, i, rv);
            st<TV>(res, i, sv);
            rn[0] += sv.re * sv.re + sv.im * sv.im;
        }
        block_sum<NT, 1>(rn, red);
        const double bt = rn[0] / rr;
#pragma unroll 4
        for (int i = threadIdx.x; i < sy.M; i += NT) {
            const zc sv = ld<TV>(res, i), dv = ld<TV>(d, i);
            st<TV>(d, i, zmk(sv.re + bt * dv.re, sv.im + bt * dv.im));
        }
        __syncthreads();
        rr = rn[0];
        ++it;
    }
    return it;
}

// x_k += ca_k p_k;  p_k = cr_k r + cb_k p_k  for the listed shifts.
// Work items are (256-element chunk, group of 8 shifts), one per wave, so
// each wave streams contiguous 1 KB segments and keeps its r chunk in
// registers across the shift group.
template <int NT, class TV>
__device__ __forceinline__ void shift_update(v2<TV>* __restrict__ x, v2<TV>* __restrict__ p,
                                             const v2<TV>* __restrict__ r, int M, int64_t Mp,
                                             const Lds& L, int nupd) {
    constexpr int NW = NT / 64, KG = 8;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nch = (M + 255) / 256;
    const int nkg = (nupd + KG - 1) / KG;
    for (int item = w; item < nch * nkg; item += NW) {
        const int kg = item / nch, ch = item - kg * nch;
        const int base = ch * 256 + lane;
        zc rv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = base + u * 64;
            rv[u] = i < M ? ld<TV>(r, i) : zmk(0.0, 0.0);
        }
        const int k1 = min(nupd, (kg + 1) * KG);
        for (int kk = kg * KG; kk < k1; ++kk) {
            const int k = L.upd[kk];
            const zc A = L.ca[k], B = L.cb[k], C = L.cr[k];
            v2<TV>* xk = x + (int64_t)k * Mp;
            v2<TV>* pk = p + (int64_t)k * Mp;
            zc xv[4], pv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = base + u * 64;
                if (i < M) {
                    xv[u] = ld<TV>(xk, i);
                    pv[u] = ld<TV>(pk, i);
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = base + u * 64;
                if (i < M) {
                    st<TV>(xk, i, zadd(xv[u], zmul(A, pv[u])));
                    st<TV>(pk, i, zadd(zmul(C, rv[u]), zmul(B, pv[u])));
                }
            }
        }
    }
}

// Set x_k = 0, p_k = r for every shift (and the FP64 accumulator x_hi = 0).
template <int NT, class TV>
__device__ void shift_init(v2<TV>* x, v2<TV>* p, double2* xhi, const v2<TV>* r, int M, int64_t Mp, int K) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nch = (M + 63) / 64;
    for (int item = w; item < nch * K; item += NW) {
        const int k = item / nch, ch = item - k * nch;
        const int i = ch * 64 + lane;
        if (i < M) {
            st<TV>(x + (int64_t)k * Mp, i, zmk(0.0, 0.0));
            st<TV>(p + (int64_t)k * Mp, i, ld<TV>(r, i));
            if (xhi) xhi[(int64_t)k * Mp + i] = make_double2(0.0, 0.0);
        }
    }
}

// Compact the shifts whose flag is set into out[] (wave 0); the count goes
// to *cnt_out and, if nd_out is given, the number of done shifts to *nd_out.
__device__ __forceinline__ void compact_flags(const unsigned char* flag, const unsigned char* done, int K,
                                              int* out, int* cnt_out, int* nd_out) {
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        int cnt = 0, nd = 0;
        for (int base = 0; base < K; base += 64) {
            const int k = base + lane;
            const bool f = k < K && flag[k];
            const bool dn = k < K && done != nullptr && done[k];
            const uint64_t m = __ballot(f);
            const uint64_t md = __ballot(dn);
            const int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
            if (f) out[cnt + below] = k;
            cnt += __popcll(m);
            nd += __popcll(md);
        }
        if (lane == 0) {
            *cnt_out = cnt;
            if (nd_out) *nd_out = nd;
        }
    }
}

// Unconverged shift with the smallest |pi| (largest residual estimate), ties
// to the lowest index; written to L.ctl[2] by wave 0.
__device__ __forceinline__ void pick_seed(const Lds& L, int K) {
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        double best = INFINITY;
        int bk = 0x7fffffff;
        for (int k = lane; k < K; k += 64) {
            if (!L.done[k]) {
                const double m = zabs(L.pi[k]);
                if (m < best) { best = m; bk = k; }
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double ob = __shfl_xor(best, off, 64);
            const int ok = __shfl_xor(bk, off, 64);
            if (ob < best || (ob == best && ok < bk)) { best = ob; bk = ok; }
        }
        if (lane == 0) L.ctl[2] = bk;
    }
}

// x_hi_k += x_lo_k; x_lo_k = 0 for the listed shifts (FP32 forms).
template <int NT>
__device__ void flush_lo(float2* xlo, double2* xhi, int M, int64_t Mp, const int* list, int n) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nch = (M + 63) / 64;
    for (int item = w; item < nch * n; item += NW) {
        const int kk = item / nch, ch = item - kk * nch;
        const int i = ch * 64 + lane;
        if (i < M) {
            const int64_t o = (int64_t)list[kk] * Mp + i;
            const float2 lo = xlo[o];
            double2 hi = xhi[o];
            hi.x += (double)lo.x;
            hi.y += (double)lo.y;
            xhi[o] = hi;
            xlo[o] = make_float2(0.f, 0.f);
        }
    }
}

// rho = b - (z S - H) x in FP64 with FP64 blocks (b = e_bl); returns ||rho||^2
// (reduced over the workgroup).  Uses q as scratch.
template <int BD, int NT, bool SID>
__device__ double true_residual(const KParams& P, const Sys& sy, zc z, const double2* x, double2* q,
                                double2* rho, int bl, double* red) {
    __syncthreads();
    (void)op_apply<BD, NT, double, double, SID>(P.Hv64, P.Sv64, sy, z, x, q);
    double nn[1] = {0.0};
#pragma unroll 4
    for (int i = threadIdx.x; i < sy.M; i += NT) {
        const zc qv = ld<double>(q, i);
        const zc v = zmk((i == bl ? 1.0 : 0.0) - qv.re, -qv.im);
        st<double>(rho, i, v);
        nn[0] += v.re * v.re + v.im * v.im;
    }
    block_sum<NT, 1>(nn, red);
    return nn[0];
}

// Single-shift FP64 COCG for (z S - H) x = b started from the given x, whose
// residual rho (and ||rho||^2 = nr2) is already in place.  Converges when
// ||rho|| < tol ||b||.  Returns the iterations used (negative if it stopped
// on a breakdown).
template <int BD, int NT, bool SID>
__device__ int fallback_cocg(const KParams& P, const Sys& sy, zc z, double2* x, double2* rho, double2* r,
                             double2* p, double2* q, double2* res, double2* d, double2* w, double nr2,
                             int maxit, double* red) {
    const int M = sy.M;
    double2* rr = SID ? rho : r;
    if (!SID) (void)inner_cg<BD, NT, double, double>(P.Sv64, sy, rho, rr, res, d, w, nr2, P.inner_tol,
                                                     P.inner_maxiter, red);
    double g[2] = {0.0, 0.0};
    for (int i = threadIdx.x; i < M; i += NT) {
        const zc t = zmul(ld<double>(rho, i), ld<double>(rr, i));
        g[0] += t.re;
        g[1] += t.im;
        p[i] = rr[i];
    }
    block_sum<NT, 2>(g, red);
    zc gamma = zmk(g[0], g[1]);
    const double stop = P.tol;   // ||b|| = 1
    int it = 0;
    for (; it < maxit; ++it) {
        if (sqrt(nr2) < stop) break;
        const zc mup = op_apply<BD, NT, double, double, SID>(P.Hv64, P.Sv64, sy, z, p, q);
        double m2[2] = {mup.re, mup.im};
        block_sum<NT, 2>(m2, red);
        const zc mu = zmk(m2[0], m2[1]);
        if (!zfinite(mu) || zzero(mu)) return -1 - it;
        const zc alpha = zdiv(gamma, mu);
        double nn[1] = {0.0};
        for (int i = threadIdx.x; i < M; i += NT) {
            const zc pv = ld<double>(p, i);
            st<double>(x, i, zadd(ld<double>(x, i), zmul(alpha, pv)));
            const zc v = zsub(ld<double>(rho, i), zmul(alpha, ld<double>(q, i)));
            st<double>(rho, i, v);
            nn[0] += v.re * v.re + v.im * v.im;
        }
        block_sum<NT, 1>(nn, red);
        nr2 = nn[0];
        if (!SID) (void)inner_cg<BD, NT, double, double>(P.Sv64, sy, rho, rr, res, d, w, nr2, P.inner_tol,
                                                         P.inner_maxiter, red);
        double gn[2] = {0.0, 0.0};
        for (int i = threadIdx.x; i < M; i += NT) {
            const zc t = zmul(ld<double>(rho, i), ld<double>(rr, i));
            gn[0] += t.re;
            gn[1] += t.im;
        }
        block_sum<NT, 2>(gn, red);
        const zc gnew = zmk(gn[0], gn[1]);
        if (!zfinite(gnew) || zzero(gamma)) return -1 - it;
        const zc beta = zdiv(gnew, gamma);
        gamma = gnew;
        for (int i = threadIdx.x; i < M; i += NT)
            st<double>(p, i, zadd(ld<double>(rr, i), zmul(beta, ld<double>(p, i))));
        __syncthreads();
    }
    return it;
}

// Bytes of one workgroup slot for K shifts and Mp padded rows.
__host__ __device__ inline int64_t slot_bytes_for(int K, int64_t Mp, bool lo) {
    const int64_t b = lo ? (32 * (int64_t)K + 6 * 8 + 7 * 16) * Mp : (32 * (int64_t)K + 7 * 16) * Mp;
    return (b + 255) / 256 * 256;
}

template <int BD, int NT, class TV, class TB, bool SID>
__device__ void solve_one(const KParams& P, int rj, char* ws, const Lds& L) {
    constexpr bool LO = sizeof(TV) == 4;
    const int tid = threadIdx.x;
    const int K = P.K;
    const RhsInfo ri = P.rhs[rj];
    const SysInfo si = P.sys[ri.sys];
    Sys sy;
    sy.rowptr = P.rowptr_l + si.row_base;
    sy.ecol = P.ecol + si.ent_base;
    sy.egid = P.egid + si.ent_base;
    sy.nrows = si.nrows;
    sy.M = si.nrows * BD;
    const int M = sy.M;
    const int64_t Mp = P.Mp;
    const TB* Hb = (const TB*)P.Hv;
    const TB* Sb = (const TB*)P.Sv;

    // ---- per-slot working memory
    v2<TV>* x = (v2<TV>*)ws;                    // FP64: x; FP32 forms: x_lo
    v2<TV>* p = x + (int64_t)K * Mp;
    double2* xhi;                                // FP64 solution accumulator
    v2<TV>* vbase;
    if constexpr (LO) {
        xhi = (double2*)(p + (int64_t)K * Mp);
        vbase = (v2<TV>*)(xhi + (int64_t)K * Mp);
    } else {
        xhi = (double2*)x;
        vbase = p + (int64_t)K * Mp;
    }
    v2<TV>* rho = vbase;
    v2<TV>* rbuf = rho + Mp;
    v2<TV>* q = rbuf + Mp;
    v2<TV>* res = q + Mp;
    v2<TV>* d = res + Mp;
    v2<TV>* w = d + Mp;
    v2<TV>* r = SID ? rho : rbuf;    // S = I: r = S^{-1} rho = rho
    // FP64 vectors for replacement, audit and fallback
    double2 *rho64, *r64, *q64, *res64, *d64, *w64, *p64;
    if constexpr (LO) {
        rho64 = (double2*)(w + Mp);
        r64 = rho64 + Mp;
        q64 = r64 + Mp;
        res64 = q64 + Mp;
        d64 = res64 + Mp;
        w64 = d64 + Mp;
        p64 = w64 + Mp;
    } else {
        rho64 = (double2*)rho;
        r64 = (double2*)rbuf;
        q64 = (double2*)q;
        res64 = (double2*)res;
        d64 = (double2*)d;
        w64 = (double2*)w;
        p64 = (double2*)(w + Mp);
    }

    const int maxiter = P.maxiter > 0 ? P.maxiter : max(1000, 4 * M);
    const double itol = LO ? P.inner_tol_lo : P.inner_tol;
    const double nu0 = 1.0;   // ||e_j||
    int64_t inner_total = 0, sum_upd = 0, nswitch = 0, nrepl = 0, nfb = 0;

    // ---- init: rho = e_j, r = S^{-1} rho, gamma = rho^T r, x_k = 0, p_k = r
    for (int i = tid; i < M; i += NT) st<TV>(rho, i, zmk(i == ri.b_local ? 1.0 : 0.0, 0.0));
    __syncthreads();
    if constexpr (!SID) inner_total += inner_cg<BD, NT, TV, TB>(Sb, sy, rho, r, res, d, w, 1.0, itol,
                                                                P.inner_maxiter, L.red);
    double gp[2] = {0.0, 0.0};
    for (int i = tid; i < M; i += NT) {
        const zc t = zmul(ld<TV>(rho, i), ld<TV>(r, i));
        gp[0] += t.re;
        gp[1] += t.im;
    }
    block_sum<NT, 2>(gp, L.red);
    zc gamma = zmk(gp[0], gp[1]);
    for (int k = tid; k < K; k += NT) {
        L.pi[k] = zmk(1.0, 0.0);
        L.piold[k] = zmk(1.0, 0.0);
        L.done[k] = 0;
        L.stat[k] = ST_MAXITER;
        L.iters[k] = -1;
        L.resid[k] = INFINITY;
        L.dirty[k] = 0;
    }
    shift_init<NT, TV>(x, p, LO ? xhi : nullptr, r, M, Mp, K);
    __syncthreads();

    int s = P.seed0;
    zc alpha_prev = zmk(1.0, 0.0), beta_prev = zmk(0.0, 0.0);
    int n_outer = 0;

    for (int n = 0; n < maxiter; ++n) {
        n_outer = n + 1;
        const zc zs = zmk(P.z[2 * s], P.z[2 * s + 1]);
        // ---- q = (z_s S - H) p_s, mu = p_s^T q
        const zc mup = op_apply<BD, NT, TV, TB, SID>(Hb, Sb, sy, zs, p + (int64_t)s * Mp, q);
        double mr[2] = {mup.re, mup.im};
        block_sum<NT, 2>(mr, L.red);
        const zc mu = zmk(mr[0], mr[1]);
        if (!zfinite(mu) || zzero(mu)) {
            const unsigned char code = zfinite(mu) ? ST_BREAKDOWN : ST_NONFINITE;
            for (int k = tid; k < K; k += NT)
                if (!L.done[k]) { L.stat[k] = code; L.done[k] = 1; }
            break;
        }
        const zc alpha = zdiv(gamma, mu);
        // ---- rho -= alpha q;  nu^2 = ||rho||^2
        double nn[1] = {0.0};
        for (int i = tid; i < M; i += NT) {
            const zc b = rnd<TV>(zsub(ld<TV>(rho, i), zmul(alpha, ld<TV>(q, i))));
            st<TV>(rho, i, b);
            nn[0] += b.re * b.re + b.im * b.im;
        }
        block_sum<NT, 1>(nn, L.red);
        const double nu = sqrt(nn[0]);
        // ---- r = S^{-1} rho
        if constexpr (!SID) inner_total += inner_cg<BD, NT, TV, TB>(Sb, sy, rho, r, res, d, w, nn[0], itol,
                                                                    P.inner_maxiter, L.red);
        // ---- gamma' = rho^T r
        double gn[2] = {0.0, 0.0};
        for (int i = tid; i < M; i += NT) {
            const zc t = zmul(ld<TV>(rho, i), ld<TV>(r, i));
            gn[0] += t.re;
            gn[1] += t.im;
        }
        block_sum<NT, 2>(gn, L.red);
        const zc gamma_new = zmk(gn[0], gn[1]);
        if (!isfinite(nu) || !zfinite(gamma_new)) {
            for (int k = tid; k < K; k += NT)
                if (!L.done[k]) { L.stat[k] = ST_NONFINITE; L.done[k] = 1; }
            break;
        }
        const zc beta = zdiv(gamma_new, gamma);
        gamma = gamma_new;

        // ---- shift scalars (FP64), one thread per shift
        const zc c3 = zdiv(zmul(beta_prev, alpha), alpha_prev);
        for (int k = tid; k < K; k += NT) {
            L.updf[k] = 0;
            if (L.done[k]) continue;
            const zc pk = L.pi[k], po = L.piold[k];
            const zc dz = zmk(P.z[2 * k] - zs.re, P.z[2 * k + 1] - zs.im);
            const zc f = zadd(zmk(1.0, 0.0), zmul(alpha, dz));
            const zc pin = zadd(zmul(f, pk), zmul(c3, zsub(pk, po)));
            if (!zfinite(pin) || zzero(pin)) {
                L.stat[k] = zfinite(pin) ? ST_BREAKDOWN : ST_NONFINITE;
                L.done[k] = 1;
                continue;
            }
            const zc ratio = zdiv(pk, pin);
            L.ca[k] = zmul(ratio, alpha);
            L.cb[k] = zmul(zmul(ratio, ratio), beta);
            L.cr[k] = zdiv(zmk(1.0, 0.0), pin);
            L.piold[k] = pk;
            L.pi[k] = pin;
            const double est = nu / zabs(pin);
            L.resid[k] = est / nu0;
            L.updf[k] = 1;
            L.dirty[k] = 1;
            if (est < P.tol * nu0) {
                L.done[k] = 1;
                L.stat[k] = ST_CONVERGED;
                L.iters[k] = n + 1;
            }
        }
        __syncthreads();
        compact_flags(L.updf, L.done, K, L.upd, &L.ctl[0], &L.ctl[1]);
        __syncthreads();
        const int nupd = L.ctl[0];
        const int ndone = L.ctl[1];
        sum_upd += nupd;
        // ---- x_k += alpha_k p_k;  p_k = r/pi_k + beta_k p_k
        shift_update<NT, TV>(x, p, r, M, Mp, L, nupd);
        __syncthreads();
        if (zzero(gamma) && nu > 0.0 && ndone < K) {
            for (int k = tid; k < K; k += NT)
                if (!L.done[k]) { L.stat[k] = ST_BREAKDOWN; L.done[k] = 1; }
            break;
        }
        if (ndone == K) break;
        zc alpha_n = alpha, beta_n = beta;
        if (L.done[s]) {
            // ---- seed switch
            pick_seed(L, K);
            __syncthreads();
            const int s2 = L.ctl[2];
            const zc cn = L.pi[s2], co = L.piold[s2];
            __syncthreads();
            const zc ratio = zdiv(co, cn);
            alpha_n = zmul(ratio, alpha);
            beta_n = zmul(zmul(ratio, ratio), beta);
            for (int i = tid; i < M; i += NT) {
                st<TV>(rho, i, zdiv(ld<TV>(rho, i), cn));
                if constexpr (!SID) st<TV>(r, i, zdiv(ld<TV>(r, i), cn));
            }
            gamma = zdiv(gamma, zmul(cn, cn));
            for (int k = tid; k < K; k += NT) {
                if (!L.done[k]) {
                    L.pi[k] = zdiv(L.pi[k], cn);
                    L.piold[k] = zdiv(L.piold[k], co);
                }
            }
            s = s2;
            ++nswitch;
            __syncthreads();
        }
        if constexpr (LO) {
            if (P.replace_every > 0 && (n + 1) % P.replace_every == 0) {
                // ---- group-wise x update, then FP64 residual replacement on the seed
                compact_flags(L.dirty, nullptr, K, L.upd, &L.ctl[3], nullptr);
                __syncthreads();
                const int nd = L.ctl[3];
                flush_lo<NT>((float2*)x, xhi, M, Mp, L.upd, nd);
                __syncthreads();
                for (int k = tid; k < K; k += NT) L.dirty[k] = 0;
                const zc z2 = zmk(P.z[2 * s], P.z[2 * s + 1]);
                const double nr2 = true_residual<BD, NT, SID>(P, sy, z2, xhi + (int64_t)s * Mp, q64, rho64,
                                                              ri.b_local, L.red);
                // Replacing the recursive residual keeps the recurrences valid only while the gap
                // between it and the true residual is small against it.  A seed taken over by a
                // switch carries the FP32 gap of its whole history as a shifted system, which can
                // exceed its residual: replacing then destroys the seed's conjugacy and the
                // iteration stalls until the shifted scalars overflow.  Such replacements are skipped.
                double gd[2] = {0.0, 0.0};
                for (int i = tid; i < M; i += NT) {
                    const zc a = ld<double>(rho64, i), c = ld<TV>(rho, i);
                    const double dr = a.re - c.re, di = a.im - c.im;
                    gd[0] += dr * dr + di * di;
                    gd[1] += c.re * c.re + c.im * c.im;
                }
                block_sum<NT, 2>(gd, L.red);
                if (gd[0] <= REPLACE_GAP2 * gd[1]) {
                    double2* rr64 = SID ? rho64 : r64;
                    if constexpr (!SID) inner_total += inner_cg<BD, NT, double, double>(P.Sv64, sy, rho64, rr64, res64,
                                                                                        d64, w64, nr2, P.inner_tol,
                                                                                        P.inner_maxiter, L.red);
                    double g2[2] = {0.0, 0.0};
                    for (int i = tid; i < M; i += NT) {
                        const zc a = ld<double>(rho64, i), b = ld<double>(rr64, i);
                        const zc t = zmul(a, b);
                        g2[0] += t.re;
                        g2[1] += t.im;
                        st<TV>(rho, i, a);
                        if constexpr (!SID) st<TV>(r, i, b);
                    }
                    block_sum<NT, 2>(g2, L.red);
                    gamma = zmk(g2[0], g2[1]);
                    ++nrepl;
                }
            }
        }
        alpha_prev = alpha_n;
        beta_prev = beta_n;
    }
    __syncthreads();
    if constexpr (LO) {
        compact_flags(L.dirty, nullptr, K, L.upd, &L.ctl[3], nullptr);
        __syncthreads();
        flush_lo<NT>((float2*)x, xhi, M, Mp, L.upd, L.ctl[3]);
        __syncthreads();
    }

    // ---- FP64 true-residual audit of every shift, FP64 fallback where needed
    if (P.audit > 0) {
        const bool fix = LO || P.audit >= 2;
        for (int k = 0; k < K; ++k) {
            const zc zk = zmk(P.z[2 * k], P.z[2 * k + 1]);
            double2* xk = xhi + (int64_t)k * Mp;
            double nr2 = true_residual<BD, NT, SID>(P, sy, zk, xk, q64, rho64, ri.b_local, L.red);
            const bool retry = L.stat[k] == ST_CONVERGED || L.stat[k] == ST_MAXITER;
            if (fix && retry && !(sqrt(nr2) <= P.tol)) {
                const int it = fallback_cocg<BD, NT, SID>(P, sy, zk, xk, rho64, r64, p64, q64, res64, d64, w64,
                                                          nr2, maxiter, L.red);
                nfb += it < 0 ? -it : it;
                nr2 = true_residual<BD, NT, SID>(P, sy, zk, xk, q64, rho64, ri.b_local, L.red);
                // the audited residual is the judge: converged only if it is <= tol
                if (tid == 0) L.stat[k] = it < 0 ? ST_BREAKDOWN : (sqrt(nr2) <= P.tol ? ST_CONVERGED : ST_MAXITER);
            }
            if (tid == 0) L.resid[k] = sqrt(nr2);
        }
        __syncthreads();
    }

    // ---- outputs: G rows (or all of x), iteration counts, codes, residuals
    const int nout = ri.full_x ? M : ri.nout;
    const int64_t obase = P.out_off[rj] * (int64_t)K;
    const int32_t* ol = P.out_local + ri.out_base;
    for (int64_t idx = tid; idx < (int64_t)K * nout; idx += NT) {
        const int k = (int)(idx / nout), o = (int)(idx - (int64_t)k * nout);
        const int row = ri.full_x ? o : ol[o];
        const double2 v = xhi[(int64_t)k * Mp + row];
        P.out[2 * (obase + idx)] = v.x;
        P.out[2 * (obase + idx) + 1] = v.y;
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
        st_[3] = nswitch;
        st_[4] = M;
        st_[5] = sy.rowptr[sy.nrows] - sy.rowptr[0];
        st_[6] = nrepl;
        st_[7] = nfb;
    }
    __syncthreads();
}

// Bytes of one workgroup slot in projected mode (FP64): seven vectors of the
// seed process plus x_k and p_k on the requested rows of every shift.
__host__ __device__ inline int64_t slot_bytes_proj(int K, int64_t Mp, int64_t nIp) {
    return ((7 * Mp + 2 * (int64_t)K * nIp) * 16 + 255) / 256 * 256;
}

// Projected solve of one RHS: x_k and p_k live only on the rows whose G
// elements are requested; the seed runs the three-term form of COCG
//   mu_n = r_n^T q_n - beta_{n-1} gamma_n / alpha_{n-1},   q_n = (z_s S - H) r_n
//   rho_{n+1} = (1 + c_n) rho_n - alpha_n q_n - c_n rho_{n-1},  c_n = alpha_n beta_{n-1} / alpha_{n-1}
// so that a seed switch only rescales the two latest residuals.  The shifted
// scalars and the per-shift updates are those of the two-term form.
template <int BD, int NT, bool SID>
__device__ void solve_one_proj(const KParams& P, int rj, char* ws, const Lds& L) {
    const int tid = threadIdx.x;
    const int K = P.K;
    const RhsInfo ri = P.rhs[rj];
    const SysInfo si = P.sys[ri.sys];
    Sys sy;
    sy.rowptr = P.rowptr_l + si.row_base;
    sy.ecol = P.ecol + si.ent_base;
    sy.egid = P.egid + si.ent_base;
    sy.nrows = si.nrows;
    sy.M = si.nrows * BD;
    const int M = sy.M;
    const int64_t Mp = P.Mp, nIp = P.nIp;
    const double* Hb = (const double*)P.Hv;
    const double* Sb = (const double*)P.Sv;
    const int nI = ri.nout;
    const int32_t* rows = P.out_local + ri.out_base;

    double2* rhoA = (double2*)ws;
    double2* rhoB = rhoA + Mp;
    double2* rbuf = rhoB + Mp;
    double2* q = rbuf + Mp;
    double2* res = q + Mp;
    double2* d = res + Mp;
    double2* w = d + Mp;
    double2* xI = w + Mp;
    double2* pI = xI + (int64_t)K * nIp;
    double2* rho = rhoA;
    double2* rho_old = rhoB;
    double2* r = SID ? rho : rbuf;

    const int maxiter = P.maxiter > 0 ? P.maxiter : max(1000, 4 * M);
    const double nu0 = 1.0;
    int64_t inner_total = 0, sum_upd = 0, nswitch = 0;

    for (int i = tid; i < M; i += NT) {
        st<double>(rho, i, zmk(i == ri.b_local ? 1.0 : 0.0, 0.0));
        st<double>(rho_old, i, zmk(0.0, 0.0));
    }
    __syncthreads();
    if constexpr (!SID) inner_total += inner_cg<BD, NT, double, double>(Sb, sy, rho, r, res, d, w, 1.0, P.inner_tol,
                                                                        P.inner_maxiter, L.red);
    double gp[2] = {0.0, 0.0};
    for (int i = tid; i < M; i += NT) {
        const zc t = zmul(ld<double>(rho, i), ld<double>(r, i));
        gp[0] += t.re;
        gp[1] += t.im;
    }
    block_sum<NT, 2>(gp, L.red);
    zc gamma = zmk(gp[0], gp[1]);
    for (int k = tid; k < K; k += NT) {
        L.pi[k] = zmk(1.0, 0.0);
        L.piold[k] = zmk(1.0, 0.0);
        L.done[k] = 0;
        L.stat[k] = ST_MAXITER;
        L.iters[k] = -1;
        L.resid[k] = INFINITY;
    }
    for (int idx = tid; idx < K * nI; idx += NT) {
        const int k = idx / nI, o = idx - k * nI;
        xI[(int64_t)k * nIp + o] = make_double2(0.0, 0.0);
        pI[(int64_t)k * nIp + o] = r[rows[o]];
    }
    __syncthreads();

    int s = P.seed0;
    zc alpha_prev = zmk(1.0, 0.0), beta_prev = zmk(0.0, 0.0);
    int n_outer = 0;
    for (int n = 0; n < maxiter; ++n) {
        n_outer = n + 1;
        const zc zs = zmk(P.z[2 * s], P.z[2 * s + 1]);
        // ---- q = (z_s S - H) r, t = r^T q
        const zc tp = op_apply<BD, NT, double, double, SID>(Hb, Sb, sy, zs, r, q);
        double tr[2] = {tp.re, tp.im};
        block_sum<NT, 2>(tr, L.red);
        const zc mu = zsub(zmk(tr[0], tr[1]), zdiv(zmul(beta_prev, gamma), alpha_prev));
        if (!zfinite(mu) || zzero(mu)) {
            const unsigned char code = zfinite(mu) ? ST_BREAKDOWN : ST_NONFINITE;
            for (int k = tid; k < K; k += NT)
                if (!L.done[k]) { L.stat[k] = code; L.done[k] = 1; }
            break;
        }
        const zc alpha = zdiv(gamma, mu);
        const zc c = zdiv(zmul(alpha, beta_prev), alpha_prev);
        const zc c1 = zadd(zmk(1.0, 0.0), c);
        // ---- rho_{n+1} = (1 + c) rho_n - alpha q - c rho_{n-1}, written over rho_{n-1}
        double nn[1] = {0.0};
        for (int i = tid; i < M; i += NT) {
            const zc v = zsub(zsub(zmul(c1, ld<double>(rho, i)), zmul(alpha, ld<double>(q, i))),
                              zmul(c, ld<double>(rho_old, i)));
            st<double>(rho_old, i, v);
            nn[0] += v.re * v.re + v.im * v.im;
        }
        {
            double2* t = rho;
            rho = rho_old;
            rho_old = t;
        }
        if constexpr (SID) r = rho;
        block_sum<NT, 1>(nn, L.red);
        const double nu = sqrt(nn[0]);
        if constexpr (!SID) inner_total += inner_cg<BD, NT, double, double>(Sb, sy, rho, r, res, d, w, nn[0],
                                                                            P.inner_tol, P.inner_maxiter, L.red);
        double gn[2] = {0.0, 0.0};
        for (int i = tid; i < M; i += NT) {
            const zc t = zmul(ld<double>(rho, i), ld<double>(r, i));
            gn[0] += t.re;
            gn[1] += t.im;
        }
        block_sum<NT, 2>(gn, L.red);
        const zc gamma_new = zmk(gn[0], gn[1]);
        if (!isfinite(nu) || !zfinite(gamma_new)) {
            for (int k = tid; k < K; k += NT)
                if (!L.done[k]) { L.stat[k] = ST_NONFINITE; L.done[k] = 1; }
            break;
        }
        const zc beta = zdiv(gamma_new, gamma);
        gamma = gamma_new;

        // ---- shift scalars (FP64)
        const zc c3 = zdiv(zmul(beta_prev, alpha), alpha_prev);
        for (int k = tid; k < K; k += NT) {
            L.updf[k] = 0;
            if (L.done[k]) continue;
            const zc pk = L.pi[k], po = L.piold[k];
            const zc dz = zmk(P.z[2 * k] - zs.re, P.z[2 * k + 1] - zs.im);
            const zc f = zadd(zmk(1.0, 0.0), zmul(alpha, dz));
            const zc pin = zadd(zmul(f, pk), zmul(c3, zsub(pk, po)));
            if (!zfinite(pin) || zzero(pin)) {
                L.stat[k] = zfinite(pin) ? ST_BREAKDOWN : ST_NONFINITE;
                L.done[k] = 1;
                continue;
            }
            const zc ratio = zdiv(pk, pin);
            L.ca[k] = zmul(ratio, alpha);
            L.cb[k] = zmul(zmul(ratio, ratio), beta);
            L.cr[k] = zdiv(zmk(1.0, 0.0), pin);
            L.piold[k] = pk;
            L.pi[k] = pin;
            const double est = nu / zabs(pin);
            L.resid[k] = est / nu0;
            L.updf[k] = 1;
            if (est < P.tol * nu0) {
                L.done[k] = 1;
                L.stat[k] = ST_CONVERGED;
                L.iters[k] = n + 1;
            }
        }
        __syncthreads();
        compact_flags(L.updf, L.done, K, L.upd, &L.ctl[0], &L.ctl[1]);
        __syncthreads();
        const int nupd = L.ctl[0];
        const int ndone = L.ctl[1];
        sum_upd += nupd;
        // ---- x_k += alpha_k p_k;  p_k = r/pi_k + beta_k p_k  on the requested rows
        for (int idx = tid; idx < nupd * nI; idx += NT) {
            const int kk = idx / nI, o = idx - kk * nI;
            const int k = L.upd[kk];
            const int64_t a = (int64_t)k * nIp + o;
            const zc pv = ld<double>(pI, a);
            st<double>(xI, a, zadd(ld<double>(xI, a), zmul(L.ca[k], pv)));
            st<double>(pI, a, zadd(zmul(L.cr[k], ld<double>(r, rows[o])), zmul(L.cb[k], pv)));
        }
        __syncthreads();
        if (zzero(gamma) && nu > 0.0 && ndone < K) {
            for (int k = tid; k < K; k += NT)
                if (!L.done[k]) { L.stat[k] = ST_BREAKDOWN; L.done[k] = 1; }
            break;
        }
        if (ndone == K) break;
        zc alpha_n = alpha, beta_n = beta;
        if (L.done[s]) {
            pick_seed(L, K);
            __syncthreads();
            const int s2 = L.ctl[2];
            const zc cn = L.pi[s2], co = L.piold[s2];
            __syncthreads();
            const zc ratio = zdiv(co, cn);
            alpha_n = zmul(ratio, alpha);
            beta_n = zmul(zmul(ratio, ratio), beta);
            for (int i = tid; i < M; i += NT) {
                st<double>(rho, i, zdiv(ld<double>(rho, i), cn));
                st<double>(rho_old, i, zdiv(ld<double>(rho_old, i), co));
                if constexpr (!SID) st<double>(r, i, zdiv(ld<double>(r, i), cn));
            }
            gamma = zdiv(gamma, zmul(cn, cn));
            for (int k = tid; k < K; k += NT) {
                if (!L.done[k]) {
                    L.pi[k] = zdiv(L.pi[k], cn);
                    L.piold[k] = zdiv(L.piold[k], co);
                }
            }
            s = s2;
            ++nswitch;
            __syncthreads();
        }
        alpha_prev = alpha_n;
        beta_prev = beta_n;
    }
    __syncthreads();

    const int64_t obase = P.out_off[rj] * (int64_t)K;
    for (int idx = tid; idx < K * nI; idx += NT) {
        const int k = idx / nI, o = idx - k * nI;
        const double2 v = xI[(int64_t)k * nIp + o];
        P.out[2 * (obase + idx)] = v.x;
        P.out[2 * (obase + idx) + 1] = v.y;
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
        st_[3] = nswitch;
        st_[4] = M;
        st_[5] = sy.rowptr[sy.nrows] - sy.rowptr[0];
        st_[6] = 0;
        st_[7] = 0;
    }
    __syncthreads();
}

template <int BD, int NT, class TV, class TB, bool SID, bool PROJ>
__global__ __launch_bounds__(NT) void k_scocg(KParams P) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_job;
    const Lds L = lds_carve(smem, P.K, NT);
    char* ws = P.ws + (int64_t)blockIdx.x * P.slot_bytes;
    for (;;) {
        if (threadIdx.x == 0) s_job = atomicAdd(P.queue, 1);
        __syncthreads();
        const int job = __builtin_amdgcn_readfirstlane(s_job);   // uniform: its loads are scalar
        __syncthreads();
        if (job >= P.nrhs) break;
        if constexpr (PROJ) solve_one_proj<BD, NT, SID>(P, P.order[job], ws, L);
        else solve_one<BD, NT, TV, TB, SID>(P, P.order[job], ws, L);
    }
}

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

}  // namespace scocg

// ---------------------------------------------------------------------------
// launch table
// ---------------------------------------------------------------------------
#include "scocg_launch.hpp"

namespace scocg {

template <int BD, int NT, class TV, class TB, bool SID, bool PROJ = false>
static hipError_t launch_one(const KParams& P, int slots, hipStream_t st) {
    const size_t lds = lds_bytes(P.K, NT);
    hipLaunchKernelGGL((k_scocg<BD, NT, TV, TB, SID, PROJ>), dim3(slots), dim3(NT), lds, st, P);
    return hipGetLastError();
}

template <int BD, int NT>
static hipError_t launch_prec(const KParams& P, int prec, bool sid, int slots, hipStream_t st) {
    if (prec == 3) return sid ? launch_one<BD, NT, double, double, true, true>(P, slots, st)
                              : launch_one<BD, NT, double, double, false, true>(P, slots, st);
    if (prec == 0) return sid ? launch_one<BD, NT, double, double, true>(P, slots, st)
                              : launch_one<BD, NT, double, double, false>(P, slots, st);
    if (prec == 1) return sid ? launch_one<BD, NT, float, float, true>(P, slots, st)
                              : launch_one<BD, NT, float, float, false>(P, slots, st);
    return sid ? launch_one<BD, NT, float, bf16_t, true>(P, slots, st)
               : launch_one<BD, NT, float, bf16_t, false>(P, slots, st);
}

template <int BD>
static hipError_t launch_nt(const KParams& P, int prec, bool sid, int nt, int slots, hipStream_t st) {
    if (nt == 256) return launch_prec<BD, 256>(P, prec, sid, slots, st);
    if (nt == 1024) return launch_prec<BD, 1024>(P, prec, sid, slots, st);
    return launch_prec<BD, 512>(P, prec, sid, slots, st);
}

bool supported_bdim(int bd) { return bd == 1 || bd == 4 || bd == 9; }

size_t solver_lds_bytes(int K, int nt) { return lds_bytes(K, nt); }

int64_t solver_slot_bytes(int K, int64_t Mp, int prec) { return slot_bytes_for(K, Mp, prec != 0); }

int64_t solver_slot_bytes_proj(int K, int64_t Mp, int64_t nIp) { return slot_bytes_proj(K, Mp, nIp); }

hipError_t launch_solver(const KParams& P, int bd, int prec, bool sid, int nt, int slots, hipStream_t st) {
    switch (bd) {
        case 1: return launch_nt<1>(P, prec, sid, nt, slots, st);
        case 4: return launch_nt<4>(P, prec, sid, nt, slots, st);
        case 9: return launch_nt<9>(P, prec, sid, nt, slots, st);
        default: return hipErrorInvalidValue;
    }
}

// Private (scratch) bytes per lane of the instance launch_solver would run.
template <int BD, int NT, class TV, class TB, bool SID, bool PROJ = false>
static size_t priv_one() {
    hipFuncAttributes fa{};
    if (hipFuncGetAttributes(&fa, (const void*)k_scocg<BD, NT, TV, TB, SID, PROJ>) != hipSuccess) return (size_t)-1;
    return fa.localSizeBytes;
}
template <int BD, int NT>
static size_t priv_prec(int prec, bool sid) {
    if (prec == 3) return sid ? priv_one<BD, NT, double, double, true, true>() : priv_one<BD, NT, double, double, false, true>();
    if (prec == 0) return sid ? priv_one<BD, NT, double, double, true>() : priv_one<BD, NT, double, double, false>();
    if (prec == 1) return sid ? priv_one<BD, NT, float, float, true>() : priv_one<BD, NT, float, float, false>();
    return sid ? priv_one<BD, NT, float, bf16_t, true>() : priv_one<BD, NT, float, bf16_t, false>();
}
template <int BD>
static size_t priv_nt(int prec, bool sid, int nt) {
    if (nt == 256) return priv_prec<BD, 256>(prec, sid);
    if (nt == 1024) return priv_prec<BD, 1024>(prec, sid);
    return priv_prec<BD, 512>(prec, sid);
}
size_t solver_private_bytes(int bd, int prec, bool sid, int nt) {
    switch (bd) {
        case 1: return priv_nt<1>(prec, sid, nt);
        case 4: return priv_nt<4>(prec, sid, nt);
        case 9: return priv_nt<9>(prec, sid, nt);
        default: return (size_t)-1;
    }
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st) {

    if (n <= 0) return hipSuccess;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

}  // namespace scocg
