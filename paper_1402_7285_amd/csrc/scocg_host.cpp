// Host side of the scocg C ABI: validation, block-pattern merge, order-N
// cluster maps, device residency and kernel launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cctype>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/scocg.h"
#include "mlp_params.hpp"
#include "scocg_launch.hpp"
#include "scocg_params.hpp"

using scocg::KParams;
using scocg::RhsInfo;
using scocg::SysInfo;

namespace {

thread_local std::string g_err;

scocg_status fail(scocg_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(call)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess) {                                                              \
            if (e_ == hipErrorOutOfMemory) return fail(SCOCG_E_NOMEM, "%s: %s", #call,       \
                                                       hipGetErrorString(e_));               \
            return fail(SCOCG_E_DEVICE, "%s: %s", #call, hipGetErrorString(e_));             \
        }                                                                                    \
    } while (0)

template <class T>
scocg_status dev_upload(T** dst, const T* src, size_t n) {
    *dst = nullptr;
    if (n == 0) return SCOCG_OK;
    HIP_TRY(hipMalloc((void**)dst, n * sizeof(T)));
    HIP_TRY(hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice));
    return SCOCG_OK;
}

template <class T>
void dev_free(T*& p) {
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

uint16_t to_bf16(float f) {   // round to nearest even; NaN stays NaN
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

}  // namespace

// ---------------------------------------------------------------------------
// objects
// ---------------------------------------------------------------------------
struct scocg_matrix {
    int64_t nb = 0;
    int32_t bd = 0;
    std::vector<int64_t> rowptr;
    std::vector<int32_t> col;
    std::vector<double> val;
};

struct scocg_problem {
    int device = 0;
    int64_t nb = 0;
    int32_t bd = 0;
    bool has_S = false;
    bool s_unit_diag = false;
    std::vector<int64_t> rowptr;   // merged pattern
    std::vector<int32_t> col;
    std::vector<double> hH, hS;    // merged values (host copy, for lower-precision copies)
    double* dH = nullptr;
    double* dS = nullptr;
    float* dH32 = nullptr;
    float* dS32 = nullptr;
    uint16_t* dHbf = nullptr;
    uint16_t* dSbf = nullptr;
    int64_t* dRowptr = nullptr;    // merged pattern on device (global systems)
    int32_t* dCol = nullptr;
    int32_t* dIota = nullptr;
    // device-buffer solves enqueued by scocg_solve_device and not yet
    // synchronised: their plans stay alive until scocg_sync
    struct Pending {
        scocg_plan* pl;
        hipStream_t st;
        const int8_t* status;
        int64_t n;
    };
    std::vector<Pending> pending;
};

struct scocg_plan {
    scocg_problem* P = nullptr;
    scocg_options opt{};
    int32_t K = 0, nrhs = 0, seed0 = 0;
    int nt = 512, slots = 0, prec = 0;
    bool proj = false;        // projected (requested rows only) FP64 solve
    bool qmr = false;         // real S-Lanczos basis (QMR, or the COCG iterates if gal)
    bool gal = false;
    bool dl = false;          // Lanczos-COCG with the inner CG's direction in LDS
    bool unit = false;        // S applied as I + a copy of its off-diagonal blocks (dsrow/dscol/dsval)
    // team (panel) solver of the Lanczos-basis methods
    bool team = false;
    int G = 1, W = 1, nteams = 0, variant = 0, ri = 0, pairs_max = 0, rows_max = 0, pstride = 0;
    bool team_dl = false;
    size_t team_lds = 0;
    int64_t spin_ticks = 0;
    int32_t* dctl = nullptr;       // [0] queue, [1] abort flag, [32 ..) 32 ints per team
    double* dpart = nullptr;       // teams' reduction partials
    int64_t nIp = 0;
    int64_t Mp = 0, slot_bytes = 0, out_count = 0;
    std::vector<int64_t> out_off;
    // device arrays owned by the plan
    double* dz = nullptr;
    SysInfo* dsys = nullptr;
    RhsInfo* drhs = nullptr;
    int64_t* drowptr = nullptr;
    int32_t* decol = nullptr;
    int32_t* degid = nullptr;
    int32_t* doutl = nullptr;
    int64_t* doutoff = nullptr;
    double* dhout = nullptr;       // H_{row(o), j} of every output row o (scocg_plan_cohp)
    int64_t* dsrow = nullptr;      // S's off-diagonal blocks alone (unit)
    int32_t* dscol = nullptr;
    double* dsval = nullptr;
    int32_t* dsell_col = nullptr;  // the same blocks in ELL form (one-workgroup solver), ell_w per row
    double* dsell_val = nullptr;
    int ell_w = 0;
    bool reg = false;              // one-workgroup inner CG with its residual and solution in registers
    int32_t* dorder = nullptr;
    int32_t* dqueue = nullptr;
    char* dws = nullptr;
    int64_t* dstats = nullptr;
    bool global = true;
    hipStream_t last_stream = nullptr;
    hipGraph_t graph = nullptr;          // captured run (scocg_plan_capture)
    hipGraphExec_t gexec = nullptr;
};

// ---------------------------------------------------------------------------
// matrices
// ---------------------------------------------------------------------------
static scocg_status check_bsr(const scocg_matrix& m) {
    const int64_t nb = m.nb;
    if (m.rowptr[0] != 0) return fail(SCOCG_E_SHAPE, "rowptr[0] must be 0");
    for (int64_t a = 0; a < nb; ++a) {
        if (m.rowptr[a + 1] < m.rowptr[a]) return fail(SCOCG_E_SHAPE, "rowptr decreases at row %lld", (long long)a);
        for (int64_t e = m.rowptr[a]; e < m.rowptr[a + 1]; ++e) {
            const int32_t c = m.col[e];
            if (c < 0 || c >= nb) return fail(SCOCG_E_SHAPE, "colidx %d out of range in row %lld", c, (long long)a);
            if (e > m.rowptr[a] && m.col[e - 1] >= c)
                return fail(SCOCG_E_SHAPE, "colidx not strictly ascending in row %lld", (long long)a);
        }
    }
    // exact symmetry: block (a,b) == block (b,a)^T
    const int bd = m.bd;
    for (int64_t a = 0; a < nb; ++a) {
        for (int64_t e = m.rowptr[a]; e < m.rowptr[a + 1]; ++e) {
            const int64_t b = m.col[e];
            const int32_t* beg = m.col.data() + m.rowptr[b];
            const int32_t* end = m.col.data() + m.rowptr[b + 1];
            const int32_t* f = std::lower_bound(beg, end, (int32_t)a);
            if (f == end || *f != a)
                return fail(SCOCG_E_NOT_SYMMETRIC, "block (%lld,%lld) has no partner", (long long)b, (long long)a);
            const int64_t e2 = f - m.col.data();
            const double* A = m.val.data() + e * bd * bd;
            const double* B = m.val.data() + e2 * bd * bd;
            for (int r = 0; r < bd; ++r)
                for (int c = 0; c < bd; ++c) {
                    const double u = A[r * bd + c], v = B[c * bd + r];
                    if (!(u == v) && !(std::isnan(u) && std::isnan(v)))
                        return fail(SCOCG_E_NOT_SYMMETRIC, "block (%lld,%lld) != transpose of (%lld,%lld)",
                                    (long long)a, (long long)b, (long long)b, (long long)a);
                }
        }
    }
    return SCOCG_OK;
}

extern "C" const char* scocg_last_error(void) { return g_err.c_str(); }
extern "C" const char* scocg_version(void) { return "scocg 0.1 (gfx950)"; }

extern "C" scocg_status scocg_matrix_from_bsr(int64_t nbrows, int32_t bdim, const int64_t* rowptr,
                                              const int32_t* colidx, const double* vals, scocg_matrix** out) {
    if (!out) return fail(SCOCG_E_ARG, "out is NULL");
    *out = nullptr;
    if (nbrows <= 0 || nbrows > INT32_MAX) return fail(SCOCG_E_ARG, "nbrows must be in [1, 2^31)");
    if (bdim < 1 || bdim > 16) return fail(SCOCG_E_ARG, "bdim must be in [1, 16]");
    if (!rowptr || !colidx || !vals) return fail(SCOCG_E_ARG, "NULL array");
    const int64_t nnz = rowptr[nbrows];
    if (nnz < 0 || nnz > INT32_MAX) return fail(SCOCG_E_SHAPE, "block count out of range");
    scocg_matrix* m = new (std::nothrow) scocg_matrix;
    if (!m) return fail(SCOCG_E_NOMEM, "host allocation");
    try {
        m->nb = nbrows;
        m->bd = bdim;
        m->rowptr.assign(rowptr, rowptr + nbrows + 1);
        m->col.assign(colidx, colidx + nnz);
        m->val.assign(vals, vals + nnz * (int64_t)bdim * bdim);
    } catch (...) {
        delete m;
        return fail(SCOCG_E_NOMEM, "host allocation");
    }
    const scocg_status st = check_bsr(*m);
    if (st != SCOCG_OK) {
        delete m;
        return st;
    }
    *out = m;
    return SCOCG_OK;
}

extern "C" scocg_status scocg_matrix_from_csr(int64_t n, const int64_t* rowptr, const int32_t* colidx,
                                              const double* vals, int32_t bdim, scocg_matrix** out) {
    if (!out) return fail(SCOCG_E_ARG, "out is NULL");
    *out = nullptr;
    if (bdim < 1 || bdim > 16 || n <= 0 || n % bdim) return fail(SCOCG_E_ARG, "n must be a positive multiple of bdim");
    if (!rowptr || !colidx || !vals) return fail(SCOCG_E_ARG, "NULL array");
    const int64_t nb = n / bdim;
    std::vector<int64_t> brp(nb + 1, 0);
    std::vector<std::vector<int32_t>> cols(nb);
    for (int64_t i = 0; i < n; ++i) {
        if (rowptr[i + 1] < rowptr[i]) return fail(SCOCG_E_SHAPE, "rowptr decreases");
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            if (colidx[e] < 0 || colidx[e] >= n) return fail(SCOCG_E_SHAPE, "column out of range");
            if (e > rowptr[i] && colidx[e - 1] >= colidx[e]) return fail(SCOCG_E_SHAPE, "columns not ascending");
            cols[i / bdim].push_back(colidx[e] / bdim);
        }
    }
    std::vector<int32_t> bcol;
    for (int64_t a = 0; a < nb; ++a) {
        auto& c = cols[a];
        std::sort(c.begin(), c.end());
        c.erase(std::unique(c.begin(), c.end()), c.end());
        brp[a + 1] = brp[a] + (int64_t)c.size();
        bcol.insert(bcol.end(), c.begin(), c.end());
    }
    std::vector<double> bval((size_t)brp[nb] * bdim * bdim, 0.0);
    for (int64_t i = 0; i < n; ++i) {
        const int64_t a = i / bdim, r = i % bdim;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            const int32_t b = colidx[e] / bdim, c = colidx[e] % bdim;
            const int32_t* beg = bcol.data() + brp[a];
            const int64_t pos = std::lower_bound(beg, (const int32_t*)bcol.data() + brp[a + 1], b) - bcol.data();
            bval[(pos * bdim + r) * bdim + c] = vals[e];
        }
    }
    return scocg_matrix_from_bsr(nb, bdim, brp.data(), bcol.data(), bval.data(), out);
}

// Matrix Market coordinate files (real, symmetric or general), the format
// of published tight-binding matrix sets: entries (i, j, v) 1-based; a
// symmetric file stores one triangle and the other is mirrored here.
// Duplicate entries are summed.  The result goes through the CSR path, so
// the same exact-symmetry check applies.
extern "C" scocg_status scocg_matrix_from_mtx(const char* path, int32_t bdim, scocg_matrix** out) {
    if (!out || !path) return fail(SCOCG_E_ARG, "NULL argument");
    *out = nullptr;
    FILE* f = std::fopen(path, "r");
    if (!f) return fail(SCOCG_E_ARG, "cannot open %s", path);
    struct Closer {
        FILE* f;
        ~Closer() { std::fclose(f); }
    } closer{f};
    char line[4096];
    if (!std::fgets(line, sizeof line, f)) return fail(SCOCG_E_SHAPE, "empty file");
    std::string hdr(line);
    for (auto& ch : hdr) ch = (char)std::tolower((unsigned char)ch);
    if (hdr.rfind("%%matrixmarket", 0) != 0) return fail(SCOCG_E_SHAPE, "not a Matrix Market file");
    if (hdr.find(" matrix ") == std::string::npos || hdr.find(" coordinate ") == std::string::npos)
        return fail(SCOCG_E_SHAPE, "only 'matrix coordinate' files are read");
    if (hdr.find(" real ") == std::string::npos && hdr.find(" integer ") == std::string::npos)
        return fail(SCOCG_E_SHAPE, "only real (or integer) values are read");
    const bool sym = hdr.find(" symmetric") != std::string::npos;
    if (!sym && hdr.find(" general") == std::string::npos)
        return fail(SCOCG_E_SHAPE, "symmetry must be 'symmetric' or 'general'");
    long long nr = -1, nc = -1, nnz = -1;
    while (std::fgets(line, sizeof line, f)) {
        if (line[0] == '%' || line[0] == '\n' || line[0] == '\r') continue;
        if (std::sscanf(line, "%lld %lld %lld", &nr, &nc, &nnz) != 3) return fail(SCOCG_E_SHAPE, "bad size line");
        break;
    }
    if (nr <= 0 || nr != nc || nnz < 0 || nr > INT32_MAX) return fail(SCOCG_E_SHAPE, "matrix must be square");
    struct Ent {
        int32_t i, j;
        double v;
    };
    std::vector<Ent> e;
    e.reserve((size_t)(sym ? 2 * nnz : nnz));
    long long got = 0;
    while (got < nnz && std::fgets(line, sizeof line, f)) {
        if (line[0] == '%' || line[0] == '\n' || line[0] == '\r') continue;
        long long i, j;
        double v;
        if (std::sscanf(line, "%lld %lld %lf", &i, &j, &v) != 3) return fail(SCOCG_E_SHAPE, "bad entry line");
        if (i < 1 || j < 1 || i > nr || j > nr) return fail(SCOCG_E_SHAPE, "entry index out of range");
        e.push_back({(int32_t)(i - 1), (int32_t)(j - 1), v});
        if (sym && i != j) e.push_back({(int32_t)(j - 1), (int32_t)(i - 1), v});
        ++got;
    }
    if (got != nnz) return fail(SCOCG_E_SHAPE, "file ends after %lld of %lld entries", got, nnz);
    std::sort(e.begin(), e.end(), [](const Ent& a, const Ent& b) { return a.i != b.i ? a.i < b.i : a.j < b.j; });
    std::vector<int64_t> rp(nr + 1, 0);
    std::vector<int32_t> ci;
    std::vector<double> vv;
    for (size_t t = 0; t < e.size(); ++t) {
        if (!ci.empty() && t > 0 && e[t].i == e[t - 1].i && e[t].j == e[t - 1].j) {
            vv.back() += e[t].v;
            continue;
        }
        ci.push_back(e[t].j);
        vv.push_back(e[t].v);
        rp[e[t].i + 1] = (int64_t)ci.size();
    }
    for (long long r = 0; r < nr; ++r) rp[r + 1] = std::max(rp[r + 1], rp[r]);
    return scocg_matrix_from_csr((int64_t)nr, rp.data(), ci.data(), vv.data(), bdim, out);
}

extern "C" scocg_status scocg_matrix_shape(const scocg_matrix* m, int64_t* nbrows, int32_t* bdim, int64_t* nblocks) {
    if (!m || !nbrows || !bdim || !nblocks) return fail(SCOCG_E_ARG, "NULL argument");
    *nbrows = m->nb;
    *bdim = m->bd;
    *nblocks = (int64_t)m->col.size();
    return SCOCG_OK;
}

extern "C" scocg_status scocg_matrix_export_bsr(const scocg_matrix* m, int64_t* rowptr, int32_t* colidx,
                                                double* vals) {
    if (!m || !rowptr || !colidx || !vals) return fail(SCOCG_E_ARG, "NULL argument");
    std::copy(m->rowptr.begin(), m->rowptr.end(), rowptr);
    std::copy(m->col.begin(), m->col.end(), colidx);
    std::copy(m->val.begin(), m->val.end(), vals);
    return SCOCG_OK;
}

extern "C" void scocg_matrix_free(scocg_matrix* m) { delete m; }

// ---------------------------------------------------------------------------
// problem
// ---------------------------------------------------------------------------
extern "C" void scocg_problem_free(scocg_problem* p) {
    if (!p) return;
    (void)hipSetDevice(p->device);
    (void)scocg_sync(p);          // finishes and frees any device-buffer solve still pending
    dev_free(p->dH);
    dev_free(p->dS);
    dev_free(p->dH32);
    dev_free(p->dS32);
    dev_free(p->dHbf);
    dev_free(p->dSbf);
    dev_free(p->dRowptr);
    dev_free(p->dCol);
    dev_free(p->dIota);
    delete p;
}

extern "C" scocg_status scocg_problem_create(const scocg_matrix* H, const scocg_matrix* S, scocg_problem** out) {
    if (!out) return fail(SCOCG_E_ARG, "out is NULL");
    *out = nullptr;
    if (!H) return fail(SCOCG_E_ARG, "H is NULL");
    if (S && (S->nb != H->nb || S->bd != H->bd)) return fail(SCOCG_E_SHAPE, "H and S differ in shape");
    scocg_problem* p = new (std::nothrow) scocg_problem;
    if (!p) return fail(SCOCG_E_NOMEM, "host allocation");
    scocg_status st = SCOCG_OK;
    try {
        HIP_TRY(hipGetDevice(&p->device));
        p->nb = H->nb;
        p->bd = H->bd;
        p->has_S = S != nullptr;
        const int bd = p->bd, bb = bd * bd;
        p->rowptr.assign(p->nb + 1, 0);
        // merged pattern: per row, the sorted union of H's and S's columns and
        // the diagonal block (zero where neither has it), so that every block
        // row, also of every cluster, has at least one entry: the kernels'
        // chunked row sums re-read a row's last entry to fill a chunk.
        for (int64_t a = 0; a < p->nb; ++a) {
            int64_t i = H->rowptr[a], ie = H->rowptr[a + 1];
            int64_t j = S ? S->rowptr[a] : 0, je = S ? S->rowptr[a + 1] : 0;
            bool diag_done = false;
            while (i < ie || j < je || !diag_done) {
                const int32_t ch = i < ie ? H->col[i] : INT32_MAX;
                const int32_t cs = j < je ? S->col[j] : INT32_MAX;
                const int32_t cm = std::min(ch, cs);
                if (!diag_done && a <= cm) {
                    if (a < cm) {   // no stored diagonal block: a zero one
                        p->col.push_back((int32_t)a);
                        for (int t = 0; t < bb; ++t) p->hH.push_back(0.0);
                        if (S)
                            for (int t = 0; t < bb; ++t) p->hS.push_back(0.0);
                        diag_done = true;
                        continue;
                    }
                    diag_done = true;
                }
                const bool th = ch == cm && i < ie;
                const bool ts = cs == cm && j < je;
                p->col.push_back(cm);
                for (int t = 0; t < bb; ++t) p->hH.push_back(th ? H->val[i * bb + t] : 0.0);
                if (S)
                    for (int t = 0; t < bb; ++t) p->hS.push_back(ts ? S->val[j * bb + t] : 0.0);
                if (th) ++i;
                if (ts) ++j;
            }
            p->rowptr[a + 1] = (int64_t)p->col.size();
        }
        if (p->col.size() > (size_t)INT32_MAX) {
            scocg_problem_free(p);
            return fail(SCOCG_E_SHAPE, "too many blocks");
        }
        const int64_t nblk = (int64_t)p->col.size();
        // S diagonal: unit? (only needs SPD; a unit diagonal is the LCAO norm)
        if (S) {
            bool unit = true, unit_diag_elems = true;
            for (int64_t a = 0; a < p->nb; ++a) {
                const int32_t* beg = p->col.data() + p->rowptr[a];
                const int64_t e = std::lower_bound(beg, (const int32_t*)p->col.data() + p->rowptr[a + 1], (int32_t)a) - p->col.data();
                if (e >= p->rowptr[a + 1] || p->col[e] != a) {
                    unit = unit_diag_elems = false;
                    break;
                }
                for (int r = 0; r < bd; ++r)
                    for (int c = 0; c < bd; ++c) {
                        const double v = p->hS[e * bb + r * bd + c];
                        if (v != (r == c ? 1.0 : 0.0)) unit = false;
                        if (r == c && v != 1.0) unit_diag_elems = false;
                    }
            }
            p->s_unit_diag = unit;
            if (!unit_diag_elems) st = SCOCG_W_S_DIAG;
        }
        scocg_status e;
        if ((e = dev_upload(&p->dH, p->hH.data(), p->hH.size())) != SCOCG_OK) { scocg_problem_free(p); return e; }
        if (S && (e = dev_upload(&p->dS, p->hS.data(), p->hS.size())) != SCOCG_OK) { scocg_problem_free(p); return e; }
        if ((e = dev_upload(&p->dRowptr, p->rowptr.data(), p->rowptr.size())) != SCOCG_OK) { scocg_problem_free(p); return e; }
        if ((e = dev_upload(&p->dCol, p->col.data(), p->col.size())) != SCOCG_OK) { scocg_problem_free(p); return e; }
        std::vector<int32_t> iota(nblk);
        for (int64_t t = 0; t < nblk; ++t) iota[t] = (int32_t)t;
        if ((e = dev_upload(&p->dIota, iota.data(), iota.size())) != SCOCG_OK) { scocg_problem_free(p); return e; }
    } catch (const std::bad_alloc&) {
        scocg_problem_free(p);
        return fail(SCOCG_E_NOMEM, "host allocation");
    }
    *out = p;
    if (st != SCOCG_OK) fail(st, "S has a diagonal element different from 1");
    return st;
}

static scocg_status ensure_lowp(scocg_problem* p, int prec) {
    if (prec == SCOCG_FP32 && !p->dH32) {
        std::vector<float> h(p->hH.begin(), p->hH.end());
        scocg_status e = dev_upload(&p->dH32, h.data(), h.size());
        if (e) return e;
        if (p->has_S) {
            std::vector<float> s(p->hS.begin(), p->hS.end());
            if ((e = dev_upload(&p->dS32, s.data(), s.size()))) return e;
        }
    }
    if (prec == SCOCG_FP32_BF16 && !p->dHbf) {
        std::vector<uint16_t> h(p->hH.size());
        for (size_t i = 0; i < h.size(); ++i) h[i] = to_bf16((float)p->hH[i]);
        scocg_status e = dev_upload(&p->dHbf, h.data(), h.size());
        if (e) return e;
        if (p->has_S) {
            std::vector<uint16_t> s(p->hS.size());
            for (size_t i = 0; i < s.size(); ++i) s[i] = to_bf16((float)p->hS[i]);
            if ((e = dev_upload(&p->dSbf, s.data(), s.size()))) return e;
        }
    }
    return SCOCG_OK;
}

// ---------------------------------------------------------------------------
// options
// ---------------------------------------------------------------------------
extern "C" void scocg_options_default(scocg_options* o) {
    if (!o) return;
    o->tol = 1e-10;
    o->maxiter = 0;
    o->precision = SCOCG_FP64;
    o->replace_every = 0;
    o->inner_maxiter = 1000;
    o->inner_tol = 1e-13;
    o->inner_tol_lo = 1e-6;
    o->seed_index = -1;
    o->threads = 0;
    o->slots = 0;
    o->audit = 1;
    o->projected = 1;
    o->method = SCOCG_METHOD_COCG;
    o->team_size = 0;
    o->panel_width = 0;
    o->team_registers = 1;
}

// Initial seed: smallest |Im z|, then Re z closest to the median of Re z
// (mean of the two middle values for an even count), then lowest index.
static int initial_seed(const scocg_z* z, int K) {
    std::vector<double> E(K);
    for (int k = 0; k < K; ++k) E[k] = z[k].re;
    std::sort(E.begin(), E.end());
    const double med = (K % 2) ? E[K / 2] : (E[K / 2 - 1] + E[K / 2]) / 2.0;
    int best = 0;
    for (int k = 1; k < K; ++k) {
        const double ai = std::fabs(z[k].im), bi = std::fabs(z[best].im);
        const double ar = std::fabs(z[k].re - med), br = std::fabs(z[best].re - med);
        if (ai < bi || (ai == bi && ar < br)) best = k;
    }
    return best;
}

// ---------------------------------------------------------------------------
// plans
// ---------------------------------------------------------------------------
extern "C" void scocg_plan_free(scocg_plan* pl) {
    if (!pl) return;
    (void)hipSetDevice(pl->P->device);
    if (pl->last_stream) (void)hipStreamSynchronize(pl->last_stream);
    else (void)hipDeviceSynchronize();
    if (pl->gexec) (void)hipGraphExecDestroy(pl->gexec);
    if (pl->graph) (void)hipGraphDestroy(pl->graph);
    dev_free(pl->dz);
    dev_free(pl->dsys);
    dev_free(pl->drhs);
    if (!pl->global) {
        dev_free(pl->drowptr);
        dev_free(pl->decol);
        dev_free(pl->degid);
    }
    dev_free(pl->doutl);
    dev_free(pl->doutoff);
    dev_free(pl->dhout);
    dev_free(pl->dsrow);
    dev_free(pl->dscol);
    dev_free(pl->dsval);
    dev_free(pl->dsell_col);
    dev_free(pl->dsell_val);
    dev_free(pl->dorder);
    dev_free(pl->dqueue);
    dev_free(pl->dws);
    dev_free(pl->dstats);
    dev_free(pl->dctl);
    dev_free(pl->dpart);
    delete pl;
}

namespace {

struct HostMaps {
    std::vector<SysInfo> sys;
    std::vector<RhsInfo> rhs;
    std::vector<int64_t> rowptr;
    std::vector<int32_t> ecol, egid, outl;
    std::vector<int64_t> outoff;
    int64_t maxM = 0;
};

template <class F>
void parallel_for(int64_t n, F f) {
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (n < 64) nth = 1;
    std::vector<std::thread> th;
    std::atomic<int64_t> next{0};
    auto body = [&]() {
        for (;;) {
            const int64_t i = next.fetch_add(16);
            if (i >= n) break;
            for (int64_t t = i; t < std::min(n, i + 16); ++t) f(t);
        }
    };
    for (unsigned t = 1; t < nth; ++t) th.emplace_back(body);
    body();
    for (auto& t : th) t.join();
}

scocg_status build_maps(const scocg_problem* P, int32_t nrhs, const int32_t* rhs_index,
                        const scocg_rhs_spec* spec, HostMaps& hm) {
    const int bd = P->bd;
    const int64_t nb = P->nb, M = nb * bd;
    const bool cluster = spec && spec->cluster_ptr;
    const bool full = spec && spec->out_mode == SCOCG_OUT_FULL_X;
    if (spec && spec->out_mode != SCOCG_OUT_FULL_X && spec->out_mode != SCOCG_OUT_SELECTED_G)
        return fail(SCOCG_E_ARG, "unknown out_mode %d", spec->out_mode);
    if (!full && (!spec || !spec->out_ptr || !spec->out_rows))
        return fail(SCOCG_E_ARG, "SELECTED_G needs out_ptr and out_rows");
    if (cluster && !spec->cluster_atoms) return fail(SCOCG_E_ARG, "cluster_atoms is NULL");
    for (int32_t r = 0; r < nrhs; ++r)
        if (rhs_index[r] < 0 || rhs_index[r] >= M) return fail(SCOCG_E_ARG, "rhs_index[%d] out of range", r);
    if (!full) {
        if (spec->out_ptr[0] != 0) return fail(SCOCG_E_ARG, "out_ptr[0] must be 0");
        for (int32_t r = 0; r < nrhs; ++r)
            if (spec->out_ptr[r + 1] < spec->out_ptr[r]) return fail(SCOCG_E_ARG, "out_ptr decreases");
    }
    if (cluster) {
        if (spec->cluster_ptr[0] != 0) return fail(SCOCG_E_ARG, "cluster_ptr[0] must be 0");
        for (int32_t r = 0; r < nrhs; ++r) {
            const int64_t c0 = spec->cluster_ptr[r], c1 = spec->cluster_ptr[r + 1];
            if (c1 <= c0) return fail(SCOCG_E_ARG, "cluster of RHS %d is empty", r);
            if ((c1 - c0) * bd > INT32_MAX / 2) return fail(SCOCG_E_ARG, "cluster too large");
            for (int64_t t = c0; t < c1; ++t) {
                const int32_t a = spec->cluster_atoms[t];
                if (a < 0 || a >= nb) return fail(SCOCG_E_ARG, "cluster atom out of range (RHS %d)", r);
                if (t > c0 && spec->cluster_atoms[t - 1] >= a)
                    return fail(SCOCG_E_ARG, "cluster atoms of RHS %d not strictly ascending", r);
            }
        }
    }
    hm.rhs.resize(nrhs);
    hm.outoff.assign(nrhs + 1, 0);
    if (!cluster) {
        SysInfo s{0, 0, (int32_t)nb, 0};
        hm.sys.push_back(s);
        hm.maxM = M;
        for (int32_t r = 0; r < nrhs; ++r) {
            RhsInfo& ri = hm.rhs[r];
            ri.sys = 0;
            ri.b_local = rhs_index[r];
            ri.full_x = full ? 1 : 0;
            if (full) {
                ri.out_base = 0;
                ri.nout = (int32_t)M;
            } else {
                ri.out_base = spec->out_ptr[r];
                ri.nout = (int32_t)(spec->out_ptr[r + 1] - spec->out_ptr[r]);
                for (int64_t t = spec->out_ptr[r]; t < spec->out_ptr[r + 1]; ++t)
                    if (spec->out_rows[t] < 0 || spec->out_rows[t] >= M)
                        return fail(SCOCG_E_ARG, "out row out of range (RHS %d)", r);
            }
            hm.outoff[r + 1] = hm.outoff[r] + ri.nout;
        }
        if (!full) hm.outl.assign(spec->out_rows, spec->out_rows + spec->out_ptr[nrhs]);
        return SCOCG_OK;
    }
    // ---- order-N clusters: principal submatrix on each RHS's atoms
    std::vector<int64_t> ecount(nrhs, 0);
    std::atomic<int> bad{-1};
    std::atomic<int> badkind{0};
    const int64_t* rp = P->rowptr.data();
    const int32_t* cl = P->col.data();
    auto count_fn = [&](int64_t r) {
        const int64_t c0 = spec->cluster_ptr[r], c1 = spec->cluster_ptr[r + 1];
        const int32_t* at = spec->cluster_atoms + c0;
        const int64_t n = c1 - c0;
        int64_t cnt = 0;
        for (int64_t t = 0; t < n; ++t) {
            const int32_t a = at[t];
            for (int64_t e = rp[a]; e < rp[a + 1]; ++e)
                if (std::binary_search(at, at + n, cl[e])) ++cnt;
        }
        ecount[r] = cnt;
        const int32_t ja = rhs_index[r] / bd;
        if (!std::binary_search(at, at + n, ja)) { bad = (int)r; badkind = 1; }
        if (!full) {
            for (int64_t t = spec->out_ptr[r]; t < spec->out_ptr[r + 1]; ++t) {
                const int32_t o = spec->out_rows[t];
                if (o < 0 || o >= M || !std::binary_search(at, at + n, o / bd)) { bad = (int)r; badkind = 2; }
            }
        }
    };
    parallel_for(nrhs, count_fn);
    if (bad >= 0)
        return fail(SCOCG_E_ARG, badkind == 1 ? "RHS %d: its orbital's atom is not in its cluster"
                                              : "RHS %d: an out row is not in its cluster", (int)bad);
    hm.sys.resize(nrhs);
    int64_t rbase = 0, ebase = 0, obase = 0;
    for (int32_t r = 0; r < nrhs; ++r) {
        const int64_t n = spec->cluster_ptr[r + 1] - spec->cluster_ptr[r];
        hm.sys[r] = SysInfo{rbase, ebase, (int32_t)n, 0};
        rbase += n + 1;
        ebase += ecount[r];
        RhsInfo& ri = hm.rhs[r];
        ri.sys = r;
        ri.full_x = full ? 1 : 0;
        ri.nout = full ? (int32_t)(n * bd) : (int32_t)(spec->out_ptr[r + 1] - spec->out_ptr[r]);
        ri.out_base = obase;
        if (!full) obase += ri.nout;
        hm.outoff[r + 1] = hm.outoff[r] + ri.nout;
        hm.maxM = std::max<int64_t>(hm.maxM, n * bd);
    }
    hm.rowptr.assign(rbase, 0);
    hm.ecol.assign(ebase, 0);
    hm.egid.assign(ebase, 0);
    hm.outl.assign(obase, 0);
    auto fill_fn = [&](int64_t r) {
        const int64_t c0 = spec->cluster_ptr[r], c1 = spec->cluster_ptr[r + 1];
        const int32_t* at = spec->cluster_atoms + c0;
        const int64_t n = c1 - c0;
        int64_t* rowp = hm.rowptr.data() + hm.sys[r].row_base;
        int32_t* ec = hm.ecol.data() + hm.sys[r].ent_base;
        int32_t* eg = hm.egid.data() + hm.sys[r].ent_base;
        int64_t cnt = 0;
        rowp[0] = 0;
        for (int64_t t = 0; t < n; ++t) {
            const int32_t a = at[t];
            for (int64_t e = rp[a]; e < rp[a + 1]; ++e) {
                const int32_t* f = std::lower_bound(at, at + n, cl[e]);
                if (f != at + n && *f == cl[e]) {
                    ec[cnt] = (int32_t)(f - at);
                    eg[cnt] = (int32_t)e;
                    ++cnt;
                }
            }
            rowp[t + 1] = cnt;
        }
        const int32_t j = rhs_index[r];
        hm.rhs[r].b_local = (int32_t)((std::lower_bound(at, at + n, j / bd) - at) * bd + j % bd);
        if (!full) {
            int32_t* ol = hm.outl.data() + hm.rhs[r].out_base;
            for (int64_t t = spec->out_ptr[r]; t < spec->out_ptr[r + 1]; ++t) {
                const int32_t o = spec->out_rows[t];
                ol[t - spec->out_ptr[r]] = (int32_t)((std::lower_bound(at, at + n, o / bd) - at) * bd + o % bd);
            }
        }
    };
    parallel_for(nrhs, fill_fn);
    return SCOCG_OK;
}

// H_{i, j} for every output row of every RHS (i the output row's global
// orbital, j the RHS's orbital), from the merged block pattern; 0 where the
// block (atom(i), atom(j)) is not in the pattern.
void output_h(const scocg_problem* P, int32_t nrhs, const int32_t* rhs_index, const scocg_rhs_spec* spec,
              const HostMaps& hm, std::vector<double>& h) {
    const int bd = P->bd;
    const bool cluster = spec && spec->cluster_ptr;
    const bool full = spec && spec->out_mode == SCOCG_OUT_FULL_X;
    h.assign((size_t)hm.outoff[nrhs], 0.0);
    auto fn = [&](int64_t r) {
        const int32_t j = rhs_index[r];
        const int32_t ja = j / bd, jr = j % bd;
        const int64_t n = hm.outoff[r + 1] - hm.outoff[r];
        double* hr = h.data() + hm.outoff[r];
        for (int64_t t = 0; t < n; ++t) {
            int64_t i;
            if (!full) i = spec->out_rows[spec->out_ptr[r] + t];
            else if (cluster) i = (int64_t)spec->cluster_atoms[spec->cluster_ptr[r] + t / bd] * bd + t % bd;
            else i = t;
            const int64_t ia = i / bd;
            const int32_t* beg = P->col.data() + P->rowptr[ia];
            const int32_t* end = P->col.data() + P->rowptr[ia + 1];
            const int32_t* f = std::lower_bound(beg, end, ja);
            if (f == end || *f != ja) continue;
            const int64_t e = f - P->col.data();
            hr[t] = P->hH[(size_t)e * bd * bd + (size_t)(i % bd) * bd + jr];
        }
    };
    parallel_for(nrhs, fn);
}

}  // namespace

extern "C" scocg_status scocg_plan_create(scocg_problem* P, const scocg_options* opt_in, int32_t nshift,
                                          const scocg_z* shifts, int32_t nrhs, const int32_t* rhs_index,
                                          const scocg_rhs_spec* spec, scocg_plan** out) {
    if (!out) return fail(SCOCG_E_ARG, "out is NULL");
    *out = nullptr;
    if (!P) return fail(SCOCG_E_ARG, "problem is NULL");
    scocg_options opt;
    if (opt_in) opt = *opt_in; else scocg_options_default(&opt);
    if (!(opt.tol > 0.0)) return fail(SCOCG_E_ARG, "tol must be > 0");
    if (opt.maxiter < 0 || opt.inner_maxiter < 0) return fail(SCOCG_E_ARG, "negative iteration cap");
    if (opt.precision < SCOCG_FP64 || opt.precision > SCOCG_FP32_BF16) return fail(SCOCG_E_ARG, "unknown precision");
    if (!(opt.inner_tol > 0.0) || !(opt.inner_tol_lo > 0.0)) return fail(SCOCG_E_ARG, "inner tolerances must be > 0");
    if (opt.threads != 0 && opt.threads != 256 && opt.threads != 512 && opt.threads != 1024)
        return fail(SCOCG_E_ARG, "threads must be 0, 256, 512 or 1024");
    if (opt.slots < 0) return fail(SCOCG_E_ARG, "slots must be >= 0");
    if (nshift < 1 || nshift > 512) return fail(nshift < 1 ? SCOCG_E_ARG : SCOCG_E_UNSUPPORTED, "nshift must be in [1, 512]");
    if (!shifts) return fail(SCOCG_E_ARG, "shifts is NULL");
    for (int k = 0; k < nshift; ++k)
        if (!std::isfinite(shifts[k].re) || !std::isfinite(shifts[k].im)) return fail(SCOCG_E_ARG, "shift %d not finite", k);
    if (nrhs < 0 || (nrhs > 0 && !rhs_index)) return fail(SCOCG_E_ARG, "bad RHS list");
    if (opt.seed_index < -1 || opt.seed_index >= nshift) return fail(SCOCG_E_ARG, "seed_index out of range");
    if (!scocg::supported_bdim(P->bd)) return fail(SCOCG_E_UNSUPPORTED, "block size %d not compiled in", P->bd);
    if (spec && spec->order) {
        std::vector<char> seen(nrhs, 0);
        for (int32_t r = 0; r < nrhs; ++r) {
            const int32_t o = spec->order[r];
            if (o < 0 || o >= nrhs || seen[o]) return fail(SCOCG_E_ARG, "order is not a permutation");
            seen[o] = 1;
        }
    }
    HIP_TRY(hipSetDevice(P->device));
    HostMaps hm;
    scocg_status st;
    try {
        st = build_maps(P, nrhs, rhs_index, spec, hm);
    } catch (const std::bad_alloc&) {
        return fail(SCOCG_E_NOMEM, "host allocation");
    }
    if (st != SCOCG_OK) return st;
    if ((st = ensure_lowp(P, opt.precision)) != SCOCG_OK) return st;

    scocg_plan* pl = new (std::nothrow) scocg_plan;
    if (!pl) return fail(SCOCG_E_NOMEM, "host allocation");
    pl->P = P;
    pl->opt = opt;
    pl->K = nshift;
    pl->nrhs = nrhs;
    pl->prec = opt.precision;
    pl->seed0 = opt.seed_index >= 0 ? opt.seed_index : initial_seed(shifts, nshift);
    pl->global = !(spec && spec->cluster_ptr);
    pl->out_off = hm.outoff;
    pl->out_count = hm.outoff[nrhs] * (int64_t)nshift;
    pl->nt = opt.threads ? opt.threads : 512;
    pl->Mp = std::max<int64_t>(64, (hm.maxM + 63) / 64 * 64);
    pl->proj = opt.projected && opt.precision == SCOCG_FP64 && !(spec && spec->out_mode == SCOCG_OUT_FULL_X);
    pl->qmr = opt.method == SCOCG_METHOD_QMR || opt.method == SCOCG_METHOD_COCG_LANCZOS;
    pl->gal = opt.method == SCOCG_METHOD_COCG_LANCZOS;
    if (opt.method != SCOCG_METHOD_COCG && opt.method != SCOCG_METHOD_QMR && opt.method != SCOCG_METHOD_COCG_LANCZOS) {
        scocg_plan_free(pl);
        return fail(SCOCG_E_ARG, "unknown method %d", opt.method);
    }
    if (pl->qmr && (opt.precision != SCOCG_FP64 || (spec && spec->out_mode == SCOCG_OUT_FULL_X))) {
        scocg_plan_free(pl);
        return fail(SCOCG_E_UNSUPPORTED, "the Lanczos-basis methods run in FP64 with SELECTED_G output");
    }
    if (pl->qmr) {
        int64_t maxout = 1;
        for (const auto& r : hm.rhs) maxout = std::max<int64_t>(maxout, r.nout);
        pl->nIp = (maxout + 63) / 64 * 64;
        pl->slot_bytes = scocg::qmr_slot_bytes(nshift, pl->Mp, pl->nIp);
        pl->proj = false;
    } else if (pl->proj) {
        int64_t maxout = 1;
        for (const auto& r : hm.rhs) maxout = std::max<int64_t>(maxout, r.nout);
        pl->nIp = (maxout + 63) / 64 * 64;
        pl->slot_bytes = scocg::solver_slot_bytes_proj(nshift, pl->Mp, pl->nIp);
    } else {
        pl->slot_bytes = scocg::solver_slot_bytes(nshift, pl->Mp, opt.precision);
    }

    auto bail = [&](scocg_status e) { scocg_plan_free(pl); return e; };
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, P->device) != hipSuccess || cus <= 0) cus = 256;
    // the generalized Lanczos-basis forms keep the inner CG's direction in LDS when it fits
    pl->dl = pl->qmr && P->has_S && scocg::qmr_lds_bytes(nshift, pl->nt, pl->Mp, true) <= 160 * 1024;
    const size_t lds = pl->qmr ? scocg::qmr_lds_bytes(nshift, pl->nt, pl->Mp, pl->dl)
                               : scocg::solver_lds_bytes(nshift, pl->nt);
    if (lds > 160 * 1024) return bail(fail(SCOCG_E_UNSUPPORTED, "too many shifts for LDS"));
    // S = I + its off-diagonal blocks (Lanczos-basis forms on a global system whose diagonal blocks of S
    // are exactly I): a copy of the nonzero off-diagonal blocks in their own CSR, so that the inner CG
    // never reads an identity block
    std::vector<int64_t> srow_h;
    std::vector<int32_t> scol_h;
    std::vector<double> sval_h;
    if (pl->qmr && P->has_S && pl->global && P->s_unit_diag) {
        const int bd = P->bd;
        const size_t bb = (size_t)bd * bd;
        srow_h.assign((size_t)P->nb + 1, 0);
        for (int64_t a = 0; a < P->nb; ++a) {
            for (int64_t e = P->rowptr[a]; e < P->rowptr[a + 1]; ++e) {
                if (P->col[e] == a) continue;
                const double* blk = P->hS.data() + (size_t)e * bb;
                bool any = false;
                for (size_t t = 0; t < bb && !any; ++t) any = blk[t] != 0.0;
                if (!any) continue;
                scol_h.push_back(P->col[e]);
                sval_h.insert(sval_h.end(), blk, blk + bb);
            }
            srow_h[a + 1] = (int64_t)scol_h.size();
        }
        if (scol_h.empty()) srow_h.clear();
        else pl->unit = true;
    }
    // The same blocks in ELL form (every block row padded to the longest with its own column and a zero
    // block) for the one-workgroup solver, when the rows are near-uniform (at most a quarter padding):
    // its row product then needs no row extent and issues a row's index and block loads together.
    std::vector<int32_t> ecol_ell;
    std::vector<double> eval_ell;
    if (pl->unit) {
        const size_t bb = (size_t)P->bd * P->bd;
        int64_t wmax = 0;
        for (int64_t a = 0; a < P->nb; ++a) wmax = std::max<int64_t>(wmax, srow_h[a + 1] - srow_h[a]);
        const int64_t total = srow_h[(size_t)P->nb];
        if (wmax > 0 && wmax <= 16 && 4 * total >= 3 * wmax * P->nb) {
            pl->ell_w = (int)wmax;
            ecol_ell.assign((size_t)(P->nb * wmax), 0);
            eval_ell.assign((size_t)(P->nb * wmax) * bb, 0.0);
            for (int64_t a = 0; a < P->nb; ++a) {
                for (int64_t u = 0; u < wmax; ++u) {
                    const int64_t e = srow_h[a] + u;
                    const size_t o = (size_t)(a * wmax + u);
                    if (e < srow_h[a + 1]) {
                        ecol_ell[o] = scol_h[(size_t)e];
                        std::copy(sval_h.begin() + (size_t)e * bb, sval_h.begin() + (size_t)(e + 1) * bb,
                                  eval_ell.begin() + o * bb);
                    } else {
                        ecol_ell[o] = (int32_t)a;
                    }
                }
            }
        }
    }

    // a workgroup size whose kernel instance would spill registers to private memory is not launched:
    // the first of (requested, 512, 256, 1024) that keeps every value in registers runs instead
    // (the Lanczos-basis forms on the ELL blocks at 512 threads first try the instance that keeps the inner
    // CG's residual and solution in registers, when a thread's rows fit it)
    if (!pl->team) {
        const int tries[4] = {pl->nt, 512, 256, 1024};
        bool found = false;
        for (int nt : tries) {
            const size_t dl_lds = pl->qmr ? scocg::qmr_lds_bytes(nshift, nt, pl->Mp, pl->dl) : 0;
            if (pl->qmr && dl_lds > 160 * 1024) continue;
            const bool reg = pl->qmr && pl->unit && pl->dl && pl->ell_w > 0 && P->bd == 4 && nt == 512 &&
                             pl->Mp <= 32 * 512;
            for (int um : {reg ? 2 : -1, pl->unit && pl->dl ? 1 : 0}) {
                if (um < 0) continue;
                const size_t priv = pl->qmr ? scocg::qmr_private_bytes(P->bd, !P->has_S, pl->gal, pl->dl, um, nt)
                                            : scocg::solver_private_bytes(P->bd, pl->proj ? 3 : pl->prec, !P->has_S, nt);
                if (priv == 0) {
                    pl->nt = nt;
                    pl->reg = um == 2;
                    found = true;
                    break;
                }
            }
            if (found) break;
        }
    }
    const size_t lds_nt = pl->qmr ? scocg::qmr_lds_bytes(nshift, pl->nt, pl->Mp, pl->dl)
                                  : scocg::solver_lds_bytes(nshift, pl->nt);
    int per_cu = std::max(1, 2048 / pl->nt);
    per_cu = std::min<int>(per_cu, (int)std::max<size_t>(1, (160 * 1024) / lds_nt));
    per_cu = std::min(per_cu, 2);
    int slots = opt.slots ? opt.slots : cus * per_cu;
    slots = std::max(1, std::min(slots, std::max(1, nrhs)));
    size_t freeb = 0, totb = 0;
    if (hipMemGetInfo(&freeb, &totb) == hipSuccess && freeb > 0) {
        const int64_t cap = (int64_t)(0.8 * (double)freeb) / std::max<int64_t>(1, pl->slot_bytes);
        if (cap < 1) return bail(fail(SCOCG_E_NOMEM, "one workgroup slot (%lld bytes) exceeds free memory",
                                      (long long)pl->slot_bytes));
        slots = (int)std::min<int64_t>(slots, cap);
    }
    pl->slots = slots;

    // ---- team (panel) solver of the Lanczos-basis methods
    if (pl->qmr && opt.team_size >= 0 && nrhs > 0) {
        int W = opt.panel_width, G = opt.team_size;
        const bool can_panel = pl->global && P->bd == 4;
        if (W != 0 && W != 1 && W != 4 && W != 8) return bail(fail(SCOCG_E_ARG, "panel_width must be 0, 1, 4 or 8"));
        if (W > 1 && !can_panel)
            return bail(fail(SCOCG_E_UNSUPPORTED, "panels of several RHS need 4x4 blocks and the whole system"));
        if (G > 32) return bail(fail(SCOCG_E_ARG, "team_size must be -1 .. 32"));
        // Chosen by the library: the one-workgroup solver whenever the right-hand sides alone fill the
        // compute units (measured faster there: every workgroup then streams its own vectors without team
        // waits); teams when there are fewer RHS than compute units on a large system, or order-N
        // clusters large enough that one workgroup per RHS would bound the launch by its latency.
        const bool auto_shape = G == 0 && W == 0;
        if (W == 0) W = can_panel && nrhs < cus ? (nrhs >= 64 ? 8 : (nrhs >= 16 ? 4 : 1)) : 1;
        const int npanels = (nrhs + W - 1) / W;
        if (G == 0) {
            if (pl->global) {
                // enough teams to fill the compute units, at least 64 block rows per workgroup
                G = 1;
                while (G < 8 && (int64_t)npanels * G * 2 <= cus && P->nb >= (int64_t)G * 2 * 64) G *= 2;
                if (auto_shape && nrhs >= cus) G = 1;
            } else {
                // (measured on a launch of 64 order-N clusters of an fcc crystal with 9x9 blocks and 256
                // shifts, the largest with M_j = 9,495 rows: 43.5 s with teams of 8, 35.0 s with 16, 52.2 s
                // with 32)
                G = hm.maxM >= 8192 ? 16 : (hm.maxM >= 6144 ? 8 : (hm.maxM >= 3072 ? 4 : (hm.maxM >= 1536 ? 2 : 1)));
            }
        }
        if (G > 1 || W > 1) {
            if (opt.threads != 0 && opt.threads != 512 && opt.threads != 1024)
                return bail(fail(SCOCG_E_ARG, "the team solver runs 512 or 1024 threads per workgroup"));
            pl->team = true;
            pl->G = G;
            pl->W = W;
            pl->pairs_max = (W * nshift + G - 1) / G;
            int64_t maxshare = 0;
            for (const auto& sy : hm.sys) maxshare = std::max<int64_t>(maxshare, ((int64_t)sy.nrows + G - 1) / G);
            pl->rows_max = (int)(maxshare * P->bd);
            // 160 KB of LDS per workgroup, less the kernel's own few static words
            const size_t lds_cap = 160 * 1024 - 256;
            pl->team_dl = P->has_S && scocg::team_lds_bytes(512, W, pl->pairs_max, pl->rows_max, true) <= lds_cap;
            // Launch shapes in order of preference; the first whose kernel fits a compute unit and keeps
            // every value in registers (no scratch: private-memory spills are never launched) is taken.
            // (threads is a request: the other size runs if the requested one would spill or not fit)
            std::vector<int> nts;
            if (opt.threads) nts = {opt.threads, opt.threads == 1024 ? 512 : 1024};
            else if (W >= 8) nts = {1024, 512};
            else nts = {512, 1024};
            int per_cu = 0;
            bool found = false;
            for (int nt : nts) {
                for (int rv = opt.team_registers ? 1 : 0; rv >= 0 && !found; --rv) {
                    int variant = !P->has_S ? 0 : (pl->team_dl ? (pl->unit ? 2 : 1) : 3);
                    int ri = 0;
                    size_t lds = scocg::team_lds_bytes(nt, W, pl->pairs_max, pl->rows_max, pl->team_dl);
                    if (rv) {
                        // the inner CG's vectors in registers (its residual in the LDS region of the direction)
                        // when a compiled instance covers this workgroup's share of block rows
                        if (!(P->has_S && pl->team_dl && P->bd == 4 && W % 4 == 0)) continue;
                        const int nw = nt / 64;
                        const int need = (int)((maxshare + 4 * nw - 1) / (4 * nw));
                        const size_t lds_rv = scocg::team_lds_bytes(nt, W, pl->pairs_max, pl->rows_max, true, true);
                        for (int r : {4, 8, 16})
                            if (r >= need && scocg::team_rv_ok(nt, W, r) && lds_rv <= lds_cap) {
                                ri = r;
                                break;
                            }
                        if (!ri) continue;
                        variant = pl->unit ? 4 : 5;
                        lds = lds_rv;
                    }
                    if (lds > lds_cap) continue;
                    int pc = 0;
                    size_t priv = 0;
                    if (scocg::team_occupancy(P->bd, pl->gal, variant, ri, nt, W, lds, &pc, &priv) != hipSuccess ||
                        pc < 1 || priv > 0)
                        continue;
                    pl->nt = nt;
                    pl->variant = variant;
                    pl->ri = ri;
                    pl->team_lds = lds;
                    per_cu = pc;
                    found = true;
                }
                if (found) break;
            }
            if (!found)
                return bail(fail(SCOCG_E_UNSUPPORTED, "no team launch shape for this problem fits a compute unit "
                                                      "without private-memory spills (threads %d)", opt.threads));
            const int maxwg = cus * per_cu;
            if (G > maxwg) return bail(fail(SCOCG_E_UNSUPPORTED, "team larger than the resident workgroups"));
            int nteams = std::min(npanels, maxwg / G);
            if (opt.slots) nteams = std::min(nteams, std::max(1, opt.slots / G));
            if (nteams >= 8) nteams -= nteams % 8;   // whole teams on every XCD
            pl->slot_bytes = scocg::team_ws_bytes(W, nshift, pl->Mp, pl->nIp, !pl->gal);
            if (hipMemGetInfo(&freeb, &totb) == hipSuccess && freeb > 0) {
                const int64_t cap = (int64_t)(0.8 * (double)freeb) / std::max<int64_t>(1, pl->slot_bytes);
                if (cap < 1) return bail(fail(SCOCG_E_NOMEM, "one team's memory (%lld bytes) exceeds free memory",
                                              (long long)pl->slot_bytes));
                nteams = (int)std::min<int64_t>(nteams, cap);
            }
            pl->nteams = nteams;
            pl->slots = nteams * G;
            pl->pstride = (2 * W + 15) / 16 * 16;
            int rate_khz = 0;
            if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, P->device) != hipSuccess ||
                rate_khz <= 0)
                rate_khz = 100000;
            pl->spin_ticks = (int64_t)rate_khz * 1000 * 5;     // a wait is abandoned after 5 s
        }
    }

    std::vector<double> zz(2 * nshift);
    for (int k = 0; k < nshift; ++k) {
        zz[2 * k] = shifts[k].re;
        zz[2 * k + 1] = shifts[k].im;
    }
    std::vector<int32_t> order(nrhs);
    for (int32_t r = 0; r < nrhs; ++r) order[r] = (spec && spec->order) ? spec->order[r] : r;
    if ((st = dev_upload(&pl->dz, zz.data(), zz.size()))) return bail(st);
    if ((st = dev_upload(&pl->dsys, hm.sys.data(), hm.sys.size()))) return bail(st);
    if ((st = dev_upload(&pl->drhs, hm.rhs.data(), hm.rhs.size()))) return bail(st);
    if (pl->global) {
        pl->drowptr = P->dRowptr;
        pl->decol = P->dCol;
        pl->degid = P->dIota;
    } else {
        if ((st = dev_upload(&pl->drowptr, hm.rowptr.data(), hm.rowptr.size()))) return bail(st);
        if ((st = dev_upload(&pl->decol, hm.ecol.data(), hm.ecol.size()))) return bail(st);
        if ((st = dev_upload(&pl->degid, hm.egid.data(), hm.egid.size()))) return bail(st);
    }
    if ((st = dev_upload(&pl->doutl, hm.outl.data(), hm.outl.size()))) return bail(st);
    if ((st = dev_upload(&pl->doutoff, hm.outoff.data(), hm.outoff.size()))) return bail(st);
    {
        std::vector<double> hout;
        output_h(P, nrhs, rhs_index, spec, hm, hout);
        if ((st = dev_upload(&pl->dhout, hout.data(), hout.size()))) return bail(st);
    }
    if (!srow_h.empty()) {
        if ((st = dev_upload(&pl->dsrow, srow_h.data(), srow_h.size()))) return bail(st);
        if ((st = dev_upload(&pl->dscol, scol_h.data(), scol_h.size()))) return bail(st);
        if ((st = dev_upload(&pl->dsval, sval_h.data(), sval_h.size()))) return bail(st);
    }
    if (!ecol_ell.empty()) {
        if ((st = dev_upload(&pl->dsell_col, ecol_ell.data(), ecol_ell.size()))) return bail(st);
        if ((st = dev_upload(&pl->dsell_val, eval_ell.data(), eval_ell.size()))) return bail(st);
    }
    if ((st = dev_upload(&pl->dorder, order.data(), order.size()))) return bail(st);
    if (hipMalloc((void**)&pl->dqueue, sizeof(int32_t)) != hipSuccess) return bail(fail(SCOCG_E_NOMEM, "queue"));
    if (pl->team) {
        if (hipMalloc((void**)&pl->dctl, sizeof(int32_t) * 32 * (size_t)(pl->nteams + 1)) != hipSuccess ||
            hipMalloc((void**)&pl->dpart, sizeof(double) * 2 * (size_t)pl->G * pl->pstride * pl->nteams) != hipSuccess)
            return bail(fail(SCOCG_E_NOMEM, "team synchronisation buffers"));
    }
    if (nrhs > 0) {
        const int64_t units = pl->team ? pl->nteams : pl->slots;
        if (hipMalloc((void**)&pl->dws, (size_t)pl->slot_bytes * units) != hipSuccess)
            return bail(fail(SCOCG_E_NOMEM, "workspace of %lld bytes", (long long)pl->slot_bytes * units));
        if (hipMalloc((void**)&pl->dstats, sizeof(int64_t) * scocg::NSTAT * nrhs) != hipSuccess)
            return bail(fail(SCOCG_E_NOMEM, "stats"));
    }
    *out = pl;
    return SCOCG_OK;
}

extern "C" int64_t scocg_plan_out_count(const scocg_plan* pl) { return pl ? pl->out_count : -1; }

extern "C" scocg_status scocg_plan_info(const scocg_plan* pl, int64_t* info) {
    if (!pl || !info) return fail(SCOCG_E_ARG, "NULL argument");
    info[0] = pl->slots;
    info[1] = pl->nt;
    info[2] = pl->Mp;
    info[3] = pl->slot_bytes;
    info[4] = pl->seed0;
    info[5] = (int64_t)(pl->qmr ? scocg::qmr_lds_bytes(pl->K, pl->nt, pl->Mp, pl->dl)
                                : scocg::solver_lds_bytes(pl->K, pl->nt));
    info[6] = pl->prec;
    const bool dl = pl->team ? pl->team_dl : pl->dl;
    const bool unit = pl->team ? (pl->variant == 2 || pl->variant == 4) : (pl->unit && pl->dl);
    const bool mfma = pl->team && pl->P->bd == 4 && pl->W % 4 == 0;
    info[7] = (pl->global ? 1 : 0) | (pl->proj ? 2 : 0) | (pl->qmr ? 4 : 0) | (pl->gal ? 8 : 0) | (dl ? 16 : 0) |
              (unit ? 32 : 0) | (pl->team ? 64 : 0) | (mfma ? 128 : 0) |
              ((pl->team && pl->ri) || (!pl->team && unit && pl->reg) ? 256 : 0) |
              (unit && !pl->team && pl->ell_w ? 512 : 0);
    if (pl->team) info[5] = (int64_t)pl->team_lds;
    info[8] = pl->team ? pl->G : 1;
    info[9] = pl->team ? pl->W : 1;
    return SCOCG_OK;
}

extern "C" scocg_status scocg_plan_out_offsets(const scocg_plan* pl, int64_t* offsets) {
    if (!pl || !offsets) return fail(SCOCG_E_ARG, "NULL argument");
    std::memcpy(offsets, pl->out_off.data(), sizeof(int64_t) * pl->out_off.size());
    return SCOCG_OK;
}

static KParams make_kparams(const scocg_plan* pl, scocg_z* out, int32_t* iters, int8_t* status, double* resid) {
    const scocg_problem* P = pl->P;
    KParams k{};
    if (pl->prec == SCOCG_FP64) {
        k.Hv = P->dH;
        k.Sv = P->dS;
    } else if (pl->prec == SCOCG_FP32) {
        k.Hv = P->dH32;
        k.Sv = P->dS32;
    } else {
        k.Hv = P->dHbf;
        k.Sv = P->dSbf;
    }
    k.Hv64 = P->dH;
    k.Sv64 = P->dS;
    k.rowptr_l = pl->drowptr;
    k.ecol = pl->decol;
    k.egid = pl->degid;
    k.sys = pl->dsys;
    k.rhs = pl->drhs;
    k.out_local = pl->doutl;
    k.out_off = pl->doutoff;
    k.order = pl->dorder;
    k.z = pl->dz;
    k.nrhs = pl->nrhs;
    k.K = pl->K;
    k.seed0 = pl->seed0;
    k.maxiter = pl->opt.maxiter;
    k.tol = pl->opt.tol;
    k.inner_tol = pl->opt.inner_tol;
    k.inner_tol_lo = pl->opt.inner_tol_lo;
    k.inner_maxiter = pl->opt.inner_maxiter;
    k.replace_every = pl->opt.replace_every;
    k.audit = pl->opt.audit;
    k.s_unit_diag = P->s_unit_diag ? 1 : 0;
    k.ent_direct = pl->global ? 1 : 0;     // the global system's egid is dIota
    k.s_rowptr = pl->unit ? pl->dsrow : nullptr;
    k.s_ecol = pl->unit ? pl->dscol : nullptr;
    k.s_vals = pl->unit ? pl->dsval : nullptr;
    k.s_ell_col = pl->unit && pl->ell_w ? pl->dsell_col : nullptr;
    k.s_ell_val = pl->unit && pl->ell_w ? pl->dsell_val : nullptr;
    k.s_ell_w = pl->unit ? pl->ell_w : 0;
    k.queue = pl->dqueue;
    k.ws = pl->dws;
    k.slot_bytes = pl->slot_bytes;
    k.Mp = pl->Mp;
    k.nIp = pl->nIp;
    k.out = (double*)out;
    k.iters = iters;
    k.status = status;
    k.resid = resid;
    k.stats = pl->dstats;
    return k;
}

extern "C" scocg_status scocg_plan_run(scocg_plan* pl, void* stream, scocg_z* out, int32_t* iters,
                                       int8_t* status, double* resid) {
    if (!pl) return fail(SCOCG_E_ARG, "plan is NULL");
    if (!out && pl->out_count > 0) return fail(SCOCG_E_ARG, "out is NULL");
    if (pl->nrhs == 0) return SCOCG_OK;
    HIP_TRY(hipSetDevice(pl->P->device));
    hipStream_t st = (hipStream_t)stream;
    pl->last_stream = st;
    const scocg_problem* P = pl->P;
    KParams k = make_kparams(pl, out, iters, status, resid);
    (void)hipGetLastError();   // drop any error another caller left on this thread
    if (pl->team) {
        // queue, abort flag and every team's counters start at zero; the per-RHS counters too (the
        // teams add their shift updates into them)
        HIP_TRY(scocg::launch_fill_i32(pl->dctl, 0, 32 * (int64_t)(pl->nteams + 1), st));
        HIP_TRY(scocg::launch_fill_i32((int32_t*)pl->dstats, 0, 2 * (int64_t)scocg::NSTAT * pl->nrhs, st));
        scocg::TParams T{};
        T.k = k;
        T.k.queue = pl->dctl;
        T.G = pl->G;
        T.W = pl->W;
        T.nteams = pl->nteams;
        T.npanels = (pl->nrhs + pl->W - 1) / pl->W;
        T.pairs_max = pl->pairs_max;
        T.rows_max = pl->rows_max;
        T.team_bytes = pl->slot_bytes;
        T.vec_stride = pl->Mp * pl->W;
        T.tws = pl->dws;
        T.sync = pl->dctl + 32;
        T.part = pl->dpart;
        T.pstride = pl->pstride;
        T.abort_flag = pl->dctl + 1;
        T.spin_ticks = pl->spin_ticks;
        HIP_TRY(scocg::launch_team(T, P->bd, pl->gal, pl->variant, pl->ri, pl->nt, pl->slots, pl->team_lds, st));
        return SCOCG_OK;
    }
    HIP_TRY(scocg::launch_fill_i32(pl->dqueue, 0, 1, st));
    if (pl->qmr)
        HIP_TRY(scocg::launch_qmr(k, P->bd, !P->has_S, pl->gal, pl->dl, pl->unit && pl->dl ? (pl->reg ? 2 : 1) : 0,
                                  pl->nt, pl->slots, st));
    else HIP_TRY(scocg::launch_solver(k, P->bd, pl->proj ? 3 : pl->prec, !P->has_S, pl->nt, pl->slots, st));
    return SCOCG_OK;
}

extern "C" scocg_status scocg_plan_integrate(scocg_plan* pl, void* stream, const scocg_z* G, const double* weights,
                                             double mu, double kT, double* rho, double* ldos) {
    if (!pl || !G || !weights || !rho) return fail(SCOCG_E_ARG, "NULL argument");
    if (!std::isfinite(mu) || !std::isfinite(kT) || kT < 0.0) return fail(SCOCG_E_ARG, "mu must be finite, kT >= 0");
    if (pl->nrhs == 0) return SCOCG_OK;
    HIP_TRY(hipSetDevice(pl->P->device));
    hipStream_t st = (hipStream_t)stream;
    (void)hipGetLastError();
    HIP_TRY(scocg::launch_integrate((const double*)G, pl->dz, weights, pl->drhs, pl->doutoff, pl->doutl, pl->nrhs,
                                    pl->K, mu, kT, rho, ldos, st));
    return SCOCG_OK;
}

extern "C" scocg_status scocg_plan_cohp(scocg_plan* pl, void* stream, const double* rho, double* cohp) {
    if (!pl || !rho || !cohp) return fail(SCOCG_E_ARG, "NULL argument");
    if (pl->nrhs == 0) return SCOCG_OK;
    HIP_TRY(hipSetDevice(pl->P->device));
    (void)hipGetLastError();
    HIP_TRY(scocg::launch_cohp(pl->dhout, rho, cohp, pl->out_off[pl->nrhs], (hipStream_t)stream));
    return SCOCG_OK;
}

extern "C" scocg_status scocg_plan_stats(scocg_plan* pl, int64_t* stats) {
    if (!pl || !stats) return fail(SCOCG_E_ARG, "NULL argument");
    if (pl->nrhs == 0) return SCOCG_OK;
    HIP_TRY(hipSetDevice(pl->P->device));
    if (pl->last_stream) HIP_TRY(hipStreamSynchronize(pl->last_stream));
    else HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(stats, pl->dstats, sizeof(int64_t) * scocg::NSTAT * pl->nrhs, hipMemcpyDeviceToHost));
    if (pl->team) {
        int32_t ab = 0;
        HIP_TRY(hipMemcpy(&ab, pl->dctl + 1, sizeof(int32_t), hipMemcpyDeviceToHost));
        if (ab) return fail(SCOCG_E_DEVICE, "a wait between the workgroups of a team exceeded its bound; "
                                            "the run was abandoned (status ABORTED)");
    }
    return SCOCG_OK;
}

extern "C" scocg_status scocg_solve(scocg_problem* P, const scocg_options* opt, int32_t nshift,
                                    const scocg_z* shifts, int32_t nrhs, const int32_t* rhs_index,
                                    const scocg_rhs_spec* spec, scocg_z* out, int32_t* iters, int8_t* status,
                                    double* resid) {
    scocg_plan* pl = nullptr;
    scocg_status st = scocg_plan_create(P, opt, nshift, shifts, nrhs, rhs_index, spec, &pl);
    if (st < 0) return st;
    if (nrhs == 0) {
        scocg_plan_free(pl);
        return SCOCG_OK;
    }
    if (!out) {
        scocg_plan_free(pl);
        return fail(SCOCG_E_ARG, "out is NULL");
    }
    const size_t nk = (size_t)nrhs * nshift;
    scocg_z* dout = nullptr;
    int32_t* dit = nullptr;
    int8_t* dst = nullptr;
    double* dres = nullptr;
    auto cleanup = [&]() {
        dev_free(dout);
        dev_free(dit);
        dev_free(dst);
        dev_free(dres);
        scocg_plan_free(pl);
    };
    if (hipMalloc((void**)&dout, sizeof(scocg_z) * std::max<int64_t>(1, pl->out_count)) != hipSuccess ||
        hipMalloc((void**)&dit, sizeof(int32_t) * nk) != hipSuccess ||
        hipMalloc((void**)&dst, nk) != hipSuccess || hipMalloc((void**)&dres, sizeof(double) * nk) != hipSuccess) {
        cleanup();
        return fail(SCOCG_E_NOMEM, "output buffers");
    }
    st = scocg_plan_run(pl, nullptr, dout, dit, dst, dres);
    if (st == SCOCG_OK) {
        hipError_t e = hipDeviceSynchronize();
        if (e == hipSuccess) e = hipMemcpy(out, dout, sizeof(scocg_z) * pl->out_count, hipMemcpyDeviceToHost);
        std::vector<int8_t> hst(nk);
        if (e == hipSuccess) e = hipMemcpy(hst.data(), dst, nk, hipMemcpyDeviceToHost);
        if (e == hipSuccess && iters) e = hipMemcpy(iters, dit, sizeof(int32_t) * nk, hipMemcpyDeviceToHost);
        if (e == hipSuccess && resid) e = hipMemcpy(resid, dres, sizeof(double) * nk, hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
            cleanup();
            return fail(SCOCG_E_DEVICE, "solve: %s", hipGetErrorString(e));
        }
        if (status) std::memcpy(status, hst.data(), nk);
        for (size_t t = 0; t < nk; ++t)
            if (hst[t] != SCOCG_CONVERGED) { st = SCOCG_W_PARTIAL; break; }
    }
    cleanup();
    return st;
}

// ---------------------------------------------------------------------------
// device-buffer solve: plan_create + plan_run, the plan kept until scocg_sync
// ---------------------------------------------------------------------------
extern "C" scocg_status scocg_solve_device(scocg_problem* P, const scocg_options* opt, int32_t nshift,
                                           const scocg_z* shifts, int32_t nrhs, const int32_t* rhs_index,
                                           const scocg_rhs_spec* spec, scocg_z* out, int32_t* iters, int8_t* status,
                                           double* resid, void* stream) {
    if (!P) return fail(SCOCG_E_ARG, "problem is NULL");
    scocg_plan* pl = nullptr;
    scocg_status st = scocg_plan_create(P, opt, nshift, shifts, nrhs, rhs_index, spec, &pl);
    if (st < 0) return st;
    if (nrhs == 0) {
        scocg_plan_free(pl);
        return SCOCG_OK;
    }
    st = scocg_plan_run(pl, stream, out, iters, status, resid);
    if (st < 0) {
        const std::string msg = scocg_last_error();
        (void)hipStreamSynchronize((hipStream_t)stream);
        scocg_plan_free(pl);
        return fail(st, "%s", msg.c_str());
    }
    try {
        P->pending.push_back(scocg_problem::Pending{pl, (hipStream_t)stream, status, (int64_t)nrhs * nshift});
    } catch (...) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        scocg_plan_free(pl);
        return fail(SCOCG_E_NOMEM, "host allocation");
    }
    return SCOCG_OK;
}

// ---------------------------------------------------------------------------
// allocation-free device-buffer solve: the one-workgroup Lanczos-basis solver
// with every piece of per-call device memory taken from the library's fixed
// per-device array
// ---------------------------------------------------------------------------
extern "C" scocg_status scocg_solve_device_noalloc(scocg_problem* P, const scocg_options* opt_in, int32_t nshift,
                                                   const scocg_z* shifts, int32_t nrhs, const int32_t* rhs_index,
                                                   const scocg_rhs_spec* spec, scocg_z* out, int32_t* iters,
                                                   int8_t* status, double* resid, void* stream) {
    if (!P) return fail(SCOCG_E_ARG, "problem is NULL");
    scocg_options opt;
    if (opt_in) opt = *opt_in; else scocg_options_default(&opt);
    if (opt.method != SCOCG_METHOD_COCG_LANCZOS && opt.method != SCOCG_METHOD_QMR)
        return fail(SCOCG_E_UNSUPPORTED, "the allocation-free solve runs the Lanczos-basis methods");
    if (opt.precision != SCOCG_FP64) return fail(SCOCG_E_UNSUPPORTED, "the allocation-free solve runs in FP64");
    if (spec && spec->cluster_ptr) return fail(SCOCG_E_UNSUPPORTED, "the allocation-free solve needs the whole system");
    if (spec && spec->out_mode == SCOCG_OUT_FULL_X) return fail(SCOCG_E_UNSUPPORTED, "SELECTED_G output only");
    if (!(opt.tol > 0.0) || !(opt.inner_tol > 0.0) || opt.maxiter < 0 || opt.inner_maxiter < 0)
        return fail(SCOCG_E_ARG, "bad tolerance or iteration cap");
    if (nshift < 1 || nshift > 512) return fail(nshift < 1 ? SCOCG_E_ARG : SCOCG_E_UNSUPPORTED, "nshift must be in [1, 512]");
    if (!shifts) return fail(SCOCG_E_ARG, "shifts is NULL");
    for (int k = 0; k < nshift; ++k)
        if (!std::isfinite(shifts[k].re) || !std::isfinite(shifts[k].im)) return fail(SCOCG_E_ARG, "shift %d not finite", k);
    if (nrhs < 0 || (nrhs > 0 && !rhs_index)) return fail(SCOCG_E_ARG, "bad RHS list");
    if (nrhs == 0) return SCOCG_OK;
    if (!out) return fail(SCOCG_E_ARG, "out is NULL");
    if (!scocg::supported_bdim(P->bd)) return fail(SCOCG_E_UNSUPPORTED, "block size %d not compiled in", P->bd);
    if (spec && spec->order) {
        std::vector<char> seen(nrhs, 0);
        for (int32_t r = 0; r < nrhs; ++r) {
            const int32_t o = spec->order[r];
            if (o < 0 || o >= nrhs || seen[o]) return fail(SCOCG_E_ARG, "order is not a permutation");
            seen[o] = 1;
        }
    }
    HIP_TRY(hipSetDevice(P->device));
    void* base = nullptr;
    HIP_TRY(scocg::noalloc_scratch(P->device, &base));
    HostMaps hm;
    scocg_status st;
    try {
        st = build_maps(P, nrhs, rhs_index, spec, hm);
    } catch (const std::bad_alloc&) {
        return fail(SCOCG_E_NOMEM, "host allocation");
    }
    if (st != SCOCG_OK) return st;

    // launch shape: the one-workgroup Lanczos-basis kernel, CG direction in LDS when it fits, S as stored
    const bool gal = opt.method == SCOCG_METHOD_COCG_LANCZOS;
    const int64_t Mp = std::max<int64_t>(64, (hm.maxM + 63) / 64 * 64);
    int64_t maxout = 1;
    for (const auto& r : hm.rhs) maxout = std::max<int64_t>(maxout, r.nout);
    const int64_t nIp = (maxout + 63) / 64 * 64;
    int nt = 0;
    bool dl = false;
    for (int cand : {opt.threads ? opt.threads : 1024, 1024, 512, 256}) {
        if (cand != 256 && cand != 512 && cand != 1024) return fail(SCOCG_E_ARG, "threads must be 0, 256, 512 or 1024");
        const bool d = P->has_S && scocg::qmr_lds_bytes(nshift, cand, Mp, true) <= 160 * 1024;
        if (scocg::qmr_lds_bytes(nshift, cand, Mp, d) > 160 * 1024) continue;
        if (scocg::qmr_private_bytes(P->bd, !P->has_S, gal, d, false, cand) == 0) {
            nt = cand;
            dl = d;
            break;
        }
    }
    if (!nt) return fail(SCOCG_E_UNSUPPORTED, "no spill-free launch shape for this problem");
    const int64_t slot_bytes = scocg::qmr_slot_bytes(nshift, Mp, nIp);

    // the fixed array, carved: queue | shifts | RHS and system records | requested rows | row offsets |
    // queue order | per-RHS counters | workgroup slots (each carve 256-byte aligned)
    const size_t cap = scocg::NOALLOC_SCRATCH_BYTES;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = (off + bytes + 255) & ~(size_t)255;
        return at;
    };
    const size_t o_queue = take(sizeof(int32_t));
    const size_t o_z = take(sizeof(double) * 2 * nshift);
    const size_t o_rhs = take(sizeof(RhsInfo) * hm.rhs.size());
    const size_t o_sys = take(sizeof(SysInfo) * hm.sys.size());
    const size_t o_outl = take(sizeof(int32_t) * std::max<size_t>(1, hm.outl.size()));
    const size_t o_outoff = take(sizeof(int64_t) * hm.outoff.size());
    const size_t o_order = take(sizeof(int32_t) * nrhs);
    const size_t o_stats = take(sizeof(int64_t) * scocg::NSTAT * nrhs);
    const size_t o_ws = off;
    if (o_ws + (size_t)slot_bytes > cap)
        return fail(SCOCG_E_ARG, "the allocation-free solve needs %zu bytes of working memory for one workgroup; "
                                 "its fixed per-device array holds %zu", o_ws + (size_t)slot_bytes, cap);
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, P->device) != hipSuccess || cus <= 0) cus = 256;
    const size_t lds = scocg::qmr_lds_bytes(nshift, nt, Mp, dl);
    int per_cu = std::min(2, std::max(1, 2048 / nt));
    per_cu = std::min<int>(per_cu, (int)std::max<size_t>(1, (160 * 1024) / lds));
    int64_t slots = std::min<int64_t>({(int64_t)nrhs, (int64_t)cus * per_cu, (int64_t)((cap - o_ws) / slot_bytes)});
    if (opt.slots > 0) slots = std::min<int64_t>(slots, opt.slots);

    char* b = (char*)base;
    std::vector<double> zz(2 * (size_t)nshift);
    for (int k = 0; k < nshift; ++k) {
        zz[2 * k] = shifts[k].re;
        zz[2 * k + 1] = shifts[k].im;
    }
    std::vector<int32_t> order(nrhs);
    for (int32_t r = 0; r < nrhs; ++r) order[r] = (spec && spec->order) ? spec->order[r] : r;
    hipStream_t hs = (hipStream_t)stream;
    // the host arrays are copied before this call returns (the copies end before the solve is enqueued)
    HIP_TRY(hipMemcpyAsync(b + o_z, zz.data(), sizeof(double) * zz.size(), hipMemcpyHostToDevice, hs));
    HIP_TRY(hipMemcpyAsync(b + o_rhs, hm.rhs.data(), sizeof(RhsInfo) * hm.rhs.size(), hipMemcpyHostToDevice, hs));
    HIP_TRY(hipMemcpyAsync(b + o_sys, hm.sys.data(), sizeof(SysInfo) * hm.sys.size(), hipMemcpyHostToDevice, hs));
    if (!hm.outl.empty())
        HIP_TRY(hipMemcpyAsync(b + o_outl, hm.outl.data(), sizeof(int32_t) * hm.outl.size(), hipMemcpyHostToDevice, hs));
    HIP_TRY(hipMemcpyAsync(b + o_outoff, hm.outoff.data(), sizeof(int64_t) * hm.outoff.size(), hipMemcpyHostToDevice,
                           hs));
    HIP_TRY(hipMemcpyAsync(b + o_order, order.data(), sizeof(int32_t) * order.size(), hipMemcpyHostToDevice, hs));
    HIP_TRY(hipStreamSynchronize(hs));

    KParams k{};
    k.Hv = P->dH;
    k.Sv = P->dS;
    k.Hv64 = P->dH;
    k.Sv64 = P->dS;
    k.rowptr_l = P->dRowptr;
    k.ecol = P->dCol;
    k.egid = P->dIota;
    k.sys = (const SysInfo*)(b + o_sys);
    k.rhs = (const RhsInfo*)(b + o_rhs);
    k.out_local = (const int32_t*)(b + o_outl);
    k.out_off = (const int64_t*)(b + o_outoff);
    k.order = (const int32_t*)(b + o_order);
    k.z = (const double*)(b + o_z);
    k.nrhs = nrhs;
    k.K = nshift;
    k.maxiter = opt.maxiter;
    k.tol = opt.tol;
    k.inner_tol = opt.inner_tol;
    k.inner_tol_lo = opt.inner_tol_lo;
    k.inner_maxiter = opt.inner_maxiter;
    k.s_unit_diag = P->s_unit_diag ? 1 : 0;
    k.ent_direct = 1;
    k.queue = (int32_t*)(b + o_queue);
    k.ws = b + o_ws;
    k.slot_bytes = slot_bytes;
    k.Mp = Mp;
    k.nIp = nIp;
    k.out = (double*)out;
    k.iters = iters;
    k.status = status;
    k.resid = resid;
    k.stats = (int64_t*)(b + o_stats);
    (void)hipGetLastError();
    // the queue counter starts at zero (a fill kernel: the last call's value is still there)
    HIP_TRY(scocg::launch_fill_i32(k.queue, 0, 1, hs));
    HIP_TRY(scocg::launch_qmr(k, P->bd, !P->has_S, gal, dl, false, nt, (int)slots, hs));
    return SCOCG_OK;
}

extern "C" scocg_status scocg_sync(scocg_problem* P) {
    if (!P) return fail(SCOCG_E_ARG, "problem is NULL");
    if (P->pending.empty()) return SCOCG_OK;
    scocg_status res = SCOCG_OK;
    bool partial = false;
    std::string err;
    if (hipSetDevice(P->device) != hipSuccess) err = "hipSetDevice failed";
    std::vector<int8_t> h;
    for (const auto& q : P->pending) {
        hipError_t e = q.st ? hipStreamSynchronize(q.st) : hipDeviceSynchronize();
        if (e == hipSuccess && q.status && q.n > 0) {
            h.resize((size_t)q.n);
            e = hipMemcpy(h.data(), q.status, (size_t)q.n, hipMemcpyDeviceToHost);
            if (e == hipSuccess)
                for (int8_t v : h)
                    if (v != SCOCG_CONVERGED) { partial = true; break; }
        }
        if (e != hipSuccess && err.empty()) err = hipGetErrorString(e);
        scocg_plan_free(q.pl);
    }
    P->pending.clear();
    if (!err.empty()) return fail(SCOCG_E_DEVICE, "scocg_sync: %s", err.c_str());
    if (partial) res = SCOCG_W_PARTIAL;
    return res;
}

// ---------------------------------------------------------------------------
// graph capture / replay
// ---------------------------------------------------------------------------
extern "C" scocg_status scocg_plan_capture(scocg_plan* pl, void* stream, scocg_z* out, int32_t* iters,
                                           int8_t* status, double* resid) {
    if (!pl) return fail(SCOCG_E_ARG, "plan is NULL");
    if (!stream) return fail(SCOCG_E_ARG, "capture needs a non-default stream");
    HIP_TRY(hipSetDevice(pl->P->device));
    if (pl->gexec) { (void)hipGraphExecDestroy(pl->gexec); pl->gexec = nullptr; }
    if (pl->graph) { (void)hipGraphDestroy(pl->graph); pl->graph = nullptr; }
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    const scocg_status rs = scocg_plan_run(pl, stream, out, iters, status, resid);
    hipGraph_t g = nullptr;
    const hipError_t ee = hipStreamEndCapture(st, &g);
    if (rs != SCOCG_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rs;
    }
    if (ee != hipSuccess) return fail(SCOCG_E_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(ee));
    pl->graph = g;
    HIP_TRY(hipGraphInstantiate(&pl->gexec, pl->graph, nullptr, nullptr, 0));
    return SCOCG_OK;
}

extern "C" scocg_status scocg_plan_replay(scocg_plan* pl, void* stream) {
    if (!pl) return fail(SCOCG_E_ARG, "plan is NULL");
    if (!pl->gexec) return fail(SCOCG_E_ARG, "no captured graph: call scocg_plan_capture first");
    HIP_TRY(hipSetDevice(pl->P->device));
    pl->last_stream = (hipStream_t)stream;
    HIP_TRY(hipGraphLaunch(pl->gexec, (hipStream_t)stream));
    return SCOCG_OK;
}

// ---------------------------------------------------------------------------
// autotuner: workgroup size x resident workgroups per CU
// ---------------------------------------------------------------------------
extern "C" scocg_status scocg_autotune(scocg_problem* P, const scocg_options* opt_in, int32_t nshift,
                                       const scocg_z* shifts, int32_t nrhs, const int32_t* rhs_index,
                                       const scocg_rhs_spec* spec, int32_t probe_iters, int32_t* best_threads,
                                       int32_t* best_slots, double* best_seconds) {
    if (!P || !best_threads || !best_slots) return fail(SCOCG_E_ARG, "NULL argument");
    if (probe_iters <= 0) return fail(SCOCG_E_ARG, "probe_iters must be > 0");
    scocg_options opt;
    if (opt_in) opt = *opt_in; else scocg_options_default(&opt);
    HIP_TRY(hipSetDevice(P->device));
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, P->device) != hipSuccess || cus <= 0)
        cus = 256;
    hipStream_t st = nullptr;
    HIP_TRY(hipStreamCreate(&st));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    double best = 1e300;
    int bt = 0, bs = 0;
    scocg_status result = SCOCG_OK;
    const int threads_c[3] = {256, 512, 1024};
    for (int ti = 0; ti < 3 && result == SCOCG_OK; ++ti) {
        for (int per_cu = 1; per_cu <= 2 && result == SCOCG_OK; ++per_cu) {
            scocg_options o = opt;
            o.maxiter = probe_iters;
            o.team_size = -1;                  // this search is over the one-workgroup solver's launch
            o.threads = threads_c[ti];
            o.slots = std::max(1, std::min(nrhs, cus * per_cu));
            scocg_plan* pl = nullptr;
            scocg_status s2 = scocg_plan_create(P, &o, nshift, shifts, nrhs, rhs_index, spec, &pl);
            if (s2 < 0) { result = s2; break; }
            if (pl->slots != o.slots) { scocg_plan_free(pl); continue; }   // memory-capped duplicate
            const size_t nk = (size_t)std::max(1, nrhs) * nshift;
            scocg_z* dout = nullptr;
            if (hipMalloc((void**)&dout, sizeof(scocg_z) * std::max<int64_t>(1, pl->out_count)) != hipSuccess) {
                scocg_plan_free(pl);
                result = fail(SCOCG_E_NOMEM, "autotune output buffer");
                break;
            }
            (void)nk;
            float ms = 0.f;
            hipError_t he = hipSuccess;
            if ((s2 = scocg_plan_run(pl, st, dout, nullptr, nullptr, nullptr)) == SCOCG_OK &&   // warm-up
                (he = hipStreamSynchronize(st)) == hipSuccess &&
                (he = hipEventRecord(e0, st)) == hipSuccess &&
                (s2 = scocg_plan_run(pl, st, dout, nullptr, nullptr, nullptr)) == SCOCG_OK &&
                (he = hipEventRecord(e1, st)) == hipSuccess && (he = hipEventSynchronize(e1)) == hipSuccess &&
                (he = hipEventElapsedTime(&ms, e0, e1)) == hipSuccess) {
                if (ms < best) { best = ms; bt = pl->nt; bs = o.slots; }
            }
            dev_free(dout);
            scocg_plan_free(pl);
            if (s2 != SCOCG_OK) { result = s2; break; }
            if (he != hipSuccess) { result = fail(SCOCG_E_DEVICE, "autotune: %s", hipGetErrorString(he)); break; }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(st);
    if (result != SCOCG_OK) return result;
    *best_threads = bt;
    *best_slots = bs;
    if (best_seconds) *best_seconds = best / 1e3;
    return SCOCG_OK;
}

// ---------------------------------------------------------------------------
// autotuner of the team solver: panel width x workgroups per team x workgroup size
// ---------------------------------------------------------------------------
namespace {
// One timed probe of a plan (warm-up, then one run); ms < 0 if the plan could not be made.
scocg_status probe_plan(scocg_problem* P, const scocg_options& o, int32_t nshift, const scocg_z* shifts,
                        int32_t nrhs, const int32_t* rhs_index, const scocg_rhs_spec* spec, hipStream_t st,
                        hipEvent_t e0, hipEvent_t e1, float* ms, scocg_options* used) {
    *ms = -1.f;
    scocg_plan* pl = nullptr;
    scocg_status s2 = scocg_plan_create(P, &o, nshift, shifts, nrhs, rhs_index, spec, &pl);
    if (s2 == SCOCG_E_UNSUPPORTED || s2 == SCOCG_E_NOMEM) return SCOCG_OK;   // not a candidate here
    if (s2 < 0) return s2;
    scocg_z* dout = nullptr;
    if (hipMalloc((void**)&dout, sizeof(scocg_z) * std::max<int64_t>(1, pl->out_count)) != hipSuccess) {
        scocg_plan_free(pl);
        return fail(SCOCG_E_NOMEM, "autotune output buffer");
    }
    hipError_t he = hipSuccess;
    if ((s2 = scocg_plan_run(pl, st, dout, nullptr, nullptr, nullptr)) == SCOCG_OK &&
        (he = hipStreamSynchronize(st)) == hipSuccess && (he = hipEventRecord(e0, st)) == hipSuccess &&
        (s2 = scocg_plan_run(pl, st, dout, nullptr, nullptr, nullptr)) == SCOCG_OK &&
        (he = hipEventRecord(e1, st)) == hipSuccess && (he = hipEventSynchronize(e1)) == hipSuccess) {
        he = hipEventElapsedTime(ms, e0, e1);
    }
    *used = o;
    used->threads = pl->nt;
    used->slots = pl->slots;
    used->team_size = pl->team ? pl->G : -1;
    used->panel_width = pl->team ? pl->W : 1;
    if (pl->team) {
        int32_t ab = 0;
        if (he == hipSuccess) he = hipMemcpy(&ab, pl->dctl + 1, sizeof(int32_t), hipMemcpyDeviceToHost);
        if (ab) *ms = -1.f;     // an abandoned run is no candidate
    }
    dev_free(dout);
    scocg_plan_free(pl);
    if (s2 != SCOCG_OK) return s2;
    if (he != hipSuccess) return fail(SCOCG_E_DEVICE, "autotune: %s", hipGetErrorString(he));
    return SCOCG_OK;
}
}  // namespace

extern "C" scocg_status scocg_autotune_team(scocg_problem* P, const scocg_options* opt_in, int32_t nshift,
                                            const scocg_z* shifts, int32_t nrhs, const int32_t* rhs_index,
                                            const scocg_rhs_spec* spec, int32_t probe_iters, scocg_options* best,
                                            double* best_seconds) {
    if (!P || !best) return fail(SCOCG_E_ARG, "NULL argument");
    if (probe_iters <= 0) return fail(SCOCG_E_ARG, "probe_iters must be > 0");
    scocg_options opt;
    if (opt_in) opt = *opt_in; else scocg_options_default(&opt);
    if (opt.method != SCOCG_METHOD_QMR && opt.method != SCOCG_METHOD_COCG_LANCZOS)
        return fail(SCOCG_E_ARG, "the team solver runs the Lanczos-basis methods");
    HIP_TRY(hipSetDevice(P->device));
    const bool global = !(spec && spec->cluster_ptr);
    struct Cand { int W, G, nt; };
    std::vector<Cand> cands = {{1, -1, 1024}, {1, -1, 512}};
    if (global && P->bd == 4) {
        const Cand c4[] = {{8, 8, 1024}, {8, 8, 512}, {8, 16, 1024}, {4, 8, 512}, {4, 4, 512}, {8, 4, 1024}};
        cands.insert(cands.end(), std::begin(c4), std::end(c4));
    } else {
        const Cand c1[] = {{1, 2, 512}, {1, 4, 512}, {1, 8, 512}, {1, 4, 1024}, {1, 8, 1024}};
        cands.insert(cands.end(), std::begin(c1), std::end(c1));
    }
    hipStream_t st = nullptr;
    HIP_TRY(hipStreamCreate(&st));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    float bestms = 1e30f;
    scocg_status result = SCOCG_OK;
    bool found = false;
    for (const Cand& c : cands) {
        scocg_options o = opt;
        o.maxiter = probe_iters;
        o.panel_width = c.W;
        o.team_size = c.G;
        o.threads = c.nt;
        o.slots = 0;
        float ms = -1.f;
        scocg_options used;
        result = probe_plan(P, o, nshift, shifts, nrhs, rhs_index, spec, st, e0, e1, &ms, &used);
        if (result != SCOCG_OK) break;
        if (ms >= 0.f && ms < bestms) {
            bestms = ms;
            *best = used;
            best->maxiter = opt.maxiter;
            found = true;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(st);
    if (result != SCOCG_OK) return result;
    if (!found) return fail(SCOCG_E_UNSUPPORTED, "no launch shape fits this problem");
    if (best_seconds) *best_seconds = bestms / 1e3;
    return SCOCG_OK;
}

// ---------------------------------------------------------------------------
// learned RHS-cost predictor: features, MLP forward, training step
// ---------------------------------------------------------------------------
extern "C" int64_t scocg_mlp_nparams(void) { return scocg::NPARAM; }

extern "C" int64_t scocg_mlp_work_floats(void) {
    return (int64_t)scocg::GRAD_BLOCKS * 4 * (scocg::NPARAM + 1);
}

extern "C" scocg_status scocg_features(scocg_plan* pl, float* feats, void* stream) {
    if (!pl) return fail(SCOCG_E_ARG, "plan is NULL");
    if (pl->nrhs == 0) return SCOCG_OK;
    if (!feats) return fail(SCOCG_E_ARG, "feats is NULL");
    HIP_TRY(hipSetDevice(pl->P->device));
    const KParams k = make_kparams(pl, nullptr, nullptr, nullptr, nullptr);
    (void)hipGetLastError();
    HIP_TRY(scocg::launch_features(k, pl->P->bd, pl->P->has_S ? 1 : 0, feats, (hipStream_t)stream));
    return SCOCG_OK;
}

extern "C" scocg_status scocg_mlp_forward(const float* w, const float* x, int64_t n, float* y, void* stream) {
    if (n < 0) return fail(SCOCG_E_ARG, "n < 0");
    if (n == 0) return SCOCG_OK;
    if (!w || !x || !y) return fail(SCOCG_E_ARG, "NULL argument");
    (void)hipGetLastError();
    HIP_TRY(scocg::launch_mlp_forward(w, x, n, y, (hipStream_t)stream));
    return SCOCG_OK;
}

extern "C" scocg_status scocg_mlp_train_step(float* w, float* adam_m, float* adam_v, const float* x, const float* t,
                                             const int32_t* idx, int64_t m, float lr, int32_t step, float* loss,
                                             float* grad, float* work, void* stream) {
    if (!w || !x || !t || !work || m <= 0) return fail(SCOCG_E_ARG, "bad argument");
    if (lr > 0.f && (!adam_m || !adam_v || step < 1)) return fail(SCOCG_E_ARG, "Adam needs m, v and step >= 1");
    hipStream_t st = (hipStream_t)stream;
    const int64_t nparts = (int64_t)scocg::GRAD_BLOCKS * 4;
    float* partial = work;
    float* loss_part = work + nparts * scocg::NPARAM;
    (void)hipGetLastError();
    HIP_TRY(scocg::launch_mlp_grad(w, x, t, idx, m, partial, loss_part, scocg::GRAD_BLOCKS, st));
    HIP_TRY(scocg::launch_mlp_adam(w, adam_m, adam_v, partial, loss_part, nparts, m, lr, step, grad, loss, st));
    return SCOCG_OK;
}

// ---------------------------------------------------------------------------
// whole training run and prediction on host buffers
// ---------------------------------------------------------------------------
namespace {

// splitmix64: the initial weights and the batch order of scocg_mlp_train
struct Mix64 {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
    int64_t below(int64_t n) { return (int64_t)(uniform() * (double)n); }
};

void shuffle(std::vector<int32_t>& v, Mix64& r) {
    for (int64_t i = (int64_t)v.size() - 1; i > 0; --i) std::swap(v[i], v[r.below(i + 1)]);
}

struct DevBuf {
    void* p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
    bool alloc(size_t b) { return hipMalloc(&p, std::max<size_t>(b, 16)) == hipSuccess; }
    template <class T> T* as() const { return (T*)p; }
};

}  // namespace

extern "C" int64_t scocg_mlp_model_floats(void) { return scocg::NPARAM + 2 * scocg::NIN; }

extern "C" void scocg_mlp_cfg_default(scocg_mlp_cfg* cfg) {
    if (!cfg) return;
    cfg->epochs = 200;
    cfg->batch = 256;
    cfg->lr = 1e-3f;
    cfg->val_frac = 0.2f;
    cfg->seed = 0x14027285ull;
    cfg->init_weights = nullptr;
}

extern "C" scocg_status scocg_mlp_train(const float* feats, const float* log_iters, int64_t n,
                                        const scocg_mlp_cfg* cfg_in, float* model_out, double* val_loss) {
    using namespace scocg;
    if (!feats || !log_iters || !model_out || n < 2) return fail(SCOCG_E_ARG, "bad argument (n >= 2 needed)");
    scocg_mlp_cfg cfg;
    scocg_mlp_cfg_default(&cfg);
    if (cfg_in) cfg = *cfg_in;
    if (cfg.epochs < 1 || cfg.batch < 1 || !(cfg.lr > 0.f) || !(cfg.val_frac >= 0.f && cfg.val_frac < 1.f))
        return fail(SCOCG_E_ARG, "epochs, batch >= 1, lr > 0, 0 <= val_frac < 1");
    // z-score every feature (constant features keep sd = 1)
    std::vector<double> mu(NIN, 0.0), sd(NIN, 0.0);
    for (int64_t r = 0; r < n; ++r)
        for (int f = 0; f < NIN; ++f) mu[f] += feats[r * NIN + f];
    for (int f = 0; f < NIN; ++f) mu[f] /= (double)n;
    for (int64_t r = 0; r < n; ++r)
        for (int f = 0; f < NIN; ++f) {
            const double d = feats[r * NIN + f] - mu[f];
            sd[f] += d * d;
        }
    for (int f = 0; f < NIN; ++f) {
        sd[f] = std::sqrt(sd[f] / (double)n);
        if (!(sd[f] > 0.0)) sd[f] = 1.0;
    }
    std::vector<float> X((size_t)n * NIN), T((size_t)n);
    for (int64_t r = 0; r < n; ++r) {
        for (int f = 0; f < NIN; ++f) X[r * NIN + f] = (float)((feats[r * NIN + f] - mu[f]) / sd[f]);
        T[r] = log_iters[r];
        if (!std::isfinite(T[r])) return fail(SCOCG_E_ARG, "log_iters[%lld] is not finite", (long long)r);
    }
    Mix64 rng{cfg.seed};
    std::vector<float> w(NPARAM, 0.f);
    if (cfg.init_weights) {
        std::memcpy(w.data(), cfg.init_weights, sizeof(float) * NPARAM);
    } else {
        // Kaiming-uniform weights (bound sqrt(6 / fan_in)), zero biases
        auto fill = [&](int off, int cnt, int fan_in) {
            const double b = std::sqrt(6.0 / fan_in);
            for (int i = 0; i < cnt; ++i) w[off + i] = (float)((2.0 * rng.uniform() - 1.0) * b);
        };
        fill(OFF_W1, NH * NIN, NIN);
        fill(OFF_W2, NH * NH, NH);
        fill(OFF_W3, NH, NH);
    }
    std::vector<int32_t> perm((size_t)n);
    for (int64_t r = 0; r < n; ++r) perm[r] = (int32_t)r;
    shuffle(perm, rng);
    const int64_t nval = (int64_t)std::llround((double)cfg.val_frac * (double)n);
    if (n - nval < 1) return fail(SCOCG_E_ARG, "no training samples left after the validation split");
    std::vector<int32_t> val(perm.begin(), perm.begin() + nval), tr(perm.begin() + nval, perm.end());

    DevBuf dX, dT, dw, dm, dv, didx, dloss, dwork;
    const int64_t nwork = scocg_mlp_work_floats();
    if (!dX.alloc(sizeof(float) * X.size()) || !dT.alloc(sizeof(float) * T.size()) ||
        !dw.alloc(sizeof(float) * NPARAM) || !dm.alloc(sizeof(float) * NPARAM) || !dv.alloc(sizeof(float) * NPARAM) ||
        !didx.alloc(sizeof(int32_t) * (size_t)n) || !dloss.alloc(sizeof(float)) ||
        !dwork.alloc(sizeof(float) * (size_t)nwork))
        return fail(SCOCG_E_NOMEM, "training buffers");
    HIP_TRY(hipMemcpy(dX.p, X.data(), sizeof(float) * X.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(dT.p, T.data(), sizeof(float) * T.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(dw.p, w.data(), sizeof(float) * NPARAM, hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(dm.p, 0, sizeof(float) * NPARAM));
    HIP_TRY(hipMemset(dv.p, 0, sizeof(float) * NPARAM));
    std::vector<float> best = w;
    double best_loss = INFINITY;
    int32_t step = 0;
    const int64_t ntr = (int64_t)tr.size();
    for (int ep = 0; ep < cfg.epochs; ++ep) {
        shuffle(tr, rng);
        // the epoch's batch order goes up once; each step reads its slice
        HIP_TRY(hipMemcpy(didx.p, tr.data(), sizeof(int32_t) * (size_t)ntr, hipMemcpyHostToDevice));
        for (int64_t b0 = 0; b0 < ntr; b0 += cfg.batch) {
            const int64_t m = std::min<int64_t>(cfg.batch, ntr - b0);
            scocg_status st = scocg_mlp_train_step(dw.as<float>(), dm.as<float>(), dv.as<float>(), dX.as<float>(),
                                                   dT.as<float>(), didx.as<int32_t>() + b0, m, cfg.lr, ++step,
                                                   nullptr, nullptr, dwork.as<float>(), nullptr);
            if (st < 0) return st;
        }
        if (nval > 0) {
            HIP_TRY(hipMemcpy(didx.p, val.data(), sizeof(int32_t) * (size_t)nval, hipMemcpyHostToDevice));
            scocg_status st = scocg_mlp_train_step(dw.as<float>(), nullptr, nullptr, dX.as<float>(), dT.as<float>(),
                                                   didx.as<int32_t>(), nval, 0.f, 1, dloss.as<float>(), nullptr,
                                                   dwork.as<float>(), nullptr);
            if (st < 0) return st;
            float vl = 0.f;
            HIP_TRY(hipMemcpy(&vl, dloss.p, sizeof(float), hipMemcpyDeviceToHost));
            if (vl < best_loss) {
                best_loss = vl;
                HIP_TRY(hipMemcpy(best.data(), dw.p, sizeof(float) * NPARAM, hipMemcpyDeviceToHost));
            }
        }
    }
    if (nval == 0) HIP_TRY(hipMemcpy(best.data(), dw.p, sizeof(float) * NPARAM, hipMemcpyDeviceToHost));
    HIP_TRY(hipDeviceSynchronize());
    std::memcpy(model_out, best.data(), sizeof(float) * NPARAM);
    for (int f = 0; f < NIN; ++f) {
        model_out[NPARAM + f] = (float)mu[f];
        model_out[NPARAM + NIN + f] = (float)sd[f];
    }
    if (val_loss) *val_loss = nval > 0 ? best_loss : NAN;
    return SCOCG_OK;
}

extern "C" scocg_status scocg_mlp_predict(const float* model, const float* feats, int64_t n, float* pred) {
    using namespace scocg;
    if (n < 0) return fail(SCOCG_E_ARG, "n < 0");
    if (n == 0) return SCOCG_OK;
    if (!model || !feats || !pred) return fail(SCOCG_E_ARG, "NULL argument");
    const float* mu = model + NPARAM;
    const float* sd = model + NPARAM + NIN;
    for (int f = 0; f < NIN; ++f)
        if (!(sd[f] > 0.f)) return fail(SCOCG_E_ARG, "model: feature %d has sd <= 0", f);
    std::vector<float> X((size_t)n * NIN);
    for (int64_t r = 0; r < n; ++r)
        for (int f = 0; f < NIN; ++f) X[r * NIN + f] = (feats[r * NIN + f] - mu[f]) / sd[f];
    DevBuf dX, dw, dy;
    if (!dX.alloc(sizeof(float) * X.size()) || !dw.alloc(sizeof(float) * NPARAM) || !dy.alloc(sizeof(float) * n))
        return fail(SCOCG_E_NOMEM, "prediction buffers");
    HIP_TRY(hipMemcpy(dX.p, X.data(), sizeof(float) * X.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(dw.p, model, sizeof(float) * NPARAM, hipMemcpyHostToDevice));
    scocg_status st = scocg_mlp_forward(dw.as<float>(), dX.as<float>(), n, dy.as<float>(), nullptr);
    if (st < 0) return st;
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(pred, dy.p, sizeof(float) * n, hipMemcpyDeviceToHost));
    return SCOCG_OK;
}

// ---------------------------------------------------------------------------
// work-queue order of a plan: set directly, or scheduled from predicted costs
// ---------------------------------------------------------------------------
extern "C" scocg_status scocg_plan_set_order(scocg_plan* pl, const int32_t* order) {
    if (!pl) return fail(SCOCG_E_ARG, "plan is NULL");
    const int32_t nrhs = pl->nrhs;
    if (nrhs == 0) return SCOCG_OK;
    std::vector<int32_t> o(nrhs);
    if (order) {
        std::vector<char> seen(nrhs, 0);
        for (int32_t r = 0; r < nrhs; ++r) {
            if (order[r] < 0 || order[r] >= nrhs || seen[order[r]]) return fail(SCOCG_E_ARG, "order is not a permutation");
            seen[order[r]] = 1;
            o[r] = order[r];
        }
    } else {
        for (int32_t r = 0; r < nrhs; ++r) o[r] = r;
    }
    HIP_TRY(hipSetDevice(pl->P->device));
    HIP_TRY(hipDeviceSynchronize());   // no launch of this plan may still read the old order
    HIP_TRY(hipMemcpy(pl->dorder, o.data(), sizeof(int32_t) * (size_t)nrhs, hipMemcpyHostToDevice));
    return SCOCG_OK;
}

extern "C" scocg_status scocg_schedule(scocg_plan* pl, const float* model, int32_t* order_out, float* cost_out) {
    using namespace scocg;
    if (!pl) return fail(SCOCG_E_ARG, "plan is NULL");
    const int32_t nrhs = pl->nrhs;
    if (nrhs == 0) return SCOCG_OK;
    HIP_TRY(hipSetDevice(pl->P->device));
    DevBuf df;
    if (!df.alloc(sizeof(float) * (size_t)nrhs * NIN)) return fail(SCOCG_E_NOMEM, "feature buffer");
    scocg_status st = scocg_features(pl, df.as<float>(), nullptr);
    if (st < 0) return st;
    HIP_TRY(hipDeviceSynchronize());
    std::vector<float> F((size_t)nrhs * NIN), pred(nrhs, 0.f);
    HIP_TRY(hipMemcpy(F.data(), df.p, sizeof(float) * F.size(), hipMemcpyDeviceToHost));
    if (model && (st = scocg_mlp_predict(model, F.data(), nrhs, pred.data())) < 0) return st;
    // cost = predicted outer iterations x block entries of the local pattern (features 0 and 1)
    std::vector<double> cost(nrhs);
    for (int32_t r = 0; r < nrhs; ++r) {
        const double ent = (double)F[(size_t)r * NIN + 0] * (double)F[(size_t)r * NIN + 1];
        cost[r] = (model ? std::exp((double)pred[r]) : 1.0) * ent;
        if (!std::isfinite(cost[r])) return fail(SCOCG_E_ARG, "predicted cost of RHS %d is not finite", r);
    }
    std::vector<int32_t> o(nrhs);
    for (int32_t r = 0; r < nrhs; ++r) o[r] = r;
    std::stable_sort(o.begin(), o.end(), [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
    if ((st = scocg_plan_set_order(pl, o.data())) < 0) return st;
    if (order_out) std::memcpy(order_out, o.data(), sizeof(int32_t) * (size_t)nrhs);
    if (cost_out)
        for (int32_t r = 0; r < nrhs; ++r) cost_out[r] = (float)cost[r];
    return SCOCG_OK;
}
