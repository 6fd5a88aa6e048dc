// Host side of the C ABI declared in include/ecount.h: argument validation,
// workspace carving and the launch sequence of the estimator (Algorithm 2
// over a block of probes and shifts, Algorithm 1 inside).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <complex>
#include <mutex>
#include <string>
#include <vector>

#include "ecount.h"
#include "ecount_internal.h"

namespace ecnt {

// ------------------------------------------------------------------ profiling
enum Family { F_CHEB = 0, F_CSR, F_DOTS, F_UPDATE, F_SETUP, F_FIN, F_QUAD, F_BDOTS, F_BUPD,
              F_VGRAD, F_CHEB2, F_LDL, F_LDLE, F_BKDOTS, F_BKUPD, F_BKNORM, F_BKQUAD,
              F_STA, F_FUSED, F_COUNT };
static const char *kFamilyName[F_COUNT] = {"op_cheb_sweep", "op_csr", "lz_dots", "lz_update",
                                           "lz_setup", "lz_finalize", "quadrature", "bw_dots",
                                           "bw_update", "bw_vgrad", "op_cheb_quad",
                                           "op_ldl_solve", "op_ldl_elementwise", "blk_dots",
                                           "blk_update", "blk_normalize", "blk_quadrature",
                                           "op_a_stencil", "lz_fused"};
static std::mutex g_prof_mu;
static bool g_prof_on = false;
static ecnt_kernel_stat g_stats[F_COUNT];
struct PendingEvent {
    int fam;
    hipEvent_t a, b;
    double bytes;
    int gate;   // 0: always runs; 1: runs only in the stencil form of A; 2: only in the CSR form
};
static thread_local std::vector<PendingEvent> t_pending;
static thread_local std::vector<hipEvent_t> t_event_pool;
static thread_local bool t_prof = false;

static hipEvent_t get_event()
{
    if (!t_event_pool.empty()) {
        hipEvent_t e = t_event_pool.back();
        t_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

struct Timed {
    int fam;
    double bytes;
    hipStream_t st;
    int gate;
    hipEvent_t a = nullptr;
    Timed(int f, double b, hipStream_t s, int g = 0) : fam(f), bytes(b), st(s), gate(g)
    {
        if (t_prof && (a = get_event())) (void)hipEventRecord(a, st);
    }
    ~Timed()
    {
        if (!a) return;
        hipEvent_t b = get_event();
        if (!b) return;
        (void)hipEventRecord(b, st);
        t_pending.push_back({fam, a, b, bytes, gate});
    }
};

// stencil_form: whether the stencil form applied A in the run (flags[2] == 0);
// a gated launch that returned at once is counted with no bytes
static void collect_profile(bool stencil_form = false)
{
    if (t_pending.empty()) return;
    std::lock_guard<std::mutex> g(g_prof_mu);
    for (auto &pe : t_pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, pe.a, pe.b) == hipSuccess) {
            const bool idle = (pe.gate == 1 && !stencil_form) || (pe.gate == 2 && stencil_form);
            g_stats[pe.fam].launches += 1;
            g_stats[pe.fam].total_ms += ms;
            g_stats[pe.fam].bytes += idle ? 0.0 : pe.bytes;
        }
        t_event_pool.push_back(pe.a);
        t_event_pool.push_back(pe.b);
    }
    t_pending.clear();
}

static thread_local std::string g_err;

static ecnt_status fail(ecnt_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

int32_t set_error(int32_t st, const char *msg)
{
    g_err = msg;
    return st;
}

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

static void col_geometry(Plan &p);

size_t plan_layout(Plan &p, char *base)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        off = align_up(off, 256);
        char *ptr = base ? base + off : nullptr;
        off += bytes;
        return ptr;
    };
    const size_t bv = p.vec_f32 ? 4 : 8;
    const size_t blk = (size_t)p.n * p.wave_cols * bv;
    const size_t NC = (size_t)p.nseg * p.wave_cols;   // virtual columns of one wave
    const size_t NCt = (size_t)p.nseg * p.Ct;         // of the whole run
    const bool pow2 = blk != 0 && (blk & (blk - 1)) == 0;
    p.slot_pad = pow2 ? kSlotPadBytes / bv : 0;
    const size_t slot = blk + p.slot_pad * bv;   // slot stride of the widest wave
    p.basis = take(slot * (p.k + 1));
    const int ntmp = p.prec_kind == ECNT_PREC_CHEB_LAPLACIAN ? 3 : (p.prec_kind == ECNT_PREC_LDL ? 2 : 0);
    for (int t = 0; t < 3; ++t) p.tmp[t] = t < ntmp ? take(blk) : nullptr;
    p.part = (double *)take(sizeof(double) * (size_t)p.nchunk * kPartRows * p.wave_cols);
    p.sig = (double *)take(sizeof(double) * (p.k + 1) * NC);
    p.alpha = (double *)take(sizeof(double) * p.k * NC);
    p.beta = (double *)take(sizeof(double) * (p.k + 1) * NC);
    p.cf = (double *)take(sizeof(double) * (p.k + 1) * NC);
    p.kappa = (double *)take(sizeof(double) * NC);
    p.runmax = (double *)take(sizeof(double) * NC);
    p.nu = (double *)take(sizeof(double) * NC);
    p.s_out = (double *)take(sizeof(double) * NCt);
    p.minabs = (double *)take(sizeof(double) * NCt);
    p.jac = (double *)take(p.prec_kind == ECNT_PREC_JACOBI ? sizeof(double) * p.S * p.n : 0);
    p.st_diag = (double *)take(p.stencil_a ? sizeof(double) * p.n : 0);
    p.st_coff = (double *)take(p.stencil_a ? sizeof(double) : 0);
    p.e_blk = (double *)take(p.prec_kind == ECNT_PREC_LDL ? sizeof(double) * 2 * p.S * p.n : 0);
    p.band = (double *)take(p.prec_kind == ECNT_PREC_LDL ? ldl_band_bytes(p.n, p.S) : 0);
    p.result = (double *)take(sizeof(double) * kResStride * p.nseg);
    p.active = (int32_t *)take(sizeof(int32_t) * NC);
    p.kused = (int32_t *)take(sizeof(int32_t) * NCt);
    p.flags = (int32_t *)take(sizeof(int32_t) * 4);
    p.seg_row = (int64_t *)take(sizeof(int64_t) * (p.nseg + 1));
    p.seg_chunk = (int64_t *)take(sizeof(int64_t) * (p.nseg + 1));
    p.seg_tile = (int64_t *)take(sizeof(int64_t) * (p.nseg + 1));
    p.seg_dims = (int32_t *)take(sizeof(int32_t) * 3 * p.nseg);
    p.seg_taus = (double *)take(sizeof(double) * p.S * p.nseg);
    if (p.arnoldi) {
        const size_t k = p.k;
        p.H = (double *)take(sizeof(double) * k * (k + 1) * NC);
    }
    if (p.block) {
        // row chunks of the block reductions: about 2048 workgroups of 4
        // wavefronts, 16-row tiles
        p.nblk = p.wave_cols / kBlk;
        const int64_t tiles = (p.n + 15) / 16;
        int64_t nch = (2048 + p.nblk - 1) / p.nblk;
        if (nch > tiles) nch = tiles;
        if (nch < 1) nch = 1;
        p.bk_rpc = ((p.n + nch - 1) / nch + 15) / 16 * 16;
        p.bk_nchunk = (int)((p.n + p.bk_rpc - 1) / p.bk_rpc);
        const size_t mat = sizeof(double) * 256 * (size_t)p.nblk;
        p.bk_part = (double *)take(mat * (size_t)p.bk_nchunk * kBlkChunk);
        p.bk_S = (double *)take(mat * (p.k + 1));
        p.bk_K = (double *)take(mat * p.k);
        p.bk_A = (double *)take(mat * p.k);
        p.bk_B = (double *)take(mat * (p.k + 1));
        p.bk_R0 = (double *)take(mat);
        p.bk_R1 = (double *)take(mat);
        p.bk_T = (double *)take(mat);
        p.bk_rm = (double *)take(sizeof(double) * p.nblk);
        p.bk_act = (int32_t *)take(sizeof(int32_t) * p.nblk);
    }
    if (p.grad) {
        const size_t k = p.k, C = p.wave_cols;
        p.g_tslots = take(slot * k);
        p.g_qbar = (double *)take(slot * k);
        p.g_ybar = (double *)take(blk);
        p.g_tbar = (double *)take(blk);
        p.g_gall = (double *)take(sizeof(double) * k * k * C);
        p.g_pall = (double *)take(sizeof(double) * k * k * C);
        p.g_Z = (double *)take(sizeof(double) * k * k * C);
        p.g_theta = (double *)take(sizeof(double) * k * C);
        p.g_sval = (double *)take(sizeof(double) * k * C);
        p.g_abar = (double *)take(sizeof(double) * k * C);
        p.g_bbar = (double *)take(sizeof(double) * (k + 1) * C);
        p.g_coef = (double *)take(sizeof(double) * 4 * 32 * C);
        p.g_scal = (double *)take(sizeof(double) * 5 * C);
        p.g_vpart = (double *)take(sizeof(double) * ((C + 63) / 64) * (size_t)p.n);
        p.g_taubar = (double *)take(sizeof(double) * C);
        p.g_sums = (double *)take(sizeof(double) * 64 * C);
    }
    p.bytes = align_up(off, 256) + 256;   // slack for aligning the caller's pointer
    return p.bytes;
}

// Column geometry of a wave of width p.C.
static void col_geometry(Plan &p)
{
    // columns per lane: 16-byte accesses where the column count allows it
    if (p.vec_f32) p.vw = (p.C % 4 == 0) ? 4 : (p.C % 2 == 0 ? 2 : 1);
    else p.vw = (p.C % 2 == 0) ? 2 : 1;
    if (p.req_vw > 0 && p.req_vw <= p.vw && p.C % p.req_vw == 0) p.vw = p.req_vw;
    p.nct = (p.C + kColTile - 1) / kColTile;
}

// Row geometry (once per run): rows per reduction chunk, chunk and stencil
// line-block offsets of every segment.  `sh.row` and `sh.dims` must be set.
static void row_geometry(Plan &p, SegHost &sh)
{
    // reductions: one wavefront per (row chunk, tile of 64 lanes); about 2048 of them
    const int vwr = (p.vec_f32 && p.wave_cols % 2 == 0) ? 2 : 1;
    const int nctr = (p.wave_cols + 64 * vwr - 1) / (64 * vwr);
    const int waves = p.req_red_waves > 0 ? p.req_red_waves : 2048;
    int64_t target = (waves + nctr - 1) / nctr;
    const int64_t maxchunks = (p.n + 15) / 16;
    if (target > maxchunks) target = maxchunks;
    if (target < 1) target = 1;
    p.rpc = (p.n + target - 1) / target;
    sh.chunk.assign(p.nseg + 1, 0);
    sh.tile.assign(p.nseg + 1, 0);
    bool thin = false;
    for (int b = 0; b < p.nseg; ++b) thin = thin || sh.dims[3 * b] < 4;
    // 8 x 8 workgroup blocks serve the fused quadratic sweep only: every factor
    // of the preconditioner must be quadratic
    bool all_quad = p.prec_kind == ECNT_PREC_CHEB_LAPLACIAN && p.product && p.nfac > 0;
    for (int f = 0; f < p.nfac; ++f) all_quad = all_quad && p.fac_quad[f];
    int shape = p.req_tile > 0 ? p.req_tile : (thin ? 3 : (all_quad ? 5 : 1));
    if (shape == 5 && !all_quad) shape = 1;
    p.tx = (shape == 1 || shape == 4) ? 4 : (shape == 2 ? 2 : (shape == 5 ? 8 : 1));
    p.ty = (shape == 3 || shape == 5) ? 8 : 4;
    p.no_fuse = shape == 4 ? 1 : 0;
    for (int b = 0; b < p.nseg; ++b) {
        const int64_t nb = sh.row[b + 1] - sh.row[b];
        sh.chunk[b + 1] = sh.chunk[b] + (nb + p.rpc - 1) / p.rpc;
        const int64_t tiles = (int64_t)((sh.dims[3 * b] + p.tx - 1) / p.tx) *
                              ((sh.dims[3 * b + 1] + p.ty - 1) / p.ty);
        sh.tile[b + 1] = sh.tile[b] + tiles;
    }
    p.nchunk = (int)sh.chunk[p.nseg];
    p.ntiles = sh.tile[p.nseg];
    p.max_d2 = 1;
    for (int b = 0; b < p.nseg; ++b) p.max_d2 = sh.dims[3 * b + 2] > p.max_d2 ? sh.dims[3 * b + 2] : p.max_d2;
    p.max_rows = 0;
    for (int b = 0; b < p.nseg; ++b)
        p.max_rows = sh.row[b + 1] - sh.row[b] > p.max_rows ? sh.row[b + 1] - sh.row[b] : p.max_rows;
}

// ---- product form of the preconditioner polynomial ----
// p(t) = sum_j c_j T_j(t) and p'(t) by Clenshaw's recurrence (complex t).
static std::complex<double> cheb_eval(const double *c, int d, std::complex<double> t,
                                      std::complex<double> *dp)
{
    std::complex<double> b1 = 0, b2 = 0, d1 = 0, d2 = 0;
    for (int j = d; j >= 1; --j) {
        std::complex<double> b = c[j] + 2.0 * t * b1 - b2;
        std::complex<double> db = 2.0 * b1 + 2.0 * t * d1 - d2;
        b2 = b1;
        b1 = b;
        d2 = d1;
        d1 = db;
    }
    if (dp) *dp = b1 + t * d1 - d2;
    return c[0] + t * b1 - b2;
}

// Roots by the Aberth-Ehrlich simultaneous iteration, paired into real
// linear / quadratic factors; accepted only if lead * prod (t - r) reproduces
// p on [-1, 1] to 1e-12 relative.  Returns false otherwise (Clenshaw is used).
static bool factorize(Plan &p)
{
    const int d = p.degree;
    if (d < 2 || d > 16 || p.coef[d] == 0.0) return false;
    typedef std::complex<double> cd;
    cd z[16];
    for (int i = 0; i < d; ++i) z[i] = std::polar(1.3, 2.0 * M_PI * (i + 0.25) / d);
    for (int it = 0; it < 500; ++it) {
        double maxstep = 0.0;
        for (int i = 0; i < d; ++i) {
            cd dp;
            const cd pv = cheb_eval(p.coef, d, z[i], &dp);
            if (std::abs(pv) == 0.0) continue;
            const cd ratio = pv / dp;
            cd sum = 0;
            for (int j = 0; j < d; ++j)
                if (j != i) sum += 1.0 / (z[i] - z[j]);
            const cd step = ratio / (1.0 - ratio * sum);
            z[i] -= step;
            maxstep = fmax(maxstep, std::abs(step) / fmax(1.0, std::abs(z[i])));
        }
        if (maxstep < 1e-15) break;
    }
    bool used[16] = {false};
    int nf = 0;
    for (int i = 0; i < d; ++i) {
        if (used[i]) continue;
        used[i] = true;
        if (fabs(z[i].imag()) <= 1e-10 * fmax(1.0, std::abs(z[i]))) {
            p.fac_quad[nf] = 0;
            p.fac_a[nf] = z[i].real();
            p.fac_b[nf] = 0.0;
            ++nf;
            continue;
        }
        int best = -1;
        double bd = 1e300;
        for (int j = 0; j < d; ++j) {
            if (used[j]) continue;
            const double dd = std::abs(z[j] - std::conj(z[i]));
            if (dd < bd) {
                bd = dd;
                best = j;
            }
        }
        if (best < 0 || bd > 1e-8 * fmax(1.0, std::abs(z[i]))) return false;
        used[best] = true;
        const cd r = 0.5 * (z[i] + std::conj(z[best]));
        p.fac_quad[nf] = 1;
        p.fac_a[nf] = r.real();
        p.fac_b[nf] = std::norm(r);
        ++nf;
    }
    p.nfac = nf;
    p.lead = p.coef[d] * ldexp(1.0, d - 1);
    // validate on Chebyshev points of [-1, 1]
    double maxp = 0.0, maxerr = 0.0;
    for (int k = 0; k < 4 * d + 1; ++k) {
        const double t = cos(M_PI * (k + 0.5) / (4 * d + 1));
        const double pv = cheb_eval(p.coef, d, cd(t, 0.0), nullptr).real();
        double q = p.lead;
        for (int f = 0; f < nf; ++f)
            q *= p.fac_quad[f] ? (t * t - 2.0 * p.fac_a[f] * t + p.fac_b[f]) : (t - p.fac_a[f]);
        maxp = fmax(maxp, fabs(pv));
        maxerr = fmax(maxerr, fabs(q - pv));
    }
    return maxerr <= 1e-12 * maxp;
}

static ecnt_status make_plan(Plan &p, int64_t n, int64_t m, int S, const ecnt_prec *T,
                             const ecnt_opts *o)
{
    if (!T || !o) return fail(ECNT_EINVAL, "null preconditioner or options");
    if (n < 1) return fail(ECNT_EINVAL, "n must be >= 1 (got %lld)", (long long)n);
    if (n > INT32_MAX) return fail(ECNT_EUNSUPPORTED, "n above 2^31-1 is not supported");
    if (m < 1) return fail(ECNT_EINVAL, "m must be >= 1 (got %lld)", (long long)m);
    if (S < 1 || S > kMaxShifts) return fail(ECNT_EINVAL, "nshift must be in 1..%d", kMaxShifts);
    if ((int64_t)m * S > (1 << 24)) return fail(ECNT_EUNSUPPORTED, "too many probe columns");
    if (o->k < 1 || o->k > n) return fail(ECNT_EINVAL, "k must satisfy 1 <= k <= n (got %d)", o->k);
    if (o->vec_type != ECNT_F64 && o->vec_type != ECNT_F32)
        return fail(ECNT_EINVAL, "vec_type must be ECNT_F64 or ECNT_F32");
    if (o->rule != ECNT_RULE_GAUSS && o->rule != ECNT_RULE_GA)
        return fail(ECNT_EINVAL, "unknown quadrature rule %d", o->rule);
    if (o->max_cols < 0) return fail(ECNT_EINVAL, "opts.max_cols must be >= 0");
    if (!(o->smooth_w >= 0.0) || !isfinite(o->smooth_w))
        return fail(ECNT_EINVAL, "smooth_w must be finite and >= 0");
    if (o->tile < 0 || o->tile > 5) return fail(ECNT_EINVAL, "opts.tile must be 0..5");
    if (o->red_waves != 0 && (o->red_waves < 64 || o->red_waves > 65536))
        return fail(ECNT_EINVAL, "opts.red_waves must be 0 or 64..65536");
    if (o->csr_vw != 0 && o->csr_vw != 1 && o->csr_vw != 2 && o->csr_vw != 4)
        return fail(ECNT_EINVAL, "opts.csr_vw must be 0, 1, 2 or 4");
    if (o->a_form != 0 && o->a_form != 1) return fail(ECNT_EINVAL, "opts.a_form must be 0 or 1");
    if (o->fused != 0 && o->fused != 1) return fail(ECNT_EINVAL, "opts.fused must be 0 or 1");
    const int kmax = o->rule == ECNT_RULE_GA ? kMaxK / 2 : kMaxK;
    if (o->k > kmax) return fail(ECNT_EUNSUPPORTED, "k above %d is not supported", kmax);
    p.n = n;
    p.m = (int)m;
    p.S = S;
    p.Ct = (int)(m * S);
    p.wave_cols = (o->max_cols > 0 && o->max_cols < p.Ct) ? o->max_cols : p.Ct;
    p.C = p.wave_cols;
    p.k = o->k;
    p.vec_f32 = o->vec_type == ECNT_F32;
    p.rule = o->rule;
    p.smooth_w = o->smooth_w;
    p.req_tile = o->tile;
    p.req_red_waves = o->red_waves;
    p.req_vw = o->csr_vw;
    p.prec_kind = T->kind;
    switch (T->kind) {
    case ECNT_PREC_NONE:
    case ECNT_PREC_JACOBI:
        break;
    case ECNT_PREC_CHEB_LAPLACIAN: {
        if (T->ndim < 1 || T->ndim > 3) return fail(ECNT_EINVAL, "prec.ndim must be 1..3");
        int64_t prod = 1;
        int d[3] = {1, 1, 1};
        for (int a = 0; a < T->ndim; ++a) {
            if (T->dims[a] < 1) return fail(ECNT_EINVAL, "prec.dims must be >= 1");
            prod *= T->dims[a];
            d[3 - T->ndim + a] = T->dims[a];
        }
        if (prod != n) return fail(ECNT_EINVAL, "prec grid (%lld points) does not match n", (long long)prod);
        if (T->degree < 0 || T->degree > 16) return fail(ECNT_EINVAL, "prec.degree must be 0..16");
        if (T->eval != ECNT_EVAL_AUTO && T->eval != ECNT_EVAL_CLENSHAW)
            return fail(ECNT_EINVAL, "prec.eval must be ECNT_EVAL_AUTO or ECNT_EVAL_CLENSHAW");
        if (!T->coef) return fail(ECNT_EINVAL, "prec.coef is null");
        if (!isfinite(T->s) || !isfinite(T->lo) || !isfinite(T->hi) || !(T->hi > T->lo))
            return fail(ECNT_EINVAL, "prec interval must be finite with hi > lo");
        for (int j = 0; j <= T->degree; ++j) {
            if (!isfinite(T->coef[j])) return fail(ECNT_EINVAL, "prec.coef[%d] is not finite", j);
            p.coef[j] = T->coef[j];
        }
        p.ndim = T->ndim;
        p.dims[0] = d[0];
        p.dims[1] = d[1];
        p.dims[2] = d[2];
        p.degree = T->degree;
        p.s = T->s;
        p.lo = T->lo;
        p.hi = T->hi;
        break;
    }
    case ECNT_PREC_LDL: {
        if (!T->ldl) return fail(ECNT_EINVAL, "prec.ldl is null (one factor per shift)");
        for (int s = 0; s < S; ++s) {
            const ecnt_ldl_factor &f = T->ldl[s];
            if (!f.perm || !f.l_row_ptr || !f.d_diag || !f.d_off)
                return fail(ECNT_EINVAL, "factor %d: null array", s);
            if (f.nnz < 0 || f.nnz >= INT32_MAX) return fail(ECNT_EINVAL, "factor %d: bad nnz", s);
            if (f.nnz > 0 && (!f.l_col_idx || !f.l_val))
                return fail(ECNT_EINVAL, "factor %d: null entry arrays", s);
            if (f.reserved != 0) return fail(ECNT_EINVAL, "factor %d: reserved must be 0", s);
            if (f.bandwidth < 0 || f.bandwidth >= n)
                return fail(ECNT_EINVAL, "factor %d: bandwidth out of range", s);
            if (f.bandwidth > ldl_ring_rows())
                return fail(ECNT_EUNSUPPORTED, "factor %d: bandwidth %d above %d", s, f.bandwidth,
                            ldl_ring_rows());
            LdlDev &d = p.ldl[s];
            d.perm = f.perm;
            d.lrp = f.l_row_ptr;
            d.lci = f.l_col_idx;
            d.lval = f.l_val;
            d.dd = f.d_diag;
            d.doff = f.d_off;
            d.nnz = f.nnz;
            d.bw = f.bandwidth;
        }
        break;
    }
    default:
        return fail(ECNT_EINVAL, "unknown preconditioner kind %d", T->kind);
    }
    if (p.prec_kind == ECNT_PREC_CHEB_LAPLACIAN && T->eval == ECNT_EVAL_AUTO)
        p.product = factorize(p) ? 1 : 0;
    // the grid of the Laplacian preconditioner is where A may be a stencil
    p.stencil_a = (p.prec_kind == ECNT_PREC_CHEB_LAPLACIAN && o->a_form == 0) ? 1 : 0;
    p.req_fused = o->fused;
    return ECNT_OK;
}

// Segment tables: nseg problems of ns[b] rows (grids dims[3b..3b+2], d2
// contiguous) and shifts taus[b*S..]; then geometry and workspace size.
static ecnt_status set_segments(Plan &p, SegHost &sh, int nseg, const int64_t *ns,
                                const int32_t *dims, const double *taus)
{
    p.nseg = nseg;
    sh.row.assign(nseg + 1, 0);
    sh.dims.assign(3 * (size_t)nseg, 1);
    sh.taus.assign((size_t)nseg * p.S, 0.0);
    for (int b = 0; b < nseg; ++b) {
        if (ns[b] < 1) return fail(ECNT_EINVAL, "problem %d has no rows", b);
        if (p.k > ns[b]) return fail(ECNT_EINVAL, "k = %d exceeds the size of problem %d", p.k, b);
        sh.row[b + 1] = sh.row[b] + ns[b];
        int64_t prod = 1;
        for (int a = 0; a < 3; ++a) {
            const int32_t d = dims ? dims[3 * b + a] : (a == 2 ? (int32_t)ns[b] : 1);
            if (d < 1) return fail(ECNT_EINVAL, "grid extents of problem %d must be >= 1", b);
            sh.dims[3 * b + a] = d;
            prod *= d;
        }
        if (prod != ns[b])
            return fail(ECNT_EINVAL, "grid of problem %d (%lld points) does not match its %lld rows", b,
                        (long long)prod, (long long)ns[b]);
        for (int t = 0; t < p.S; ++t) {
            const double tau = taus[(size_t)b * p.S + t];
            if (!isfinite(tau)) return fail(ECNT_EINVAL, "shift %d of problem %d is not finite", t, b);
            sh.taus[(size_t)b * p.S + t] = tau;
        }
    }
    if (sh.row[nseg] != p.n) return fail(ECNT_EINVAL, "problem sizes do not add up to n");
    p.st_ref_row = -1;   // the first row of the first problem with an off-diagonal entry
    for (int b = 0; b < nseg && p.st_ref_row < 0; ++b)
        if (ns[b] >= 2) p.st_ref_row = sh.row[b];
    col_geometry(p);
    row_geometry(p, sh);
    plan_layout(p, nullptr);
    return ECNT_OK;
}

// One problem: one segment, grid from the preconditioner (a single line otherwise).
static ecnt_status single_segment(Plan &p, SegHost &sh, const double *taus)
{
    const int64_t n = p.n;
    int32_t d[3] = {1, 1, (int32_t)n};
    if (p.prec_kind == ECNT_PREC_CHEB_LAPLACIAN) {
        d[0] = p.dims[0];
        d[1] = p.dims[1];
        d[2] = p.dims[2];
    }
    return set_segments(p, sh, 1, &n, d, taus);
}

__global__ void k_init(int32_t *flags)
{
    if (threadIdx.x < 4) flags[threadIdx.x] = 0;
}

// M x by Clenshaw's recurrence (R of degree d), with x = xs .* X.
// b_{d+1} = b_{d+2} = 0; b_j = c_j x + 2 B b_{j+1} - b_{j+2}; M x = c_0 x + B b_1 - b_2.
// Uses the two scratch blocks `t0`, `t1`; writes `out` (which may alias t0 or t1
// only where noted by the caller: here it must differ from both).
static double block_bytes(const Plan &p) { return (double)p.n * p.C * (p.vec_f32 ? 4 : 8); }

static void sweep(const Plan &p, const void *X, const double *xs, double cx, const void *IN,
                  bool in_is_x, double cb, const void *Z, double cz, void *out, hipStream_t st)
{
    // distinct block vectors read, plus the one written
    int nread = 1 + ((IN && IN != X) ? 1 : 0) + ((Z && Z != X && Z != IN) ? 1 : 0);
    Timed t(F_CHEB, (nread + 1) * block_bytes(p), st);
    launch_stencil(p, X, xs, cx, IN, in_is_x, cb, Z, cz, out, st);
}

// M x in product form, x = xs .* X:  M = lead * prod_f F_f(B), applied factor by
// factor; a quadratic factor (B^2 - 2aB + b) takes two sweeps,
//   t = B x - 2a x ;  y = B t + b x.
// Scratch: t0 (quadratic intermediate); factor outputs alternate between t1
// and t2 so that the last one lands in `out` (t2 may be `out` itself unless
// accumulating).  accum: out += M x instead of out = M x.
static void apply_M_product(const Plan &p, const void *X, const double *xs, void *t0, void *t1,
                            void *t2, void *out, bool accum, hipStream_t st)
{
    const void *in = X;
    const double *insc = xs;
    double scale = p.lead;
    for (int f = 0; f < p.nfac; ++f) {
        const bool last = f == p.nfac - 1;
        void *dst = last ? out : (((p.nfac - 2 - f) % 2 == 0) ? t1 : t2);
        const void *Z = (last && accum) ? out : nullptr;
        const double cz = (last && accum) ? -1.0 : 0.0;
        const double a = p.fac_a[f];
        if (!p.fac_quad[f]) {
            sweep(p, in, insc, -a * scale, in, insc != nullptr, scale, Z, cz, dst, st);
        } else if (quad_sweep_supported(p)) {
            Timed t(F_CHEB2, (Z ? 3 : 2) * block_bytes(p), st);
            launch_quad_sweep(p, in, insc, -2.0 * a * scale, scale, p.fac_b[f] * scale, Z, cz, dst, st);
        } else {
            sweep(p, in, insc, -2.0 * a * scale, in, insc != nullptr, scale, nullptr, 0.0, t0, st);
            sweep(p, in, insc, p.fac_b[f] * scale, t0, false, 1.0, Z, cz, dst, st);
        }
        in = dst;
        insc = nullptr;
        scale = 1.0;
    }
}

// M x by Clenshaw's recurrence, x = xs .* X:
// b_{d+1} = b_{d+2} = 0; b_j = c_j x + 2 B b_{j+1} - b_{j+2}; M x = c_0 x + B b_1 - b_2.
// Scratch t0, t1; `out` must differ from both.
static void apply_M_clenshaw(const Plan &p, const void *X, const double *xs, void *t0, void *t1,
                             void *out, hipStream_t st)
{
    const double *c = p.coef;
    const int d = p.degree;
    if (d == 0) {
        sweep(p, X, xs, c[0], nullptr, false, 0.0, nullptr, 0.0, out, st);
        return;
    }
    if (d == 1) {
        sweep(p, X, xs, c[0], X, true, c[1], nullptr, 0.0, out, st);
        return;
    }
    // b_{d-1} = c_{d-1} x + 2 c_d B x
    void *bj1 = t0;   // b_{j+1}
    sweep(p, X, xs, c[d - 1], X, true, 2.0 * c[d], nullptr, 0.0, bj1, st);
    if (d == 2) {
        // M x = c_0 x + B b_1 - b_2, b_2 = c_2 x
        sweep(p, X, xs, c[0] - c[2], bj1, false, 1.0, nullptr, 0.0, out, st);
        return;
    }
    // b_{d-2} = (c_{d-2} - c_d) x + 2 B b_{d-1}
    void *bj = t1;
    sweep(p, X, xs, c[d - 2] - c[d], bj1, false, 2.0, nullptr, 0.0, bj, st);
    void *bj2 = bj1;  // b_{j+2}
    bj1 = bj;
    for (int j = d - 3; j >= 1; --j) {
        // b_j = c_j x + 2 B b_{j+1} - b_{j+2}, written over b_{j+2} (read point-wise only)
        sweep(p, X, xs, c[j], bj1, false, 2.0, bj2, 1.0, bj2, st);
        void *tmp = bj2;
        bj2 = bj1;
        bj1 = tmp;
    }
    sweep(p, X, xs, c[0], bj1, false, 1.0, bj2, 1.0, out, st);
}

// out = M x (or out += M x when accum).  Scratch t0, t1, t2, all distinct from
// X; t2 may equal out when not accumulating.
static void apply_M(const Plan &p, const void *X, const double *xs, void *t0, void *t1, void *t2,
                    void *out, bool accum, hipStream_t st)
{
    if (p.product) {
        apply_M_product(p, X, xs, t0, t1, t2, out, accum, st);
    } else if (!accum) {
        apply_M_clenshaw(p, X, xs, t0, t1, out, st);
    } else {
        apply_M_clenshaw(p, X, xs, t0, t1, t2, st);
        sweep(p, t2, nullptr, 1.0, nullptr, false, 0.0, out, -1.0, out, st);   // out += t2
    }
}

static void enqueue_wave(const Plan &p, const ecnt_csr *A, const void *probes, hipStream_t st);

static void enqueue(const Plan &p, const ecnt_csr *A, const void *probes, ecnt_info *info,
                    hipStream_t st)
{
    k_init<<<1, 64, 0, st>>>(p.flags);
    const double csr_b = (double)(p.n + 1) * 4 + (double)A->nnz * (4 + (p.val_f32 ? 4 : 8));
    if (p.stencil_a && p.a_mode == 0) {
        Timed t(F_SETUP, csr_b + 8.0 * p.n, st);
        launch_stencil_check(p, A->row_ptr, A->col_idx, A->val, st);
    }
    if (p.prec_kind == ECNT_PREC_JACOBI) {
        Timed t(F_SETUP, csr_b + 8.0 * p.S * p.n, st);
        launch_jacobi_diag(p, A->row_ptr, A->col_idx, A->val, st);
    }
    if (p.prec_kind == ECNT_PREC_LDL) {
        Timed t(F_SETUP, (32.0 + 2 * 8.0 * ldl_ring_rows()) * p.S * p.n, st);
        launch_ldl_eblocks(p, st);
    }
    for (int c_off = 0; c_off < p.Ct; c_off += p.wave_cols) {
        Plan w = p;
        w.c_off = c_off;
        w.C = (p.Ct - c_off) < p.wave_cols ? (p.Ct - c_off) : p.wave_cols;
        if (w.block) w.nblk = w.C / kBlk;   // whole blocks: m and wave_cols are multiples of kBlk
        col_geometry(w);
        enqueue_wave(w, A, probes, st);
        // diagnostics of a single problem: alpha/beta of this wave into the caller's arrays
        if (p.nseg == 1 && !p.arnoldi && !p.block && info && info->alpha)
            (void)hipMemcpy2DAsync(info->alpha + c_off, sizeof(double) * p.Ct, w.alpha,
                                   sizeof(double) * w.C, sizeof(double) * w.C, p.k,
                                   hipMemcpyDeviceToDevice, st);
        if (p.nseg == 1 && !p.arnoldi && !p.block && info && info->beta)
            (void)hipMemcpy2DAsync(info->beta + c_off, sizeof(double) * p.Ct, w.beta,
                                   sizeof(double) * w.C, sizeof(double) * w.C, p.k + 1,
                                   hipMemcpyDeviceToDevice, st);
    }
    Timed t(F_QUAD, 0.0, st);
    launch_reduce(p, st);
}

// y = xs .* ((A - tau_c I) x) on the wave's columns.  With the Laplacian
// preconditioner, A is applied by the stencil sweep when it was found to be a
// stencil on the grid, else by the CSR sweep.  The single-problem calls learn
// which before their launches (a_mode 1 or 2); a batch's launch sequence,
// which takes no host synchronization, launches both, each returning at once
// when the other one applies (a_mode 0).
static void apply_A(const Plan &p, const ecnt_csr *A, const void *x, const double *xs, void *y,
                    hipStream_t st)
{
    const double blk_b = block_bytes(p);
    const double csr_b = (double)(p.n + 1) * 4 + (double)A->nnz * (4 + (p.val_f32 ? 4 : 8));
    if (p.stencil_a && p.a_mode == 1) {
        Timed t(F_STA, 2 * blk_b + 8.0 * p.n, st);
        launch_stencil_a(p, x, xs, y, st);
        return;
    }
    if (p.stencil_a && p.a_mode == 0) {
        {
            Timed t(F_STA, 2 * blk_b + 8.0 * p.n, st, 1);
            launch_stencil_a(p, x, xs, y, st);
        }
        Timed t(F_CSR, 2 * blk_b + csr_b, st, 2);
        launch_csr_op(p, A->row_ptr, A->col_idx, A->val, x, xs, nullptr, y, st, p.flags);
        return;
    }
    Timed t(F_CSR, 2 * blk_b + csr_b, st);
    launch_csr_op(p, A->row_ptr, A->col_idx, A->val, x, xs, nullptr, y, st);
}

// One wave of columns for the Arnoldi estimator (Algorithms 3 and 4):
// w = T (A - tau I) q_j, two classical Gram-Schmidt passes building column j
// of H, h_{j+1,j} = |w|; then the quadrature of every column.
static void enqueue_wave_arnoldi(const Plan &p, const ecnt_csr *A, const void *probes,
                                 hipStream_t st)
{
    const double blk_b = block_bytes(p);
    const double csr_b = (double)(p.n + 1) * 4 + (double)A->nnz * (4 + (p.val_f32 ? 4 : 8));
    {
        Timed t(F_SETUP, blk_b + (double)p.n * p.C * (p.vec_f32 ? 4 : 8) / p.S, st);
        launch_setup(p, probes, st);
    }
    {
        Timed t(F_FIN, 0.0, st);
        launch_setup_fin(p, st);
    }
    const size_t slot = slot_bytes(p);
    char *basis = (char *)p.basis;
    for (int j = 1; j <= p.k; ++j) {
        void *x = basis + (size_t)(j - 1) * slot;   // slot j-1 holds q_j (unnormalized)
        void *y = basis + (size_t)j * slot;         // slot j receives C q_j
        const double *xs = p.sig + (size_t)(j - 1) * p.nseg * p.C;
        if (p.prec_kind == ECNT_PREC_CHEB_LAPLACIAN) {
            apply_A(p, A, x, xs, p.tmp[0], st);
            apply_M(p, p.tmp[0], nullptr, p.tmp[1], p.tmp[2], y, y, false, st);   // T u
        } else {
            Timed t(F_CSR, 2 * blk_b + csr_b, st);
            launch_csr_op(p, A->row_ptr, A->col_idx, A->val, x, xs, nullptr, y, st);
        }
        for (int pass = 1; pass <= 2; ++pass) {
            for (int l0 = 0; l0 < j; l0 += kBasisChunk) {
                const int nb = (j - l0) < kBasisChunk ? (j - l0) : kBasisChunk;
                {
                    Timed t(F_DOTS, (nb + 1) * blk_b, st);
                    launch_dots(p, j, l0, nb, false, st);
                }
                Timed t(F_FIN, 0.0, st);
                launch_arn_fin(p, j, l0, nb, pass, st);
            }
            for (int l0 = 0; l0 < j; l0 += kBasisChunk) {
                const int nb = (j - l0) < kBasisChunk ? (j - l0) : kBasisChunk;
                Timed t(F_UPDATE, (nb + 2) * blk_b, st);
                launch_update(p, j, l0, nb, false, pass == 2 && l0 + kBasisChunk >= j, st);
            }
        }
        Timed t(F_FIN, 0.0, st);
        launch_arn_norm_fin(p, j, st);
    }
    Timed t(F_QUAD, 0.0, st);
    launch_arn_quad(p, st);
}

// y = C x = M (A - tau I) M^* x on the columns of the wave, x = xs .* X (xs may
// be null).  Step i only matters to the differentiated form, which keeps M q_i.
static void apply_op(const Plan &p, const ecnt_csr *A, void *x, const double *xs, void *y, int i,
                     hipStream_t st)
{
    const double blk_b = block_bytes(p);
    const double csr_b = (double)(p.n + 1) * 4 + (double)A->nnz * (4 + (p.val_f32 ? 4 : 8));
    const size_t slot = slot_bytes(p);
    const double jac_b = p.prec_kind == ECNT_PREC_JACOBI ? 8.0 * p.S * p.n : 0.0;
    // factor bytes a triangular solve streams (the band rows of one triangle)
    // and an elementwise pass (|D|^{-1/2} blocks and D's structure, or P)
    const double ldl_b = p.prec_kind == ECNT_PREC_LDL ? 8.0 * ldl_ring_rows() * p.S * p.n : 0.0;
    const double ldle_b = p.prec_kind == ECNT_PREC_LDL ? 24.0 * p.S * p.n : 0.0;
    if (p.prec_kind == ECNT_PREC_CHEB_LAPLACIAN) {
        // t = M q ; u = (A - tau I) t ; y = M u   (t kept per step for the backward)
        void *t = p.grad ? (char *)p.g_tslots + (size_t)(i - 1) * slot : p.tmp[2];
        apply_M(p, x, xs, p.tmp[0], p.tmp[1], t, t, false, st);
        apply_A(p, A, t, nullptr, p.tmp[0], st);
        apply_M(p, p.tmp[0], nullptr, p.tmp[1], p.tmp[2], y, y, false, st);
    } else if (p.prec_kind == ECNT_PREC_LDL) {
        // t = M^* q = P^T L^{-T} (|D|^{-1/2} q) ; u = (A - tau I) t ;
        // y = M u = |D|^{-1/2} (L^{-1} (P u))
        auto elem = [&](int what, const void *in, const double *sc, void *out) {
            Timed tm(F_LDLE, 2 * blk_b + ldle_b, st);
            launch_ldl(p, what, in, sc, out, st);
        };
        auto solve = [&](int what, const void *in, void *out) {
            Timed tm(F_LDL, 2 * blk_b + ldl_b, st);
            launch_ldl(p, what, in, nullptr, out, st);
        };
        elem(0, x, xs, p.tmp[0]);
        solve(2, p.tmp[0], p.tmp[1]);
        elem(4, p.tmp[1], nullptr, p.tmp[0]);
        {
            Timed tm(F_CSR, 2 * blk_b + csr_b, st);
            launch_csr_op(p, A->row_ptr, A->col_idx, A->val, p.tmp[0], nullptr, nullptr, p.tmp[1], st);
        }
        elem(3, p.tmp[1], nullptr, p.tmp[0]);
        solve(1, p.tmp[0], p.tmp[1]);
        elem(0, p.tmp[1], nullptr, y);
    } else {
        Timed t(F_CSR, 2 * blk_b + csr_b + jac_b, st);
        launch_csr_op(p, A->row_ptr, A->col_idx, A->val, x, xs,
                      p.prec_kind == ECNT_PREC_JACOBI ? p.jac : nullptr, y, st);
    }
}

// One wave of columns in the block-Lanczos form (blocks of kBlk columns):
// orthonormalize every probe block (two Cholesky QR passes), then k block
// steps, each one Gram-Schmidt pass against the whole basis followed by two
// Cholesky QR passes; then the block Gauss rule of every block.
static void enqueue_wave_block(const Plan &p, const ecnt_csr *A, const void *probes, hipStream_t st)
{
    const double blk_b = block_bytes(p);
    {
        Timed t(F_SETUP, blk_b + (double)p.n * p.C * 8 / p.S, st);
        launch_setup(p, probes, st);
    }
    auto dots = [&](int l0, int nb, int ys) {
        Timed t(F_BKDOTS, (nb + 1) * blk_b, st);
        launch_blk_dots(p, l0, nb, ys, st);
    };
    auto normalize = [&](int ws) {
        Timed t(F_BKNORM, 2 * blk_b, st);
        launch_blk_normalize(p, ws, st);
    };
    auto fin = [&](int mode, int step) {
        Timed t(F_FIN, 0.0, st);
        launch_blk_norm_fin(p, mode, step, st);
    };
    dots(0, 1, 0);
    fin(2, 0);
    normalize(0);
    fin(3, 0);
    const size_t slot = slot_bytes(p);
    char *basis = (char *)p.basis;
    for (int i = 1; i <= p.k; ++i) {
        apply_op(p, A, basis + (size_t)(i - 1) * slot, nullptr, basis + (size_t)i * slot, i, st);
        for (int l0 = 0; l0 < i; l0 += kBlkChunk) {
            const int nb = (i - l0) < kBlkChunk ? (i - l0) : kBlkChunk;
            dots(l0, nb, i);
            Timed t(F_FIN, 0.0, st);
            launch_blk_dots_fin(p, l0, nb, i - 1, st);
        }
        for (int l0 = 0; l0 < i; l0 += kBlkChunk) {
            const int nb = (i - l0) < kBlkChunk ? (i - l0) : kBlkChunk;
            Timed t(F_BKUPD, (nb + 2) * blk_b, st);
            launch_blk_update(p, l0, nb, i, l0 + kBlkChunk >= i, st);
        }
        fin(0, i);
        normalize(i);
        fin(1, i);
    }
    Timed t(F_BKQUAD, 0.0, st);
    launch_blk_quad(p, st);
}

// One wave of columns: Algorithm 1 on every column, then the quadrature.
static void enqueue_wave(const Plan &p, const ecnt_csr *A, const void *probes, hipStream_t st)
{
    if (p.arnoldi) {
        enqueue_wave_arnoldi(p, A, probes, st);
        return;
    }
    if (p.block) {
        enqueue_wave_block(p, A, probes, st);
        return;
    }
    const double blk_b = block_bytes(p);
    if (fused_applies(p, A->nnz)) {
        // a small problem: all k steps in one launch (one workgroup per column)
        {
            Timed t(F_FUSED, 0.0, st);
            launch_lanczos_fused(p, A->row_ptr, A->col_idx, A->val, A->nnz, probes, st);
        }
        Timed t(F_QUAD, 0.0, st);
        launch_tridiag(p, st);
        return;
    }
    {
        Timed t(F_SETUP, blk_b + (double)p.n * p.C * (p.vec_f32 ? 4 : 8) / p.S, st);
        launch_setup(p, probes, st);
    }
    {
        Timed t(F_FIN, 0.0, st);
        launch_setup_fin(p, st);
    }
    const size_t slot = slot_bytes(p);
    char *basis = (char *)p.basis;
    for (int i = 1; i <= p.k; ++i) {
        void *x = basis + (size_t)(i - 1) * slot;   // slot i-1 holds q_i (unnormalized)
        void *y = basis + (size_t)i * slot;         // slot i receives C q_i
        const double *xs = p.sig + (size_t)(i - 1) * p.nseg * p.C;
        apply_op(p, A, x, xs, y, i, st);
        const int sm = i >= 2 ? i - 2 : -1;
        // the Gram column of q_i makes the single pass take alpha_i first as
        // Algorithm 1 does (the reverse sweep of the differentiated form
        // follows the same coefficients)
        const bool gram = true;
        // the launch that holds q_i first: its finalize yields alpha_i for the others
        const int lq = (i - 1) / kBasisChunk * kBasisChunk;
        for (int c = 0; c * kBasisChunk < i; ++c) {
            const int l0 = c == 0 ? lq : (c - 1) * kBasisChunk;
            const int nb = (i - l0) < kBasisChunk ? (i - l0) : kBasisChunk;
            const bool m_in = sm >= l0 && sm < l0 + nb;
            const bool q_in = i - 1 >= l0 && i - 1 < l0 + nb;
            {
                Timed t(F_DOTS,
                        (nb + 1 + ((sm >= 0 && !m_in) ? 1 : 0) + ((gram && !q_in) ? 1 : 0)) * blk_b,
                        st);
                launch_dots(p, i, l0, nb, gram, st);
            }
            Timed t(F_FIN, 0.0, st);
            launch_dots_fin(p, i, l0, nb, gram, st);
        }
        for (int l0 = 0; l0 < i; l0 += kBasisChunk) {
            const int nb = (i - l0) < kBasisChunk ? (i - l0) : kBasisChunk;
            const bool first = l0 == 0;
            const bool m_in = sm >= l0 && sm < l0 + nb;
            Timed t(F_UPDATE, (nb + 2 + ((first && sm >= 0 && !m_in) ? 1 : 0)) * blk_b, st);
            launch_update(p, i, l0, nb, first, l0 + kBasisChunk >= i, st);
        }
        Timed t(F_FIN, 0.0, st);
        launch_norm_fin(p, i, st);
    }
    Timed t(F_QUAD, 0.0, st);
    launch_tridiag(p, st);
}

// Reverse sweep of the smoothed count (see k_backward.hip for the recurrences).
static void enqueue_backward(const Plan &p, const ecnt_csr *A, double g_out, double *dV,
                             hipStream_t st)
{
    const size_t slot = slot_bytes(p);
    const double blk_b = block_bytes(p);
    {
        Timed t(F_QUAD, 0.0, st);
        launch_tridiag_bwd(p, g_out, st);
    }
    for (int i = p.k; i >= 1; --i) {
        const bool last = i == p.k;
        if (!last) {
            Timed t(F_BDOTS, (i + 2) * blk_b, st);
            launch_bdots(p, i, st);
        }
        {
            Timed t(F_FIN, 0.0, st);
            launch_bdots_fin(p, i, !last, st);
        }
        {
            // reads: slots 0..i, qbar_{i+1}, qbar_0..i-1; writes: ybar, qbar_0..i-1
            Timed t(F_BUPD, ((i + 1) + (last ? 0 : 1) + (last ? 0 : i) + (1 + i)) * blk_b, st);
            launch_bupdate(p, i, last, st);
        }
        {
            Timed t(F_FIN, 0.0, st);
            launch_bnorm_fin(p, i, st);
        }
        // qbar_i += C ybar:  tbar = M ybar ; u = (A - tau I) tbar ; qbar_i += M u
        apply_M(p, p.g_ybar, nullptr, p.tmp[0], p.tmp[1], p.g_tbar, p.g_tbar, false, st);
        apply_A(p, A, p.g_tbar, nullptr, p.tmp[2], st);
        double *qbi = (double *)((char *)p.g_qbar + (size_t)(i - 1) * slot);
        apply_M(p, p.tmp[2], nullptr, p.tmp[0], p.tmp[1], p.g_ybar, qbi, true, st);
        {
            Timed t(F_VGRAD, 2 * blk_b, st);
            launch_vgrad(p, (const double *)((char *)p.g_tslots + (size_t)(i - 1) * slot), last, st);
        }
    }
    Timed t(F_FIN, 0.0, st);
    launch_grad_out(p, dV, st);
}

static ecnt_status check_common(const ecnt_csr *A, const void *probes, const ecnt_opts *o,
                                void *ws, const Plan &p, size_t ws_bytes)
{
    if (!A) return fail(ECNT_EINVAL, "A is null");
    if (!A->row_ptr || !A->col_idx || !A->val) return fail(ECNT_EINVAL, "A has null arrays");
    if (A->nnz < 0) return fail(ECNT_EINVAL, "A.nnz must be >= 0");
    if (A->val_type != ECNT_F64 && A->val_type != ECNT_F32)
        return fail(ECNT_EINVAL, "A.val_type must be ECNT_F64 or ECNT_F32");
    if (!probes) return fail(ECNT_EINVAL, "probes is null");
    (void)o;
    if (!ws) return fail(ECNT_EWORKSPACE, "workspace is null");
    if (ws_bytes < p.bytes)
        return fail(ECNT_EWORKSPACE, "workspace too small: %zu bytes given, %zu needed", ws_bytes, p.bytes);
    return ECNT_OK;
}

static ecnt_status upload_tables(const Plan &p, const SegHost &sh, hipStream_t st)
{
    hipError_t e = hipMemcpyAsync(p.seg_row, sh.row.data(), sizeof(int64_t) * (p.nseg + 1),
                                  hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p.seg_chunk, sh.chunk.data(), sizeof(int64_t) * (p.nseg + 1),
                           hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p.seg_tile, sh.tile.data(), sizeof(int64_t) * (p.nseg + 1),
                           hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p.seg_dims, sh.dims.data(), sizeof(int32_t) * 3 * p.nseg,
                           hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p.seg_taus, sh.taus.data(), sizeof(double) * p.S * p.nseg,
                           hipMemcpyHostToDevice, st);
    // the host tables are locals of the caller: complete the copies before returning
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(ECNT_EDEVICE, "HIP error: %s", hipGetErrorString(e));
    return ECNT_OK;
}

// Copy results (nseg * kResStride doubles) and flags back; synchronizes the stream.
static ecnt_status finish(const Plan &p, hipStream_t st, double *res_host, ecnt_info *info)
{
    int32_t flags[4] = {0, 0, 0, 0};
    hipError_t e = hipMemcpyAsync(res_host, p.result, sizeof(double) * kResStride * p.nseg,
                                  hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(flags, p.flags, sizeof flags, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && info) {
        const size_t NCt = (size_t)p.nseg * p.Ct;
        if (info->per_probe)
            e = hipMemcpyAsync(info->per_probe, p.s_out, sizeof(double) * NCt, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess && info->k_used)
            e = hipMemcpyAsync(info->k_used, p.kused, sizeof(int32_t) * NCt, hipMemcpyDeviceToDevice, st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(ECNT_EDEVICE, "HIP error: %s", hipGetErrorString(e));
    collect_profile(p.a_mode == 1 || (p.stencil_a && p.a_mode == 0 && flags[2] == 0));
    if (flags[0]) return fail(ECNT_ENOTHPD, "Jacobi preconditioner singular: a_rr == tau for some row");
    if (flags[1]) return fail(ECNT_EDEVICE, "tridiagonal eigensolver did not converge");
    return ECNT_OK;
}

// Restrictions of the differentiated form: FP64 Gauss rule with a smoothed
// step, the Laplacian-polynomial preconditioner (M independent of V and tau),
// one wave of columns, k <= 32.
static ecnt_status grad_plan(Plan &p, SegHost &sh, int64_t n, int64_t m, const ecnt_prec *T,
                             const ecnt_opts *o, const double *taus)
{
    ecnt_status rc = make_plan(p, n, m, 2, T, o);
    if (rc) return rc;
    if (!(o->smooth_w > 0.0)) return fail(ECNT_EINVAL, "the smoothed count needs opts.smooth_w > 0");
    if (o->vec_type != ECNT_F64) return fail(ECNT_EUNSUPPORTED, "gradients need FP64 vectors");
    if (o->rule != ECNT_RULE_GAUSS) return fail(ECNT_EUNSUPPORTED, "gradients need the Gauss rule");
    if (T->kind != ECNT_PREC_CHEB_LAPLACIAN)
        return fail(ECNT_EUNSUPPORTED, "gradients need the Laplacian-polynomial preconditioner");
    if (o->k > kBasisChunk) return fail(ECNT_EUNSUPPORTED, "gradients need k <= %d", kBasisChunk);
    if (p.wave_cols != p.Ct) return fail(ECNT_EUNSUPPORTED, "gradients need a single column wave");
    p.grad = 1;
    return single_segment(p, sh, taus);
}

// The Arnoldi estimator: T itself is the preconditioner description (not a
// factor of it); one problem, the paper's step h, no GA rule.
static ecnt_status arnoldi_plan(Plan &p, SegHost &sh, int64_t n, int64_t m, const ecnt_prec *T,
                                const ecnt_opts *o, const double *taus)
{
    ecnt_status rc = make_plan(p, n, m, 2, T, o);
    if (rc) return rc;
    if (T->kind == ECNT_PREC_JACOBI || T->kind == ECNT_PREC_LDL)
        return fail(ECNT_EUNSUPPORTED, "the Arnoldi estimator takes T = I or a Laplacian polynomial");
    if (o->rule != ECNT_RULE_GAUSS) return fail(ECNT_EUNSUPPORTED, "the Arnoldi estimator has no GA rule");
    if (o->smooth_w != 0.0) return fail(ECNT_EUNSUPPORTED, "the Arnoldi estimator uses the step h");
    if (o->k > 64) return fail(ECNT_EUNSUPPORTED, "the Arnoldi estimator needs k <= 64");
    p.arnoldi = 1;
    return single_segment(p, sh, taus);
}

// The block-Lanczos form: FP64, one problem, probes in blocks of kBlk
// (m and the wave width multiples of kBlk), Gauss rule, k <= kBlkMaxK.
static ecnt_status block_plan(Plan &p, SegHost &sh, int64_t n, int64_t m, const ecnt_prec *T,
                              const ecnt_opts *o, const double *taus)
{
    ecnt_status rc = make_plan(p, n, m, 2, T, o);
    if (rc) return rc;
    if (o->vec_type != ECNT_F64) return fail(ECNT_EUNSUPPORTED, "the block form needs FP64 vectors");
    if (o->rule != ECNT_RULE_GAUSS) return fail(ECNT_EUNSUPPORTED, "the block form has no GA rule");
    if (m % kBlk != 0) return fail(ECNT_EINVAL, "the block form needs m a multiple of %d (got %lld)", kBlk, (long long)m);
    if (p.wave_cols % kBlk != 0)
        return fail(ECNT_EINVAL, "the block form needs opts.max_cols a multiple of %d", kBlk);
    if (o->k > kBlkMaxK) return fail(ECNT_EUNSUPPORTED, "the block form needs k <= %d", kBlkMaxK);
    if (T->kind == ECNT_PREC_LDL)
        return fail(ECNT_EUNSUPPORTED, "the block form takes no LDL preconditioner");
    p.block = 1;
    return single_segment(p, sh, taus);
}

static void begin_launches()
{
    (void)hipGetLastError();
    std::lock_guard<std::mutex> g(g_prof_mu);
    t_prof = g_prof_on;
}

// mode: 0 count, 1 forward keeping backward state, 2 backward on kept state,
//       3 forward + backward (recompute), 4 Arnoldi count.
static ecnt_status run(const ecnt_csr *A, const ecnt_prec *T, const double *taus, int S,
                       const void *probes, int64_t m, const ecnt_opts *o, void *ws,
                       size_t ws_bytes, void *stream, double *res_host, ecnt_info *info, Plan &p,
                       int mode = 0, double g_out = 0.0, double *dV = nullptr)
{
    SegHost sh;
    ecnt_status rc;
    if (mode == 0) {
        rc = make_plan(p, A ? A->n : 0, m, S, T, o);
        if (!rc) rc = single_segment(p, sh, taus);
    } else if (mode == 4) {
        rc = arnoldi_plan(p, sh, A ? A->n : 0, m, T, o, taus);
    } else if (mode == 5) {
        rc = block_plan(p, sh, A ? A->n : 0, m, T, o, taus);
    } else {
        rc = grad_plan(p, sh, A ? A->n : 0, m, T, o, taus);
    }
    if (rc) return rc;
    if ((mode == 2 || mode == 3) && !dV) return fail(ECNT_EINVAL, "dV is null");
    if (mode >= 1 && mode <= 3 && A && A->val_type != ECNT_F64)
        return fail(ECNT_EUNSUPPORTED, "gradients need FP64 matrix values");
    rc = check_common(A, probes, o, ws, p, ws_bytes);
    if (rc) return rc;
    p.val_f32 = A->val_type == ECNT_F32;
    char *base = (char *)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
    plan_layout(p, base);
    hipStream_t st = (hipStream_t)stream;
    rc = upload_tables(p, sh, st);
    if (rc) return rc;
    if (p.stencil_a) {   // which form applies A: check once, before the launch sequence
        int32_t flag = 1;
        k_init<<<1, 64, 0, st>>>(p.flags);
        launch_stencil_check(p, A->row_ptr, A->col_idx, A->val, st);
        hipError_t e = hipMemcpyAsync(&flag, p.flags + 2, sizeof flag, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return fail(ECNT_EDEVICE, "HIP error: %s", hipGetErrorString(e));
        p.a_mode = flag == 0 ? 1 : 2;
    }
    begin_launches();
    if (mode != 2) enqueue(p, A, probes, info, st);
    if (mode == 2 || mode == 3) enqueue_backward(p, A, g_out, dV, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(ECNT_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return finish(p, st, res_host, info);
}

// ---- batches of independent problems (block-diagonal A) ----
static ecnt_status batch_plan(Plan &p, SegHost &sh, const ecnt_batch_item *items, int32_t nprob,
                              int32_t nshift, int64_t m, const ecnt_prec *T, const ecnt_opts *o)
{
    if (!items || nprob < 1) return fail(ECNT_EINVAL, "need at least one problem");
    if (nprob > (1 << 20)) return fail(ECNT_EUNSUPPORTED, "too many problems");
    if (nshift < 1 || nshift > kMaxShifts) return fail(ECNT_EINVAL, "nshift must be in 1..%d", kMaxShifts);
    int64_t n = 0;
    std::vector<int64_t> ns(nprob);
    std::vector<int32_t> dims(3 * (size_t)nprob);
    std::vector<double> taus((size_t)nprob * (nshift > 0 ? nshift : 1));
    for (int b = 0; b < nprob; ++b) {
        ns[b] = items[b].n;
        if (ns[b] < 1) return fail(ECNT_EINVAL, "problem %d has no rows", b);
        n += ns[b];
        if (!items[b].taus) return fail(ECNT_EINVAL, "shifts of problem %d are null", b);
        for (int a = 0; a < 3; ++a)   // the grid matters to the stencil preconditioner only
            dims[3 * b + a] = T && T->kind == ECNT_PREC_CHEB_LAPLACIAN
                                  ? items[b].dims[a]
                                  : (a == 2 ? (int32_t)(ns[b] < INT32_MAX ? ns[b] : INT32_MAX) : 1);
        for (int t = 0; t < nshift; ++t) taus[(size_t)b * nshift + t] = items[b].taus[t];
    }
    if (!T) return fail(ECNT_EINVAL, "null preconditioner");
    if (T->kind == ECNT_PREC_LDL)
        return fail(ECNT_EUNSUPPORTED, "batches do not take the LDL preconditioner");
    if (T->kind == ECNT_PREC_CHEB_LAPLACIAN && T->ndim != 3)
        return fail(ECNT_EINVAL, "batches with the Laplacian preconditioner need prec.ndim = 3");
    ecnt_prec Tb = *T;
    if (Tb.kind == ECNT_PREC_CHEB_LAPLACIAN) {   // per-problem grids come from the items
        Tb.ndim = 3;
        Tb.dims[0] = 1;
        Tb.dims[1] = 1;
        Tb.dims[2] = (int32_t)(n < INT32_MAX ? n : INT32_MAX);
    }
    ecnt_status rc = make_plan(p, n, m, nshift, &Tb, o);
    if (rc) return rc;
    p.ndim = T->ndim;
    return set_segments(p, sh, nprob, ns.data(), dims.data(), taus.data());
}


// ---- fixed device array behind ecnt_count_noalloc ----
// Each GPU the library runs on holds one copy, for the life of the process.
// In host code `scratch` names a host-side stand-in: its device address on the
// current GPU comes from hipGetSymbolAddress and is used everywhere instead.
static __device__ __align__(256) unsigned char scratch[ECNT_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;                  // guards g_scratch_ptr
static void *g_scratch_ptr[kMaxDevices];         // device address of `scratch`, per device
static std::mutex g_scratch_run_mu[kMaxDevices]; // one call at a time per device

// Device address of the array on the current device (looked up once per device).
static ecnt_status scratch_address(int dev, void **out)
{
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(ECNT_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return ECNT_OK;
}

}  // namespace ecnt

using namespace ecnt;

extern "C" {

size_t ecnt_workspace_bytes(int64_t n, int64_t m, int32_t nshift, const ecnt_prec *T,
                            const ecnt_opts *opts)
{
    Plan p;
    SegHost sh;
    if (make_plan(p, n, m, nshift, T, opts) != ECNT_OK) return 0;
    std::vector<double> taus((size_t)nshift, 0.0);   // values do not affect the size
    if (single_segment(p, sh, taus.data()) != ECNT_OK) return 0;
    return p.bytes;
}

ecnt_status ecnt_count(const ecnt_csr *A, const ecnt_prec *T, double xi, double eta,
                       const void *probes, int64_t m, const ecnt_opts *opts, void *ws,
                       size_t ws_bytes, void *stream, double *estimate, double *variance,
                       ecnt_info *info)
{
    g_err.clear();
    if (!estimate || !variance) return fail(ECNT_EINVAL, "estimate/variance output is null");
    if (!isfinite(xi) || !isfinite(eta)) return fail(ECNT_EINVAL, "xi and eta must be finite");
    if (!(xi < eta)) return fail(ECNT_EINVAL, "need xi < eta (got %g, %g)", xi, eta);
    const double taus[2] = {xi, eta};
    double res[kResStride];
    Plan p;
    ecnt_status rc = run(A, T, taus, 2, probes, m, opts, ws, ws_bytes, stream, res, info, p);
    if (rc) return rc;
    *estimate = res[2];
    *variance = res[3];
    if (info) {
        info->neg_xi = res[0];
        info->neg_eta = res[1];
        info->min_abs_ritz = res[4];
    }
    return ECNT_OK;
}

ecnt_status ecnt_count_noalloc(const ecnt_csr *A, const ecnt_prec *T, double xi, double eta,
                               const void *probes, int64_t m, const ecnt_opts *opts, void *stream,
                               double *estimate, double *variance, ecnt_info *info)
{
    g_err.clear();
    // Validation and the size check run on the host first, as in ecnt_count:
    // a refused call (including a count too large for the fixed array) makes
    // no device call at all.
    if (!estimate || !variance) return fail(ECNT_EINVAL, "estimate/variance output is null");
    if (!isfinite(xi) || !isfinite(eta)) return fail(ECNT_EINVAL, "xi and eta must be finite");
    if (!(xi < eta)) return fail(ECNT_EINVAL, "need xi < eta (got %g, %g)", xi, eta);
    {
        Plan p;
        SegHost sh;
        const double taus[2] = {xi, eta};
        ecnt_status rc = make_plan(p, A ? A->n : 0, m, 2, T, opts);
        if (!rc) rc = single_segment(p, sh, taus);
        if (!rc) rc = check_common(A, probes, opts, (void *)&p, p, p.bytes);
        if (rc) return rc;
        if (p.bytes > ECNT_NOALLOC_SCRATCH_BYTES)
            return fail(ECNT_EWORKSPACE,
                        "ecnt_count_noalloc: this count needs %zu bytes of device scratch, the fixed "
                        "array holds %zu; use ecnt_count with a caller workspace",
                        p.bytes, (size_t)ECNT_NOALLOC_SCRATCH_BYTES);
    }
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(ECNT_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(ECNT_EUNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
    if (stream) {
        hipDevice_t sd = -1;
        e = hipStreamGetDevice((hipStream_t)stream, &sd);
        if (e != hipSuccess) return fail(ECNT_EDEVICE, "hipStreamGetDevice: %s", hipGetErrorString(e));
        if (sd != dev)
            return fail(ECNT_EINVAL, "the stream belongs to device %d but device %d is current", (int)sd, dev);
    }
    void *ws = nullptr;
    ecnt_status rc = scratch_address(dev, &ws);
    if (rc) return rc;
    std::lock_guard<std::mutex> g(g_scratch_run_mu[dev]);
    rc = ecnt_count(A, T, xi, eta, probes, m, opts, ws, ECNT_NOALLOC_SCRATCH_BYTES, stream, estimate,
                    variance, info);
    // nothing of this call may still use the array when the next one starts
    // (ecnt_count returns after synchronizing the stream unless it failed early)
    if (rc) (void)hipStreamSynchronize((hipStream_t)stream);
    return rc;
}

ecnt_status ecnt_negcounts(const ecnt_csr *A, const ecnt_prec *T, const double *taus,
                           int32_t nshift, const void *probes, int64_t m, const ecnt_opts *opts,
                           void *ws, size_t ws_bytes, void *stream, double *negcounts,
                           double *counts, double *variances, ecnt_info *info)
{
    g_err.clear();
    if (!taus || !negcounts) return fail(ECNT_EINVAL, "taus/negcounts is null");
    if (nshift < 1 || nshift > kMaxShifts) return fail(ECNT_EINVAL, "nshift must be in 1..%d", kMaxShifts);
    double res[kResStride];
    Plan p;
    ecnt_status rc = run(A, T, taus, nshift, probes, m, opts, ws, ws_bytes, stream, res, info, p);
    if (rc) return rc;
    const int S = nshift;
    for (int s = 0; s < S; ++s) negcounts[s] = res[s];
    for (int t = 0; t + 1 < S; ++t) {
        if (counts) counts[t] = res[S + t];
        if (variances) variances[t] = res[2 * S - 1 + t];
    }
    if (info) {
        info->neg_xi = res[0];
        info->neg_eta = S > 1 ? res[1] : res[0];
        info->min_abs_ritz = res[3 * S - 2];
    }
    return ECNT_OK;
}

size_t ecnt_arnoldi_workspace_bytes(int64_t n, int64_t m, const ecnt_prec *T, const ecnt_opts *opts)
{
    Plan p;
    SegHost sh;
    const double taus[2] = {0.0, 1.0};
    if (arnoldi_plan(p, sh, n, m, T, opts, taus) != ECNT_OK) return 0;
    return p.bytes;
}

ecnt_status ecnt_count_arnoldi(const ecnt_csr *A, const ecnt_prec *T, double xi, double eta,
                               const void *probes, int64_t m, const ecnt_opts *opts, void *ws,
                               size_t ws_bytes, void *stream, double *estimate, double *variance,
                               ecnt_info *info)
{
    g_err.clear();
    if (!estimate || !variance) return fail(ECNT_EINVAL, "estimate/variance output is null");
    if (!isfinite(xi) || !isfinite(eta)) return fail(ECNT_EINVAL, "xi and eta must be finite");
    if (!(xi < eta)) return fail(ECNT_EINVAL, "need xi < eta (got %g, %g)", xi, eta);
    const double taus[2] = {xi, eta};
    double res[kResStride];
    Plan p;
    ecnt_status rc = run(A, T, taus, 2, probes, m, opts, ws, ws_bytes, stream, res, info, p, 4);
    if (rc) return rc;
    *estimate = res[2];
    *variance = res[3];
    if (info) {
        info->neg_xi = res[0];
        info->neg_eta = res[1];
        info->min_abs_ritz = INFINITY;
    }
    return ECNT_OK;
}

size_t ecnt_block_workspace_bytes(int64_t n, int64_t m, const ecnt_prec *T, const ecnt_opts *opts)
{
    Plan p;
    SegHost sh;
    const double taus[2] = {0.0, 1.0};
    if (block_plan(p, sh, n, m, T, opts, taus) != ECNT_OK) return 0;
    return p.bytes;
}

ecnt_status ecnt_count_block(const ecnt_csr *A, const ecnt_prec *T, double xi, double eta,
                             const void *probes, int64_t m, const ecnt_opts *opts, void *ws,
                             size_t ws_bytes, void *stream, double *estimate, double *variance,
                             ecnt_info *info)
{
    g_err.clear();
    if (!estimate || !variance) return fail(ECNT_EINVAL, "estimate/variance output is null");
    if (!isfinite(xi) || !isfinite(eta)) return fail(ECNT_EINVAL, "xi and eta must be finite");
    if (!(xi < eta)) return fail(ECNT_EINVAL, "need xi < eta (got %g, %g)", xi, eta);
    const double taus[2] = {xi, eta};
    double res[kResStride];
    Plan p;
    ecnt_status rc = run(A, T, taus, 2, probes, m, opts, ws, ws_bytes, stream, res, info, p, 5);
    if (rc) return rc;
    *estimate = res[2];
    *variance = res[3];
    if (info) {
        info->neg_xi = res[0];
        info->neg_eta = res[1];
        info->min_abs_ritz = res[4];
    }
    return ECNT_OK;
}

ecnt_status ecnt_profile_enable(int32_t on)
{
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof_on = on != 0;
    if (g_prof_on) {
        for (int f = 0; f < F_COUNT; ++f) {
            memset(&g_stats[f], 0, sizeof g_stats[f]);
            snprintf(g_stats[f].name, sizeof g_stats[f].name, "%s", kFamilyName[f]);
        }
    }
    return ECNT_OK;
}

int32_t ecnt_profile_read(ecnt_kernel_stat *out, int32_t max)
{
    std::lock_guard<std::mutex> g(g_prof_mu);
    int32_t n = 0;
    for (int f = 0; f < F_COUNT && n < max && out; ++f) out[n++] = g_stats[f];
    return n;
}

size_t ecnt_smooth_workspace_bytes(int64_t n, int64_t m, const ecnt_prec *T, const ecnt_opts *opts)
{
    Plan p;
    SegHost sh;
    const double taus[2] = {0.0, 1.0};
    if (grad_plan(p, sh, n, m, T, opts, taus) != ECNT_OK) return 0;
    return p.bytes;
}

size_t ecnt_batch_workspace_bytes(const ecnt_batch_item *items, int32_t nprob, int32_t nshift,
                                  int64_t m, const ecnt_prec *T, const ecnt_opts *opts)
{
    Plan p;
    SegHost sh;
    if (batch_plan(p, sh, items, nprob, nshift, m, T, opts) != ECNT_OK) return 0;
    return p.bytes;
}

// prepare: validate, carve, upload the segment tables (synchronous)
ecnt_status ecnt_batch_prepare(const ecnt_csr *A, const ecnt_prec *T, const ecnt_batch_item *items,
                               int32_t nprob, int32_t nshift, const void *probes, int64_t m,
                               const ecnt_opts *opts, void *ws, size_t ws_bytes, void *stream)
{
    g_err.clear();
    Plan p;
    SegHost sh;
    ecnt_status rc = batch_plan(p, sh, items, nprob, nshift, m, T, opts);
    if (rc) return rc;
    if (A && A->n != p.n) return fail(ECNT_EINVAL, "A has %lld rows, the problems %lld",
                                      (long long)A->n, (long long)p.n);
    rc = check_common(A, probes, opts, ws, p, ws_bytes);
    if (rc) return rc;
    char *base = (char *)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
    plan_layout(p, base);
    return upload_tables(p, sh, (hipStream_t)stream);
}

// enqueue: kernel launches only (no host synchronization, no copies): may be
// captured into a hipGraph and replayed; results stay in the workspace.
ecnt_status ecnt_batch_enqueue(const ecnt_csr *A, const ecnt_prec *T, const ecnt_batch_item *items,
                               int32_t nprob, int32_t nshift, const void *probes, int64_t m,
                               const ecnt_opts *opts, void *ws, size_t ws_bytes, void *stream)
{
    g_err.clear();
    Plan p;
    SegHost sh;
    ecnt_status rc = batch_plan(p, sh, items, nprob, nshift, m, T, opts);
    if (rc) return rc;
    rc = check_common(A, probes, opts, ws, p, ws_bytes);
    if (rc) return rc;
    p.val_f32 = A->val_type == ECNT_F32;
    char *base = (char *)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
    plan_layout(p, base);
    begin_launches();
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing((hipStream_t)stream, &cap) == hipSuccess && cap != hipStreamCaptureStatusNone)
        t_prof = false;   // no timing events inside a captured graph
    enqueue(p, A, probes, nullptr, (hipStream_t)stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(ECNT_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return ECNT_OK;
}

// results: copy the per-problem results back (synchronizes the stream)
ecnt_status ecnt_batch_results(const ecnt_batch_item *items, int32_t nprob, int32_t nshift,
                               int64_t m, const ecnt_prec *T, const ecnt_opts *opts, void *ws,
                               size_t ws_bytes, void *stream, double *negcounts, double *counts,
                               double *variances, ecnt_info *info)
{
    g_err.clear();
    Plan p;
    SegHost sh;
    ecnt_status rc = batch_plan(p, sh, items, nprob, nshift, m, T, opts);
    if (rc) return rc;
    if (!ws || ws_bytes < p.bytes) return fail(ECNT_EWORKSPACE, "workspace missing or too small");
    if (!negcounts) return fail(ECNT_EINVAL, "negcounts is null");
    char *base = (char *)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
    plan_layout(p, base);
    std::vector<double> res((size_t)kResStride * nprob);
    rc = finish(p, (hipStream_t)stream, res.data(), info);
    if (rc) return rc;
    const int S = nshift;
    for (int b = 0; b < nprob; ++b) {
        const double *r = res.data() + (size_t)b * kResStride;
        for (int s = 0; s < S; ++s) negcounts[(size_t)b * S + s] = r[s];
        for (int t = 0; t + 1 < S; ++t) {
            if (counts) counts[(size_t)b * (S - 1) + t] = r[S + t];
            if (variances) variances[(size_t)b * (S - 1) + t] = r[2 * S - 1 + t];
        }
    }
    return ECNT_OK;
}

ecnt_status ecnt_count_batched(const ecnt_csr *A, const ecnt_prec *T, const ecnt_batch_item *items,
                               int32_t nprob, int32_t nshift, const void *probes, int64_t m,
                               const ecnt_opts *opts, void *ws, size_t ws_bytes, void *stream,
                               double *negcounts, double *counts, double *variances,
                               ecnt_info *info)
{
    ecnt_status rc = ecnt_batch_prepare(A, T, items, nprob, nshift, probes, m, opts, ws, ws_bytes, stream);
    if (rc) return rc;
    rc = ecnt_batch_enqueue(A, T, items, nprob, nshift, probes, m, opts, ws, ws_bytes, stream);
    if (rc) return rc;
    return ecnt_batch_results(items, nprob, nshift, m, T, opts, ws, ws_bytes, stream, negcounts,
                              counts, variances, info);
}

static ecnt_status smooth_common_args(double xi, double eta)
{
    if (!isfinite(xi) || !isfinite(eta)) return fail(ECNT_EINVAL, "xi and eta must be finite");
    if (!(xi < eta)) return fail(ECNT_EINVAL, "need xi < eta (got %g, %g)", xi, eta);
    return ECNT_OK;
}

ecnt_status ecnt_smooth_fwd(const ecnt_csr *A, const ecnt_prec *T, double xi, double eta,
                            const void *probes, int64_t m, const ecnt_opts *opts, void *ws,
                            size_t ws_bytes, void *stream, double *estimate, double *variance,
                            ecnt_info *info)
{
    g_err.clear();
    if (!estimate || !variance) return fail(ECNT_EINVAL, "estimate/variance output is null");
    ecnt_status rc = smooth_common_args(xi, eta);
    if (rc) return rc;
    const double taus[2] = {xi, eta};
    double res[kResStride];
    Plan p;
    rc = run(A, T, taus, 2, probes, m, opts, ws, ws_bytes, stream, res, info, p, 1);
    if (rc) return rc;
    *estimate = res[2];
    *variance = res[3];
    if (info) {
        info->neg_xi = res[0];
        info->neg_eta = res[1];
        info->min_abs_ritz = res[4];
    }
    return ECNT_OK;
}

ecnt_status ecnt_smooth_bwd(const ecnt_csr *A, const ecnt_prec *T, double xi, double eta,
                            const void *probes, int64_t m, const ecnt_opts *opts, int32_t ckpt,
                            double g_est, void *ws, size_t ws_bytes, void *stream, double *dV,
                            double *dxi, double *deta)
{
    g_err.clear();
    if (!dxi || !deta) return fail(ECNT_EINVAL, "dxi/deta output is null");
    if (ckpt != ECNT_CKPT_KEEP && ckpt != ECNT_CKPT_RECOMPUTE)
        return fail(ECNT_EINVAL, "ckpt must be ECNT_CKPT_KEEP or ECNT_CKPT_RECOMPUTE");
    if (!isfinite(g_est)) return fail(ECNT_EINVAL, "g_est must be finite");
    ecnt_status rc = smooth_common_args(xi, eta);
    if (rc) return rc;
    const double taus[2] = {xi, eta};
    double res[kResStride];
    Plan p;
    rc = run(A, T, taus, 2, probes, m, opts, ws, ws_bytes, stream, res, nullptr, p,
             ckpt == ECNT_CKPT_KEEP ? 2 : 3, g_est, dV);
    if (rc) return rc;
    *dxi = res[4 * kMaxShifts + 0];
    *deta = res[4 * kMaxShifts + 1];
    return ECNT_OK;
}

ecnt_status ecnt_hbm_probe(int32_t kind, void *buf, size_t bytes, int32_t reps, void *stream,
                           double *gbs)
{
    g_err.clear();
    if (kind < 0 || kind > 2) return fail(ECNT_EINVAL, "probe kind must be 0, 1 or 2");
    if (!buf || !gbs) return fail(ECNT_EINVAL, "null buffer or output");
    if (bytes < ((size_t)64 << 20)) return fail(ECNT_EINVAL, "probe buffer below 64 MiB");
    if (reps < 1) return fail(ECNT_EINVAL, "reps must be >= 1");
    if (run_probe(kind, buf, bytes, reps, (hipStream_t)stream, gbs) != 0)
        return fail(ECNT_EDEVICE, "probe failed: %s", hipGetErrorString(hipGetLastError()));
    return ECNT_OK;
}

const char *ecnt_last_error(void) { return g_err.c_str(); }

const char *ecnt_version(void) { return "ecount-mi355x 0.1 (gfx950)"; }

}  // extern "C"
