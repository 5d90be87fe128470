// Host runtime and C ABI of the GaBP SVM solver (see include/gabp_svm.h).
//
// A solve is: validate -> stage features -> build K' (materialised tiles) ->
// row sums + diagonal weighting -> sweep 0 aggregates -> synchronous sweeps
// (sweep kernel, finalize, device-side stop rule) until the device status
// says done -> download alpha.  The host polls an 8-word status every
// `check_every` sweeps; sweeps launched after the stop are no-ops on the
// device, so the result does not depend on the polling period.
#include "../../include/gabp_svm.h"
#include "gabp_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

using namespace gabp;

namespace {

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t n) {
        if (n == 0) n = 256;
        if (p && n <= bytes) return hipSuccess;
        release();
        hipError_t e = hipMalloc(&p, n);
        if (e != hipSuccess) {
            p = nullptr;
            bytes = 0;
            (void)hipGetLastError();
            return e;
        }
        bytes = n;
        return hipSuccess;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <class T> T* as() const { return static_cast<T*>(p); }
};

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

namespace gabp {
gabp_status check_params(const gabp_svm_params* p, std::string& why) {
    if (!p) { why = "params is NULL"; return GABP_E_INVALID; }
    if (p->struct_size != sizeof(gabp_svm_params)) { why = "params.struct_size mismatch"; return GABP_E_INVALID; }
    if (p->kernel != GABP_KERNEL_RBF && p->kernel != GABP_KERNEL_PRECOMPUTED && p->kernel != GABP_KERNEL_RBF_SPARSE) { why = "unknown kernel"; return GABP_E_INVALID; }
    if (p->kernel != GABP_KERNEL_PRECOMPUTED && !(p->gamma > 0.0 && std::isfinite(p->gamma))) { why = "gamma must be > 0"; return GABP_E_INVALID; }
    if (p->kernel == GABP_KERNEL_RBF_SPARSE) {
        if (!(p->sparse_tau > 0.0 && p->sparse_tau <= 1.0)) { why = "sparse_tau must be in (0, 1]"; return GABP_E_INVALID; }
        if (p->precision == GABP_PREC_FP64) { why = "the sparsified kernel runs in FP32 or MIXED precision"; return GABP_E_INVALID; }
        if (p->schedule != GABP_SCHED_SYNC) { why = "the sparsified kernel runs the SYNC schedule"; return GABP_E_INVALID; }
        if (p->sparse_edges_hint < 0) { why = "sparse_edges_hint must be >= 0"; return GABP_E_INVALID; }
    }
    if (!(p->C > 0.0) || !std::isfinite(p->C)) { why = "C must be > 0"; return GABP_E_INVALID; }
    if (p->diag_mode < 0 || p->diag_mode > 3) { why = "unknown diag_mode"; return GABP_E_INVALID; }
    if (!(p->diag_delta >= 0.0)) { why = "diag_delta must be >= 0"; return GABP_E_INVALID; }
    if (p->box_mode < 0 || p->box_mode > 2) { why = "unknown box_mode"; return GABP_E_INVALID; }
    if (!(p->tol_abs >= 0.0) || !(p->tol_rel >= 0.0)) { why = "tolerances must be >= 0"; return GABP_E_INVALID; }
    if (p->max_sweeps < 1) { why = "max_sweeps must be >= 1"; return GABP_E_INVALID; }
    if (p->check_every < 1) { why = "check_every must be >= 1"; return GABP_E_INVALID; }
    if (p->stagnation_window < 0) { why = "stagnation_window must be >= 0"; return GABP_E_INVALID; }
    if (p->precision < 0 || p->precision > 2) { why = "unknown precision"; return GABP_E_INVALID; }
    if (p->kstore < 0 || p->kstore > 2) { why = "unknown kstore"; return GABP_E_INVALID; }
    if (p->edge_state < 0 || p->edge_state > 2) { why = "unknown edge_state"; return GABP_E_INVALID; }
    if (p->gram < 0 || p->gram > 3) { why = "unknown gram"; return GABP_E_INVALID; }
    if (p->stateless_depth < 0 || p->stateless_depth > 8) { why = "stateless_depth must be in [0, 8]"; return GABP_E_INVALID; }
    if (p->schedule < 0 || p->schedule > 1) { why = "unknown schedule"; return GABP_E_INVALID; }
    if (p->sched_groups < 0 || p->sched_groups > 4096) { why = "sched_groups must be in [0, 4096]"; return GABP_E_INVALID; }
    if (p->tile_chunk < 0 || p->tile_chunk > 2) { why = "tile_chunk must be 0, 1 or 2"; return GABP_E_INVALID; }
    return GABP_OK;
}
}  // namespace gabp

struct gabp_svm {
    gabp_svm_params p{};
    std::string err;
    bool have_result = false;
    bool rbf = true;
    // geometry of the last solve
    int64_t N = 0, m = 0, NPAD = 0, ntiles = 0;
    int NB = 0, m_pad = 0, prec = PREC_MIXED, gram = GRAM_BF16;
    double lam = 0.0;
    int32_t status = GABP_E_STATE, reason = R_NONE, sweeps = 0;
    double delta = 0.0;
    std::vector<double> alpha, ptilde, adiag, trace;
    std::vector<float> yh;
    gabp_timings tm{};
    gabp_plan plan{};
    // device memory owned by the handle
    DevBuf tiles, Kp, Pf, Pb, Ef, Eb, partP, partE, Xin, yd, mean, xs32, xhi, xlo, xlo2, x64, nrm, kdiag, rowmax, rsum,
        Adiag, Pt, S, alpha_d, blk1, blk2, one, status_d, trace_d, flag, tmp, Kin, q_rows, q_cols,
        q_out, glist, HI, HM,
        chunks,                  // 2 x 2 tile chunks of the synchronous FP32-partial sweep
        xaug,                    // training rows of the augmented decision function
        xaug0,                   // the other augmentation, for K' recomputed per band
        parena;                  // working memory of gabp_svm_predict (reused)
    int aug_kind = -1, aug_mp = 0;
    // sparsified kernel: tile counts and offsets, keys, K' per edge, edge
    // ends, degrees and offsets of the i-end and j-end lists, permutation
    DevBuf sp_cnt, sp_toff, sp_keys, sp_keys2, sp_kv, sp_kv2, sp_ei, sp_ej, sp_degi, sp_degj, sp_offi,
        sp_offj, sp_ids, sp_perm, sp_tmp, sp_order, sp_Xp, sp_cent, sp_rad, sp_keep, sp_tsel, sp_nsel, sp_xb;
    bool sparse = false;
    int64_t n_edges = 0;
    // residual certificate of the last solve (GABP_Q_RESIDUAL_BOUND), formed
    // on the first query
    bool resid_valid = false;
    double resid[3] = {0.0, 0.0, 0.0};

    DevBuf* all[72] = {&tiles, &Kp, &Pf, &Pb, &Ef, &Eb, &partP, &partE, &Xin, &yd, &mean,
                       &xs32, &xhi, &xlo, &xlo2, &x64, &nrm, &kdiag, &rowmax, &rsum, &Adiag, &Pt, &S, &alpha_d,
                       &blk1, &blk2, &one, &status_d, &trace_d, &flag, &tmp, &Kin, &q_rows,
                       &q_cols, &q_out, &glist, &sp_cnt, &sp_toff, &sp_keys, &sp_keys2, &sp_kv, &sp_kv2,
                       &sp_ei, &sp_ej, &sp_degi, &sp_degj, &sp_offi, &sp_offj, &sp_ids, &sp_perm, &sp_tmp,
                       &sp_order, &sp_Xp, &sp_cent, &sp_rad, &sp_keep, &sp_tsel, &sp_nsel, &sp_xb, &HI, &HM, &chunks, &xaug, &xaug0, &parena, nullptr};
    size_t held() const {
        size_t b = 0;
        for (int k = 0; all[k]; ++k) b += all[k]->bytes;
        return b;
    }
    void release_all() {
        for (int k = 0; all[k]; ++k) all[k]->release();
    }
};

namespace {

gabp_status fail(gabp_svm* h, gabp_status st, const std::string& msg) {
    if (h) h->err = msg;
    return st;
}

#define HIPCHK(h, expr)                                                                   \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail((h), GABP_E_DEVICE,                                               \
                        std::string(#expr ": ") + hipGetErrorString(e_));                 \
    } while (0)

struct EventPool {
    std::vector<hipEvent_t> ev;
    ~EventPool() { for (auto e : ev) (void)hipEventDestroy(e); }
    hipError_t make(size_t n) {
        while (ev.size() < n) {
            hipEvent_t e;
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return r;
            ev.push_back(e);
        }
        return hipSuccess;
    }
};

float elapsed(hipEvent_t a, hipEvent_t b) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) { (void)hipGetLastError(); return 0.0f; }
    return ms;
}

// One solve, for RBF features (X != nullptr) or a dense kernel (K != nullptr).
gabp_status solve_impl(gabp_svm* h, const float* X, const double* K, const float* y, int64_t N,
                       int64_t m, int32_t mem, hipStream_t s) {
    const double t_start = now_ms();
    const gabp_svm_params& p = h->p;
    h->have_result = false;
    h->resid_valid = false;
    h->err.clear();
    if (!y || N < 1 || (X && m < 1) || (!X && !K)) return fail(h, GABP_E_INVALID, "need N >= 1, m >= 1 and non-NULL inputs");
    if (mem != GABP_MEM_HOST && mem != GABP_MEM_DEVICE) return fail(h, GABP_E_INVALID, "unknown mem kind");
    if (N > (int64_t)TILE * 65535) return fail(h, GABP_E_INVALID, "N too large for 16-bit tile coordinates");
    const bool rbf = (X != nullptr);
    if (rbf && p.kernel != GABP_KERNEL_RBF) return fail(h, GABP_E_INVALID, "gabp_svm_solve needs kernel = RBF");
    if (!rbf && p.kernel != GABP_KERNEL_PRECOMPUTED) return fail(h, GABP_E_INVALID, "gabp_svm_solve_kernel needs kernel = PRECOMPUTED");

    // host-side validation, before any device work
    if (mem == GABP_MEM_HOST) {
        if (rbf) {
            for (int64_t k = 0; k < N * m; ++k)
                if (!std::isfinite(X[k])) return fail(h, GABP_E_INVALID, "X has a non-finite entry");
        } else {
            for (int64_t k = 0; k < N * N; ++k)
                if (!std::isfinite(K[k])) return fail(h, GABP_E_INVALID, "K has a non-finite entry");
        }
        for (int64_t k = 0; k < N; ++k)
            if (!(y[k] == 1.0f || y[k] == -1.0f)) return fail(h, GABP_E_INVALID, "labels must be +1 or -1");
    }

    // ---- plan
    const int prec = p.precision;
    int gram = GRAM_F32;
    if (prec == PREC_FP64) gram = GRAM_F64;
    else if (prec == PREC_MIXED)
        gram = (p.gram == GABP_GRAM_BF16) ? GRAM_BF16 : (p.gram == GABP_GRAM_BF16X3) ? GRAM_BF16X3 : GRAM_BF16X6;
    const int NB = (int)((N + TILE - 1) / TILE);
    const int64_t NPAD = (int64_t)NB * TILE;
    const int64_t nt = n_tiles(NB);
    const int m_pad = rbf ? (int)((m + 15) / 16 * 16) : 16;
    const size_t st_bytes = (prec == PREC_FP64) ? 8 : 4;
    const size_t plane = (size_t)nt * TT * st_bytes;
    const size_t part = (size_t)NB * (NB + 1) * TILE * sizeof(double);
    size_t feat = 0;
    if (rbf) {
        switch (gram) {
            case GRAM_F32: feat = (size_t)NPAD * m_pad * 4; break;
            case GRAM_BF16: feat = (size_t)NPAD * m_pad * 2; break;
            case GRAM_BF16X3: feat = (size_t)NPAD * m_pad * 4; break;
            case GRAM_BF16X6: feat = (size_t)NPAD * m_pad * 6; break;
            default: feat = (size_t)NPAD * m_pad * 8; break;
        }
        feat += (size_t)N * m * 4 + (size_t)NPAD * 4 + (size_t)m * 8;
        if (gram != GRAM_F64 && m + 2 <= 64) feat += (size_t)NPAD * 64 * 6;   // augmented rows (predict)
    } else if (mem == GABP_MEM_HOST) {
        feat = (size_t)N * N * 8;
    }
    const size_t vecs = (size_t)NPAD * 8 * 10 + (size_t)nt * 4 + (size_t)p.max_sweeps * 8 + 4096;
    size_t free_b = 0, total_b = 0;
    HIPCHK(h, hipSetDevice(p.device));
    HIPCHK(h, hipMemGetInfo(&free_b, &total_b));
    const size_t avail = free_b + h->held();
    const size_t budget = p.hbm_budget_bytes ? (size_t)p.hbm_budget_bytes : (size_t)(0.92 * (double)avail);
    const bool can_recompute = rbf && prec != PREC_FP64;
    // candidate plans in order of preference: (materialised K', stored edges) first
    struct Cand { bool kmat, stored; };
    const Cand cands[4] = {{true, true}, {false, true}, {true, false}, {false, false}};
    bool have = false, kmat = true, stored = true;
    size_t need = 0, need_min = SIZE_MAX;
    for (const Cand& c : cands) {
        if (p.kstore == GABP_KSTORE_MATERIALISE && !c.kmat) continue;
        if (p.kstore == GABP_KSTORE_RECOMPUTE && c.kmat) continue;
        if (p.edge_state == GABP_EDGE_STORED && !c.stored) continue;
        if (p.edge_state == GABP_EDGE_STATELESS && c.stored) continue;
        if (!c.kmat && !can_recompute) continue;
        const int R = c.stored ? 1 : 8;
        const size_t n_ = (c.stored ? 4 * plane : 0) + (c.kmat ? plane : 0) + 2 * part + feat + vecs +
                          (size_t)2 * R * NPAD * 8;
        need_min = std::min(need_min, n_);
        if (n_ <= budget) { have = true; kmat = c.kmat; stored = c.stored; need = n_; break; }
    }
    if (need_min == SIZE_MAX)
        return fail(h, GABP_E_INVALID, "no plan matches the requested kstore/edge_state/precision "
                                       "(recompute needs RBF features and FP32 or MIXED precision)");
    if (!have) {
        char msg[256];
        snprintf(msg, sizeof msg, "smallest allowed plan needs %.3f GB, budget %.3f GB", need_min / 1e9, budget / 1e9);
        return fail(h, GABP_E_NOMEM, msg);
    }
    // AUTO edge state with room for stored planes: the choice between stored
    // and stateless waits for the contraction bound computed after the
    // diagonal weighting; the planes are allocated only if stored wins.
    const bool probe = stored && p.edge_state == GABP_EDGE_AUTO;
    const int R = (stored && !probe) ? 1 : 8;
    {
        // buffers of the previous solve are reused where large enough (a
        // repeated solve of the same shape allocates nothing); everything is
        // released first only when the large buffers that must grow do not
        // fit in the free memory
        auto grow = [](const DevBuf& b, size_t n) -> size_t { return (n == 0 || (b.p && b.bytes >= n)) ? 0 : n; };
        const size_t ring = (size_t)R * NPAD * 8;
        size_t extra = grow(h->Kp, kmat ? plane : 0) + 2 * grow(h->partP, part) + grow(h->Pt, ring) +
                       grow(h->S, ring) + feat + vecs;
        if (stored && !probe)
            extra += grow(h->Pf, plane) + grow(h->Pb, plane) + grow(h->Ef, plane) + grow(h->Eb, plane);
        if (extra > free_b) h->release_all();
    }
    const int ksrc = kmat ? KSRC_PLANE : KSRC_RECOMPUTE;

    hipError_t ae = hipSuccess;
    auto A = [&](DevBuf& b, size_t n) { if (ae == hipSuccess) ae = b.ensure(n); };
    A(h->tiles, (size_t)nt * 4);
    const int NBc = (NB + 1) / 2;
    const int64_t nchunks = (int64_t)NBc * (NBc + 1) / 2;
    A(h->chunks, (size_t)nchunks * 4);
    if (kmat) A(h->Kp, plane); else h->Kp.release();
    // pair-record planes: allocated now for a stored plan, on demand after the probe
    if (stored && !probe) { A(h->Pf, plane); A(h->Pb, plane); A(h->Ef, plane); A(h->Eb, plane); }
    else { h->Pf.release(); h->Pb.release(); h->Ef.release(); h->Eb.release(); }
    A(h->partP, part); A(h->partE, part);
    A(h->yd, (size_t)N * 4);
    A(h->kdiag, (size_t)N * 8); A(h->Adiag, (size_t)N * 8); A(h->rowmax, (size_t)N * 8);
    A(h->rsum, (size_t)N * 8);
    A(h->Pt, (size_t)R * NPAD * 8); A(h->S, (size_t)R * NPAD * 8);
    A(h->alpha_d, (size_t)N * 8); A(h->tmp, (size_t)NPAD * 8);
    A(h->blk1, (size_t)(NPAD / WG + 1) * 8); A(h->blk2, (size_t)(NPAD / WG + 1) * 8);
    A(h->one, 64); A(h->status_d, sizeof(DevStatus)); A(h->flag, 64);
    A(h->trace_d, (size_t)p.max_sweeps * 8);
    if (rbf) {
        A(h->Xin, (size_t)N * m * 4); A(h->mean, (size_t)m * 8); A(h->nrm, (size_t)NPAD * 4);
        if (gram == GRAM_F32) A(h->xs32, (size_t)NPAD * m_pad * 4);
        if (gram == GRAM_BF16 || gram == GRAM_BF16X3 || gram == GRAM_BF16X6) A(h->xhi, (size_t)NPAD * m_pad * 2);
        if (gram == GRAM_BF16X3 || gram == GRAM_BF16X6) A(h->xlo, (size_t)NPAD * m_pad * 2);
        if (gram == GRAM_BF16X6) A(h->xlo2, (size_t)NPAD * m_pad * 2);
        if (gram == GRAM_F64) A(h->x64, (size_t)NPAD * m_pad * 8);
    } else if (mem == GABP_MEM_HOST) {
        A(h->Kin, (size_t)N * N * 8);
    }
    if (ae != hipSuccess) {
        h->release_all();
        return fail(h, GABP_E_NOMEM, std::string("device allocation failed: ") + hipGetErrorString(ae));
    }

    EventPool evp;
    const int ce = p.check_every;
    HIPCHK(h, evp.make(6 + 2 * (size_t)ce));
    hipEvent_t* ev = evp.ev.data();
    hipEvent_t* sev = ev + 6;

    // ---- inputs and staging
    HIPCHK(h, hipEventRecord(ev[0], s));
    const float* Xd = nullptr;
    const double* Kd = nullptr;
    if (mem == GABP_MEM_HOST) {
        HIPCHK(h, hipMemcpyAsync(h->yd.p, y, (size_t)N * 4, hipMemcpyHostToDevice, s));
        if (rbf) HIPCHK(h, hipMemcpyAsync(h->Xin.p, X, (size_t)N * m * 4, hipMemcpyHostToDevice, s));
        else HIPCHK(h, hipMemcpyAsync(h->Kin.p, K, (size_t)N * N * 8, hipMemcpyHostToDevice, s));
        Xd = h->Xin.as<float>();
        Kd = h->Kin.as<double>();
    } else {
        HIPCHK(h, hipMemcpyAsync(h->yd.p, y, (size_t)N * 4, hipMemcpyDeviceToDevice, s));
        if (rbf) HIPCHK(h, hipMemcpyAsync(h->Xin.p, X, (size_t)N * m * 4, hipMemcpyDeviceToDevice, s));
        Xd = h->Xin.as<float>();
        Kd = K;
        // device-side validation of device inputs
        HIPCHK(h, hipMemsetAsync(h->flag.p, 0, 4, s));
        HIPCHK(h, launch_validate(rbf ? Xd : nullptr, h->yd.as<float>(), N, rbf ? m : 0, h->flag.as<int32_t>(), s));
        int32_t fl = 0;
        HIPCHK(h, hipMemcpyAsync(&fl, h->flag.p, 4, hipMemcpyDeviceToHost, s));
        HIPCHK(h, hipStreamSynchronize(s));
        if (fl & 1) return fail(h, GABP_E_INVALID, "X has a non-finite entry");
        if (fl & 2) return fail(h, GABP_E_INVALID, "labels must be +1 or -1");
    }
    const double lam = (p.lambda_aug < 0.0) ? 1.0 / (double)N : p.lambda_aug;
    KernelParams kp{};
    kp.N = N;
    kp.NB = NB;
    kp.gamma = p.gamma;
    kp.neg_gamma_log2e = (float)(-p.gamma * 1.4426950408889634);
    kp.lam2 = rbf ? lam * lam : 0.0;
    Features F{};
    F.m_pad = m_pad;
    F.kind = gram;
    if (rbf) {
        if (gram != GRAM_F64) HIPCHK(h, launch_colmean(Xd, N, m, h->mean.as<double>(), s));
        HIPCHK(h, launch_stage(Xd, h->mean.as<double>(), N, m, NPAD, m_pad, gram, h->xs32.as<float>(),
                               h->xhi.as<uint16_t>(), h->xlo.as<uint16_t>(), h->xlo2.as<uint16_t>(),
                               h->x64.as<double>(), h->nrm.as<float>(), s));
        F.f32 = h->xs32.as<float>();
        F.hi = h->xhi.as<uint16_t>();
        F.lo = h->xlo.as<uint16_t>();
        F.lo2 = h->xlo2.as<uint16_t>();
        F.f64 = h->x64.as<double>();
        F.nrm = h->nrm.as<float>();
        // augmented training rows of the decision function: the solve's BF16
        // split kind (three-term split for FP32 handles), up to 62 features
        h->aug_kind = -1;
        h->aug_mp = 0;
        if (gram != GRAM_F64 && m + 2 <= 64) {
            const int ak = (gram == GRAM_F32) ? GRAM_BF16X6 : gram;
            const int amp = (m + 2 <= 32) ? 32 : 64;
            const int anp = (ak == GRAM_BF16X6) ? 3 : (ak == GRAM_BF16X3) ? 2 : 1;
            if (h->xaug.ensure((size_t)NPAD * amp * 2 * anp) == hipSuccess) {
                HIPCHK(h, launch_stage_aug(Xd, h->mean.as<double>(), N, m, NPAD, amp, ak, 1,
                                           (float)(2.0 * p.gamma * 1.4426950408889634), h->xaug.as<uint16_t>(), s));
                h->aug_kind = ak;
                h->aug_mp = amp;
            } else {
                (void)hipGetLastError();
            }
        } else {
            h->xaug.release();
        }
        // K' recomputed per band from augmented rows (the solve's own split
        // kind and width): the Gram of (x, |x|^2, 1) and (c x, -c/2, -c/2 |x|^2)
        // is the exponent, so a K' entry costs a clamped exp2 and an add
        h->xaug0.release();
        if (!kmat && h->aug_kind == gram && h->aug_mp == m_pad) {
            const int anp = (gram == GRAM_BF16X6) ? 3 : (gram == GRAM_BF16X3) ? 2 : 1;
            if (h->xaug0.ensure((size_t)NPAD * m_pad * 2 * anp) == hipSuccess) {
                HIPCHK(h, launch_stage_aug(Xd, h->mean.as<double>(), N, m, NPAD, m_pad, gram, 0, 0.0f,
                                           h->xaug0.as<uint16_t>(), s));
                F.aug0 = h->xaug0.as<uint16_t>();
                F.aug1 = h->xaug.as<uint16_t>();
                F.aug_plane = NPAD * m_pad;
            } else {
                (void)hipGetLastError();
            }
        }
    }
    HIPCHK(h, hipEventRecord(ev[1], s));

    // ---- K' tiles (materialised plan)
    HIPCHK(h, launch_fill_tiles(h->tiles.as<uint32_t>(), NB, s));
    HIPCHK(h, launch_fill_tiles(h->chunks.as<uint32_t>(), NBc, s));
    // FP32-stored K' is built together with the row-sum partials (fused_sums)
    const bool fused_sums = rbf && kmat && gram != GRAM_F64;
    if (rbf) {
        if (fused_sums) {
            // build order: super-blocks of S x S tiles (their 2 S row fragments
            // stay in one XCD's L2); the sweep keeps the row-major list
            const uint32_t* order = h->tiles.as<uint32_t>();
            const int planes = (gram == GRAM_F32) ? 2 : (gram == GRAM_BF16) ? 1 : (gram == GRAM_BF16X3) ? 2 : 3;
            const int64_t frag_bytes = (int64_t)TILE * m_pad * 2 * planes;
            const int S = (int)std::max<int64_t>(4, std::min<int64_t>(16, ((int64_t)1 << 21) / (2 * frag_bytes)));
            size_t ob = 0;
            if (h->sp_tsel.ensure((size_t)nt * 4) == hipSuccess && h->sp_keys.ensure((size_t)nt * 8) == hipSuccess &&
                h->sp_keys2.ensure((size_t)nt * 8) == hipSuccess &&
                sp_tile_order(nullptr, &ob, nullptr, nt, S, NB, nullptr, nullptr, s) == hipSuccess &&
                h->sp_tmp.ensure(ob) == hipSuccess) {
                HIPCHK(h, hipMemcpyAsync(h->sp_tsel.p, h->tiles.p, (size_t)nt * 4, hipMemcpyDeviceToDevice, s));
                HIPCHK(h, sp_tile_order(h->sp_tmp.p, &ob, h->sp_tsel.as<uint32_t>(), nt, S, NB,
                                        h->sp_keys.as<uint64_t>(), h->sp_keys2.as<uint64_t>(), s));
                order = h->sp_tsel.as<uint32_t>();
            }
            HIPCHK(h, launch_gram_sums(F, kp, order, nt, h->Kp.p, NB, h->partP.as<double>(),
                                       h->partE.as<double>(), s));
        }
        else if (kmat)
            HIPCHK(h, launch_gram(F, kp, h->tiles.as<uint32_t>(), nt, h->Kp.p, s));
        HIPCHK(h, launch_fill_value(h->kdiag.as<double>(), N, 1.0 + lam * lam, s));
    } else {
        HIPCHK(h, launch_gather_dense(Kd, kp, h->tiles.as<uint32_t>(), nt, h->Kp.p, prec,
                                      h->kdiag.as<double>(), s));
    }
    HIPCHK(h, hipEventRecord(ev[2], s));

    // ---- diagonal weighting and sweep 0
    if (!fused_sums)
        HIPCHK(h, launch_rowsum(h->Kp.p, prec, ksrc, F, kp, h->tiles.as<uint32_t>(), nt, NB,
                                h->partP.as<double>(), h->partE.as<double>(), s));
    HIPCHK(h, launch_diag(N, NB, h->partP.as<double>(), h->partE.as<double>(), h->kdiag.as<double>(),
                          p.diag_mode, p.C, p.diag_delta, h->Adiag.as<double>(), h->rowmax.as<double>(),
                          h->rsum.as<double>(), h->blk1.as<double>(), h->one.as<double>(), s));
    DevStatus* st = h->status_d.as<DevStatus>();
    const double boxC = (p.box_mode == GABP_BOX_PROJECT) ? p.C : 0.0;
    HIPCHK(h, launch_init(prec, N, NPAD, R, h->Adiag.as<double>(), h->yd.as<float>(), h->Pt.p, h->S.p,
                          h->alpha_d.as<double>(), st, s, boxC));
    HIPCHK(h, hipEventRecord(ev[3], s));

    // ---- plan of the edge state from the contraction bound (rho bounds
    // |A_ij| / Q_ij; stateless_levels_needed and stateless_series_form give
    // the level count and the reciprocal form)
    double rho = INFINITY;
    {
        double hb[2] = {0.0, 0.0};
        HIPCHK(h, launch_rho_bound(N, h->Adiag.as<double>(), h->rowmax.as<double>(), h->rsum.as<double>(),
                                   h->blk1.as<double>(), h->one.as<double>(), s));
        HIPCHK(h, hipMemcpyAsync(hb, h->one.p, 16, hipMemcpyDeviceToHost, s));
        HIPCHK(h, hipStreamSynchronize(s));
        rho = hb[1];
    }
    const double rr = 1.25 * rho;
    const int dneed = stateless_levels_needed(prec, rr);
    bool cur_stored = stored;
    int depth = 0;
    if (probe) cur_stored = dneed > 8;
    // AUTO takes the stateless form only with a depth (<= 8) whose truncation
    // the contraction bound keeps below the message precision; an explicit
    // STATELESS plan with an automatic depth takes at most 8 levels and needs
    // a bound (1.25 rho < 1) to have any; an explicit depth is taken as given.
    // The plan flags every depth below the bound's (stateless_bounded = 0).
    if (!cur_stored && p.stateless_depth == 0 &&
        (p.edge_state == GABP_EDGE_AUTO ? dneed > 8 : !(rr < 1.0))) {
        char msg[320];
        if (p.edge_state == GABP_EDGE_AUTO)
            snprintf(msg, sizeof msg, "stored pair records do not fit the budget (%.3f GB) and the stateless form "
                     "has no truncation bound within 8 levels for this system (contraction bound rho = %.4g)",
                     budget / 1e9, rho);
        else
            snprintf(msg, sizeof msg, "the stateless form has no truncation bound for this system (contraction "
                     "bound rho = %.4g); set stateless_depth to accept an unbounded truncation", rho);
        h->release_all();
        return fail(h, p.edge_state == GABP_EDGE_AUTO ? GABP_E_NOMEM : GABP_E_INVALID, msg);
    }
    if (!cur_stored) depth = (p.stateless_depth > 0) ? p.stateless_depth : std::min(dneed, 8);
    const int ser = cur_stored ? 0 : stateless_series_form(prec, depth, rr);
    if (probe && cur_stored) {
        if (h->Pf.ensure(plane) != hipSuccess || h->Pb.ensure(plane) != hipSuccess ||
            h->Ef.ensure(plane) != hipSuccess || h->Eb.ensure(plane) != hipSuccess) {
            h->release_all();
            return fail(h, GABP_E_NOMEM, "device allocation of the pair-record planes failed");
        }
    }
    if (!cur_stored) { h->Pf.release(); h->Pb.release(); h->Ef.release(); h->Eb.release(); }

    // ---- sweeps
    const size_t agg_bytes = (prec == PREC_FP32) ? 4 : 8;
    const int Rr = cur_stored ? 1 : R;
    // series sweeps: per-node 1/P~ and S/P~ rings, formed by the finalize
    // once per node (without them every tile forms the same quotients)
    void* hinv = nullptr;
    void* hmean = nullptr;
    if (ser > 0 && h->HI.ensure((size_t)Rr * NPAD * agg_bytes) == hipSuccess &&
        h->HM.ensure((size_t)Rr * NPAD * agg_bytes) == hipSuccess) {
        hinv = h->HI.p;
        hmean = h->HM.p;
        HIPCHK(h, launch_ring_recip(prec, NPAD, Rr, h->Pt.p, h->S.p, hinv, hmean, s));
    } else {
        (void)hipGetLastError();
        h->HI.release(); h->HM.release();
    }
    SweepArgs sa{};
    sa.tiles = h->tiles.as<uint32_t>();
    sa.ntiles = nt;
    sa.NB = NB;
    sa.Kp = h->Kp.p;
    sa.Pf = h->Pf.p; sa.Pb = h->Pb.p; sa.Ef = h->Ef.p; sa.Eb = h->Eb.p;
    sa.HP = h->Pt.p; sa.HS = h->S.p;
    sa.HI = hinv; sa.HM = hmean;
    sa.NPAD = NPAD;
    sa.R = Rr;
    // the FP32-message form (MIXED, series reciprocals) sums each tile's
    // messages in FP32; its partial sums are kept in FP32 (half the traffic)
    sa.part32 = (prec == PREC_MIXED && !cur_stored && ser > 0) ? 1 : 0;
    sa.partP = h->partP.p; sa.partE = h->partE.p;
    // synchronous stateless sweeps over an FP32 K' plane with FP32 partial
    // sums run over 2 x 2 chunks of tiles (half the partial-sum stores); the
    // finalize then reads NBc + 1 slots per block
    const bool chunked = p.schedule != GABP_SCHED_GROUPED && kmat && !cur_stored &&
                         chunk_sweep(prec == PREC_FP32 || sa.part32, depth, ser, NB, p.tile_chunk);
    sa.chunks = h->chunks.as<uint32_t>();
    sa.nchunks = nchunks;
    sa.chunk = chunked ? 2 : 1;
    const int nslot = chunked ? NBc : NB;
    sa.st = st;
    sa.F = F;
    sa.kp = kp;
    StopRule rule{p.tol_abs, p.tol_rel, p.stagnation_rel, p.max_sweeps, p.stagnation_window};
    const int nblk = (int)((N + WG - 1) / WG);

    // grouped schedule: groups of whole block rows, block I in group I G / NB;
    // per group the single-direction entries (stateless: every message into
    // the group; stored: the tiles crossing the group boundary) and, for
    // stored records, the tiles inside the group
    const bool grouped = p.schedule == GABP_SCHED_GROUPED;
    const int G = grouped ? std::min(p.sched_groups > 0 ? p.sched_groups : 16, NB) : 1;
    std::vector<int64_t> g_within_off(G + 1, 0), g_dir_off(G + 1, 0), g_b0(G + 1, 0);
    if (grouped) {
        auto grp = [&](int I) { return (int)((int64_t)I * G / NB); };
        std::vector<std::vector<uint32_t>> wl(G), dl(G);
        for (int I = 0; I < NB; ++I)
            for (int J = I; J < NB; ++J) {
                const uint32_t k = (uint32_t)tile_index(I, J, NB);
                const int gi = grp(I), gj = grp(J);
                if (cur_stored) {
                    if (gi == gj) wl[gi].push_back(k);
                    else { dl[gj].push_back(k); dl[gi].push_back(k | GE_BWD); }
                } else {
                    const uint32_t in = (gi == gj) ? GE_WITHIN : 0u;
                    dl[gj].push_back(k | in);
                    dl[gi].push_back(k | GE_BWD | in);
                }
            }
        std::vector<uint32_t> flat;
        for (int g = 0; g < G; ++g) {
            g_within_off[g] = (int64_t)flat.size();
            flat.insert(flat.end(), wl[g].begin(), wl[g].end());
            g_within_off[g + 1] = (int64_t)flat.size();
        }
        const int64_t nwithin_all = (int64_t)flat.size();
        for (int g = 0; g < G; ++g) {
            g_dir_off[g] = (int64_t)flat.size();
            flat.insert(flat.end(), dl[g].begin(), dl[g].end());
        }
        g_dir_off[G] = (int64_t)flat.size();
        (void)nwithin_all;
        int gcur = 0;
        for (int I = 0; I < NB; ++I)
            while (gcur <= G && grp(I) >= gcur) g_b0[gcur++] = I;
        while (gcur <= G) g_b0[gcur++] = NB;
        if (h->glist.ensure(flat.size() * 4) != hipSuccess) {
            h->release_all();
            return fail(h, GABP_E_NOMEM, "device allocation of the group lists failed");
        }
        HIPCHK(h, hipMemcpyAsync(h->glist.p, flat.data(), flat.size() * 4, hipMemcpyHostToDevice, s));
        // stored records: a visit reads the reverse message before any
        // sweep has written it, so the planes start at zero
        if (cur_stored)
            for (DevBuf* pl : {&h->Pf, &h->Pb, &h->Ef, &h->Eb})
                HIPCHK(h, hipMemsetAsync(pl->p, 0, plane, s));
        HIPCHK(h, hipStreamSynchronize(s));
    }
    DevStatus hs{};
    double sweep_kernel_ms = 0.0;
    int64_t launches = 0;
    int polled = 0;
    for (int t = 0; t < p.max_sweeps; ++t) {
        const int slot = t % ce;
        sa.slot_top = t % Rr;
        // every stateless sweep unrolls `depth` levels: the ring slots before
        // sweep 0 hold P~ = inf, S = 0, whose messages are exactly zero
        sa.levels = cur_stored ? 0 : depth;
        char* wP = static_cast<char*>(h->Pt.p) + (size_t)((t + 1) % Rr) * NPAD * agg_bytes;
        char* wS = static_cast<char*>(h->S.p) + (size_t)((t + 1) % Rr) * NPAD * agg_bytes;
        char* wI = hinv ? static_cast<char*>(hinv) + (size_t)((t + 1) % Rr) * NPAD * agg_bytes : nullptr;
        char* wM = hmean ? static_cast<char*>(hmean) + (size_t)((t + 1) % Rr) * NPAD * agg_bytes : nullptr;
        if (!grouped) {
            // the events take the sweep dispatch's own timestamps
            HIPCHK(h, launch_sweep(prec, ksrc, gram, sa.levels, t == 0, ser, sa, s,
                                   p.time_sweeps ? sev[2 * slot] : nullptr, p.time_sweeps ? sev[2 * slot + 1] : nullptr));
            HIPCHK(h, launch_finalize(prec, N, nslot, h->partP.p, h->partE.p, h->Adiag.as<double>(),
                                      h->yd.as<float>(), wP, wS, h->alpha_d.as<double>(),
                                      h->blk1.as<double>(), h->blk2.as<double>(), st, s, boxC, wI, wM,
                                      sa.part32));
        } else {
            // one visit per group: its messages, then its aggregates (the
            // timed span covers the visits and their group finalizes)
            if (p.time_sweeps) HIPCHK(h, hipEventRecord(sev[2 * slot], s));
            const uint32_t* gl = h->glist.as<uint32_t>();
            for (int g = 0; g < G; ++g) {
                HIPCHK(h, launch_sweep_grouped(prec, ksrc, gram, sa.levels, ser, sa, gl + g_within_off[g],
                                               (int)(g_within_off[g + 1] - g_within_off[g]), gl + g_dir_off[g],
                                               (int)(g_dir_off[g + 1] - g_dir_off[g]), t, s));
                const int64_t b0 = g_b0[g], b1 = std::min<int64_t>(g_b0[g + 1], nblk);
                HIPCHK(h, launch_finalize_range(prec, b0, b1 - b0, N, NB, h->partP.p, h->partE.p,
                                                h->Adiag.as<double>(), h->yd.as<float>(), wP, wS,
                                                h->alpha_d.as<double>(), h->blk1.as<double>(),
                                                h->blk2.as<double>(), st, s, boxC, wI, wM, sa.part32));
            }
            if (p.time_sweeps) HIPCHK(h, hipEventRecord(sev[2 * slot + 1], s));
        }
        HIPCHK(h, launch_status(nblk, h->blk1.as<double>(), h->blk2.as<double>(), st,
                                h->trace_d.as<double>(), rule, s));
        if ((t + 1) % ce == 0 || t + 1 == p.max_sweeps) {
            HIPCHK(h, hipMemcpyAsync(&hs, st, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
            HIPCHK(h, hipStreamSynchronize(s));
            if (p.time_sweeps) {
                for (int u = polled; u <= t; ++u) {
                    if (u >= hs.t) break;
                    sweep_kernel_ms += elapsed(sev[2 * (u % ce)], sev[2 * (u % ce) + 1]);
                    ++launches;
                }
            }
            polled = t + 1;
            if (hs.done) break;
        }
    }
    stored = cur_stored;
    HIPCHK(h, hipEventRecord(ev[4], s));
    const int final_slot = std::max(hs.t, 0) % (stored ? 1 : R);

    // ---- outputs
    h->alpha.assign((size_t)N, 0.0);
    h->ptilde.assign((size_t)N, 0.0);
    h->adiag.assign((size_t)N, 0.0);
    h->yh.assign((size_t)N, 0.0f);
    HIPCHK(h, launch_convert_agg(prec, static_cast<char*>(h->Pt.p) + (size_t)final_slot * NPAD * agg_bytes,
                                 h->tmp.as<double>(), N, s));
    HIPCHK(h, hipMemcpyAsync(h->alpha.data(), h->alpha_d.p, (size_t)N * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipMemcpyAsync(h->ptilde.data(), h->tmp.p, (size_t)N * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipMemcpyAsync(h->adiag.data(), h->Adiag.p, (size_t)N * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipMemcpyAsync(h->yh.data(), h->yd.p, (size_t)N * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipMemcpyAsync(&hs, st, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipEventRecord(ev[5], s));
    HIPCHK(h, hipStreamSynchronize(s));
    h->trace.assign((size_t)std::max(hs.t, 0), 0.0);
    if (hs.t > 0)
        HIPCHK(h, hipMemcpy(h->trace.data(), h->trace_d.p, (size_t)hs.t * 8, hipMemcpyDeviceToHost));

    h->N = N; h->m = rbf ? m : 0; h->NB = NB; h->NPAD = NPAD; h->ntiles = nt; h->m_pad = m_pad;
    h->prec = prec; h->gram = gram; h->lam = lam; h->rbf = rbf;
    h->sweeps = hs.t;
    h->delta = hs.delta;
    h->reason = hs.reason;
    switch (hs.reason) {
        case R_CONVERGED: case R_STAGNATED: h->status = GABP_OK; break;
        case R_DIVERGED: h->status = GABP_E_DIVERGED; break;
        default: h->status = GABP_E_NOT_CONVERGED; break;
    }
    h->tm = gabp_timings{};
    h->tm.stage_ms = elapsed(ev[0], ev[1]);
    h->tm.kbuild_ms = elapsed(ev[1], ev[2]);
    h->tm.diag_ms = elapsed(ev[2], ev[3]);
    h->tm.sweep_loop_ms = elapsed(ev[3], ev[4]);
    h->tm.sweep_kernel_ms = sweep_kernel_ms;
    h->tm.sweep_launches = launches;
    h->tm.d2h_ms = elapsed(ev[4], ev[5]);
    h->tm.total_ms = now_ms() - t_start;
    h->plan = gabp_plan{};
    h->plan.precision = prec;
    h->plan.kstore = kmat ? GABP_KSTORE_MATERIALISE : GABP_KSTORE_RECOMPUTE;
    h->plan.edge_state = stored ? GABP_EDGE_STORED : GABP_EDGE_STATELESS;
    h->plan.gram = (gram == GRAM_BF16X6) ? GABP_GRAM_BF16X6 : (gram == GRAM_BF16X3) ? GABP_GRAM_BF16X3
                 : (gram == GRAM_BF16 ? GABP_GRAM_BF16 : GABP_GRAM_AUTO);
    h->plan.tile = TILE;
    h->plan.stateless_depth = depth;
    h->plan.stateless_bounded = stored ? 1 : (depth >= dneed ? 1 : 0);
    h->plan.stateless_rho = rho;
    h->plan.series_reciprocal = ser;
    h->plan.tile_chunk = chunked ? 2 : 1;
    h->plan.recompute_aug = (!kmat && h->xaug0.p) ? 1 : 0;
    h->plan.sched_groups = grouped ? G : 0;
    h->plan.n_blocks = NB;
    h->plan.n_tiles = nt;
    h->plan.device_bytes = h->held();
    h->plan.alg_bytes_per_pair = (double)st_bytes * ((stored ? 8.0 : 0.0) + (kmat ? 1.0 : 0.0));
    h->plan.alg_bytes_per_sweep = (uint64_t)((double)N * (double)(N - 1) / 2.0 * h->plan.alg_bytes_per_pair);
    h->sparse = false;
    h->n_edges = 0;
    h->have_result = true;
    if (h->status != GABP_OK) {
        h->err = (h->status == GABP_E_DIVERGED) ? "GaBP diverged: a cavity precision became <= 0 or non-finite"
                                                : "max_sweeps reached before the stop rule held";
    }
    return (gabp_status)h->status;
}

// Residual certificate of the last dense solve (subsection "GaBP Algorithm
// Convergence": under diagonal dominance, Varah's bound turns the residual
// into an error bound): ||1 - A alpha||_inf over all N rows, one pass over K'
// (the plane, or K' recomputed per band as in the sweep) with FP64 sums in a
// fixed order, min_i (A_ii - r_i) and their quotient.  alpha is the solver's
// own (before any output clipping).  The handle's work buffers of the solve
// (partial sums, block maxima) are reused.
gabp_status residual_certificate(gabp_svm* h) {
    if (h->sparse) return fail(h, GABP_E_STATE, "the residual certificate is defined for dense solves");
    HIPCHK(h, hipSetDevice(h->p.device));
    const bool kmat = h->plan.kstore == GABP_KSTORE_MATERIALISE;
    Features F{};
    F.f32 = h->xs32.as<float>(); F.hi = h->xhi.as<uint16_t>(); F.lo = h->xlo.as<uint16_t>();
    F.lo2 = h->xlo2.as<uint16_t>(); F.f64 = h->x64.as<double>(); F.nrm = h->nrm.as<float>();
    F.m_pad = h->m_pad; F.kind = h->gram;
    if (h->xaug0.p) {   // the solve's K' came from the augmented rows
        F.aug0 = h->xaug0.as<uint16_t>();
        F.aug1 = h->xaug.as<uint16_t>();
        F.aug_plane = h->NPAD * h->m_pad;
    }
    KernelParams kp{};
    kp.N = h->N;
    kp.NB = h->NB;
    kp.gamma = h->p.gamma;
    kp.neg_gamma_log2e = (float)(-h->p.gamma * 1.4426950408889634);
    kp.lam2 = h->rbf ? h->lam * h->lam : 0.0;
    hipStream_t s = nullptr;
    HIPCHK(h, launch_residual(h->Kp.p, h->prec, kmat ? KSRC_PLANE : KSRC_RECOMPUTE, F, kp, h->tiles.as<uint32_t>(),
                              h->ntiles, h->NB, h->N, h->NPAD, h->alpha_d.as<double>(), h->yd.as<float>(),
                              h->Adiag.as<double>(), h->rsum.as<double>(), h->tmp.as<double>(),
                              h->partP.as<double>(), h->blk1.as<double>(), h->blk2.as<double>(),
                              h->one.as<double>(), s));
    HIPCHK(h, hipMemcpyAsync(h->resid, h->one.p, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    h->resid_valid = true;
    return GABP_OK;
}

// Sparsified RBF kernel: graph build on the device, then synchronous GaBP on
// the kept pairs with stored records per edge (see gabp_sparse.hip).
gabp_status solve_sparse_impl(gabp_svm* h, const float* X, const float* y, int64_t N, int64_t m, int32_t mem,
                              hipStream_t s) {
    const double t_start = now_ms();
    h->have_result = false;
    h->resid_valid = false;
    h->status = GABP_E_STATE;
    const gabp_svm_params& p = h->p;
    if (N < 1 || m < 1 || !y) return fail(h, GABP_E_INVALID, "N >= 1, m >= 1 and y are required");
    if (mem != GABP_MEM_HOST && mem != GABP_MEM_DEVICE) return fail(h, GABP_E_INVALID, "unknown mem kind");
    if (N > (int64_t)TILE * 65535) return fail(h, GABP_E_INVALID, "N too large for 16-bit tile coordinates");
    if (mem == GABP_MEM_HOST) {
        for (int64_t k = 0; k < N * m; ++k)
            if (!std::isfinite(X[k])) return fail(h, GABP_E_INVALID, "X has a non-finite entry");
        for (int64_t k = 0; k < N; ++k)
            if (!(y[k] == 1.0f || y[k] == -1.0f)) return fail(h, GABP_E_INVALID, "labels must be +1 or -1");
    }
    const int prec = p.precision;
    const int gram = (prec == PREC_FP32) ? GRAM_F32
                   : (p.gram == GABP_GRAM_BF16) ? GRAM_BF16 : (p.gram == GABP_GRAM_BF16X3) ? GRAM_BF16X3 : GRAM_BF16X6;
    const int NB = (int)((N + TILE - 1) / TILE);
    const int64_t NPAD = (int64_t)NB * TILE;
    const int64_t nt = n_tiles(NB);
    // two augmented columns carry the norms (the build's Gram is -d^2 / 2)
    const int m_pad = (int)((m + 2 + 15) / 16 * 16);
    const size_t agg = (prec == PREC_FP32) ? 4 : 8;
    const double lam = (p.lambda_aug < 0.0) ? 1.0 / (double)N : p.lambda_aug;
    const double cut = -std::log(p.sparse_tau) / p.gamma;
    HIPCHK(h, hipSetDevice(p.device));
    h->release_all();

    hipError_t ae = hipSuccess;
    auto A = [&](DevBuf& b, size_t n) { if (ae == hipSuccess) ae = b.ensure(std::max<size_t>(n, 16)); };
    A(h->tiles, (size_t)nt * 4);
    A(h->Xin, (size_t)N * m * 4); A(h->mean, (size_t)m * 8); A(h->nrm, (size_t)NPAD * 4);
    if (gram == GRAM_F32) A(h->xs32, (size_t)NPAD * m_pad * 4);
    else {
        A(h->xhi, (size_t)NPAD * m_pad * 2);
        if (gram != GRAM_BF16) A(h->xlo, (size_t)NPAD * m_pad * 2);
        if (gram == GRAM_BF16X6) A(h->xlo2, (size_t)NPAD * m_pad * 2);
    }
    // the B rows of the build: every plane of the kind, one after the other
    const int planes = (gram == GRAM_F32) ? 2 : (gram == GRAM_BF16) ? 1 : (gram == GRAM_BF16X3) ? 2 : 3;
    const size_t plane_b = (size_t)NPAD * m_pad * 2;
    A(h->sp_xb, plane_b * planes);
    A(h->yd, (size_t)N * 4);
    A(h->sp_cnt, (size_t)(nt / 32 + 1) * 4); A(h->sp_toff, (size_t)(nt / 32 + 1) * 8);   // sampled tiles
    A(h->partP, (size_t)NPAD * 8); A(h->partE, (size_t)NPAD * 8);
    A(h->kdiag, (size_t)N * 8); A(h->Adiag, (size_t)N * 8); A(h->rowmax, (size_t)N * 8);
    A(h->rsum, (size_t)N * 8);
    A(h->Pt, (size_t)NPAD * 8); A(h->S, (size_t)NPAD * 8);
    A(h->alpha_d, (size_t)N * 8); A(h->tmp, (size_t)NPAD * 8);
    A(h->blk1, (size_t)(NPAD / WG + 1) * 8); A(h->blk2, (size_t)(NPAD / WG + 1) * 8);
    A(h->one, 64); A(h->status_d, sizeof(DevStatus)); A(h->flag, 64);
    A(h->trace_d, (size_t)p.max_sweeps * 8);
    A(h->sp_degi, (size_t)(N + 1) * 4); A(h->sp_degj, (size_t)(N + 1) * 4);
    A(h->sp_offi, (size_t)(N + 1) * 8); A(h->sp_offj, (size_t)(N + 1) * 8);
    A(h->sp_order, (size_t)N * 4); A(h->sp_Xp, (size_t)N * m * 4);
    A(h->sp_cent, (size_t)NB * m * 8); A(h->sp_rad, (size_t)NB * 8);
    A(h->sp_keep, (size_t)nt); A(h->sp_tsel, (size_t)nt * 4);
    A(h->sp_nsel, 16);   // [0] tiles selected by the pruning, [1] the fill cursor
    if (ae != hipSuccess) {
        h->release_all();
        return fail(h, GABP_E_NOMEM, std::string("device allocation failed: ") + hipGetErrorString(ae));
    }
    EventPool evp;
    const int ce = p.check_every;
    HIPCHK(h, evp.make(6 + 2 * (size_t)ce));
    hipEvent_t* ev = evp.ev.data();
    hipEvent_t* sev = ev + 6;

    // ---- inputs and staging (as the dense RBF solve)
    HIPCHK(h, hipEventRecord(ev[0], s));
    const hipMemcpyKind kind = (mem == GABP_MEM_HOST) ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    HIPCHK(h, hipMemcpyAsync(h->yd.p, y, (size_t)N * 4, kind, s));
    HIPCHK(h, hipMemcpyAsync(h->Xin.p, X, (size_t)N * m * 4, kind, s));
    const float* Xd = h->Xin.as<float>();
    if (mem == GABP_MEM_DEVICE) {
        HIPCHK(h, hipMemsetAsync(h->flag.p, 0, 4, s));
        HIPCHK(h, launch_validate(Xd, h->yd.as<float>(), N, m, h->flag.as<int32_t>(), s));
        int32_t fl = 0;
        HIPCHK(h, hipMemcpyAsync(&fl, h->flag.p, 4, hipMemcpyDeviceToHost, s));
        HIPCHK(h, hipStreamSynchronize(s));
        if (fl & 1) return fail(h, GABP_E_INVALID, "X has a non-finite entry");
        if (fl & 2) return fail(h, GABP_E_INVALID, "labels must be +1 or -1");
    }
    // locality order: nearest of K evenly spaced landmark points, then sort
    // by (landmark, input index); every later step works on the reordered
    // points, and the outputs go back to input order
    const int K = (int)std::max<int64_t>(1, std::min<int64_t>(4096, N / 2048));
    {
        std::vector<int32_t> lm((size_t)K);
        for (int k = 0; k < K; ++k) lm[(size_t)k] = (int32_t)((int64_t)k * N / K);
        if (h->sp_ids.ensure((size_t)N * 4) != hipSuccess || h->sp_perm.ensure((size_t)K * 4) != hipSuccess ||
            h->sp_keys.ensure((size_t)N * 8) != hipSuccess || h->sp_keys2.ensure((size_t)N * 8) != hipSuccess) {
            h->release_all();
            return fail(h, GABP_E_NOMEM, "device allocation of the ordering arrays failed");
        }
        HIPCHK(h, hipMemcpyAsync(h->sp_perm.p, lm.data(), (size_t)K * 4, hipMemcpyHostToDevice, s));
        HIPCHK(h, launch_sp_order(Xd, N, m, h->sp_perm.as<int32_t>(), K, h->sp_keys.as<uint64_t>(),
                                  h->sp_ids.as<int32_t>(), s));
        size_t ob = 0;
        HIPCHK(h, sp_sort_ids(nullptr, &ob, h->sp_keys.as<uint64_t>(), h->sp_keys2.as<uint64_t>(),
                              h->sp_ids.as<int32_t>(), h->sp_order.as<int32_t>(), N, s));
        if (h->sp_tmp.ensure(ob) != hipSuccess) { h->release_all(); return fail(h, GABP_E_NOMEM, "sort storage"); }
        HIPCHK(h, sp_sort_ids(h->sp_tmp.p, &ob, h->sp_keys.as<uint64_t>(), h->sp_keys2.as<uint64_t>(),
                              h->sp_ids.as<int32_t>(), h->sp_order.as<int32_t>(), N, s));
        // labels in the new order go to yd (the sweep's b); the input order stays in Xin / the caller's y
        HIPCHK(h, hipMemcpyAsync(h->tmp.p, h->yd.p, (size_t)N * 4, hipMemcpyDeviceToDevice, s));
        HIPCHK(h, launch_sp_permute(Xd, h->tmp.as<float>(), N, m, h->sp_order.as<int32_t>(), h->sp_Xp.as<float>(),
                                    h->yd.as<float>(), s));
    }
    const float* Xp = h->sp_Xp.as<float>();
    Features F{};
    F.m_pad = m_pad;
    F.kind = gram;
    HIPCHK(h, launch_colmean(Xp, N, m, h->mean.as<double>(), s));
    HIPCHK(h, launch_stage(Xp, h->mean.as<double>(), N, m, NPAD, m_pad, gram, h->xs32.as<float>(),
                           h->xhi.as<uint16_t>(), h->xlo.as<uint16_t>(), h->xlo2.as<uint16_t>(), nullptr,
                           h->nrm.as<float>(), s));
    F.f32 = h->xs32.as<float>(); F.hi = h->xhi.as<uint16_t>(); F.lo = h->xlo.as<uint16_t>();
    F.lo2 = h->xlo2.as<uint16_t>(); F.nrm = h->nrm.as<float>();
    // augmented rows: A = (x, n, 1) in place, B = (x, -1/2, -n/2) in sp_xb
    Features FB = F;
    {
        uint16_t* b16 = h->sp_xb.as<uint16_t>();
        float* bf = h->sp_xb.as<float>();
        uint16_t* bhi = b16;
        uint16_t* blo = (planes >= 2) ? b16 + plane_b / 2 : nullptr;
        uint16_t* blo2 = (planes >= 3) ? b16 + plane_b : nullptr;
        HIPCHK(h, launch_sp_augment(NPAD, m, m_pad, gram, h->nrm.as<float>(), h->xs32.as<float>(),
                                    h->xhi.as<uint16_t>(), h->xlo.as<uint16_t>(), h->xlo2.as<uint16_t>(), bf, bhi,
                                    blo, blo2, s));
        FB.f32 = bf; FB.hi = bhi; FB.lo = blo; FB.lo2 = blo2;
    }
    HIPCHK(h, hipEventRecord(ev[1], s));

    // ---- graph: count per tile, offsets, fill, sort by (i, j), transposed order
    HIPCHK(h, launch_fill_tiles(h->tiles.as<uint32_t>(), NB, s));
    // tiles that may hold kept pairs (the others are provably beyond the cut)
    HIPCHK(h, launch_sp_prune(Xp, N, m, NB, h->tiles.as<uint32_t>(), nt, cut, h->sp_cent.as<double>(),
                              h->sp_rad.as<double>(), h->sp_keep.as<uint8_t>(), s));
    size_t pb = 0;
    HIPCHK(h, sp_select(nullptr, &pb, h->tiles.as<uint32_t>(), h->sp_keep.as<uint8_t>(), h->sp_tsel.as<uint32_t>(),
                        h->sp_nsel.as<int64_t>(), nt, s));
    if (h->sp_tmp.ensure(pb) != hipSuccess) { h->release_all(); return fail(h, GABP_E_NOMEM, "select storage"); }
    HIPCHK(h, sp_select(h->sp_tmp.p, &pb, h->tiles.as<uint32_t>(), h->sp_keep.as<uint8_t>(), h->sp_tsel.as<uint32_t>(),
                        h->sp_nsel.as<int64_t>(), nt, s));
    int64_t nts = 0;
    HIPCHK(h, hipMemcpyAsync(&nts, h->sp_nsel.p, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    // super-blocked tile order: S x S tiles share 2 S row fragments, sized to
    // stay well inside one XCD's L2
    if (nts > 0) {
        const int64_t frag_bytes = (int64_t)TILE * m_pad * 2 * planes;
        const int S = (int)std::max<int64_t>(4, std::min<int64_t>(16, ((int64_t)1 << 21) / (2 * frag_bytes)));
        A(h->sp_keys, (size_t)nts * 8); A(h->sp_keys2, (size_t)nts * 8);
        if (ae != hipSuccess) { h->release_all(); return fail(h, GABP_E_NOMEM, "tile order storage"); }
        size_t ob = 0;
        HIPCHK(h, sp_tile_order(nullptr, &ob, h->sp_tsel.as<uint32_t>(), nts, S, NB, h->sp_keys.as<uint64_t>(),
                                h->sp_keys2.as<uint64_t>(), s));
        if (h->sp_tmp.ensure(ob) != hipSuccess) { h->release_all(); return fail(h, GABP_E_NOMEM, "sort storage"); }
        HIPCHK(h, sp_tile_order(h->sp_tmp.p, &ob, h->sp_tsel.as<uint32_t>(), nts, S, NB, h->sp_keys.as<uint64_t>(),
                                h->sp_keys2.as<uint64_t>(), s));
    }
    const uint32_t* tsel = h->sp_tsel.as<uint32_t>();
    const float cutf = (float)cut;
    const float c = (float)(-p.gamma * 1.4426950408889634);
    int64_t E = 0;
    size_t tb = 0;
    if (nts > 0) {
        // capacity of the fill's output: the caller's hint, else 1.5 x the
        // kept pairs of every 32nd tile scaled to all tiles, plus 2^20; a
        // capacity that falls short costs a second fill pass, never a
        // different graph
        const int64_t emax = ((int64_t)1 << 31) - 1;
        int64_t cap = p.sparse_edges_hint;
        if (cap == 0) {
            const int64_t stride = 32, ns = (nts + stride - 1) / stride;
            HIPCHK(h, launch_sp_count(F, FB, tsel, ns, stride, N, cutf, h->sp_cnt.as<int32_t>(), s));
            HIPCHK(h, sp_scan(nullptr, &tb, h->sp_cnt.as<int32_t>(), h->sp_toff.as<int64_t>(), ns, s));
            if (h->sp_tmp.ensure(tb) != hipSuccess) { h->release_all(); return fail(h, GABP_E_NOMEM, "scan storage"); }
            HIPCHK(h, sp_scan(h->sp_tmp.p, &tb, h->sp_cnt.as<int32_t>(), h->sp_toff.as<int64_t>(), ns, s));
            int64_t last_off = 0;
            int32_t last_cnt = 0;
            HIPCHK(h, hipMemcpyAsync(&last_off, h->sp_toff.as<int64_t>() + (ns - 1), 8, hipMemcpyDeviceToHost, s));
            HIPCHK(h, hipMemcpyAsync(&last_cnt, h->sp_cnt.as<int32_t>() + (ns - 1), 4, hipMemcpyDeviceToHost, s));
            HIPCHK(h, hipStreamSynchronize(s));
            const double est = (double)(last_off + last_cnt) * ((double)nts / (double)ns);
            cap = std::min<int64_t>(emax, (int64_t)(1.5 * est) + ((int64_t)1 << 20));
        }
        unsigned long long* cursor = reinterpret_cast<unsigned long long*>(h->sp_nsel.as<int64_t>() + 1);
        for (int pass = 0; pass < 2; ++pass) {
            A(h->sp_keys, (size_t)cap * 8); A(h->sp_kv, (size_t)cap * 4);
            if (ae != hipSuccess) {
                h->release_all();
                return fail(h, GABP_E_NOMEM, std::string("device allocation of the edge list failed: ") +
                                                 hipGetErrorString(ae));
            }
            HIPCHK(h, hipMemsetAsync(cursor, 0, 8, s));
            HIPCHK(h, launch_sp_fill(F, FB, tsel, nts, N, cutf, c, (float)(lam * lam), cap, cursor,
                                     h->sp_keys.as<uint64_t>(), h->sp_kv.as<float>(), s));
            unsigned long long total = 0;
            HIPCHK(h, hipMemcpyAsync(&total, cursor, 8, hipMemcpyDeviceToHost, s));
            HIPCHK(h, hipStreamSynchronize(s));
            if ((int64_t)total > emax) return fail(h, GABP_E_INVALID, "more than 2^31 - 1 kept pairs: raise sparse_tau");
            if ((int64_t)total <= cap) { E = (int64_t)total; break; }
            if (pass == 1) return fail(h, GABP_E_DEVICE, "two fill passes of the sparse graph disagree");
            cap = (int64_t)total;
        }
    }
    const size_t st_bytes = 4;   // records and K' per edge in FP32 storage
    A(h->sp_keys, (size_t)E * 8); A(h->sp_keys2, (size_t)E * 8);
    A(h->sp_kv, (size_t)E * 4); A(h->sp_kv2, (size_t)E * 4);
    A(h->sp_ei, (size_t)E * 4); A(h->sp_ej, (size_t)E * 4);
    A(h->sp_ids, (size_t)std::max(E, N) * 4); A(h->sp_perm, (size_t)E * 4);
    // records: (P, E) pairs per edge and direction; packed aggregates
    A(h->Pf, (size_t)2 * E * st_bytes); A(h->Pb, (size_t)2 * E * st_bytes);
    A(h->Ef, (size_t)2 * NPAD * 8);
    if (ae != hipSuccess) {
        h->release_all();
        return fail(h, GABP_E_NOMEM, std::string("device allocation of the edge arrays failed: ") +
                                         hipGetErrorString(ae));
    }
    size_t sb = 0, sb2 = 0;
    HIPCHK(h, sp_sort_keys(nullptr, &sb, h->sp_keys.as<uint64_t>(), h->sp_keys2.as<uint64_t>(), h->sp_kv.as<float>(),
                           h->sp_kv2.as<float>(), E, s));
    HIPCHK(h, sp_sort_ids(nullptr, &sb2, h->sp_keys.as<uint64_t>(), h->sp_keys2.as<uint64_t>(),
                          h->sp_ids.as<int32_t>(), h->sp_perm.as<int32_t>(), E, s));
    size_t sb3 = 0;
    HIPCHK(h, sp_scan(nullptr, &sb3, h->sp_degi.as<int32_t>(), h->sp_offi.as<int64_t>(), N + 1, s));
    if (h->sp_tmp.ensure(std::max(std::max(sb, sb2), std::max(sb3, tb))) != hipSuccess) {
        h->release_all();
        return fail(h, GABP_E_NOMEM, "sort storage");
    }
    // edges in (i, j) order: keys2 / kv2 (K' per edge from here on)
    HIPCHK(h, sp_sort_keys(h->sp_tmp.p, &sb, h->sp_keys.as<uint64_t>(), h->sp_keys2.as<uint64_t>(),
                           h->sp_kv.as<float>(), h->sp_kv2.as<float>(), E, s));
    HIPCHK(h, hipMemsetAsync(h->sp_degi.p, 0, (size_t)(N + 1) * 4, s));
    HIPCHK(h, hipMemsetAsync(h->sp_degj.p, 0, (size_t)(N + 1) * 4, s));
    // ends and degrees; keys of the transposed order (j, i) into keys
    HIPCHK(h, launch_sp_unpack(h->sp_keys2.as<uint64_t>(), E, h->sp_ei.as<int32_t>(), h->sp_ej.as<int32_t>(),
                               h->sp_degi.as<int32_t>(), h->sp_degj.as<int32_t>(), h->sp_keys.as<uint64_t>(),
                               h->sp_ids.as<int32_t>(), s));
    // perm: edge ids in (j, i) order
    HIPCHK(h, sp_sort_ids(h->sp_tmp.p, &sb2, h->sp_keys.as<uint64_t>(), h->sp_keys2.as<uint64_t>(),
                          h->sp_ids.as<int32_t>(), h->sp_perm.as<int32_t>(), E, s));
    HIPCHK(h, sp_scan(h->sp_tmp.p, &sb3, h->sp_degi.as<int32_t>(), h->sp_offi.as<int64_t>(), N + 1, s));
    HIPCHK(h, sp_scan(h->sp_tmp.p, &sb3, h->sp_degj.as<int32_t>(), h->sp_offj.as<int64_t>(), N + 1, s));
    HIPCHK(h, hipEventRecord(ev[2], s));

    // ---- diagonal weighting from the sparse row sums (one partial per node)
    HIPCHK(h, hipMemsetAsync(h->partP.p, 0, (size_t)NPAD * 8, s));
    HIPCHK(h, hipMemsetAsync(h->partE.p, 0, (size_t)NPAD * 8, s));
    HIPCHK(h, launch_sp_rowsum(N, h->sp_offi.as<int64_t>(), h->sp_offj.as<int64_t>(), h->sp_perm.as<int32_t>(),
                               h->sp_kv2.as<float>(), h->partP.as<double>(), h->partE.as<double>(), s));
    HIPCHK(h, launch_fill_value(h->kdiag.as<double>(), N, 1.0 + lam * lam, s));
    HIPCHK(h, launch_diag(N, 0, h->partP.as<double>(), h->partE.as<double>(), h->kdiag.as<double>(),
                          p.diag_mode, p.C, p.diag_delta, h->Adiag.as<double>(), h->rowmax.as<double>(),
                          h->rsum.as<double>(), h->blk1.as<double>(), h->one.as<double>(), s));
    DevStatus* st = h->status_d.as<DevStatus>();
    const double boxC = (p.box_mode == GABP_BOX_PROJECT) ? p.C : 0.0;
    HIPCHK(h, launch_init(prec, N, NPAD, 1, h->Adiag.as<double>(), h->yd.as<float>(), h->Pt.p, h->S.p,
                          h->alpha_d.as<double>(), st, s, boxC));
    for (DevBuf* b : {&h->Pf, &h->Pb}) HIPCHK(h, hipMemsetAsync(b->p, 0, (size_t)2 * E * st_bytes, s));
    HIPCHK(h, hipEventRecord(ev[3], s));

    // ---- sweeps: edge update + per-node gather, finalize, stop rule
    StopRule rule{p.tol_abs, p.tol_rel, p.stagnation_rel, p.max_sweeps, p.stagnation_window};
    const int nblk = (int)((N + WG - 1) / WG);
    DevStatus hs{};
    double sweep_kernel_ms = 0.0;
    int64_t launches = 0;
    int polled = 0;
    for (int t = 0; t < p.max_sweeps; ++t) {
        const int slot = t % ce;
        if (p.time_sweeps) HIPCHK(h, hipEventRecord(sev[2 * slot], s));
        HIPCHK(h, launch_sp_sweep(prec, E, N, h->sp_ei.as<int32_t>(), h->sp_ej.as<int32_t>(), h->sp_kv2.as<float>(),
                                  h->Pt.p, h->S.p, h->Ef.p, h->Pf.p, h->Pb.p, h->sp_offi.as<int64_t>(),
                                  h->sp_offj.as<int64_t>(), h->sp_perm.as<int32_t>(), h->partP.p, h->partE.p,
                                  st, s));
        if (p.time_sweeps) HIPCHK(h, hipEventRecord(sev[2 * slot + 1], s));
        HIPCHK(h, launch_finalize(prec, N, 0, h->partP.p, h->partE.p, h->Adiag.as<double>(), h->yd.as<float>(),
                                  h->Pt.p, h->S.p, h->alpha_d.as<double>(), h->blk1.as<double>(),
                                  h->blk2.as<double>(), st, s, boxC));
        HIPCHK(h, launch_status(nblk, h->blk1.as<double>(), h->blk2.as<double>(), st, h->trace_d.as<double>(),
                                rule, s));
        if ((t + 1) % ce == 0 || t + 1 == p.max_sweeps) {
            HIPCHK(h, hipMemcpyAsync(&hs, st, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
            HIPCHK(h, hipStreamSynchronize(s));
            if (p.time_sweeps) {
                for (int u = polled; u <= t; ++u) {
                    if (u >= hs.t) break;
                    sweep_kernel_ms += elapsed(sev[2 * (u % ce)], sev[2 * (u % ce) + 1]);
                    ++launches;
                }
            }
            polled = t + 1;
            if (hs.done) break;
        }
    }
    HIPCHK(h, hipEventRecord(ev[4], s));

    // ---- outputs, back in input order (through partP as scratch)
    h->alpha.assign((size_t)N, 0.0);
    h->ptilde.assign((size_t)N, 0.0);
    h->adiag.assign((size_t)N, 0.0);
    h->yh.assign((size_t)N, 0.0f);
    double* scr = h->partP.as<double>();
    const int32_t* ord = h->sp_order.as<int32_t>();
    HIPCHK(h, launch_sp_unpermute(h->alpha_d.as<double>(), ord, N, scr, s));
    HIPCHK(h, hipMemcpyAsync(h->alpha.data(), scr, (size_t)N * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    HIPCHK(h, launch_convert_agg(prec, h->Pt.p, h->tmp.as<double>(), N, s));
    HIPCHK(h, launch_sp_unpermute(h->tmp.as<double>(), ord, N, scr, s));
    HIPCHK(h, hipMemcpyAsync(h->ptilde.data(), scr, (size_t)N * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    HIPCHK(h, launch_sp_unpermute(h->Adiag.as<double>(), ord, N, scr, s));
    HIPCHK(h, hipMemcpyAsync(h->adiag.data(), scr, (size_t)N * 8, hipMemcpyDeviceToHost, s));
    if (mem == GABP_MEM_HOST) std::copy(y, y + N, h->yh.begin());
    else HIPCHK(h, hipMemcpyAsync(h->yh.data(), y, (size_t)N * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipMemcpyAsync(&hs, st, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipEventRecord(ev[5], s));
    HIPCHK(h, hipStreamSynchronize(s));
    h->trace.assign((size_t)std::max(hs.t, 0), 0.0);
    if (hs.t > 0)
        HIPCHK(h, hipMemcpy(h->trace.data(), h->trace_d.p, (size_t)hs.t * 8, hipMemcpyDeviceToHost));

    h->N = N; h->m = m; h->NB = NB; h->NPAD = NPAD; h->ntiles = nt; h->m_pad = m_pad;
    h->prec = prec; h->gram = gram; h->lam = lam; h->rbf = true;
    h->sparse = true;
    h->n_edges = E;
    h->sweeps = hs.t;
    h->delta = hs.delta;
    h->reason = hs.reason;
    switch (hs.reason) {
        case R_CONVERGED: case R_STAGNATED: h->status = GABP_OK; break;
        case R_DIVERGED: h->status = GABP_E_DIVERGED; break;
        default: h->status = GABP_E_NOT_CONVERGED; break;
    }
    h->tm = gabp_timings{};
    h->tm.stage_ms = elapsed(ev[0], ev[1]);
    h->tm.kbuild_ms = elapsed(ev[1], ev[2]);
    h->tm.diag_ms = elapsed(ev[2], ev[3]);
    h->tm.sweep_loop_ms = elapsed(ev[3], ev[4]);
    h->tm.sweep_kernel_ms = sweep_kernel_ms;
    h->tm.sweep_launches = launches;
    h->tm.d2h_ms = elapsed(ev[4], ev[5]);
    h->tm.total_ms = now_ms() - t_start;
    h->plan = gabp_plan{};
    h->plan.precision = prec;
    h->plan.kstore = GABP_KSTORE_AUTO;      // K' kept per edge, not as tiles
    h->plan.edge_state = GABP_EDGE_STORED;
    h->plan.gram = (gram == GRAM_BF16X6) ? GABP_GRAM_BF16X6 : (gram == GRAM_BF16X3) ? GABP_GRAM_BF16X3
                 : (gram == GRAM_BF16 ? GABP_GRAM_BF16 : GABP_GRAM_AUTO);
    h->plan.tile = TILE;
    h->plan.n_blocks = NB;
    h->plan.n_tiles = nt;
    h->plan.n_edges = E;
    h->plan.device_bytes = h->held();
    // per edge and sweep: ends (8 B), K' (4 B), records read and written
    // (8 x 4 B), the gather's record reads (4 x 4 B) and permutation (4 B);
    // the packed aggregates (16 N B) are not counted
    h->plan.alg_bytes_per_pair = 8.0 + 4.0 + 8.0 * st_bytes + 4.0 * st_bytes + 4.0;
    h->plan.alg_bytes_per_sweep = (uint64_t)((double)E * h->plan.alg_bytes_per_pair);
    h->have_result = true;
    (void)agg;
    if (h->status != GABP_OK) {
        h->err = (h->status == GABP_E_DIVERGED) ? "GaBP diverged: a cavity precision became <= 0 or non-finite"
                                                : "max_sweeps reached before the stop rule held";
    }
    return (gabp_status)h->status;
}

std::vector<double> boxed_alpha(const gabp_svm* h) {
    std::vector<double> a = h->alpha;
    if (h->p.box_mode == GABP_BOX_CLIP_OUTPUT)
        for (auto& v : a) v = std::min(std::max(v, 0.0), h->p.C);
    return a;
}

}  // namespace

extern "C" {

int32_t gabp_abi_version(void) { return GABP_ABI_VERSION; }

const char* gabp_status_string(int32_t s) {
    switch (s) {
        case GABP_OK: return "ok";
        case GABP_E_INVALID: return "invalid argument";
        case GABP_E_NOMEM: return "plan does not fit the device-memory budget";
        case GABP_E_NOT_CONVERGED: return "not converged within max_sweeps";
        case GABP_E_DIVERGED: return "diverged";
        case GABP_E_DEVICE: return "device error";
        case GABP_E_STATE: return "invalid state";
        case GABP_E_BUFSIZE: return "buffer too small";
        default: return "unknown status";
    }
}

void gabp_svm_params_default(gabp_svm_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->struct_size = sizeof(gabp_svm_params);
    p->kernel = GABP_KERNEL_RBF;
    p->gamma = 1.0;
    p->C = 1.0;
    p->lambda_aug = -1.0;
    p->diag_mode = GABP_DIAG_DOMINANT_ROW;
    p->diag_delta = 0.1;
    p->box_mode = GABP_BOX_NONE;
    p->sv_tau = 0.0;
    p->tol_abs = 0.0;
    p->tol_rel = 1e-7;
    p->max_sweeps = 1000;
    p->check_every = 8;
    p->stagnation_window = 10;
    p->stagnation_rel = 1e-5;
    p->precision = GABP_PREC_MIXED;
    p->kstore = GABP_KSTORE_AUTO;
    p->edge_state = GABP_EDGE_AUTO;
    p->gram = GABP_GRAM_AUTO;
    p->stateless_depth = 0;
    p->device = 0;
    p->hbm_budget_bytes = 0;
    p->time_sweeps = 0;
    p->schedule = GABP_SCHED_SYNC;
    p->sched_groups = 0;
    p->sparse_edges_hint = 0;
    p->sparse_tau = 1e-3;
    p->tile_chunk = 0;
}

gabp_status gabp_svm_create(const gabp_svm_params* params, gabp_svm** out) {
    if (!out) return GABP_E_INVALID;
    *out = nullptr;
    std::string why;
    gabp_status st = check_params(params, why);
    if (st != GABP_OK) return st;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) { (void)hipGetLastError(); return GABP_E_DEVICE; }
    if (params->device < 0 || params->device >= ndev) return GABP_E_INVALID;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, params->device) != hipSuccess) return GABP_E_DEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return GABP_E_DEVICE;
    // set-up of the allocation-free decision function: the scratch array's
    // address on this device, looked up once per device with it current
    {
        int prev = 0;
        if (hipGetDevice(&prev) != hipSuccess) { (void)hipGetLastError(); return GABP_E_DEVICE; }
        void* sp = nullptr;
        const bool ok = hipSetDevice(params->device) == hipSuccess && predict_scratch(&sp) == hipSuccess;
        if (hipSetDevice(prev) != hipSuccess || !ok) { (void)hipGetLastError(); return GABP_E_DEVICE; }
    }
    gabp_svm* h = new (std::nothrow) gabp_svm();
    if (!h) return GABP_E_NOMEM;
    h->p = *params;
    *out = h;
    return GABP_OK;
}

gabp_status gabp_svm_solve(gabp_svm* h, const float* X, const float* y, int64_t N, int64_t m,
                           int32_t mem, void* stream) {
    if (!h) return GABP_E_INVALID;
    if (!X) return fail(h, GABP_E_INVALID, "X is NULL");
    if (h->p.kernel == GABP_KERNEL_RBF_SPARSE) return solve_sparse_impl(h, X, y, N, m, mem, (hipStream_t)stream);
    return solve_impl(h, X, nullptr, y, N, m, mem, (hipStream_t)stream);
}

gabp_status gabp_svm_solve_kernel(gabp_svm* h, const double* K, const float* y, int64_t N,
                                  int32_t mem, void* stream) {
    if (!h) return GABP_E_INVALID;
    if (!K) return fail(h, GABP_E_INVALID, "K is NULL");
    return solve_impl(h, nullptr, K, y, N, 0, mem, (hipStream_t)stream);
}

gabp_status gabp_svm_query(const gabp_svm* h, int32_t what, void* dst, size_t bytes) {
    if (!h || !dst) return GABP_E_INVALID;
    if (!h->have_result && what != GABP_Q_STATUS) return GABP_E_STATE;
    const size_t N = (size_t)h->N;
    auto put = [&](const void* src, size_t n) -> gabp_status {
        if (bytes < n) return GABP_E_BUFSIZE;
        std::memcpy(dst, src, n);
        return GABP_OK;
    };
    switch (what) {
        case GABP_Q_N: { int64_t v = h->N; return put(&v, sizeof v); }
        case GABP_Q_ALPHA: { auto a = boxed_alpha(h); return put(a.data(), N * 8); }
        case GABP_Q_PTILDE: return put(h->ptilde.data(), N * 8);
        case GABP_Q_ADIAG: return put(h->adiag.data(), N * 8);
        case GABP_Q_BIAS: {
            auto a = boxed_alpha(h);
            double b = 0.0;
            for (size_t i = 0; i < N; ++i) b += a[i] * (double)h->yh[i];
            b *= h->rbf ? h->lam * h->lam : 0.0;
            return put(&b, sizeof b);
        }
        case GABP_Q_SV_MASK: {
            if (bytes < N) return GABP_E_BUFSIZE;
            auto a = boxed_alpha(h);
            uint8_t* o = static_cast<uint8_t*>(dst);
            for (size_t i = 0; i < N; ++i) o[i] = a[i] > h->p.sv_tau ? 1 : 0;
            return GABP_OK;
        }
        case GABP_Q_SV_COUNT: {
            auto a = boxed_alpha(h);
            int64_t c = 0;
            for (size_t i = 0; i < N; ++i) c += a[i] > h->p.sv_tau ? 1 : 0;
            return put(&c, sizeof c);
        }
        case GABP_Q_SWEEPS: return put(&h->sweeps, sizeof h->sweeps);
        case GABP_Q_DELTA: return put(&h->delta, sizeof h->delta);
        case GABP_Q_STATUS: return put(&h->status, sizeof h->status);
        case GABP_Q_TIMINGS: return put(&h->tm, sizeof h->tm);
        case GABP_Q_TRACE: return put(h->trace.data(), h->trace.size() * 8);
        case GABP_Q_PLAN: return put(&h->plan, sizeof h->plan);
        case GABP_Q_REASON: return put(&h->reason, sizeof h->reason);
        case GABP_Q_RESIDUAL_BOUND: {
            if (bytes < 3 * sizeof(double)) return GABP_E_BUFSIZE;
            gabp_svm* hm = const_cast<gabp_svm*>(h);
            if (!hm->resid_valid) {
                const gabp_status rs = residual_certificate(hm);
                if (rs != GABP_OK) return rs;
            }
            return put(hm->resid, 3 * sizeof(double));
        }
        case GABP_Q_EDGES: {
            if (!h->sparse) return GABP_E_STATE;
            const size_t E = (size_t)h->n_edges;
            if (bytes < E * 16) return GABP_E_BUFSIZE;
            std::vector<int32_t> a(E), b(E), ord(N);
            if (E && (hipMemcpy(a.data(), h->sp_ei.p, E * 4, hipMemcpyDeviceToHost) != hipSuccess ||
                      hipMemcpy(b.data(), h->sp_ej.p, E * 4, hipMemcpyDeviceToHost) != hipSuccess ||
                      hipMemcpy(ord.data(), h->sp_order.p, N * 4, hipMemcpyDeviceToHost) != hipSuccess))
                return GABP_E_DEVICE;
            // input labels, i < j, lexicographic
            std::vector<uint64_t> keys(E);
            for (size_t e = 0; e < E; ++e) {
                const uint64_t u = (uint64_t)ord[(size_t)a[e]], v = (uint64_t)ord[(size_t)b[e]];
                keys[e] = (std::min(u, v) << 32) | std::max(u, v);
            }
            std::sort(keys.begin(), keys.end());
            int64_t* o = static_cast<int64_t*>(dst);
            for (size_t e = 0; e < E; ++e) { o[2 * e] = (int64_t)(keys[e] >> 32); o[2 * e + 1] = (int64_t)(keys[e] & 0xFFFFFFFFull); }
            return GABP_OK;
        }
        default: return GABP_E_INVALID;
    }
}

gabp_status gabp_svm_kernel_entries(const gabp_svm* hc, const int64_t* rows, const int64_t* cols,
                                    int64_t n, double* out) {
    gabp_svm* h = const_cast<gabp_svm*>(hc);
    if (!h || !rows || !cols || !out || n < 0) return GABP_E_INVALID;
    if (!h->have_result) return GABP_E_STATE;
    if (h->plan.kstore != GABP_KSTORE_MATERIALISE) return fail(h, GABP_E_STATE, "K' is not materialised in this plan");
    if (n == 0) return GABP_OK;
    for (int64_t k = 0; k < n; ++k)
        if (rows[k] < 0 || cols[k] < 0 || rows[k] >= h->N || cols[k] >= h->N || rows[k] == cols[k])
            return fail(h, GABP_E_INVALID, "index pair out of range or on the diagonal");
    HIPCHK(h, hipSetDevice(h->p.device));
    if (h->q_rows.ensure((size_t)n * 8) != hipSuccess || h->q_cols.ensure((size_t)n * 8) != hipSuccess ||
        h->q_out.ensure((size_t)n * 8) != hipSuccess)
        return fail(h, GABP_E_NOMEM, "device allocation failed");
    HIPCHK(h, hipMemcpy(h->q_rows.p, rows, (size_t)n * 8, hipMemcpyHostToDevice));
    HIPCHK(h, hipMemcpy(h->q_cols.p, cols, (size_t)n * 8, hipMemcpyHostToDevice));
    HIPCHK(h, launch_kernel_entries(h->Kp.p, h->prec, h->NB, h->q_rows.as<int64_t>(),
                                    h->q_cols.as<int64_t>(), n, h->q_out.as<double>(), nullptr));
    HIPCHK(h, hipMemcpy(out, h->q_out.p, (size_t)n * 8, hipMemcpyDeviceToHost));
    return GABP_OK;
}

}  // extern "C"

namespace {

// Working memory of one decision-function call for `nb` queries, as
// 256-byte aligned segments of one arena: the weights w_i = alpha_i y_i and
// their block sums first (the same offsets for every batch size), then the
// per-chunk partial sums and the staged queries of the form the handle
// uses (FP64 direct differences; augmented BF16 rows; FP32 or BF16 rows
// with norms).
struct PredictPlan {
    int form = 0;                 // 0 direct FP64, 1 augmented rows, 2 rows + norms
    int kind = 0, mp = 0, np = 0, nc = 1, bp = 1;
    int64_t qpad = 0;
    size_t o_w = 0, o_blk = 0, o_ws = 0, o_part = 0, o_nrm = 0, o_q0 = 0, o_q1 = 0, o_q2 = 0, bytes = 0;
};

PredictPlan predict_plan(const gabp_svm* h, int64_t nb) {
    PredictPlan P;
    size_t off = 0;
    auto seg = [&](size_t b) { const size_t o = off; off += (b + 255) / 256 * 256; return o; };
    const int64_t NPAD = h->NPAD;
    P.o_w = seg((size_t)NPAD * 8);
    P.o_blk = seg((size_t)(NPAD / WG + 1) * 8);
    P.o_ws = seg(64);
    if (h->prec == PREC_FP64) {
        P.form = 0;
        P.qpad = nb;
        P.o_part = seg((size_t)nb * 8);
    } else if (h->aug_kind >= 0) {
        P.form = 1;
        P.kind = h->aug_kind;
        P.mp = h->aug_mp;
        P.np = (P.kind == GRAM_BF16X6) ? 3 : (P.kind == GRAM_BF16X3) ? 2 : 1;
        P.qpad = predict_query_pad_aug(nb);
        predict_chunks_aug(NPAD, P.qpad, &P.nc, &P.bp);
        P.o_part = seg((size_t)P.nc * P.qpad * 8);
        P.o_q0 = seg((size_t)P.qpad * P.mp * 2 * P.np);
    } else {
        P.form = 2;
        P.kind = h->gram;
        P.mp = h->m_pad;
        P.qpad = predict_query_pad(nb);
        predict_chunks(NPAD, P.qpad, &P.nc, &P.bp);
        P.o_part = seg((size_t)P.nc * P.qpad * 8);
        P.o_nrm = seg((size_t)P.qpad * 4);
        const size_t fe = (size_t)P.qpad * P.mp;
        if (P.kind == GRAM_F32) P.o_q0 = seg(fe * 4);
        else P.o_q0 = seg(fe * 2);
        if (P.kind == GRAM_BF16X3 || P.kind == GRAM_BF16X6) P.o_q1 = seg(fe * 2);
        if (P.kind == GRAM_BF16X6) P.o_q2 = seg(fe * 2);
    }
    P.bytes = off;
    return P;
}

gabp_status predict_weights(gabp_svm* h, char* base, const PredictPlan& P, hipStream_t s) {
    HIPCHK(h, launch_predict_weights(h->alpha_d.as<double>(), h->yd.as<float>(), h->N, h->NPAD,
                                     h->p.box_mode == GABP_BOX_CLIP_OUTPUT, h->p.C,
                                     reinterpret_cast<double*>(base + P.o_w), reinterpret_cast<double*>(base + P.o_blk),
                                     reinterpret_cast<double*>(base + P.o_ws), s));
    return GABP_OK;
}

// One batch of nb device-resident queries into fd (device); e0 / e1 (if
// set) bracket the decision kernel.
gabp_status predict_batch(gabp_svm* h, const PredictPlan& P, char* base, const float* xqd, int64_t nb, double* fd,
                          hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    const double* w = reinterpret_cast<const double*>(base + P.o_w);
    const double* wsum = reinterpret_cast<const double*>(base + P.o_ws);
    double* part = reinterpret_cast<double*>(base + P.o_part);
    const double lam2 = h->lam * h->lam;
    if (P.form == 0) {
        if (e0) HIPCHK(h, hipEventRecord(e0, s));
        HIPCHK(h, launch_predict_direct(h->Xin.as<float>(), w, h->N, h->m, xqd, nb, h->p.gamma, part, s));
        if (e1) HIPCHK(h, hipEventRecord(e1, s));
        HIPCHK(h, launch_predict_reduce(part, 1, nb, nb, wsum, lam2, fd, s));
        return GABP_OK;
    }
    if (P.form == 1) {
        uint16_t* q = reinterpret_cast<uint16_t*>(base + P.o_q0);
        HIPCHK(h, launch_stage_aug(xqd, h->mean.as<double>(), nb, h->m, P.qpad, P.mp, P.kind, 0, 0.0f, q, s));
        // the events take the kernel dispatch's own timestamps
        HIPCHK(h, launch_predict_aug(P.kind, P.mp, h->xaug.as<uint16_t>(), h->NPAD, q, P.qpad, w, P.nc, P.bp, part, s,
                                     e0, e1));
        HIPCHK(h, launch_predict_reduce(part, P.nc, P.qpad, nb, wsum, lam2, fd, s));
        return GABP_OK;
    }
    Features Ft{}, Fq{};
    Ft.f32 = h->xs32.as<float>(); Ft.hi = h->xhi.as<uint16_t>(); Ft.lo = h->xlo.as<uint16_t>();
    Ft.lo2 = h->xlo2.as<uint16_t>(); Ft.nrm = h->nrm.as<float>(); Ft.m_pad = P.mp; Ft.kind = P.kind;
    float* qnrm = reinterpret_cast<float*>(base + P.o_nrm);
    float* qf32 = P.kind == GRAM_F32 ? reinterpret_cast<float*>(base + P.o_q0) : nullptr;
    uint16_t* qhi = P.kind != GRAM_F32 ? reinterpret_cast<uint16_t*>(base + P.o_q0) : nullptr;
    uint16_t* qlo = P.o_q1 ? reinterpret_cast<uint16_t*>(base + P.o_q1) : nullptr;
    uint16_t* qlo2 = P.o_q2 ? reinterpret_cast<uint16_t*>(base + P.o_q2) : nullptr;
    Fq.f32 = qf32; Fq.hi = qhi; Fq.lo = qlo; Fq.lo2 = qlo2; Fq.nrm = qnrm; Fq.m_pad = P.mp; Fq.kind = P.kind;
    const float c = (float)(-h->p.gamma * 1.4426950408889634);
    HIPCHK(h, launch_stage(xqd, h->mean.as<double>(), nb, h->m, P.qpad, P.mp, P.kind, qf32, qhi, qlo, qlo2, nullptr,
                           qnrm, s));
    if (e0) HIPCHK(h, hipEventRecord(e0, s));
    HIPCHK(h, launch_predict_mfma(Ft, Fq, w, h->NPAD, P.qpad, c, P.nc, P.bp, part, s));
    if (e1) HIPCHK(h, hipEventRecord(e1, s));
    HIPCHK(h, launch_predict_reduce(part, P.nc, P.qpad, nb, wsum, lam2, fd, s));
    return GABP_OK;
}

}  // namespace

extern "C" {

gabp_status gabp_svm_predict(gabp_svm* h, const float* Xq, int64_t nq, double* f_out, int32_t mem,
                             void* stream) {
    if (!h || !Xq || !f_out || nq < 0) return GABP_E_INVALID;
    if (mem != GABP_MEM_HOST && mem != GABP_MEM_DEVICE) return GABP_E_INVALID;
    if (!h->have_result || !h->rbf || h->sparse) return fail(h, GABP_E_STATE, "predict needs a finished dense RBF solve");
    if (nq == 0) return GABP_OK;
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(h, hipSetDevice(h->p.device));
    const int64_t m = h->m;
    if (mem == GABP_MEM_HOST) {
        for (int64_t k = 0; k < nq * m; ++k)
            if (!std::isfinite(Xq[k])) return fail(h, GABP_E_INVALID, "Xq has a non-finite entry");
    }
    // queries are processed in batches of at most QMAX rows; the arena holds
    // the largest batch's plan (the weights sit at the same offsets in all)
    const int64_t QMAX = int64_t(1) << 18;
    const int64_t qb = std::min(nq, QMAX);
    size_t need = predict_plan(h, qb).bytes;
    if (nq % QMAX && nq > QMAX) need = std::max(need, predict_plan(h, nq % QMAX).bytes);
    DevBuf xq, fo;
    bool ok = h->parena.ensure(need) == hipSuccess;
    if (ok && mem == GABP_MEM_HOST) ok = xq.ensure((size_t)qb * m * 4) == hipSuccess && fo.ensure((size_t)qb * 8) == hipSuccess;
    if (!ok) return fail(h, GABP_E_NOMEM, "device allocation for predict failed");
    char* base = static_cast<char*>(h->parena.p);
    const bool timed = h->p.time_sweeps != 0;
    const int64_t nbatch = (nq + QMAX - 1) / QMAX;
    EventPool pev;
    if (timed) HIPCHK(h, pev.make((size_t)(2 * nbatch)));
    const PredictPlan P0 = predict_plan(h, qb);
    if (predict_weights(h, base, P0, s) != GABP_OK) return GABP_E_DEVICE;
    for (int64_t q0 = 0; q0 < nq; q0 += QMAX) {
        const int64_t nb = std::min(QMAX, nq - q0);
        const float* xqd = Xq + q0 * m;
        if (mem == GABP_MEM_HOST) {
            HIPCHK(h, hipMemcpyAsync(xq.p, xqd, (size_t)nb * m * 4, hipMemcpyHostToDevice, s));
            xqd = xq.as<float>();
        }
        double* fd = (mem == GABP_MEM_HOST) ? fo.as<double>() : f_out + q0;
        const int64_t bi = q0 / QMAX;
        const gabp_status st = predict_batch(h, predict_plan(h, nb), base, xqd, nb, fd, s,
                                             timed ? pev.ev[2 * bi] : nullptr, timed ? pev.ev[2 * bi + 1] : nullptr);
        if (st != GABP_OK) return st;
        if (mem == GABP_MEM_HOST)
            HIPCHK(h, hipMemcpyAsync(f_out + q0, fo.p, (size_t)nb * 8, hipMemcpyDeviceToHost, s));
    }
    HIPCHK(h, hipStreamSynchronize(s));
    h->tm.predict_queries = nq;
    h->tm.predict_kernel_ms = 0.0;
    if (timed)
        for (int64_t b = 0; b < nbatch; ++b) {
            float ms = 0.0f;
            HIPCHK(h, hipEventElapsedTime(&ms, pev.ev[2 * b], pev.ev[2 * b + 1]));
            h->tm.predict_kernel_ms += ms;
        }
    return GABP_OK;
}

static_assert(GABP_PREDICT_SCRATCH_BYTES == PREDICT_SCRATCH_BYTES, "scratch size of the header and the library");

gabp_status gabp_svm_predict_noalloc(gabp_svm* h, const float* Xq, int64_t nq, double* f_out, void* stream) {
    if (!h || !Xq || !f_out || nq < 0) return GABP_E_INVALID;
    if (!h->have_result || !h->rbf || h->sparse) return fail(h, GABP_E_STATE, "predict needs a finished dense RBF solve");
    if (nq == 0) return GABP_OK;
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(h, hipSetDevice(h->p.device));
    void* base = nullptr;
    HIPCHK(h, predict_scratch(&base));
    // the whole call in one batch in the scratch array (every byte read is
    // written earlier in the same call on `stream`: nothing to clear)
    const PredictPlan P = predict_plan(h, nq);
    if (P.bytes > PREDICT_SCRATCH_BYTES) {
        char msg[200];
        snprintf(msg, sizeof msg, "%lld queries need %.1f MiB of scratch; the allocation-free predict holds %.0f MiB",
                 (long long)nq, P.bytes / 1048576.0, PREDICT_SCRATCH_BYTES / 1048576.0);
        return fail(h, GABP_E_NOMEM, msg);
    }
    char* b = static_cast<char*>(base);
    const gabp_status st = predict_weights(h, b, P, s);
    if (st != GABP_OK) return st;
    return predict_batch(h, P, b, Xq, nq, f_out, s, nullptr, nullptr);
}

void gabp_svm_destroy(gabp_svm* h) {
    if (!h) return;
    (void)hipSetDevice(h->p.device);
    h->release_all();
    delete h;
}

const char* gabp_svm_last_error(const gabp_svm* h) { return h ? h->err.c_str() : ""; }

}  // extern "C"
