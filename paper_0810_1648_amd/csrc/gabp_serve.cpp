// Serving runtime: continuous batching of GaBP SVM solves on one device
// (declared in include/gabp_svm.h, "Serving").
//
// A scheduler thread owns the device stream.  Each iteration it
//   1. admits queued requests (FIFO, bounded bypass) whose device footprint
//      fits the arena and for which a slot is free, uploads their inputs and
//      runs their setup kernels (staging, K' tiles, diagonal, sweep 0);
//   2. launches `steps_per_poll` batched steps over all active requests
//      (persistent sweep over the union of their tiles, batched finalize,
//      batched stop rule), one launch group per precision, level count and
//      reciprocal form; requests on the grouped schedule have launch groups
//      of their own, whose step is one group visit of every request (item
//      lists built per step from each request's current group);
//   3. reads back the packed statuses, downloads alpha of finished requests
//      and returns their arena blocks.
// Device memory comes from one arena allocated at creation, so no hipMalloc
// or hipFree (which synchronises the device) runs on the serving path.
#include "gabp_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

using namespace gabp;

namespace {

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

constexpr size_t kAlign = 256;
inline size_t align_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over one device allocation; blocks merge on release.
class Arena {
public:
    char* base = nullptr;
    size_t cap = 0;

    hipError_t init(size_t bytes) {
        cap = align_up(bytes);
        hipError_t e = hipMalloc((void**)&base, cap);
        if (e != hipSuccess) { base = nullptr; cap = 0; (void)hipGetLastError(); return e; }
        free_.clear();
        free_[0] = cap;
        return hipSuccess;
    }
    void destroy() {
        if (base) (void)hipFree(base);
        base = nullptr;
        cap = 0;
        free_.clear();
    }
    // Offsets for every size in `sizes` (0-byte entries get SIZE_MAX), all or none.
    bool alloc_all(const std::vector<size_t>& sizes, std::vector<size_t>& offs) {
        std::map<size_t, size_t> save = free_;
        offs.assign(sizes.size(), SIZE_MAX);
        for (size_t k = 0; k < sizes.size(); ++k) {
            if (sizes[k] == 0) continue;
            const size_t o = alloc(sizes[k]);
            if (o == SIZE_MAX) { free_ = save; offs.assign(sizes.size(), SIZE_MAX); return false; }
            offs[k] = o;
        }
        return true;
    }
    void release_all(const std::vector<size_t>& sizes, const std::vector<size_t>& offs) {
        for (size_t k = 0; k < sizes.size(); ++k)
            if (offs[k] != SIZE_MAX) release(offs[k], sizes[k]);
    }
    size_t free_bytes() const {
        size_t b = 0;
        for (auto& kv : free_) b += kv.second;
        return b;
    }

private:
    std::map<size_t, size_t> free_;  // offset -> length
    size_t alloc(size_t n) {
        n = align_up(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            const size_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > n) free_[off + n] = len - n;
            return off;
        }
        return SIZE_MAX;
    }
    void release(size_t off, size_t n) {
        n = align_up(n);
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

// Device buffers of one request, in a fixed order.
enum Buf {
    B_TILES, B_KP, B_PF, B_PB, B_EF, B_EB, B_PARTP, B_PARTE, B_X, B_Y, B_MEAN, B_X32, B_XHI, B_XLO,
    B_XLO2, B_X64, B_NRM, B_KDIAG, B_ADIAG, B_ROWMAX, B_RSUM, B_PT, B_S, B_ALPHA, B_BLK1, B_BLK2, B_ONE,
    B_STATUS, B_TRACE, B_COUNT
};

struct Req {
    uint64_t ticket = 0;
    std::vector<float> X, y;
    int64_t N = 0, m = 0;
    gabp_svm_params p{};
    int prec = PREC_FP32, gram = GRAM_F32;
    int NB = 0, m_pad = 0;
    int64_t NPAD = 0, nt = 0;
    double lam = 0.0;
    double t_submit = 0.0, t_admit = 0.0, t_done = 0.0;
    int state = 0;  // 0 queued, 1 active, 2 finished
    int32_t status = GABP_E_STATE, reason = R_NONE, sweeps = 0;
    std::vector<double> alpha;
    std::vector<size_t> sizes, offs;
    size_t footprint = 0;
    int slot = -1;
    int bypassed = 0;
    int32_t refused = 0; // set up but refused (gabp_status): no plan without a bound
    int levels = 0;      // 0: stored pair records; >= 1: stateless levels
    int ser = 0;         // stateless reciprocals: 0 exact, 1 / 2 series (top-level terms)
    bool chunked = false;  // synchronous sweeps over 2 x 2 chunks of tiles
    double rho = 0.0;    // contraction bound
    // grouped schedule: G groups of whole block rows, the group the next step
    // visits, the single-direction list entries of every group (into gent
    // from goff[g]), with stored pair records the tiles inside every group
    // (into gwin from gwoff[g]), and the first node block of every group
    bool grouped = false;
    int G = 1, gcur = 0;
    std::vector<uint32_t> gent, gwin;
    std::vector<int64_t> goff, gwoff, gb0;
};

constexpr int kRing = 8;   // aggregate ring slots (stateless form)

void plan_sizes(Req& r) {
    const size_t st = (r.prec == PREC_FP64) ? 8 : 4;
    const size_t plane = (size_t)r.nt * TT * st;
    const size_t part = (size_t)r.NB * (r.NB + 1) * TILE * 8;
    const size_t fe = (size_t)r.NPAD * r.m_pad;
    std::vector<size_t> z(B_COUNT, 0);
    z[B_TILES] = (size_t)r.nt * 4;
    z[B_KP] = z[B_PF] = z[B_PB] = z[B_EF] = z[B_EB] = plane;
    z[B_PARTP] = z[B_PARTE] = part;
    z[B_X] = (size_t)r.N * r.m * 4;
    z[B_Y] = (size_t)r.N * 4;
    z[B_MEAN] = (size_t)r.m * 8;
    if (r.gram == GRAM_F32) z[B_X32] = fe * 4;
    if (r.gram == GRAM_BF16 || r.gram == GRAM_BF16X3 || r.gram == GRAM_BF16X6) z[B_XHI] = fe * 2;
    if (r.gram == GRAM_BF16X3 || r.gram == GRAM_BF16X6) z[B_XLO] = fe * 2;
    if (r.gram == GRAM_BF16X6) z[B_XLO2] = fe * 2;
    if (r.gram == GRAM_F64) z[B_X64] = fe * 8;
    z[B_NRM] = (size_t)r.NPAD * 4;
    z[B_KDIAG] = z[B_ADIAG] = z[B_ROWMAX] = z[B_RSUM] = z[B_ALPHA] = (size_t)r.N * 8;
    z[B_PT] = z[B_S] = (size_t)kRing * r.NPAD * 8;
    z[B_BLK1] = z[B_BLK2] = (size_t)(r.NPAD / WG + 1) * 8;
    z[B_ONE] = 64;
    z[B_STATUS] = sizeof(DevStatus);
    z[B_TRACE] = (size_t)r.p.max_sweeps * 8;
    r.sizes = z;
    r.footprint = 0;
    for (size_t b : z) r.footprint += b ? align_up(b) : 0;
}

}  // namespace

struct gabp_server {
    gabp_server_params p{};
    Arena arena;
    hipStream_t stream = nullptr;
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    bool dev_error = false;
    std::deque<Req*> queue;
    std::map<uint64_t, Req*> reqs;
    std::vector<Req*> slots;          // active request per slot (nullptr = free)
    uint64_t next_ticket = 1;
    // device tables and pinned staging
    ReqDesc* d_reqs = nullptr;
    ReqDesc* h_reqs = nullptr;
    DevStatus* d_stat = nullptr;
    DevStatus* h_stat = nullptr;
    // launch groups: requests sharing schedule, precision, level count and
    // reciprocal form; a synchronous group's (request, tile) items are fixed
    // while its membership is
    struct Group {
        int prec = 0, levels = 0;
        int ser = 0;
        bool grouped = false;
        uint2* d_tiles = nullptr; uint2* h_tiles = nullptr; size_t cap_tiles = 0;
        int ntiles = 0, nslots = 0;
        std::vector<int> slot_list;
    };
    std::map<int, Group> groups;
    // every active slot, launch group by launch group (the order of d_stat)
    int* d_slots = nullptr; int* h_slots = nullptr;
    int nactive = 0;
    // per step of a poll: one upload of the grouped requests' (request,
    // entry) items and of every request's (request, node block) items
    struct StepLists { uint2* d = nullptr; uint2* h = nullptr; size_t cap = 0; };
    std::vector<StepLists> step_lists;
    // statistics
    std::vector<double> lat_ms, queue_ms;
    int64_t submitted = 0, completed = 0, failed = 0, steps = 0, active_sum = 0, max_active_seen = 0;
    double first_submit = -1.0, last_done = 0.0;

    char* ptr(const Req& r, int b) const {
        return r.offs[b] == SIZE_MAX ? nullptr : arena.base + r.offs[b];
    }
};

namespace {

hipError_t grow(uint2*& d, uint2*& h, size_t& cap, size_t need) {
    if (need <= cap) return hipSuccess;
    size_t nc = std::max<size_t>(need, cap * 2 + 1024);
    if (d) (void)hipFree(d);
    if (h) (void)hipHostFree(h);
    d = nullptr;
    h = nullptr;
    cap = 0;
    hipError_t e = hipMalloc((void**)&d, nc * sizeof(uint2));
    if (e != hipSuccess) return e;
    e = hipHostMalloc((void**)&h, nc * sizeof(uint2), hipHostMallocDefault);
    if (e != hipSuccess) return e;
    cap = nc;
    return hipSuccess;
}

// Uploads inputs and runs the setup kernels of a newly admitted request.
hipError_t setup_request(gabp_server* S, Req& r) {
    hipStream_t s = S->stream;
    auto P = [&](int b) { return S->ptr(r, b); };
    hipError_t e;
#define CK(x) do { e = (x); if (e != hipSuccess) return e; } while (0)
    CK(hipMemcpyAsync(P(B_X), r.X.data(), r.sizes[B_X], hipMemcpyHostToDevice, s));
    CK(hipMemcpyAsync(P(B_Y), r.y.data(), r.sizes[B_Y], hipMemcpyHostToDevice, s));
    KernelParams kp{};
    kp.N = r.N;
    kp.NB = r.NB;
    kp.gamma = r.p.gamma;
    kp.neg_gamma_log2e = (float)(-r.p.gamma * 1.4426950408889634);
    kp.lam2 = r.lam * r.lam;
    Features F{};
    F.m_pad = r.m_pad;
    F.kind = r.gram;
    F.f32 = (float*)P(B_X32);
    F.hi = (uint16_t*)P(B_XHI);
    F.lo = (uint16_t*)P(B_XLO);
    F.lo2 = (uint16_t*)P(B_XLO2);
    F.f64 = (double*)P(B_X64);
    F.nrm = (float*)P(B_NRM);
    if (r.gram != GRAM_F64) CK(launch_colmean((float*)P(B_X), r.N, r.m, (double*)P(B_MEAN), s));
    CK(launch_stage((float*)P(B_X), (double*)P(B_MEAN), r.N, r.m, r.NPAD, r.m_pad, r.gram,
                    (float*)P(B_X32), (uint16_t*)P(B_XHI), (uint16_t*)P(B_XLO), (uint16_t*)P(B_XLO2),
                    (double*)P(B_X64), (float*)P(B_NRM), s));
    CK(launch_fill_tiles((uint32_t*)P(B_TILES), r.NB, s));
    // same build as the single solve: FP32-stored K' with the row-sum partials
    // in one pass, FP64 K' followed by its own row-sum pass
    if (r.gram != GRAM_F64) {
        CK(launch_gram_sums(F, kp, (uint32_t*)P(B_TILES), r.nt, P(B_KP), r.NB, (double*)P(B_PARTP),
                            (double*)P(B_PARTE), s));
    } else {
        CK(launch_gram(F, kp, (uint32_t*)P(B_TILES), r.nt, P(B_KP), s));
        CK(launch_rowsum(P(B_KP), r.prec, KSRC_PLANE, F, kp, (uint32_t*)P(B_TILES), r.nt, r.NB,
                         (double*)P(B_PARTP), (double*)P(B_PARTE), s));
    }
    CK(launch_fill_value((double*)P(B_KDIAG), r.N, 1.0 + r.lam * r.lam, s));
    CK(launch_diag(r.N, r.NB, (double*)P(B_PARTP), (double*)P(B_PARTE), (double*)P(B_KDIAG),
                   r.p.diag_mode, r.p.C, r.p.diag_delta, (double*)P(B_ADIAG), (double*)P(B_ROWMAX),
                   (double*)P(B_RSUM), (double*)P(B_BLK1), (double*)P(B_ONE), s));
    // edge state from the contraction bound (same rule as a single solve)
    CK(launch_rho_bound(r.N, (double*)P(B_ADIAG), (double*)P(B_ROWMAX), (double*)P(B_RSUM),
                        (double*)P(B_BLK1), (double*)P(B_ONE), s));
    double hb[2] = {0.0, 0.0};
    CK(hipMemcpyAsync(hb, P(B_ONE), 16, hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    r.rho = hb[1];
    const double rr = 1.25 * r.rho;
    const int dneed = stateless_levels_needed(r.prec, rr);
    bool stateless = false;
    if (r.p.edge_state == GABP_EDGE_STATELESS) stateless = true;
    else if (r.p.edge_state == GABP_EDGE_AUTO) stateless = dneed <= 8;
    if (stateless && r.p.stateless_depth == 0 && !(rr < 1.0)) {
        // as in a single solve: an explicit stateless plan with an automatic
        // depth needs a contraction bound, else the request is refused
        r.refused = GABP_E_INVALID;
        return hipSuccess;
    }
    r.levels = stateless ? (r.p.stateless_depth > 0 ? r.p.stateless_depth : std::min(dneed, 8)) : 0;
    r.ser = stateless ? stateless_series_form(r.prec, r.levels, rr) : 0;
    if (stateless) {
        // the pair-record planes are not needed: give them back to the arena
        const std::vector<int> planes = {B_PF, B_PB, B_EF, B_EB};
        std::vector<size_t> sz, of;
        for (int b : planes) { sz.push_back(r.sizes[b]); of.push_back(r.offs[b]); r.offs[b] = SIZE_MAX; }
        S->arena.release_all(sz, of);
        for (int b : planes) { r.footprint -= align_up(r.sizes[b]); r.sizes[b] = 0; }
    }
    // grouped schedule (same groups and lists as a single solve): stateless
    // plans visit every message into the group; stored pair records visit
    // the tiles crossing the group boundary in one direction and the tiles
    // inside the group in both
    r.grouped = r.p.schedule == GABP_SCHED_GROUPED;
    r.G = 1;
    r.gcur = 0;
    if (r.grouped) {
        const int NB = r.NB, G = std::min(r.p.sched_groups > 0 ? r.p.sched_groups : 16, NB);
        auto grp = [&](int I) { return (int)((int64_t)I * G / NB); };
        std::vector<std::vector<uint32_t>> dl(G), wl(G);
        for (int I = 0; I < NB; ++I)
            for (int J = I; J < NB; ++J) {
                const uint32_t k = (uint32_t)tile_index(I, J, NB);
                const int gi = grp(I), gj = grp(J);
                if (!stateless) {
                    if (gi == gj) wl[gi].push_back(k);
                    else { dl[gj].push_back(k); dl[gi].push_back(k | GE_BWD); }
                } else {
                    const uint32_t in = (gi == gj) ? GE_WITHIN : 0u;
                    dl[gj].push_back(k | in);
                    dl[gi].push_back(k | GE_BWD | in);
                }
            }
        r.gent.clear();
        r.gwin.clear();
        r.goff.assign(G + 1, 0);
        r.gwoff.assign(G + 1, 0);
        for (int g = 0; g < G; ++g) {
            r.goff[g] = (int64_t)r.gent.size();
            r.gent.insert(r.gent.end(), dl[g].begin(), dl[g].end());
            r.gwoff[g] = (int64_t)r.gwin.size();
            r.gwin.insert(r.gwin.end(), wl[g].begin(), wl[g].end());
        }
        r.goff[G] = (int64_t)r.gent.size();
        r.gwoff[G] = (int64_t)r.gwin.size();
        r.gb0.assign(G + 1, NB);
        int gc = 0;
        for (int I = 0; I < NB; ++I)
            while (gc <= G && grp(I) >= gc) r.gb0[gc++] = I;
        r.G = G;
    }
    const int R = stateless ? kRing : 1;
    CK(launch_init(r.prec, r.N, r.NPAD, R, (double*)P(B_ADIAG), (float*)P(B_Y), P(B_PT), P(B_S),
                   (double*)P(B_ALPHA), (DevStatus*)P(B_STATUS), s));
    if (!stateless)
        for (int b : {B_PF, B_PB, B_EF, B_EB}) CK(hipMemsetAsync(P(b), 0, r.sizes[b], s));
    ReqDesc& d = S->h_reqs[r.slot];
    d = ReqDesc{};
    d.sw.tiles = (uint32_t*)P(B_TILES);
    d.sw.ntiles = r.nt;
    d.sw.NB = r.NB;
    d.sw.Kp = P(B_KP);
    d.sw.Pf = P(B_PF); d.sw.Pb = P(B_PB); d.sw.Ef = P(B_EF); d.sw.Eb = P(B_EB);
    d.sw.HP = P(B_PT); d.sw.HS = P(B_S);
    d.sw.NPAD = r.NPAD;
    d.sw.R = R;
    d.sw.slot_top = 0;
    d.sw.levels = r.levels;
    d.sw.part32 = (r.prec == PREC_MIXED && stateless && r.ser > 0) ? 1 : 0;   // as in a single solve
    // synchronous stateless sweeps with FP32 partial sums run over 2 x 2
    // chunks of tiles, as in a single solve (items (request, Ic << 16 | Jc))
    d.sw.chunk = (!r.grouped && stateless && chunk_sweep(r.prec == PREC_FP32 || d.sw.part32, r.levels, r.ser, r.NB,
                                                               r.p.tile_chunk)) ? 2 : 1;
    r.chunked = d.sw.chunk > 1;
    d.sw.partP = P(B_PARTP); d.sw.partE = P(B_PARTE);
    d.sw.st = (DevStatus*)P(B_STATUS);
    d.sw.F = F;
    d.sw.kp = kp;
    d.N = r.N;
    d.Adiag = (double*)P(B_ADIAG);
    d.y = (float*)P(B_Y);
    d.alpha = (double*)P(B_ALPHA);
    d.blk_delta = (double*)P(B_BLK1);
    d.blk_amax = (double*)P(B_BLK2);
    d.trace = (double*)P(B_TRACE);
    d.rule = StopRule{r.p.tol_abs, r.p.tol_rel, r.p.stagnation_rel, r.p.max_sweeps, r.p.stagnation_window};
    d.nblk = (int)((r.N + WG - 1) / WG);
    d.G = r.G;
    CK(hipMemcpyAsync(S->d_reqs + r.slot, S->h_reqs + r.slot, sizeof(ReqDesc), hipMemcpyHostToDevice, s));
#undef CK
    return hipSuccess;
}

inline int group_key(const Req& r) { return (r.grouped ? 1000 : 0) + r.prec * 100 + r.ser * 10 + r.levels; }

// Rebuilds the launch groups, their fixed tile lists and the slot order
// from the active slots.
hipError_t rebuild_lists(gabp_server* S) {
    hipError_t e;
    for (auto& kv : S->groups) kv.second.slot_list.clear();
    for (size_t k = 0; k < S->slots.size(); ++k) {
        Req* r = S->slots[k];
        if (!r) continue;
        auto& G = S->groups[group_key(*r)];
        G.prec = r->prec;
        G.levels = r->levels;
        G.ser = r->ser;
        G.grouped = r->grouped;
        G.slot_list.push_back((int)k);
    }
    if (!S->d_slots) {
        const size_t A = S->slots.size();
        if ((e = hipMalloc((void**)&S->d_slots, A * sizeof(int))) != hipSuccess) return e;
        if ((e = hipHostMalloc((void**)&S->h_slots, A * sizeof(int), hipHostMallocDefault)) != hipSuccess) return e;
    }
    int na = 0;
    for (auto& kv : S->groups) {
        auto& G = kv.second;
        G.nslots = (int)G.slot_list.size();
        for (int k : G.slot_list) S->h_slots[na++] = k;
        G.ntiles = 0;
        if (G.grouped) continue;   // per-step items (build_step)
        // items: (request, tile), or (request, Ic << 16 | Jc) for a request
        // whose sweeps run over 2 x 2 chunks of tiles
        auto nitems = [](const Req* r) {
            const int64_t nbc = (r->NB + 1) / 2;
            return r->chunked ? nbc * (nbc + 1) / 2 : r->nt;
        };
        size_t nt = 0;
        for (int k : G.slot_list) nt += (size_t)nitems(S->slots[k]);
        if ((e = grow(G.d_tiles, G.h_tiles, G.cap_tiles, std::max<size_t>(nt, 1))) != hipSuccess) return e;
        size_t it = 0;
        for (int k : G.slot_list) {
            Req* r = S->slots[k];
            if (r->chunked) {
                const int nbc = (r->NB + 1) / 2;
                for (int ic = 0; ic < nbc; ++ic)
                    for (int jc = ic; jc < nbc; ++jc)
                        G.h_tiles[it++] = make_uint2((unsigned)k, ((unsigned)ic << 16) | (unsigned)jc);
            } else {
                for (int64_t t = 0; t < r->nt; ++t) G.h_tiles[it++] = make_uint2((unsigned)k, (unsigned)t);
            }
        }
        G.ntiles = (int)it;
        if (it && (e = hipMemcpyAsync(G.d_tiles, G.h_tiles, it * sizeof(uint2), hipMemcpyHostToDevice, S->stream)) != hipSuccess)
            return e;
    }
    S->nactive = na;
    if (na && (e = hipMemcpyAsync(S->d_slots, S->h_slots, (size_t)na * sizeof(int), hipMemcpyHostToDevice, S->stream)) != hipSuccess)
        return e;
    return hipSuccess;
}

// Items of step k of the poll, uploaded at once: the (request, entry) items
// of every grouped launch group's requests' current groups, then the
// (request, node block) items of every active request (its current group's
// blocks on the grouped schedule, all of them otherwise), FP32 aggregates
// first.  The grouped requests' groups then advance.
struct StepPlan {
    std::vector<std::pair<int64_t, int>> dir;   // per launch group (map order): offset, count
    std::vector<std::pair<int64_t, int>> win;   // stored records: the (request, tile) items inside the groups
    int64_t off_f32 = 0, off_f64 = 0;
    int n_f32 = 0, n_f64 = 0;
};

hipError_t build_step(gabp_server* S, int k, StepPlan& P) {
    hipError_t e;
    if ((int)S->step_lists.size() <= k) S->step_lists.resize(k + 1);
    auto& L = S->step_lists[k];
    auto node_range = [](const Req* r, int64_t& b0, int64_t& b1) {
        const int64_t nblk = (r->N + WG - 1) / WG;
        if (r->grouped) { b0 = r->gb0[r->gcur]; b1 = std::min<int64_t>(r->gb0[r->gcur + 1], nblk); }
        else { b0 = 0; b1 = nblk; }
    };
    size_t n = 0;
    for (auto& kv : S->groups)
        if (kv.second.grouped)
            for (int q : kv.second.slot_list) {
                const Req* r = S->slots[q];
                n += (size_t)(r->goff[r->gcur + 1] - r->goff[r->gcur]);
                n += (size_t)(r->gwoff[r->gcur + 1] - r->gwoff[r->gcur]);
            }
    for (int q = 0; q < S->nactive; ++q) {
        int64_t b0, b1;
        node_range(S->slots[S->h_slots[q]], b0, b1);
        n += (size_t)std::max<int64_t>(b1 - b0, 0);
    }
    if ((e = grow(L.d, L.h, L.cap, std::max<size_t>(n, 1))) != hipSuccess) return e;
    size_t it = 0;
    P.dir.clear();
    P.win.clear();
    for (auto& kv : S->groups) {
        size_t start = it;
        if (kv.second.grouped)
            for (int q : kv.second.slot_list) {
                const Req* r = S->slots[q];
                for (int64_t u = r->goff[r->gcur]; u < r->goff[r->gcur + 1]; ++u)
                    L.h[it++] = make_uint2((unsigned)q, r->gent[(size_t)u]);
            }
        P.dir.emplace_back((int64_t)start, (int)(it - start));
        start = it;
        if (kv.second.grouped)
            for (int q : kv.second.slot_list) {
                const Req* r = S->slots[q];
                for (int64_t u = r->gwoff[r->gcur]; u < r->gwoff[r->gcur + 1]; ++u)
                    L.h[it++] = make_uint2((unsigned)q, r->gwin[(size_t)u]);
            }
        P.win.emplace_back((int64_t)start, (int)(it - start));
    }
    for (int pass = 0; pass < 2; ++pass) {
        const size_t start = it;
        for (int q = 0; q < S->nactive; ++q) {
            const int slot = S->h_slots[q];
            const Req* r = S->slots[slot];
            if ((r->prec == PREC_FP32) != (pass == 0)) continue;
            int64_t b0, b1;
            node_range(r, b0, b1);
            for (int64_t b = b0; b < b1; ++b) L.h[it++] = make_uint2((unsigned)slot, (unsigned)b);
        }
        if (pass == 0) { P.off_f32 = (int64_t)start; P.n_f32 = (int)(it - start); }
        else { P.off_f64 = (int64_t)start; P.n_f64 = (int)(it - start); }
    }
    for (auto& kv : S->groups)
        if (kv.second.grouped)
            for (int q : kv.second.slot_list) {
                Req* r = S->slots[q];
                r->gcur = (r->gcur + 1) % r->G;
            }
    if (it && (e = hipMemcpyAsync(L.d, L.h, it * sizeof(uint2), hipMemcpyHostToDevice, S->stream)) != hipSuccess)
        return e;
    return hipSuccess;
}

void finish(gabp_server* S, Req& r, int32_t status, int32_t reason, int32_t sweeps) {
    r.status = status;
    r.reason = reason;
    r.sweeps = sweeps;
    r.t_done = now_s();
    r.state = 2;
    r.X.clear(); r.X.shrink_to_fit();
    r.y.clear(); r.y.shrink_to_fit();
    if (r.p.box_mode == GABP_BOX_CLIP_OUTPUT)
        for (auto& v : r.alpha) v = std::min(std::max(v, 0.0), r.p.C);
    if (status == GABP_OK) ++S->completed; else ++S->failed;
    S->lat_ms.push_back((r.t_done - r.t_submit) * 1e3);
    S->queue_ms.push_back((r.t_admit - r.t_submit) * 1e3);
    S->last_done = r.t_done;
}

void fail_all_active(gabp_server* S) {
    for (auto& r : S->slots) {
        if (!r) continue;
        finish(S, *r, GABP_E_DEVICE, R_NONE, 0);
        r = nullptr;
    }
    while (!S->queue.empty()) {
        Req* r = S->queue.front();
        S->queue.pop_front();
        r->t_admit = now_s();
        finish(S, *r, GABP_E_DEVICE, R_NONE, 0);
    }
}

void worker_loop(gabp_server* S) {
    (void)hipSetDevice(S->p.device);
    std::vector<Req*> admitted;
    bool lists_dirty = false;
    while (true) {
        admitted.clear();
        {
            std::unique_lock<std::mutex> lk(S->mu);
            bool any_active = std::any_of(S->slots.begin(), S->slots.end(), [](Req* r) { return r != nullptr; });
            if (!any_active && S->queue.empty() && !S->stop)
                S->cv_work.wait(lk, [&] { return S->stop || !S->queue.empty(); });
            if (S->stop) return;
            // admission: FIFO; requests behind a head that does not fit may
            // pass it at most max_bypass times, after which the head blocks
            Req* head = S->queue.empty() ? nullptr : S->queue.front();
            bool head_waits = false;
            int looked = 0;
            for (auto it = S->queue.begin(); it != S->queue.end();) {
                auto fs = std::find(S->slots.begin(), S->slots.end(), nullptr);
                if (fs == S->slots.end()) break;
                Req* r = *it;
                if (r != head && head_waits && head->bypassed >= S->p.max_bypass) break;
                if (S->arena.alloc_all(r->sizes, r->offs)) {
                    r->slot = (int)(fs - S->slots.begin());
                    *fs = r;
                    r->state = 1;
                    r->t_admit = now_s();
                    admitted.push_back(r);
                    if (r != head && head_waits) ++head->bypassed;
                    it = S->queue.erase(it);
                    continue;
                }
                if (r == head) head_waits = true;
                ++it;
                if (++looked > S->p.max_bypass) break;
            }
        }
        for (Req* r : admitted) {
            if (setup_request(S, *r) != hipSuccess) {
                std::lock_guard<std::mutex> lk(S->mu);
                S->dev_error = true;
                fail_all_active(S);
                S->cv_done.notify_all();
                return;
            }
            if (r->refused) {
                std::lock_guard<std::mutex> lk(S->mu);
                S->arena.release_all(r->sizes, r->offs);
                S->slots[r->slot] = nullptr;
                finish(S, *r, r->refused, R_NONE, 0);
                S->cv_done.notify_all();
                continue;
            }
            lists_dirty = true;
        }
        if (lists_dirty) {
            if (rebuild_lists(S) != hipSuccess) {
                std::lock_guard<std::mutex> lk(S->mu);
                S->dev_error = true;
                fail_all_active(S);
                S->cv_done.notify_all();
                return;
            }
            lists_dirty = false;
        }
        const int nactive = S->nactive;
        if (nactive == 0) continue;
        hipError_t e = hipSuccess;
        // a step: the sweep (or group visit) of every launch group, then the
        // finalize of every request's node blocks, then every stop rule
        StepPlan plan;
        for (int k = 0; k < S->p.steps_per_poll && e == hipSuccess; ++k) {
            e = build_step(S, k, plan);
            const uint2* items = S->step_lists.empty() ? nullptr : S->step_lists[k].d;
            size_t gi = 0;
            for (auto& kv : S->groups) {
                auto& G = kv.second;
                const auto dir = plan.dir[gi], win = plan.win[gi];
                ++gi;
                if (!G.nslots || e != hipSuccess) continue;
                if (G.grouped) {
                    // stored records: the tiles inside the group (both directions), then the crossing ones
                    if (win.second)
                        e = launch_served_sweep(G.prec, G.levels, G.ser, false, S->d_reqs, items + win.first, win.second,
                                                S->stream);
                    if (e == hipSuccess)
                        e = launch_served_sweep(G.prec, G.levels, G.ser, true, S->d_reqs, items + dir.first,
                                                dir.second, S->stream);
                } else
                    e = launch_served_sweep(G.prec, G.levels, G.ser, false, S->d_reqs, G.d_tiles, G.ntiles, S->stream);
            }
            if (e == hipSuccess && plan.n_f32)
                e = launch_served_finalize(true, S->d_reqs, items + plan.off_f32, plan.n_f32, S->stream);
            if (e == hipSuccess && plan.n_f64)
                e = launch_served_finalize(false, S->d_reqs, items + plan.off_f64, plan.n_f64, S->stream);
            if (e == hipSuccess) e = launch_served_status(S->d_reqs, S->d_slots, nactive, S->d_stat, S->stream);
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(S->h_stat, S->d_stat, (size_t)nactive * sizeof(DevStatus), hipMemcpyDeviceToHost,
                               S->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(S->stream);
        // retire finished requests
        std::vector<std::pair<Req*, DevStatus>> done;
        int base = 0;
        for (auto& kv : S->groups) {
            auto& G = kv.second;
            for (int q = 0; q < G.nslots; ++q) {
                const DevStatus& ds = S->h_stat[base + q];
                if (ds.done) done.emplace_back(S->slots[G.slot_list[q]], ds);
            }
            base += G.nslots;
        }
        for (auto& d : done) {
            Req* r = d.first;
            r->alpha.assign((size_t)r->N, 0.0);
            if (e == hipSuccess)
                e = hipMemcpyAsync(r->alpha.data(), S->ptr(*r, B_ALPHA), (size_t)r->N * 8, hipMemcpyDeviceToHost, S->stream);
        }
        if (!done.empty() && e == hipSuccess) e = hipStreamSynchronize(S->stream);
        std::lock_guard<std::mutex> lk(S->mu);
        S->steps += S->p.steps_per_poll;
        S->active_sum += (int64_t)nactive * S->p.steps_per_poll;
        S->max_active_seen = std::max<int64_t>(S->max_active_seen, nactive);
        if (e != hipSuccess) {
            S->dev_error = true;
            fail_all_active(S);
            S->cv_done.notify_all();
            return;
        }
        for (auto& d : done) {
            Req* r = d.first;
            const DevStatus& ds = d.second;
            int32_t st = GABP_E_NOT_CONVERGED;
            if (ds.reason == R_CONVERGED || ds.reason == R_STAGNATED) st = GABP_OK;
            else if (ds.reason == R_DIVERGED) st = GABP_E_DIVERGED;
            S->arena.release_all(r->sizes, r->offs);
            S->slots[r->slot] = nullptr;
            finish(S, *r, st, ds.reason, ds.t);
            lists_dirty = true;
        }
        if (!done.empty()) S->cv_done.notify_all();
    }
}

gabp_status check_server_params(const gabp_server_params* p) {
    if (!p || p->struct_size != sizeof(gabp_server_params)) return GABP_E_INVALID;
    if (p->max_active < 1 || p->max_active > 1024) return GABP_E_INVALID;
    if (p->steps_per_poll < 1 || p->steps_per_poll > 64) return GABP_E_INVALID;
    if (p->max_bypass < 0) return GABP_E_INVALID;
    return GABP_OK;
}

}  // namespace

extern "C" {

void gabp_server_params_default(gabp_server_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->struct_size = sizeof(gabp_server_params);
    p->device = 0;
    p->arena_bytes = 0;
    p->max_active = 64;
    p->steps_per_poll = 2;
    p->max_bypass = 8;
}

gabp_status gabp_server_create(const gabp_server_params* params, gabp_server** out) {
    if (!out) return GABP_E_INVALID;
    *out = nullptr;
    if (check_server_params(params) != GABP_OK) return GABP_E_INVALID;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) { (void)hipGetLastError(); return GABP_E_DEVICE; }
    if (params->device < 0 || params->device >= ndev) return GABP_E_INVALID;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, params->device) != hipSuccess) return GABP_E_DEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return GABP_E_DEVICE;
    if (hipSetDevice(params->device) != hipSuccess) return GABP_E_DEVICE;
    gabp_server* S = new (std::nothrow) gabp_server();
    if (!S) return GABP_E_NOMEM;
    S->p = *params;
    size_t fb = 0, tb = 0;
    if (hipMemGetInfo(&fb, &tb) != hipSuccess) { delete S; return GABP_E_DEVICE; }
    const size_t arena = params->arena_bytes ? (size_t)params->arena_bytes : (size_t)(0.8 * (double)fb);
    const int A = params->max_active;
    bool ok = S->arena.init(arena) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipMalloc((void**)&S->d_reqs, (size_t)A * sizeof(ReqDesc)) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&S->h_reqs, (size_t)A * sizeof(ReqDesc), hipHostMallocDefault) == hipSuccess;
    ok = ok && hipMalloc((void**)&S->d_stat, (size_t)A * sizeof(DevStatus)) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&S->h_stat, (size_t)A * sizeof(DevStatus), hipHostMallocDefault) == hipSuccess;

    if (!ok) {
        (void)hipGetLastError();
        gabp_server_destroy(S);
        return GABP_E_NOMEM;
    }
    S->slots.assign((size_t)A, nullptr);
    S->worker = std::thread(worker_loop, S);
    *out = S;
    return GABP_OK;
}

gabp_status gabp_server_submit(gabp_server* S, const float* X, const float* y, int64_t N, int64_t m,
                               const gabp_svm_params* params, uint64_t* ticket) {
    if (!S || !X || !y || !params || !ticket || N < 1 || m < 1) return GABP_E_INVALID;
    std::string why;
    if (check_params(params, why) != GABP_OK) return GABP_E_INVALID;
    if (params->kernel != GABP_KERNEL_RBF) return GABP_E_INVALID;
    if (params->kstore == GABP_KSTORE_RECOMPUTE || params->box_mode == GABP_BOX_PROJECT)
        return GABP_E_INVALID;
    if (N > (int64_t)TILE * 65535) return GABP_E_INVALID;
    for (int64_t k = 0; k < N * m; ++k)
        if (!std::isfinite(X[k])) return GABP_E_INVALID;
    for (int64_t k = 0; k < N; ++k)
        if (!(y[k] == 1.0f || y[k] == -1.0f)) return GABP_E_INVALID;
    Req* r = new (std::nothrow) Req();
    if (!r) return GABP_E_NOMEM;
    r->X.assign(X, X + N * m);
    r->y.assign(y, y + N);
    r->N = N;
    r->m = m;
    r->p = *params;
    r->prec = params->precision;
    r->gram = (r->prec == PREC_FP64) ? GRAM_F64 : (r->prec == PREC_FP32) ? GRAM_F32
            : (params->gram == GABP_GRAM_BF16) ? GRAM_BF16 : (params->gram == GABP_GRAM_BF16X3) ? GRAM_BF16X3 : GRAM_BF16X6;
    r->NB = (int)((N + TILE - 1) / TILE);
    r->NPAD = (int64_t)r->NB * TILE;
    r->nt = n_tiles(r->NB);
    r->m_pad = (int)((m + 15) / 16 * 16);
    r->lam = (params->lambda_aug < 0.0) ? 1.0 / (double)N : params->lambda_aug;
    plan_sizes(*r);
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->dev_error) { delete r; return GABP_E_DEVICE; }
    if (r->footprint > S->arena.cap) { delete r; return GABP_E_NOMEM; }
    r->ticket = S->next_ticket++;
    r->t_submit = now_s();
    if (S->first_submit < 0.0) S->first_submit = r->t_submit;
    ++S->submitted;
    S->reqs[r->ticket] = r;
    S->queue.push_back(r);
    *ticket = r->ticket;
    S->cv_work.notify_one();
    return GABP_OK;
}

gabp_status gabp_server_poll(gabp_server* S, uint64_t ticket, int32_t* done) {
    if (!S || !done) return GABP_E_INVALID;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return GABP_E_INVALID;
    *done = it->second->state == 2 ? 1 : 0;
    return GABP_OK;
}

gabp_status gabp_server_wait(gabp_server* S, uint64_t ticket, double timeout_s) {
    if (!S) return GABP_E_INVALID;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return GABP_E_INVALID;
    Req* r = it->second;
    auto pred = [&] { return r->state == 2; };
    if (timeout_s < 0) S->cv_done.wait(lk, pred);
    else if (!S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred)) return GABP_E_STATE;
    return GABP_OK;
}

gabp_status gabp_server_result(gabp_server* S, uint64_t ticket, double* alpha, size_t bytes,
                               gabp_request_info* info) {
    if (!S) return GABP_E_INVALID;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return GABP_E_INVALID;
    Req* r = it->second;
    if (r->state != 2) return GABP_E_STATE;
    if (alpha) {
        if (bytes < r->alpha.size() * 8) return GABP_E_BUFSIZE;
        std::memcpy(alpha, r->alpha.data(), r->alpha.size() * 8);
    }
    if (info) {
        info->status = r->status;
        info->reason = r->reason;
        info->sweeps = r->sweeps;
        info->stateless_levels = r->levels;
        info->N = r->N;
        info->latency_ms = (r->t_done - r->t_submit) * 1e3;
        info->queue_ms = (r->t_admit - r->t_submit) * 1e3;
        info->device_bytes = (double)r->footprint;
    }
    return GABP_OK;
}

gabp_status gabp_server_stats_get(gabp_server* S, gabp_server_stats* out) {
    if (!S || !out) return GABP_E_INVALID;
    std::lock_guard<std::mutex> lk(S->mu);
    std::memset(out, 0, sizeof *out);
    out->submitted = S->submitted;
    out->completed = S->completed;
    out->failed = S->failed;
    std::vector<double> l = S->lat_ms;
    std::sort(l.begin(), l.end());
    auto pct = [&](double q) {
        if (l.empty()) return 0.0;
        const double pos = q * (double)(l.size() - 1);
        const size_t lo = (size_t)std::floor(pos), hi = (size_t)std::ceil(pos);
        return l[lo] + (l[hi] - l[lo]) * (pos - (double)lo);
    };
    out->p50_ms = pct(0.50);
    out->p99_ms = pct(0.99);
    out->max_ms = l.empty() ? 0.0 : l.back();
    double sm = 0.0, sq = 0.0;
    for (double v : l) sm += v;
    for (double v : S->queue_ms) sq += v;
    out->mean_ms = l.empty() ? 0.0 : sm / (double)l.size();
    out->mean_queue_ms = S->queue_ms.empty() ? 0.0 : sq / (double)S->queue_ms.size();
    const double span = S->last_done - S->first_submit;
    out->throughput_per_s = (span > 0.0) ? (double)(S->completed + S->failed) / span : 0.0;
    out->mean_active = S->steps ? (double)S->active_sum / (double)S->steps : 0.0;
    out->max_active_seen = S->max_active_seen;
    out->steps = S->steps;
    return GABP_OK;
}

void gabp_server_destroy(gabp_server* S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    if (S->worker.joinable()) S->worker.join();
    (void)hipSetDevice(S->p.device);
    if (S->stream) (void)hipStreamSynchronize(S->stream);
    for (auto& kv : S->groups) {
        auto& G = kv.second;
        if (G.d_tiles) (void)hipFree(G.d_tiles);
        if (G.h_tiles) (void)hipHostFree(G.h_tiles);
    }
    for (auto& L : S->step_lists) {
        if (L.d) (void)hipFree(L.d);
        if (L.h) (void)hipHostFree(L.h);
    }
    if (S->d_slots) (void)hipFree(S->d_slots);
    if (S->h_slots) (void)hipHostFree(S->h_slots);
    if (S->d_reqs) (void)hipFree(S->d_reqs);
    if (S->h_reqs) (void)hipHostFree(S->h_reqs);
    if (S->d_stat) (void)hipFree(S->d_stat);
    if (S->h_stat) (void)hipHostFree(S->h_stat);
    S->arena.destroy();
    if (S->stream) (void)hipStreamDestroy(S->stream);
    for (auto& kv : S->reqs) delete kv.second;
    delete S;
}

}  // extern "C"
