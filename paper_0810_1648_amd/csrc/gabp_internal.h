// Internal declarations shared by the host runtime and the HIP kernels of
// the GaBP SVM solver.  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>

#include <string>

#include "../../include/gabp_svm.h"

namespace gabp {

// Pairs {i, j}, i < j, are processed in TILE x TILE tiles of the upper
// triangle; every per-pair device array is a sequence of full tiles stored
// row-major (tile-local row r, column c at r * TILE + c).
constexpr int TILE = 256;
constexpr int TT = TILE * TILE;
constexpr int WG = 256;               // threads per workgroup (4 wave64)

enum Prec : int { PREC_FP64 = 0, PREC_FP32 = 1, PREC_MIXED = 2 };
enum GramKind : int { GRAM_F32 = 0, GRAM_BF16 = 1, GRAM_BF16X3 = 2, GRAM_F64 = 3, GRAM_BF16X6 = 4 };
enum KSrc : int { KSRC_PLANE = 0, KSRC_RECOMPUTE = 1 };
enum Reason : int { R_NONE = 0, R_CONVERGED = 1, R_MAX_SWEEPS = 2, R_DIVERGED = 3, R_STAGNATED = 4 };

// Device-resident solve status, advanced by k_status once per sweep.  Every
// sweep kernel returns at once when `done` is set, so the state a solve
// stops in does not depend on how often the host polls.
struct DevStatus {
    int32_t t;           // completed sweeps
    int32_t done;
    int32_t reason;
    int32_t since_best;  // sweeps since the smallest change so far
    int32_t bad;         // set when a cavity precision <= 0 or a value is not finite
    int32_t g;           // served grouped schedule: the group the next step visits
    double delta;        // ||alpha^t - alpha^(t-1)||_inf
    double amax;         // ||alpha^t||_inf
    double best_delta;
};

struct StopRule {
    double tol_abs, tol_rel, stag_rel;
    int32_t max_sweeps, stag_window;
};

// Features staged for the Gram: row-major NPAD x m_pad, zero padded.
struct Features {
    const float* f32;        // GRAM_F32: centred FP32
    const uint16_t* hi;      // GRAM_BF16/BF16X3: centred, rounded to BF16
    const uint16_t* lo;      // GRAM_BF16X3/X6: BF16 of the rounding remainder x - hi
    const uint16_t* lo2;     // GRAM_BF16X6: BF16 of the second remainder x - hi - lo
    const double* f64;       // GRAM_F64: uncentred FP64
    const float* nrm;        // squared norms of the staged rows (FP32)
    int32_t m_pad;
    int32_t kind;            // GramKind
    // BF16 kinds with m + 2 <= m_pad, K' recomputed: the training rows
    // augmented as (x, |x|^2, 1) (aug0) and (c x, -c/2, -c/2 |x|^2) (aug1,
    // c = 2 gamma log2(e)), in the kind's split planes `aug_plane` apart, so
    // that their Gram is the exponent -gamma log2(e) |x_i - x_j|^2 itself
    // (null: K' from the plain Gram and the norms)
    const uint16_t* aug0;
    const uint16_t* aug1;
    int64_t aug_plane;
};

struct KernelParams {
    int64_t N;
    int32_t NB;
    float neg_gamma_log2e;   // -gamma * log2(e): K = exp2(neg_gamma_log2e * d2)
    double gamma;
    double lam2;             // lambda^2 added to every RBF entry
};

// Validates a parameter struct (shared by the solver and the server).
gabp_status check_params(const gabp_svm_params* p, std::string& why);

inline int64_t n_tiles(int NB) { return (int64_t)NB * (NB + 1) / 2; }

// Stateless plan from the contraction bound.  rr = 1.25 rho bounds
// |A_ij| / Q_ij, the factor with which a reverse message enters the next
// one, so unrolling `levels` levels truncates the recursion by about
// rr^levels.  Levels needed: the smallest count with rr^levels below the
// path's message precision, 2^-24 (FP32), 2^-30 (MIXED, FP32-stored
// messages), 2^-50 (FP64); 9 when no count up to 8 suffices.
inline int stateless_levels_needed(int prec, double rr) {
    const double eps = (prec == PREC_FP32) ? std::ldexp(1.0, -24)
                     : (prec == PREC_MIXED) ? std::ldexp(1.0, -30) : std::ldexp(1.0, -50);
    if (rr == 0.0) return 1;
    if (!(rr < 1.0)) return 9;
    return std::max(1, (int)std::ceil(std::log(eps) / std::log(rr)));
}
// Reciprocal form of a stateless plan: 0 exact reciprocals; 1 / 2 series
// around 1/P~ with a one- / two-term top level; 3 a one-term top level over
// lower levels that take G = 1/P~ (no series term).  |e| <= rr^2, so the
// one-term lower levels err by rr^4, entering the top level scaled by rr,
// and the top level errs by rr^4 (one term) or rr^6 (two terms).  Form 3
// drops the lower levels' e: G errs by rr^2, which reaches the top level's
// precision term scaled by rr^2 (rr^4) and its mean term through F scaled by
// rr (rr^3); it needs a middle level (levels >= 3).  Each error must stay
// below the precision of the message arithmetic (FP32 messages: FP32 and
// MIXED; FP64 messages: FP64).
inline int stateless_series_form(int prec, int levels, double rr) {
    const double eps = (prec == PREC_FP64) ? std::ldexp(1.0, -52) : std::ldexp(1.0, -24);
    if (levels < 1 || levels > 6 || !(rr < 0.25) || std::pow(rr, 5) > eps) return 0;
    if (std::pow(rr, 4) <= eps) return (levels >= 3 && std::pow(rr, 3) <= eps) ? 3 : 1;
    if (std::pow(rr, 6) <= eps) return 2;
    return 0;
}
// Entries of the grouped schedule's visit lists: bit 31 = messages into the
// row block (BWD; clear: into the column block), bit 30 = both blocks lie in
// the visited group, low 30 bits = tile index.
constexpr uint32_t GE_BWD = 0x80000000u, GE_WITHIN = 0x40000000u, GE_TILE = 0x3FFFFFFFu;
// Synchronous stateless sweeps over an FP32 K' plane with FP32 partial sums
// (FP32 plan, or FP32 messages) run over 2 x 2 chunks of tiles where the
// chunk's sums fit beside the message recursion in the registers of four
// waves per SIMD: one level, two with series reciprocals, three with series
// form 3.
__host__ __device__ constexpr bool chunk_plan(bool fp32_partials, int levels, int ser) {
    return fp32_partials && (levels == 1 || (levels == 2 && ser > 0) || (levels == 3 && ser == 3));
}
// The choice for one solve (`mode`: the tile_chunk parameter): automatic
// (0) takes chunks only with at least four per workgroup slot of the GPU (256
// CUs x 4 workgroups), since fewer balance worse than single tiles; 1 never,
// 2 wherever the plan allows.
constexpr int64_t kChunkMin = 4096;
inline bool chunk_sweep(bool fp32_partials, int levels, int ser, int NB, int mode) {
    const int64_t nbc = (NB + 1) / 2;
    if (mode == 1 || !chunk_plan(fp32_partials, levels, ser)) return false;
    return mode == 2 || nbc * (nbc + 1) / 2 >= kChunkMin;
}
// Storage index of tile (I, J), I <= J: row-major over the upper triangle.
__host__ __device__ inline int64_t tile_index(int I, int J, int NB) {
    return (int64_t)I * NB - (int64_t)I * (I - 1) / 2 + (J - I);
}

// ---- launchers (gabp_kernels.hip); all asynchronous on `s` ----
hipError_t launch_fill_tiles(uint32_t* tiles, int NB, hipStream_t s);
hipError_t launch_validate(const float* X, const float* y, int64_t N, int64_t m,
                           int32_t* flag, hipStream_t s);
hipError_t launch_colmean(const float* X, int64_t N, int64_t m, double* mean, hipStream_t s);
hipError_t launch_stage(const float* X, const double* mean, int64_t N, int64_t m,
                        int64_t NPAD, int m_pad, int kind, float* f32, uint16_t* hi,
                        uint16_t* lo, uint16_t* lo2, double* f64, float* nrm, hipStream_t s);
// FP32-stored K' (every Gram kind but FP64) together with the row/column
// sum and maximum partials of k_rowsum, in one pass.  `tiles` lists the
// upper tiles in any order (each is written at its tile_index position).
hipError_t launch_gram_sums(const Features& F, const KernelParams& kp, const uint32_t* tiles, int64_t ntiles,
                            void* Kp, int NB, double* psum, double* pmax, hipStream_t s);
hipError_t launch_gram(const Features& F, const KernelParams& kp, const uint32_t* tiles,
                       int64_t ntiles, void* Kp, hipStream_t s);
hipError_t launch_gather_dense(const double* K, const KernelParams& kp,
                               const uint32_t* tiles, int64_t ntiles, void* Kp, int prec,
                               double* kdiag, hipStream_t s);
hipError_t launch_fill_value(double* dst, int64_t n, double v, hipStream_t s);
hipError_t launch_rowsum(const void* Kp, int prec, int ksrc, const Features& F,
                         const KernelParams& kp, const uint32_t* tiles, int64_t ntiles, int NB,
                         double* psum, double* pmax, hipStream_t s);
hipError_t launch_diag(int64_t N, int NB, const double* psum, const double* pmax,
                       const double* kdiag, int mode, double C, double delta, double* Adiag,
                       double* rowmax, double* rsum, double* scratch_blk, double* scratch_one,
                       hipStream_t s);
// boxC > 0 (here and in the finalize launchers): belief means projected
// onto [0, boxC] (the box-projected variant); 0: no projection.
hipError_t launch_init(int prec, int64_t N, int64_t NPAD, int R, const double* Adiag, const float* y,
                       void* Pt, void* S, double* alpha, DevStatus* st, hipStream_t s, double boxC = 0.0);

// Arguments of one sweep launch.  HP/HS are rings of R aggregate vectors
// (NPAD entries each); slot_top holds the aggregates of the previous sweep,
// slot_top - k (mod R) those k sweeps earlier.
struct SweepArgs {
    const uint32_t* tiles;
    int64_t ntiles;
    int NB;
    const void* Kp;               // K' plane (KSRC_PLANE)
    void *Pf, *Pb, *Ef, *Eb;      // pair planes: P_ij, P_ji, E_ij, E_ji (i < j), stored state
    const void *HP, *HS;          // aggregate rings
    const void *HI, *HM;          // series: rings of 1/P~ and S/P~ (null: formed in the tile)
    int64_t NPAD;
    int R, slot_top, levels;      // ring depth, top slot, stateless levels in use
    int part32;                   // 1: partial sums stored in FP32 (FP32-message plans)
    void *partP, *partE;          // [NB][NB+1][TILE] partial sums (aggregate type, or FP32); chunked
                                  // sweeps: [NB][NBc+1][TILE], NBc = ceil(NB / chunk)
    const uint32_t* chunks;       // chunked synchronous sweep: Ic << 16 | Jc, Ic <= Jc < NBc (row-major)
    int64_t nchunks;
    int chunk;                    // tiles per chunk side (0 or 1: one tile per workgroup)
    DevStatus* st;
    Features F;                   // KSRC_RECOMPUTE
    KernelParams kp;
};
// Per-request state of the served form: sweep arguments plus what the
// finalize and stop-rule steps need.  Aggregates live in sw.HP / sw.HS (ring
// of sw.R slots: 1 for stored pair records, 8 for the stateless form; the
// slot of a sweep follows from the request's sweep count).
struct ReqDesc {
    SweepArgs sw;
    int64_t N;
    const double* Adiag;
    const float* y;
    double* alpha;
    double* blk_delta;
    double* blk_amax;
    double* trace;
    StopRule rule;
    int nblk;
    int G;               // groups of the grouped schedule (1: synchronous)
};
// One served step for the requests of one group (precision, level count:
// 0 = stored pair records, >= 1 stateless; series reciprocals): batched sweep
// over the (request, tile) items, batched finalize over the (request, node
// block) items, batched stop rule for the request slots listed in `slots`,
// whose statuses are copied to status_out[0..nslots).
// A served step, launched in this order on one stream: the batched sweep of
// every launch group (items (request, tile); grouped: (request, list entry)
// of each request's current group), the batched finalize of the (request,
// node block) items of each aggregate type (grouped: the current group's
// blocks), and the stop rule of every active request (grouped: after the
// visit of its last group; G = 1 is the synchronous schedule), whose
// statuses are copied to status_out[0..nslots).
hipError_t launch_served_sweep(int prec, int levels, int ser, bool grouped, const ReqDesc* reqs, const uint2* items,
                               int n, hipStream_t s);
hipError_t launch_served_finalize(bool agg_f32, const ReqDesc* reqs, const uint2* items, int n, hipStream_t s);
hipError_t launch_served_status(const ReqDesc* reqs, const int* slots, int nslots, DevStatus* status_out,
                                hipStream_t s);
hipError_t launch_served_sweep_f32(int levels, int ser, bool grouped, const ReqDesc* reqs, const uint2* items, int n,
                                   hipStream_t s);
hipError_t launch_served_sweep_mixed(int levels, int ser, bool grouped, const ReqDesc* reqs, const uint2* items,
                                     int n, hipStream_t s);
hipError_t launch_served_sweep_f64(int levels, int ser, bool grouped, const ReqDesc* reqs, const uint2* items, int n,
                                   hipStream_t s);
// depth 0 = stored edge state, 1..8 = stateless with up to `depth` levels.
// levels: 0 = stored edge state, >= 1 = stateless with that many levels in
// this launch; ser: stateless reciprocals by the series around 1/P~;
// e0 / e1 (optional): events that take the kernel's begin / end timestamps.
hipError_t launch_sweep(int prec, int ksrc, int gram, int levels, bool first, int ser, const SweepArgs& a,
                        hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_sweep_f32(int ksrc, int gram, int levels, bool first, int ser, const SweepArgs& a,
                            hipStream_t s, hipEvent_t e0, hipEvent_t e1);
hipError_t launch_sweep_mixed(int ksrc, int gram, int levels, bool first, int ser, const SweepArgs& a,
                              hipStream_t s, hipEvent_t e0, hipEvent_t e1);
hipError_t launch_sweep_f64(int ksrc, int gram, int levels, bool first, int ser, const SweepArgs& a,
                            hipStream_t s, hipEvent_t e0, hipEvent_t e1);
// Inv / Mean (optional, with Pt / S): the new 1/P~ and S/P~ of the series
// sweeps, formed once per node here instead of in every tile.  part32: the
// partial sums are FP32 (SweepArgs::part32).
hipError_t launch_finalize(int prec, int64_t N, int NB, const void* partP, const void* partE,
                           const double* Adiag, const float* y, void* Pt, void* S,
                           double* alpha, double* blk_delta, double* blk_amax,
                           DevStatus* st, hipStream_t s, double boxC = 0.0, void* Inv = nullptr,
                           void* Mean = nullptr, int part32 = 0);
// Inv / Mean of every ring slot from Pt / S (R slots of NPAD entries).
hipError_t launch_ring_recip(int prec, int64_t NPAD, int R, const void* Pt, const void* S, void* Inv, void* Mean,
                             hipStream_t s);
// Grouped schedule: one group visit.  `within` lists the stored-record tiles
// inside the group (both directions), `dir` the single-direction entries
// (tile index | GE_BWD | GE_WITHIN bits, see gabp_device.h); t = sweep index.
hipError_t launch_sweep_grouped(int prec, int ksrc, int gram, int levels, int ser, const SweepArgs& a,
                                const uint32_t* within, int nwithin, const uint32_t* dir, int ndir, int t,
                                hipStream_t s);
hipError_t launch_sweep_grouped_f32(int ksrc, int gram, int levels, int ser, const SweepArgs& a,
                                    const uint32_t* within, int nwithin, const uint32_t* dir, int ndir, int t,
                                    hipStream_t s);
hipError_t launch_sweep_grouped_mixed(int ksrc, int gram, int levels, int ser, const SweepArgs& a,
                                      const uint32_t* within, int nwithin, const uint32_t* dir, int ndir, int t,
                                      hipStream_t s);
hipError_t launch_sweep_grouped_f64(int ksrc, int gram, int levels, int ser, const SweepArgs& a,
                                    const uint32_t* within, int nwithin, const uint32_t* dir, int ndir, int t,
                                    hipStream_t s);
// Sparsified kernel (gabp_sparse.hip): build passes, sorts and scans (the
// temporary storage size comes back in *bytes when tmp is NULL), and the
// sweep (edge update + per-node gather into one partial per node).
// count: kept pairs of tiles[0], tiles[stride], ... (ntiles launched);
// fill: every listed tile's kept pairs appended at *cursor (slots >= cap
// counted, not written).
// FA, FB: the augmented A and B rows (launch_sp_augment), whose Gram is
// -d^2 / 2.
hipError_t launch_sp_count(const Features& FA, const Features& FB, const uint32_t* tiles, int64_t ntiles,
                           int64_t stride, int64_t N, float cut, int32_t* counts, hipStream_t s);
hipError_t launch_sp_fill(const Features& FA, const Features& FB, const uint32_t* tiles, int64_t ntiles, int64_t N,
                          float cut, float neg_gamma_log2e, float lam2, int64_t cap, unsigned long long* cursor,
                          uint64_t* keys, float* kv, hipStream_t s);
// Columns m, m + 1 (< m_pad) of the staged rows: A planes (n_i, 1), B planes
// the first m columns of A and (-1/2, -n_i/2); NPAD rows.
hipError_t launch_sp_augment(int64_t NPAD, int64_t m, int m_pad, int kind, const float* nrm, float* f32a,
                             uint16_t* hia, uint16_t* loa, uint16_t* lo2a, float* f32b, uint16_t* hib,
                             uint16_t* lob, uint16_t* lo2b, hipStream_t s);
hipError_t sp_scan(void* tmp, size_t* bytes, const int32_t* in, int64_t* out, int64_t n, hipStream_t s);
// The tile list in super-blocked order (S x S tiles per super-block, NB
// blocks per side), through the key buffers k0, k1 (nt entries each).
hipError_t sp_tile_order(void* tmp, size_t* bytes, uint32_t* tiles, int64_t nt, int S, int NB, uint64_t* k0,
                         uint64_t* k1, hipStream_t s);
// Locality order: nearest of the K landmark points lm[] for every point
// (key = landmark << 32 | point, ids = point), rows permuted into that order,
// block centroids / radii and the tiles that may hold kept pairs, compaction
// of the tile list, and per-node arrays back to input order.
hipError_t launch_sp_order(const float* X, int64_t N, int64_t m, const int32_t* lm, int K, uint64_t* key,
                           int32_t* ids, hipStream_t s);
hipError_t launch_sp_permute(const float* X, const float* y, int64_t N, int64_t m, const int32_t* order, float* Xp,
                             float* yp, hipStream_t s);
hipError_t launch_sp_prune(const float* Xp, int64_t N, int64_t m, int NB, const uint32_t* tiles, int64_t nt,
                           double cut, double* cent, double* rad, uint8_t* keep, hipStream_t s);
hipError_t sp_select(void* tmp, size_t* bytes, const uint32_t* in, const uint8_t* flags, uint32_t* out,
                     int64_t* nsel, int64_t n, hipStream_t s);
hipError_t launch_sp_unpermute(const double* in, const int32_t* order, int64_t N, double* out, hipStream_t s);
hipError_t sp_sort_keys(void* tmp, size_t* bytes, const uint64_t* kin, uint64_t* kout, const float* vin,
                        float* vout, int64_t n, hipStream_t s);
hipError_t sp_sort_ids(void* tmp, size_t* bytes, const uint64_t* kin, uint64_t* kout, const int32_t* vin,
                       int32_t* vout, int64_t n, hipStream_t s);
hipError_t launch_sp_unpack(const uint64_t* keys, int64_t E, int32_t* ei, int32_t* ej, int32_t* deg_i,
                            int32_t* deg_j, uint64_t* keys_t, int32_t* ids, hipStream_t s);
hipError_t launch_sp_rowsum(int64_t N, const int64_t* off_i, const int64_t* off_j, const int32_t* perm,
                            const float* kv, double* psum, double* pmax, hipStream_t s);
// PS: 2 N aggregates packed (P~, S); RF / RB: 2 E records packed (P, E) of
// the messages i -> j / j -> i of every edge.
hipError_t launch_sp_sweep(int prec, int64_t E, int64_t N, const int32_t* ei, const int32_t* ej, const float* kv,
                           const void* Pt, const void* S, void* PS, void* RF, void* RB, const int64_t* off_i,
                           const int64_t* off_j, const int32_t* perm, void* partP, void* partE, DevStatus* st,
                           hipStream_t s);
// Finalize of the node blocks [b0, b0 + nb) only (the group just visited).
hipError_t launch_finalize_range(int prec, int64_t b0, int64_t nb, int64_t N, int NB, const void* partP,
                                 const void* partE, const double* Adiag, const float* y, void* Pt, void* S,
                                 double* alpha, double* blk_delta, double* blk_amax, DevStatus* st,
                                 hipStream_t s, double boxC = 0.0, void* Inv = nullptr, void* Mean = nullptr,
                                 int part32 = 0);
hipError_t launch_status(int nblk, const double* blk_delta, const double* blk_amax,
                         DevStatus* st, double* trace, StopRule rule, hipStream_t s);
// A-priori contraction bound: one[0] = -m* (minus the aggregate lower
// bound), one[1] = rho (+inf when no bound exists).
hipError_t launch_rho_bound(int64_t N, const double* Adiag, const double* rowmax, const double* rsum,
                            double* blk, double* one, hipStream_t s);
// Residual certificate of a finished dense solve: out[0] = ||1 - A alpha||_inf,
// out[1] = min_i (A_ii - sum_{j != i} |A_ij|), out[2] = out[0] / out[1]
// (Varah's bound on ||alpha - A^-1 1||_inf; +inf unless out[1] > 0).  K'
// from the plane or recomputed; w (NPAD), part (partial-sum layout), blk1,
// blk2 (grid1(N)) are work buffers.
hipError_t launch_residual(const void* Kp, int prec, int ksrc, const Features& F, const KernelParams& kp,
                           const uint32_t* tiles, int64_t ntiles, int NB, int64_t N, int64_t NPAD,
                           const double* alpha, const float* y, const double* Adiag, const double* rsum,
                           double* w, double* part, double* blk1, double* blk2, double* out, hipStream_t s);
hipError_t launch_kernel_entries(const void* Kp, int prec, int NB, const int64_t* rows,
                                 const int64_t* cols, int64_t n, double* out, hipStream_t s);
// Decision function (gabp_predict.hip).  Queries are padded to
// predict_query_pad(nq) rows; the MFMA form splits the training rows into
// nchunk chunks of bpc 32-row blocks (predict_chunks) and writes
// part[nchunk][NQPAD]; the direct FP64 form writes part[nq].
int64_t predict_query_pad(int64_t nq);
// Bytes of the per-device scratch array of the allocation-free decision
// function (gabp_svm_predict_noalloc), and its device address on the current
// device (looked up once per device, then cached).
constexpr size_t PREDICT_SCRATCH_BYTES = size_t(64) << 20;
hipError_t predict_scratch(void** ptr);
void predict_chunks(int64_t NPAD, int64_t NQPAD, int* nchunk, int* bpc);
hipError_t launch_predict_weights(const double* alpha, const float* y, int64_t N, int64_t NPAD, bool box,
                                  double C, double* w, double* blk, double* wsum, hipStream_t s);
hipError_t launch_predict_direct(const float* Xtr, const double* w, int64_t N, int64_t m, const float* Xq,
                                 int64_t nq, double gamma, double* part, hipStream_t s);
hipError_t launch_predict_mfma(const Features& Ft, const Features& Fq, const double* w, int64_t NPAD,
                               int64_t NQPAD, float neg_gamma_log2e, int nchunk, int bpc, double* part,
                               hipStream_t s);
// Augmented form (BF16 split kinds, m + 2 <= mp, mp = 32 or 64): rows staged
// by launch_stage_aug (side 0 queries (x, n, 1); side 1 training rows
// c (x, -1/2, -n/2), c = 2 gamma log2(e); `out` holds np planes of NPAD x mp
// BF16); queries padded to predict_query_pad_aug, part[nchunk][NQPAD].
int64_t predict_query_pad_aug(int64_t nq);
void predict_chunks_aug(int64_t NPAD, int64_t NQPAD, int* nchunk, int* bpc);
hipError_t launch_stage_aug(const float* X, const double* mean, int64_t n, int64_t m, int64_t NPAD, int mp, int kind,
                            int side, float c, uint16_t* out, hipStream_t s);
// e0 / e1 (optional): events that take the kernel's begin / end timestamps.
hipError_t launch_predict_aug(int kind, int mp, const uint16_t* Bt, int64_t NPAD, const uint16_t* Aq, int64_t NQPAD,
                              const double* w, int nchunk, int bpc, double* part, hipStream_t s,
                              hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_predict_reduce(const double* part, int nchunk, int64_t stride, int64_t nq, const double* wsum,
                                 double lam2, double* f, hipStream_t s);
hipError_t launch_convert_agg(int prec, const void* src, double* dst, int64_t n, hipStream_t s);

}  // namespace gabp
