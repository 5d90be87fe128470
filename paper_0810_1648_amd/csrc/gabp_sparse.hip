// Sparsified kernel (the closing discussion's route to millions of points):
// the message graph keeps the pairs with exp(-gamma d^2) >= tau, i.e.
// d^2 <= cut = -ln(tau) / gamma, with K'_ij = exp(-gamma d^2) + lambda^2 on
// them and no message on the others.  GaBP itself is unchanged (Algorithm 2
// with N(i) the kept neighbours); the pair records live in edge order.
//
// Build (every pair is examined once, on MFMA, as for the dense K'):
//   k_sp_count  per 256 x 256 tile: kept pairs i < j;
//   k_sp_fill   per tile: 64-bit keys (i << 32 | j) and K' at the tile's
//               offset (order inside a tile is arbitrary);
//   radix sort of the keys: edges in (i, j) order, so every node's edges
//   with the node as i-end are contiguous; a second sort by (j, i) gives
//   the permutation listing each node's edges as j-end.
// Sweep (Algorithm 2, synchronous, information form): one thread per edge
// updates both directions from the previous records and aggregates; one
// thread per node adds its incoming messages in a fixed order (its i-end
// edges, then its j-end edges), so every result is reproducible.
#include "gabp_device.h"

#include <hipcub/hipcub.hpp>

namespace gabp {

namespace {

// Thresholded distances of one tile on MFMA.  Wave w walks the 32-row bands
// w and w + 4 and the eight 32-column blocks; `visit(i, j, d2)` is called for
// every kept pair i < j < N with lane-uniform control flow.
template <int KIND, int MP, class Visit>
__device__ inline void sp_tile(const Features& F, const TileCoord& tc, int64_t N, float cut, Visit&& visit) {
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6, h = l >> 5, l32 = l & 31;
    const int64_t i0 = (int64_t)tc.I * TILE, j0 = (int64_t)tc.J * TILE;
#pragma unroll 1
    for (int pass = 0; pass < 2; ++pass) {
        const int band = w + 4 * pass;
        const int64_t rowA = i0 + band * 32 + l32;
        float ni[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) ni[r] = F.nrm[i0 + band * 32 + 8 * (r >> 2) + 4 * h + (r & 3)];
        RowFrag<KIND, MP> fa;
        fa.load(F, rowA);
#pragma unroll 1
        for (int cb = 0; cb < TILE / 32; ++cb) {
            // blocks wholly below the diagonal hold no pair i < j
            if (j0 + cb * 32 + 31 < i0 + band * 32) continue;
            const int64_t j = j0 + cb * 32 + l32;
            const f32x16 acc = fa.gram(F, rowA, F, j);
            const float nj = F.nrm[j];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t i = i0 + band * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
                // one explicit FMA: the count and fill passes round identically
                const float d2 = fmaxf(fmaf(-2.0f, acc[r], ni[r] + nj), 0.0f);
                const bool keep = (i < j) && (j < N) && (d2 <= cut);
                visit(keep, i, j, d2);
            }
        }
    }
}

template <int KIND, int MP>
__global__ __launch_bounds__(WG) void k_sp_count(Features F, const uint32_t* __restrict__ tiles, int64_t N,
                                                 float cut, int32_t* __restrict__ counts) {
    __shared__ int wsum[4];
    const TileCoord tc = tile_of(tiles);
    int c = 0;
    sp_tile<KIND, MP>(F, tc, N, cut, [&](bool keep, int64_t, int64_t, float) { c += keep ? 1 : 0; });
    // wave sum, then workgroup sum (integer: order does not matter)
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) counts[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// Writes never leave the tile's range [offsets[t], offsets[t] + counts[t]);
// a pass that keeps a different number of pairs than the count pass sets
// *flag (the host then stops with an error instead of using the graph).
template <int KIND, int MP>
__global__ __launch_bounds__(WG) void k_sp_fill(Features F, const uint32_t* __restrict__ tiles, int64_t N,
                                                float cut, float neg_gamma_log2e, float lam2,
                                                const int64_t* __restrict__ offsets,
                                                const int32_t* __restrict__ counts, uint64_t* __restrict__ keys,
                                                float* __restrict__ kv, int32_t* __restrict__ flag) {
    __shared__ int cursor;
    const TileCoord tc = tile_of(tiles);
    if (threadIdx.x == 0) cursor = 0;
    __syncthreads();
    const int64_t base = offsets[blockIdx.x];
    const int cap = counts[blockIdx.x];
    const int l = threadIdx.x & 63;
    sp_tile<KIND, MP>(F, tc, N, cut, [&](bool keep, int64_t i, int64_t j, float d2) {
        // one LDS atomic per wave and register: the wave's kept lanes take
        // consecutive slots in lane order
        const uint64_t mask = __ballot(keep);
        if (mask == 0) return;
        int first = 0;
        if (l == __builtin_ctzll(mask)) first = atomicAdd(&cursor, __popcll(mask));
        first = __shfl(first, __builtin_ctzll(mask));
        if (keep) {
            const int slot = first + __popcll(mask & ((1ull << l) - 1ull));
            if (slot < cap) {
                keys[base + slot] = ((uint64_t)i << 32) | (uint64_t)j;
                kv[base + slot] = exp2f(neg_gamma_log2e * d2) + lam2;
            } else {
                atomicOr(flag, 1);
            }
        }
    });
    __syncthreads();
    if (threadIdx.x == 0 && cursor != cap) atomicOr(flag, 2);
}

// i, j of every sorted edge; node degrees as i-end and as j-end.
__global__ void k_sp_unpack(const uint64_t* __restrict__ keys, int64_t E, int32_t* __restrict__ ei,
                            int32_t* __restrict__ ej, int32_t* __restrict__ deg_i, int32_t* __restrict__ deg_j,
                            uint64_t* __restrict__ keys_t, int32_t* __restrict__ ids) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    const uint64_t k = keys[e];
    const int32_t i = (int32_t)(k >> 32), j = (int32_t)(k & 0xFFFFFFFFull);
    ei[e] = i;
    ej[e] = j;
    atomicAdd(&deg_i[i], 1);
    atomicAdd(&deg_j[j], 1);
    keys_t[e] = ((uint64_t)j << 32) | (uint64_t)i;
    ids[e] = (int32_t)e;
}

// Row sums and maxima of K' over each node's edges (the sparse r_i), written
// as one partial per node (the dense layout with a single slot); sixteen
// lanes per node as in k_sp_gather.
__global__ __launch_bounds__(WG) void k_sp_rowsum(int64_t N, const int64_t* __restrict__ off_i,
                                                  const int64_t* __restrict__ off_j,
                                                  const int32_t* __restrict__ perm, const float* __restrict__ kv,
                                                  double* __restrict__ psum, double* __restrict__ pmax) {
    const int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
    const int q = threadIdx.x & 15;
    double s = 0.0, m = 0.0;
    if (k < N) {
        for (int64_t e = off_i[k] + q; e < off_i[k + 1]; e += 16) { s += (double)kv[e]; m = fmax(m, (double)kv[e]); }
        for (int64_t t = off_j[k] + q; t < off_j[k + 1]; t += 16) {
            const double v = (double)kv[perm[t]];
            s += v;
            m = fmax(m, v);
        }
    }
    s = sum16(s);
    m = fmax(m, dpp<0xB1>(m));
    m = fmax(m, dpp<0x4E>(m));
    m = fmax(m, dpp<0x141>(m));
    m = fmax(m, dpp<0x140>(m));
    if (k < N && q == 0) { psum[k] = s; pmax[k] = m; }
}

// Aggregates of every node packed as (P~, S) pairs, so that the sweep's
// reads of a random neighbour fetch one 8- or 16-byte item.
template <class AT>
__global__ void k_sp_pack(int64_t N, const AT* __restrict__ Pt, const AT* __restrict__ S, AT* __restrict__ PS,
                          const DevStatus* st) {
    if (st->done) return;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < N) { PS[2 * k] = Pt[k]; PS[2 * k + 1] = S[k]; }
}

// One synchronous sweep over the edges: both directions of edge (i, j) from
// the previous records and aggregates.  Records are (P, E) pairs: RF[e] the
// message i -> j, RB[e] the message j -> i (ST), aggregates (P~, S) pairs
// (AT), arithmetic in MT.
template <class ST, class MT, class AT>
__global__ __launch_bounds__(WG) void k_sp_sweep(int64_t E, const int32_t* __restrict__ ei,
                                                 const int32_t* __restrict__ ej, const float* __restrict__ kv,
                                                 const AT* __restrict__ PS, ST* __restrict__ RF,
                                                 ST* __restrict__ RB, DevStatus* st) {
    if (st->done) return;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false;
    if (e < E) {
        const int32_t i = ei[e], j = ej[e];
        const MT a = (MT)kv[e];
        const MT pf = (MT)RF[2 * e], ef = (MT)RF[2 * e + 1], pb = (MT)RB[2 * e], eb = (MT)RB[2 * e + 1];
        const MT Pi = (MT)PS[2 * (int64_t)i], Si = (MT)PS[2 * (int64_t)i + 1];
        const MT Pj = (MT)PS[2 * (int64_t)j], Sj = (MT)PS[2 * (int64_t)j + 1];
        const MT qf = Pi - pb;      // P~_i - P_ji
        const MT qb = Pj - pf;      // P~_j - P_ij
        bad = !(qf > (MT)0) || !(qb > (MT)0);
        const MT rf = rcp_fast(qf), rb = rcp_fast(qb);
        const MT a2 = a * a;
        RF[2 * e] = (ST)(-a2 * rf);
        RF[2 * e + 1] = (ST)(-a * (Si - eb) * rf);
        RB[2 * e] = (ST)(-a2 * rb);
        RB[2 * e + 1] = (ST)(-a * (Sj - ef) * rb);
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) st->bad = 1;
}

// Incoming messages of every node: sixteen lanes (one DPP row) per node
// stride over its i-end edges (the reverse records j -> i) and its j-end
// edges (the records i -> j), then add their partial sums in a fixed tree,
// so every result is reproducible and the reads of a segment coalesce.
template <class ST, class AT>
__global__ __launch_bounds__(WG) void k_sp_gather(int64_t N, const int64_t* __restrict__ off_i,
                                                  const int64_t* __restrict__ off_j,
                                                  const int32_t* __restrict__ perm, const ST* __restrict__ RF,
                                                  const ST* __restrict__ RB, AT* __restrict__ partP,
                                                  AT* __restrict__ partE, const DevStatus* st) {
    if (st->done) return;
    const int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
    const int q = threadIdx.x & 15;
    AT p = 0, e = 0;
    if (k < N) {
        const int64_t a0 = off_i[k], a1 = off_i[k + 1];
        for (int64_t t = a0 + q; t < a1; t += 16) { p += (AT)RB[2 * t]; e += (AT)RB[2 * t + 1]; }
        const int64_t b0 = off_j[k], b1 = off_j[k + 1];
        for (int64_t t = b0 + q; t < b1; t += 16) {
            const int64_t x = perm[t];
            p += (AT)RF[2 * x];
            e += (AT)RF[2 * x + 1];
        }
    }
    p = sum16(p);
    e = sum16(e);
    if (k < N && q == 0) { partP[k] = p; partE[k] = e; }
}

template <int KIND>
void sp_build_kind(bool fill, int mp, dim3 g, const Features& F, const uint32_t* tiles, int64_t N, float cut,
                   float c, float lam2, int32_t* counts, const int64_t* offsets, uint64_t* keys, float* kv,
                   int32_t* flag, hipStream_t s) {
#define GABP_SP_LAUNCH(MPV)                                                                                  \
    do {                                                                                                     \
        if (fill)                                                                                            \
            hipLaunchKernelGGL((k_sp_fill<KIND, MPV>), g, dim3(WG), 0, s, F, tiles, N, cut, c, lam2, offsets, \
                               counts, keys, kv, flag);                                                      \
        else                                                                                                 \
            hipLaunchKernelGGL((k_sp_count<KIND, MPV>), g, dim3(WG), 0, s, F, tiles, N, cut, counts);        \
    } while (0)
    if (mp <= 32) GABP_SP_LAUNCH(32);
    else if (mp <= 64) GABP_SP_LAUNCH(64);
    else if (mp <= 128) GABP_SP_LAUNCH(128);
    else GABP_SP_LAUNCH(0);
#undef GABP_SP_LAUNCH
}

hipError_t sp_build(bool fill, const Features& F, const uint32_t* tiles, int64_t ntiles, int64_t N, float cut,
                    float c, float lam2, int32_t* counts, const int64_t* offsets, uint64_t* keys, float* kv,
                    int32_t* flag, hipStream_t s) {
    const dim3 g((unsigned)ntiles);
    switch (F.kind) {
        case GRAM_F32: sp_build_kind<GRAM_F32>(fill, F.m_pad, g, F, tiles, N, cut, c, lam2, counts, offsets, keys, kv, flag, s); break;
        case GRAM_BF16: sp_build_kind<GRAM_BF16>(fill, F.m_pad, g, F, tiles, N, cut, c, lam2, counts, offsets, keys, kv, flag, s); break;
        case GRAM_BF16X3: sp_build_kind<GRAM_BF16X3>(fill, F.m_pad, g, F, tiles, N, cut, c, lam2, counts, offsets, keys, kv, flag, s); break;
        case GRAM_BF16X6: sp_build_kind<GRAM_BF16X6>(fill, F.m_pad, g, F, tiles, N, cut, c, lam2, counts, offsets, keys, kv, flag, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + WG - 1) / WG); }

}  // namespace

hipError_t launch_sp_count(const Features& F, const uint32_t* tiles, int64_t ntiles, int64_t N, float cut,
                           int32_t* counts, hipStream_t s) {
    return sp_build(false, F, tiles, ntiles, N, cut, 0.0f, 0.0f, counts, nullptr, nullptr, nullptr, nullptr, s);
}

hipError_t launch_sp_fill(const Features& F, const uint32_t* tiles, int64_t ntiles, int64_t N, float cut,
                          float neg_gamma_log2e, float lam2, const int64_t* offsets, const int32_t* counts,
                          uint64_t* keys, float* kv, int32_t* flag, hipStream_t s) {
    return sp_build(true, F, tiles, ntiles, N, cut, neg_gamma_log2e, lam2, const_cast<int32_t*>(counts), offsets,
                    keys, kv, flag, s);
}

hipError_t sp_scan(void* tmp, size_t* bytes, const int32_t* in, int64_t* out, int64_t n, hipStream_t s) {
    return hipcub::DeviceScan::ExclusiveSum(tmp, *bytes, in, out, (int)n, s);
}

hipError_t sp_sort_keys(void* tmp, size_t* bytes, const uint64_t* kin, uint64_t* kout, const float* vin,
                        float* vout, int64_t n, hipStream_t s) {
    return hipcub::DeviceRadixSort::SortPairs(tmp, *bytes, kin, kout, vin, vout, (int)n, 0, 64, s);
}

hipError_t sp_sort_ids(void* tmp, size_t* bytes, const uint64_t* kin, uint64_t* kout, const int32_t* vin,
                       int32_t* vout, int64_t n, hipStream_t s) {
    return hipcub::DeviceRadixSort::SortPairs(tmp, *bytes, kin, kout, vin, vout, (int)n, 0, 64, s);
}

hipError_t launch_sp_unpack(const uint64_t* keys, int64_t E, int32_t* ei, int32_t* ej, int32_t* deg_i,
                            int32_t* deg_j, uint64_t* keys_t, int32_t* ids, hipStream_t s) {
    if (E > 0)
        hipLaunchKernelGGL(k_sp_unpack, dim3(blocks(E)), dim3(WG), 0, s, keys, E, ei, ej, deg_i, deg_j, keys_t, ids);
    return hipGetLastError();
}

hipError_t launch_sp_rowsum(int64_t N, const int64_t* off_i, const int64_t* off_j, const int32_t* perm,
                            const float* kv, double* psum, double* pmax, hipStream_t s) {
    hipLaunchKernelGGL(k_sp_rowsum, dim3(blocks(16 * N)), dim3(WG), 0, s, N, off_i, off_j, perm, kv, psum, pmax);
    return hipGetLastError();
}

hipError_t launch_sp_sweep(int prec, int64_t E, int64_t N, const int32_t* ei, const int32_t* ej, const float* kv,
                           const void* Pt, const void* S, void* PS, void* RF, void* RB, const int64_t* off_i,
                           const int64_t* off_j, const int32_t* perm, void* partP, void* partE, DevStatus* st,
                           hipStream_t s) {
    const dim3 ge(blocks(std::max<int64_t>(E, 1))), gn(blocks(16 * N)), g1(blocks(N)), b(WG);
    switch (prec) {
        case PREC_FP32:
            hipLaunchKernelGGL(k_sp_pack<float>, g1, b, 0, s, N, (const float*)Pt, (const float*)S, (float*)PS, st);
            hipLaunchKernelGGL((k_sp_sweep<float, float, float>), ge, b, 0, s, E, ei, ej, kv, (const float*)PS,
                               (float*)RF, (float*)RB, st);
            hipLaunchKernelGGL((k_sp_gather<float, float>), gn, b, 0, s, N, off_i, off_j, perm, (const float*)RF,
                               (const float*)RB, (float*)partP, (float*)partE, st);
            break;
        case PREC_MIXED:
            hipLaunchKernelGGL(k_sp_pack<double>, g1, b, 0, s, N, (const double*)Pt, (const double*)S,
                               (double*)PS, st);
            hipLaunchKernelGGL((k_sp_sweep<float, double, double>), ge, b, 0, s, E, ei, ej, kv, (const double*)PS,
                               (float*)RF, (float*)RB, st);
            hipLaunchKernelGGL((k_sp_gather<float, double>), gn, b, 0, s, N, off_i, off_j, perm, (const float*)RF,
                               (const float*)RB, (double*)partP, (double*)partE, st);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace gabp
