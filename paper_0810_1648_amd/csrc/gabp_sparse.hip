// Sparsified kernel (the closing discussion's route to millions of points):
// the message graph keeps the pairs with exp(-gamma d^2) >= tau, i.e.
// d^2 <= cut = -ln(tau) / gamma, with K'_ij = exp(-gamma d^2) + lambda^2 on
// them and no message on the others.  GaBP itself is unchanged (Algorithm 2
// with N(i) the kept neighbours); the pair records live in edge order.
//
// Build (every pair of the unpruned tiles is examined on MFMA, over rows
// augmented so that the Gram is -d^2 / 2):
//   k_sp_augment the A and B rows of the build;
//   k_sp_count  kept pairs i < j of every 32nd tile: an estimate that sizes
//               the fill's output;
//   k_sp_fill   per tile: 64-bit keys (i << 32 | j) and K' appended at a
//               global cursor (arbitrary order); a second pass runs only if
//               the estimate fell short;
//   radix sort of the keys: edges in (i, j) order, so every node's edges
//   with the node as i-end are contiguous; a second sort by (j, i) gives
//   the permutation listing each node's edges as j-end.
// Sweep (Algorithm 2, synchronous, information form): one thread per edge
// updates both directions from the previous records and aggregates;
// sixteen lanes per node add its incoming messages in a fixed order (its
// i-end edges, then its j-end edges), so every result is reproducible.
#include "gabp_device.h"

#include <hipcub/hipcub.hpp>

namespace gabp {

namespace {

// Thresholded distances of the listed tiles tiles[p0, p1) on MFMA.  The rows
// are augmented (k_sp_augment): A row a_i = (x_i, n_i, 1), B row
// b_j = (x_j, -1/2, -n_j/2) with n = ||x||^2, so the Gram a_i . b_j is
// -d_ij^2 / 2 and the keep test d^2 <= cut is a single compare of the MFMA
// output with -cut / 2.  Wave w computes the 32-row bands w and w + 4 of a
// tile together (their A fragments in registers, reloaded only when the row
// block changes, each B fragment loaded once for both) and walks the
// tiles' 32-column blocks in order, the next block's B fragment (across
// tile boundaries too) in flight during the current MFMAs.  For every
// block, `visit(g0, g1, i0r, jcol, hc)` receives the Gram values of both
// bands, where the pair of register r of a lane is kept iff its value is
// >= hc = -cut / 2 (its ballot is the block's mask for that register).
// Blocks off the diagonal tile and before the last column hold only pairs
// i < j < N; in the others the pairs outside i < j < N get -inf first, so
// that the test stays one compare everywhere.
template <int KIND, int MP, class Visit>
__device__ inline void sp_tiles(const Features& FA, const Features& FB, const uint32_t* __restrict__ tiles,
                                int64_t p0, int64_t p1, int64_t N, float cut, Visit&& visit) {
    if (p0 >= p1) return;
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6, h = l >> 5, l32 = l & 31;
    const float hc = -0.5f * cut;
    auto coord = [&](int64_t p) {
        const uint32_t ij = tiles[p];
        return TileCoord{(int)(ij >> 16), (int)(ij & 0xFFFFu)};
    };
    // first column block with a pair i < j for the wave's lower band
    auto first_cb = [&](const TileCoord& t) {
        int c = 0;
        while (c < TILE / 32 && (int64_t)t.J * TILE + c * 32 + 31 < (int64_t)t.I * TILE + w * 32) ++c;
        return c;
    };
    int64_t p = p0;
    TileCoord tc = coord(p);
    int cb = first_cb(tc);
    RowFrag<KIND, MP> fa0, fa1, fb;
    fa0.load(FA, (int64_t)tc.I * TILE + w * 32 + l32);
    fa1.load(FA, (int64_t)tc.I * TILE + (w + 4) * 32 + l32);
    if constexpr (MP > 0) fb.load(FB, (int64_t)tc.J * TILE + cb * 32 + l32);
    while (true) {
        // the next (tile, block) of the walk
        int64_t pn = p;
        TileCoord tn = tc;
        int cbn = cb + 1;
        if (cbn == TILE / 32) {
            pn = p + 1;
            if (pn < p1) {
                tn = coord(pn);
                cbn = first_cb(tn);
            }
        }
        const bool more = pn < p1;
        const int64_t i0 = (int64_t)tc.I * TILE, j0 = (int64_t)tc.J * TILE;
        const int64_t rowA0 = i0 + w * 32 + l32, rowA1 = i0 + (w + 4) * 32 + l32;
        const int64_t j = j0 + cb * 32 + l32;
        f32x16 g0 = {}, g1 = {};
        if constexpr (MP > 0) {
            RowFrag<KIND, MP> fn;
            fn.load(FB, more ? (int64_t)tn.J * TILE + cbn * 32 + l32 : j);
            frag_mma(fa0, fb, g0, FA.m_pad);
            frag_mma(fa1, fb, g1, FA.m_pad);
            fb = fn;
        } else {
            RowFrag<KIND, MP>::gram2(fa0, fa1, FA, rowA0, rowA1, FB, j, g0, g1);
        }
        if (!((tc.I < tc.J) && (j0 + cb * 32 + 31 < N))) {
            // register r of lane l holds row 8 (r / 4) + 4 (l / 32) + r % 4 of its band
            const int64_t dj = j - (i0 + w * 32 + 4 * h);
            const bool jn = j < N;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int ro = 8 * (r >> 2) + (r & 3);
                if (!(jn && dj > ro)) g0[r] = -INFINITY;
                if (!(jn && dj > ro + 128)) g1[r] = -INFINITY;
            }
        }
        visit(g0, g1, i0 + w * 32, j, hc);
        if (!more) break;
        if (tn.I != tc.I) {
            fa0.load(FA, (int64_t)tn.I * TILE + w * 32 + l32);
            fa1.load(FA, (int64_t)tn.I * TILE + (w + 4) * 32 + l32);
        }
        p = pn;
        tc = tn;
        cb = cbn;
    }
}

// Kept pairs of every stride-th listed tile (stride 1: all of them), one
// count per launched tile; the host sums a strided sample to size the fill.
template <int KIND, int MP>
__global__ __launch_bounds__(WG) void k_sp_count(Features FA, Features FB, const uint32_t* __restrict__ tiles, int64_t stride,
                                                 int64_t N, float cut, int32_t* __restrict__ counts) {
    __shared__ int wsum[4];
    int c = 0;   // wave-uniform
    sp_tiles<KIND, MP>(FA, FB, tiles + (int64_t)blockIdx.x * stride, 0, 1, N, cut, [&](const f32x16& g0, const f32x16& g1, int64_t, int64_t, float hc) {
#pragma unroll
        for (int r = 0; r < 16; ++r) c += __popcll(__ballot(g0[r] >= hc)) + __popcll(__ballot(g1[r] >= hc));
    });
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) counts[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

constexpr int SP_TPW = 16;   // listed tiles per workgroup of the fill

// Kept pairs appended at a global cursor.  A wave collects its kept pairs
// (key and K' value) in an LDS buffer, register by register in lane order;
// a full buffer is drained to slots reserved by one atomic, and at the end
// of its tiles one atomic reserves the slots of all four waves' remainders.
// The order across waves and tiles is arbitrary: the (i, j) sort that
// follows fixes it, and every pair's key and K' value do not depend on it.
// Slots at or beyond cap are not written but still counted, so the cursor
// ends at the exact number of kept pairs and the host repeats the pass with
// room for all of them.
template <int KIND, int MP>
__global__ __launch_bounds__(WG) void k_sp_fill(Features FA, Features FB, const uint32_t* __restrict__ tiles,
                                                int64_t ntiles, int64_t N,
                                                float cut, float neg_gamma_log2e, float lam2, int64_t cap,
                                                unsigned long long* __restrict__ cursor,
                                                uint64_t* __restrict__ keys, float* __restrict__ kv) {
    constexpr int BW = 512;   // entries buffered per wave
    __shared__ uint64_t bkey[4][BW];
    __shared__ float bval[4][BW];
    __shared__ unsigned long long wbase[4];
    __shared__ int wcnt[4];
    // SP_TPW consecutive listed tiles per workgroup (mostly one row block of a
    // super-block: the A fragments stay in registers)
    const int64_t p0 = xcd_contiguous(blockIdx.x, gridDim.x) * SP_TPW;
    const int64_t p1 = (p0 + SP_TPW < ntiles) ? p0 + SP_TPW : ntiles;
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6, h = l >> 5;
    const uint64_t below = (1ull << l) - 1ull;
    int n = 0;   // wave-uniform: entries in the wave's buffer
    // the wave's n buffered entries to slots base, base + 1, ...
    auto drain = [&](unsigned long long base) {
        for (int k = l; k < n; k += 64) {
            const int64_t slot = (int64_t)base + k;
            if (slot < cap) {
                keys[slot] = bkey[w][k];
                kv[slot] = bval[w][k];
            }
        }
    };
    sp_tiles<KIND, MP>(FA, FB, tiles, p0, p1, N, cut, [&](const f32x16& g0, const f32x16& g1, int64_t ib, int64_t j,
                                                          float hc) {
#pragma unroll
        for (int half = 0; half < 2; ++half) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const float gv = half ? g1[r] : g0[r];
                const uint64_t mask = __ballot(gv >= hc);
                if (mask == 0) continue;
                if (n + 64 > BW) {
                    wave_lds_sync();
                    unsigned long long first = 0;
                    if (l == 0) first = atomicAdd(cursor, (unsigned long long)n);
                    drain(__shfl(first, 0));
                    n = 0;
                    wave_lds_sync();
                }
                if ((mask >> l) & 1ull) {
                    const int k = n + __popcll(mask & below);
                    const int64_t i = ib + 128 * half + 8 * (r >> 2) + 4 * h + (r & 3);
                    bkey[w][k] = ((uint64_t)i << 32) | (uint64_t)j;
                    bval[w][k] = __builtin_amdgcn_exp2f(neg_gamma_log2e * fmaxf(-2.0f * gv, 0.0f)) + lam2;
                }
                n += __popcll(mask);
            }
        }
    });
    if (l == 0) wcnt[w] = n;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long c0 = wcnt[0], c1 = wcnt[1], c2 = wcnt[2], c3 = wcnt[3];
        const unsigned long long tot = c0 + c1 + c2 + c3;
        const unsigned long long b = tot ? atomicAdd(cursor, tot) : 0ull;
        wbase[0] = b;
        wbase[1] = b + c0;
        wbase[2] = b + c0 + c1;
        wbase[3] = b + c0 + c1 + c2;
    }
    __syncthreads();
    drain(wbase[w]);
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
    const int64_t e = xcd_contiguous(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
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
    const int64_t k = (xcd_contiguous(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x) >> 4;
    const int q = threadIdx.x & 15;
    AT p = 0, e = 0;
    if (k < N) {
        const int64_t a0 = off_i[k], a1 = off_i[k + 1];
        int64_t u = a0 + q;
        for (; u + 48 < a1; u += 64) {
            const ST p0 = RB[2 * u], e0 = RB[2 * u + 1], p1 = RB[2 * u + 32], e1 = RB[2 * u + 33];
            const ST p2 = RB[2 * u + 64], e2 = RB[2 * u + 65], p3 = RB[2 * u + 96], e3 = RB[2 * u + 97];
            p += (AT)p0; e += (AT)e0;
            p += (AT)p1; e += (AT)e1;
            p += (AT)p2; e += (AT)e2;
            p += (AT)p3; e += (AT)e3;
        }
        for (; u < a1; u += 16) { p += (AT)RB[2 * u]; e += (AT)RB[2 * u + 1]; }
        const int64_t b0 = off_j[k], b1 = off_j[k + 1];
        // four edge ids, then their four records, in flight at once; the
        // additions keep the edge order
        int64_t t = b0 + q;
        for (; t + 48 < b1; t += 64) {
            const int64_t x0 = perm[t], x1 = perm[t + 16], x2 = perm[t + 32], x3 = perm[t + 48];
            const ST p0 = RF[2 * x0], e0 = RF[2 * x0 + 1], p1 = RF[2 * x1], e1 = RF[2 * x1 + 1];
            const ST p2 = RF[2 * x2], e2 = RF[2 * x2 + 1], p3 = RF[2 * x3], e3 = RF[2 * x3 + 1];
            p += (AT)p0; e += (AT)e0;
            p += (AT)p1; e += (AT)e1;
            p += (AT)p2; e += (AT)e2;
            p += (AT)p3; e += (AT)e3;
        }
        for (; t < b1; t += 16) {
            const int64_t x = perm[t];
            p += (AT)RF[2 * x];
            e += (AT)RF[2 * x + 1];
        }
    }
    p = sum16(p);
    e = sum16(e);
    if (k < N && q == 0) { partP[k] = p; partE[k] = e; }
}

// ---- locality order and tile pruning
//
// Points are reordered so that each 256-point block is compact: every point
// goes to its nearest landmark (landmarks: K evenly spaced input points;
// ties to the smaller landmark index) and points are sorted by (landmark,
// input index).  Then a tile whose blocks are provably farther apart than
// the cut is skipped by the build (triangle inequality on block centroids
// and radii), and the neighbours of a node sit in few cache lines during the
// sweep.  GaBP is equivariant under the relabelling; results are returned in
// input order.

// Nearest landmark of every point by direct FP32 differences; landmarks are
// staged through LDS in chunks.  key = (landmark << 32) | point.
__global__ __launch_bounds__(WG) void k_sp_assign(const float* __restrict__ X, int64_t N, int64_t m,
                                                  const int32_t* __restrict__ lm, int K, uint64_t* __restrict__ key,
                                                  int32_t* __restrict__ ids) {
    extern __shared__ float sl[];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int chunk = (int)(8192 / m) > 0 ? (int)(8192 / m) : 1;
    float best = INFINITY;
    int arg = 0;
    for (int k0 = 0; k0 < K; k0 += chunk) {
        const int kc = (K - k0 < chunk) ? K - k0 : chunk;
        __syncthreads();
        for (int64_t t = threadIdx.x; t < (int64_t)kc * m; t += blockDim.x)
            sl[t] = X[(int64_t)lm[k0 + t / m] * m + t % m];
        __syncthreads();
        if (i < N) {
            for (int k = 0; k < kc; ++k) {
                float d2 = 0.0f;
                for (int64_t c = 0; c < m; ++c) {
                    const float d = X[i * m + c] - sl[(int64_t)k * m + c];
                    d2 = fmaf(d, d, d2);
                }
                if (d2 < best) { best = d2; arg = k0 + k; }
            }
        }
    }
    if (i < N) {
        key[i] = ((uint64_t)(uint32_t)arg << 32) | (uint64_t)i;
        ids[i] = (int32_t)i;
    }
}

// Super-blocked order of the tile list: key = (super-block of (I, J), tile
// code), super-blocks of S x S tiles in row-major order, tiles inside one in
// row-major order.  With the XCD-contiguous workgroup index, the tiles of a
// super-block run on one XCD and share its L2 for their 2 S row fragments.
__global__ void k_sp_tile_keys(const uint32_t* __restrict__ tiles, int64_t nt, int S, int NSB,
                               uint64_t* __restrict__ keys) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    const uint32_t ij = tiles[t];
    const uint32_t I = ij >> 16, J = ij & 0xFFFFu;
    keys[t] = ((uint64_t)((I / S) * (uint32_t)NSB + J / S) << 32) | (uint64_t)ij;
}

__global__ void k_sp_tile_codes(const uint64_t* __restrict__ keys, int64_t nt, uint32_t* __restrict__ tiles) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nt) tiles[t] = (uint32_t)(keys[t] & 0xFFFFFFFFull);
}

// Rows of X and labels in the new order: Xp[r] = X[order[r]].
__global__ void k_sp_permute(const float* __restrict__ X, const float* __restrict__ y, int64_t N, int64_t m,
                             const int32_t* __restrict__ order, float* __restrict__ Xp, float* __restrict__ yp) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * m) return;
    const int64_t r = t / m, c = t % m;
    Xp[t] = X[(int64_t)order[r] * m + c];
    if (c == 0) yp[r] = y[order[r]];
}

// Centroid (FP64) and radius (max distance to it, FP64) of each block of
// 256 reordered points; one workgroup per block.
__global__ __launch_bounds__(WG) void k_sp_block_bounds(const float* __restrict__ Xp, int64_t N, int64_t m,
                                                        double* __restrict__ cent, double* __restrict__ rad) {
    __shared__ double sh[WG];
    __shared__ double sh4[4];
    const int64_t b = blockIdx.x;
    const int64_t r0 = b * TILE;
    const int64_t nr = (N - r0 < TILE) ? N - r0 : TILE;
    for (int64_t c = 0; c < m; ++c) {
        double v = (threadIdx.x < nr) ? (double)Xp[(r0 + threadIdx.x) * m + c] : 0.0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int o = WG / 2; o > 0; o >>= 1) {
            if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) cent[b * m + c] = sh[0] / (double)nr;
        __syncthreads();
    }
    double d2 = 0.0;
    if (threadIdx.x < nr)
        for (int64_t c = 0; c < m; ++c) {
            const double d = (double)Xp[(r0 + threadIdx.x) * m + c] - cent[b * m + c];
            d2 += d * d;
        }
    d2 = block_max(threadIdx.x < nr ? d2 : 0.0, sh4);
    if (threadIdx.x == 0) rad[b] = sqrt(d2);
}

// keep[t] = 1 unless every pair of tile t is provably beyond the cut:
// ||x_i - x_j|| >= ||c_I - c_J|| - r_I - r_J.  The margin makes the test
// conservative against the rounding of the bounds and of the device's own
// distances (a skipped pair has d^2 > 1.001 cut).
__global__ void k_sp_prune(const uint32_t* __restrict__ tiles, int64_t nt, int64_t m, const double* __restrict__ cent,
                           const double* __restrict__ rad, double cut, uint8_t* __restrict__ keep) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    const uint32_t ij = tiles[t];
    const int I = (int)(ij >> 16), J = (int)(ij & 0xFFFFu);
    double dc2 = 0.0;
    for (int64_t c = 0; c < m; ++c) {
        const double d = cent[(int64_t)I * m + c] - cent[(int64_t)J * m + c];
        dc2 += d * d;
    }
    const double gap = sqrt(dc2) - (rad[I] + rad[J]) * (1.0 + 1e-6) - 1e-6;
    keep[t] = (gap > 0.0 && gap * gap > 1.001 * cut) ? 0 : 1;
}

// Augmented rows of the build: A row i gets (n_i, 1) in columns m, m + 1,
// B row i (a copy of A's first m columns) gets (-1/2, -n_i/2), each value
// split into the Gram kind's planes as the features are (hi, then the BF16
// remainders), so that sum_k a_ik b_jk = x_i . x_j - n_i/2 - n_j/2 for the
// products the kind forms.  One thread per row; columns past m + 1 stay 0.
__global__ void k_sp_augment(int64_t NPAD, int64_t m, int m_pad, int kind, const float* __restrict__ nrm,
                             float* f32a, uint16_t* hia, uint16_t* loa, uint16_t* lo2a, float* f32b,
                             uint16_t* hib, uint16_t* lob, uint16_t* lo2b) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NPAD) return;
    const int64_t o = i * m_pad;
    const float n = nrm[i], nb = -0.5f * n;
    if (kind == GRAM_F32) {
        for (int64_t k = 0; k < m; ++k) f32b[o + k] = f32a[o + k];
        f32a[o + m] = n;
        f32a[o + m + 1] = 1.0f;
        f32b[o + m] = -0.5f;
        f32b[o + m + 1] = nb;
        for (int64_t k = m + 2; k < m_pad; ++k) f32b[o + k] = 0.0f;
        return;
    }
    const bool x3 = (kind == GRAM_BF16X3 || kind == GRAM_BF16X6), x6 = (kind == GRAM_BF16X6);
    for (int64_t k = 0; k < m_pad; ++k) {
        hib[o + k] = (k < m) ? hia[o + k] : 0;
        if (x3) lob[o + k] = (k < m) ? loa[o + k] : 0;
        if (x6) lo2b[o + k] = (k < m) ? lo2a[o + k] : 0;
    }
    uint16_t h, l, l2;
    split3(n, h, l, l2);
    hia[o + m] = h;
    hia[o + m + 1] = f2bf(1.0f);
    hib[o + m] = f2bf(-0.5f);
    if (x3) { loa[o + m] = l; loa[o + m + 1] = 0; lob[o + m] = 0; }
    if (x6) { lo2a[o + m] = l2; lo2a[o + m + 1] = 0; lo2b[o + m] = 0; }
    split3(nb, h, l, l2);
    hib[o + m + 1] = h;
    if (x3) lob[o + m + 1] = l;
    if (x6) lo2b[o + m + 1] = l2;
}

// out[order[r]] = in[r]: a per-node array back to input order.
__global__ void k_sp_unpermute(const double* __restrict__ in, const int32_t* __restrict__ order, int64_t N,
                               double* __restrict__ out) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < N) out[order[r]] = in[r];
}

template <int KIND>
void sp_build_kind(bool fill, int mp, dim3 g, const Features& FA, const Features& FB, const uint32_t* tiles, int64_t stride, int64_t N,
                   float cut, float c, float lam2, int32_t* counts, int64_t cap, unsigned long long* cursor,
                   uint64_t* keys, float* kv, hipStream_t s) {
    const dim3 gf((unsigned)(((int64_t)g.x + SP_TPW - 1) / SP_TPW));
#define GABP_SP_LAUNCH(MPV)                                                                                  \
    do {                                                                                                     \
        if (fill)                                                                                            \
            hipLaunchKernelGGL((k_sp_fill<KIND, MPV>), gf, dim3(WG), 0, s, FA, FB, tiles, (int64_t)g.x, N, cut,   \
                               c, lam2, cap, cursor, keys, kv);                                              \
        else                                                                                                 \
            hipLaunchKernelGGL((k_sp_count<KIND, MPV>), g, dim3(WG), 0, s, FA, FB, tiles, stride, N, cut,     \
                               counts);                                                                      \
    } while (0)
    // register-held fragments of two bands plus the prefetched B fragment
    // fit up to 64 features; beyond, fragments are reloaded per block
    if (mp <= 32) GABP_SP_LAUNCH(32);
    else if (mp <= 64) GABP_SP_LAUNCH(64);
    else GABP_SP_LAUNCH(0);
#undef GABP_SP_LAUNCH
}

hipError_t sp_build(bool fill, const Features& FA, const Features& FB, const uint32_t* tiles, int64_t ntiles,
                    int64_t stride, int64_t N, float cut, float c, float lam2, int32_t* counts, int64_t cap,
                    unsigned long long* cursor, uint64_t* keys, float* kv, hipStream_t s) {
    const dim3 g((unsigned)ntiles);
#define GABP_SP_KIND(K) sp_build_kind<K>(fill, FA.m_pad, g, FA, FB, tiles, stride, N, cut, c, lam2, counts, cap, cursor, keys, kv, s)
    switch (FA.kind) {
        case GRAM_F32: GABP_SP_KIND(GRAM_F32); break;
        case GRAM_BF16: GABP_SP_KIND(GRAM_BF16); break;
        case GRAM_BF16X3: GABP_SP_KIND(GRAM_BF16X3); break;
        case GRAM_BF16X6: GABP_SP_KIND(GRAM_BF16X6); break;
        default: return hipErrorInvalidValue;
    }
#undef GABP_SP_KIND
    return hipGetLastError();
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + WG - 1) / WG); }

}  // namespace

hipError_t launch_sp_count(const Features& FA, const Features& FB, const uint32_t* tiles, int64_t ntiles,
                           int64_t stride, int64_t N, float cut, int32_t* counts, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    return sp_build(false, FA, FB, tiles, ntiles, stride, N, cut, 0.0f, 0.0f, counts, 0, nullptr, nullptr, nullptr,
                    s);
}

hipError_t launch_sp_fill(const Features& FA, const Features& FB, const uint32_t* tiles, int64_t ntiles, int64_t N,
                          float cut, float neg_gamma_log2e, float lam2, int64_t cap, unsigned long long* cursor,
                          uint64_t* keys, float* kv, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    return sp_build(true, FA, FB, tiles, ntiles, 1, N, cut, neg_gamma_log2e, lam2, nullptr, cap, cursor, keys, kv, s);
}

hipError_t launch_sp_augment(int64_t NPAD, int64_t m, int m_pad, int kind, const float* nrm, float* f32a,
                             uint16_t* hia, uint16_t* loa, uint16_t* lo2a, float* f32b, uint16_t* hib,
                             uint16_t* lob, uint16_t* lo2b, hipStream_t s) {
    if (m + 2 > m_pad) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sp_augment, dim3(blocks(NPAD)), dim3(WG), 0, s, NPAD, m, m_pad, kind, nrm, f32a, hia, loa,
                       lo2a, f32b, hib, lob, lo2b);
    return hipGetLastError();
}

hipError_t launch_sp_order(const float* X, int64_t N, int64_t m, const int32_t* lm, int K, uint64_t* key,
                           int32_t* ids, hipStream_t s) {
    const int chunk = (int)(8192 / m) > 0 ? (int)(8192 / m) : 1;
    const size_t lds = (size_t)std::min<int64_t>(chunk, K) * m * sizeof(float);
    hipLaunchKernelGGL(k_sp_assign, dim3(blocks(N)), dim3(WG), lds, s, X, N, m, lm, K, key, ids);
    return hipGetLastError();
}

hipError_t launch_sp_permute(const float* X, const float* y, int64_t N, int64_t m, const int32_t* order, float* Xp,
                             float* yp, hipStream_t s) {
    hipLaunchKernelGGL(k_sp_permute, dim3(blocks(N * m)), dim3(WG), 0, s, X, y, N, m, order, Xp, yp);
    return hipGetLastError();
}

hipError_t launch_sp_prune(const float* Xp, int64_t N, int64_t m, int NB, const uint32_t* tiles, int64_t nt,
                           double cut, double* cent, double* rad, uint8_t* keep, hipStream_t s) {
    hipLaunchKernelGGL(k_sp_block_bounds, dim3((unsigned)NB), dim3(WG), 0, s, Xp, N, m, cent, rad);
    hipLaunchKernelGGL(k_sp_prune, dim3(blocks(nt)), dim3(WG), 0, s, tiles, nt, m, cent, rad, cut, keep);
    return hipGetLastError();
}

hipError_t sp_select(void* tmp, size_t* bytes, const uint32_t* in, const uint8_t* flags, uint32_t* out,
                     int64_t* nsel, int64_t n, hipStream_t s) {
    return hipcub::DeviceSelect::Flagged(tmp, *bytes, in, flags, out, nsel, (int)n, s);
}

hipError_t sp_tile_order(void* tmp, size_t* bytes, uint32_t* tiles, int64_t nt, int S, int NB, uint64_t* k0,
                         uint64_t* k1, hipStream_t s) {
    if (tmp == nullptr) return hipcub::DeviceRadixSort::SortKeys(tmp, *bytes, k0, k1, (int)nt, 0, 64, s);
    if (nt <= 0) return hipSuccess;
    const int NSB = (NB + S - 1) / S;
    hipLaunchKernelGGL(k_sp_tile_keys, dim3(blocks(nt)), dim3(WG), 0, s, tiles, nt, S, NSB, k0);
    hipError_t e = hipcub::DeviceRadixSort::SortKeys(tmp, *bytes, k0, k1, (int)nt, 0, 64, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sp_tile_codes, dim3(blocks(nt)), dim3(WG), 0, s, k1, nt, tiles);
    return hipGetLastError();
}

hipError_t launch_sp_unpermute(const double* in, const int32_t* order, int64_t N, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_sp_unpermute, dim3(blocks(N)), dim3(WG), 0, s, in, order, N, out);
    return hipGetLastError();
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
