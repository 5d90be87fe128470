// HIP kernels of the GaBP SVM solver for gfx950 (MI355X).
//
// Method: Bickson, Yom-Tov, Dolev, arXiv 0810.1648.  The sweep is Algorithm
// 2 (section "Algorithm Optimization") in synchronous rounds (section
// "Experimental Results"), with messages kept in information form
// E_ij = P_ij mu_ij:
//     Q_ij = P~_i - P_ji,   P_ij <- -A_ij^2 / Q_ij,   E_ij <- -A_ij (S_i - E_ji) / Q_ij,
//     P~_j = A_jj + sum_i P_ij,   S_j = b_j + sum_i E_ij,   mu_j = S_j / P~_j.
// Labels are folded into the right-hand side: with Y = diag(y), A = Y(K'+W)Y,
// so GaBP on (K' + W, b = y) yields the same iterates up to exact sign flips
// and alpha = y * mu.  The kernels therefore never multiply by labels.
//
// Data layout: the unordered pairs {i, j}, i < j, live in TILE x TILE tiles of
// the upper triangle, row-major inside a tile.  Pair-record planes keep both
// directions of a pair at the same offset (P_ij, P_ji, E_ij, E_ji), so the
// update of a pair reads and writes one position of five planes with no
// transpose.  Entries below the diagonal of diagonal tiles and entries of
// padded rows/columns hold K' = 0, which makes their messages exactly zero.
//
// Lane layout of the streaming kernels: a workgroup (4 wave64) owns one tile;
// wave w owns the 64-column strip [64w, 64w + 64); in step s, lane (g, q) =
// (lane / 16, lane % 16) handles row 4s + g and the four columns
// 64w + 4q .. 64w + 4q + 3, so each plane access of a wave is four 256-byte
// contiguous segments of 16-byte loads.  Row sums (messages received by the
// row node) are reduced over 16 lanes with DPP; column sums (messages
// received by the column node) accumulate in registers and are combined
// across the four lane groups once per tile.  Partial sums go to a
// [block][slot][TILE] array that a second kernel reduces in a fixed order,
// so results are bitwise reproducible.
//
// K' comes either from the materialised plane (one 16-byte load per lane
// and row) or is recomputed per 32-row band: each wave forms the Gram
// products of its 32 x 64 block on MFMA, applies exp, and passes the block
// through a wave-private LDS buffer into the row layout above.  Messages come
// either from the pair-record planes (stored edge state) or are rebuilt from
// a ring of earlier aggregates (stateless edge state): the message i -> j of
// sweep t needs only the reverse message of sweep t - 1, which needs i -> j
// of sweep t - 2, and so on, so unrolling L levels from zero reproduces the
// stored recursion exactly while t <= L and truncates it after.
#include "gabp_device.h"

namespace gabp {

// ------------------------------------------------------- setup kernels --

__global__ void k_fill_tiles(uint32_t* tiles, int NB) {
    const int I = blockIdx.x;
    for (int J = I + threadIdx.x; J < NB; J += blockDim.x)
        tiles[tile_index(I, J, NB)] = ((uint32_t)I << 16) | (uint32_t)J;
}

__global__ void k_validate(const float* __restrict__ X, const float* __restrict__ y, int64_t N,
                           int64_t m, int32_t* flag) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int bad = 0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < N * m; k += stride)
        if (!isfinite(X[k])) bad |= 1;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < N; k += stride)
        if (!(y[k] == 1.0f || y[k] == -1.0f)) bad |= 2;
    if (bad) atomicOr(flag, bad);
}

// Column means in FP64 (the RBF kernel is translation invariant, so
// centring is exact math; it shrinks ||x||^2 before the Gram expansion).
__global__ void k_colmean(const float* __restrict__ X, int64_t N, int64_t m, double* mean) {
    __shared__ double sh[WG];
    const int64_t k = blockIdx.x;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < N; i += WG) acc += (double)X[i * m + k];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = WG / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) mean[k] = sh[0] / (double)N;
}

// One thread per staged row: writes the zero-padded row and its squared
// norm, computed from the values actually staged (so that d^2 of a point
// with itself is 0 up to the Gram's own rounding).
__global__ void k_stage(const float* __restrict__ X, const double* __restrict__ mean, int64_t N,
                        int64_t m, int64_t NPAD, int m_pad, int kind, float* f32, uint16_t* hi,
                        uint16_t* lo, uint16_t* lo2, double* f64, float* nrm) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NPAD) return;
    float acc = 0.0f;
    for (int k = 0; k < m_pad; ++k) {
        const bool in = (i < N) && (k < m);
        const float raw = in ? X[i * m + k] : 0.0f;
        if (kind == GRAM_F64) {
            f64[i * m_pad + k] = (double)raw;
            continue;
        }
        const float xc = in ? (float)((double)raw - mean[k]) : 0.0f;
        if (kind == GRAM_F32) {
            f32[i * m_pad + k] = xc;
            acc = fmaf(xc, xc, acc);
        } else {
            const uint16_t h = f2bf(xc);
            float v = bf2f(h);
            hi[i * m_pad + k] = h;
            if (kind == GRAM_BF16X3 || kind == GRAM_BF16X6) {
                const uint16_t l = f2bf(xc - v);
                lo[i * m_pad + k] = l;
                if (kind == GRAM_BF16X6) {
                    const uint16_t l2 = f2bf((xc - v) - bf2f(l));
                    lo2[i * m_pad + k] = l2;
                    v += bf2f(l) + bf2f(l2);
                } else {
                    v += bf2f(l);
                }
            }
            acc = fmaf(v, v, acc);
        }
    }
    if (nrm) nrm[i] = acc;
}

// Materialise the K' tiles.  Wave w computes the 32-row bands w and w + 4,
// one 32 x 32 block at a time, and stores straight from the MFMA layout.
template <int KIND>
__global__ __launch_bounds__(WG) void k_gram_mfma(Features F, KernelParams kp,
                                                 const uint32_t* __restrict__ tiles,
                                                 float* __restrict__ Kp) {
    const TileCoord tc = tile_of(tiles);
    const size_t tbase = (size_t)blockIdx.x * TT;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, h = l >> 5, l32 = l & 31;
    for (int band = w; band < TILE / 32; band += 4) {
        const int64_t rowA = (int64_t)tc.I * TILE + band * 32 + l32;
        float ni[16];
#pragma unroll
        for (int r = 0; r < 16; ++r)
            ni[r] = F.nrm[(int64_t)tc.I * TILE + band * 32 + 8 * (r >> 2) + 4 * h + (r & 3)];
        for (int cb = 0; cb < TILE / 32; ++cb) {
            const int64_t colB = (int64_t)tc.J * TILE + cb * 32 + l32;
            const f32x16 acc = mfma_gram_32x32<KIND>(F, rowA, colB);
            const float nj = F.nrm[colB];
            const int col = cb * 32 + l32;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = band * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
                Kp[tbase + (size_t)row * TILE + col] =
                    kernel_entry(ni[r], nj, acc[r], (int64_t)tc.I * TILE + row, colB, kp);
            }
        }
    }
}

// Materialise the K' tiles and, in the same pass, the partial row and column
// sums and maxima of K' (>= 0) that the diagonal weighting needs, in the
// layout of k_rowsum.  Wave w computes the 32-row bands w and w + 4 with the
// band's A fragments in registers, walking the eight 32-column blocks.  Each
// 32 x 32 block goes through LDS once: column sums come from the MFMA layout
// (a lane holds 16 rows of one column), row sums and the 16-byte row stores
// from the transposed read (eight lanes per row).  All sums in a fixed order.
// BF16 Gram kinds: the four waves walk the same column blocks, so each
// block's B fragments are staged once in LDS in fragment order (BStage), the
// next block's chunks loaded into registers while the current one is
// multiplied (one barrier per block; the products in the same order as from
// registers, so K' is the same to the bit).
template <int KIND, int MP>
__global__ __launch_bounds__(WG) void k_gram_sums(Features F, KernelParams kp, const uint32_t* __restrict__ tiles,
                                                 float* __restrict__ Kp, int NB, double* __restrict__ psum,
                                                 double* __restrict__ pmax) {
    // tiles in list order (any order of the upper tiles, read XCD-contiguously);
    // each is written at its own position of the plane
    const uint32_t ij = tiles[xcd_contiguous(blockIdx.x, gridDim.x)];
    const TileCoord tc{(int)(ij >> 16), (int)(ij & 0xFFFFu)};
    const size_t tbase = (size_t)tile_index(tc.I, tc.J, NB) * TT;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, h = l >> 5, l32 = l & 31;
    __shared__ double csum[4][TILE];
    __shared__ float cmax[4][TILE];
    __shared__ float blk[4][32][33];
    const int64_t i0 = (int64_t)tc.I * TILE, j0 = (int64_t)tc.J * TILE;
    const int rr = l >> 3, cq = 4 * (l & 7);       // transposed read: row rr + 8 k, columns cq .. cq + 3
    constexpr bool STG = (KIND != GRAM_F32) && (MP > 0);
    using BS = BStage<KIND>;
    constexpr int CH = STG ? BS::NP * (MP / 16) * 64 : 1;                  // 16-byte chunks per block
    constexpr int PR = (CH + WG - 1) / WG;                                 // per thread
    __shared__ bf16x8 sb[2][CH];
    const int ns = F.m_pad / 16, ch = BS::NP * ns * 64;
    int cur = 0;
    if constexpr (STG) {
#pragma unroll
        for (int i = 0; i < PR; ++i) {
            const int k = tid + WG * i;
            if (k < ch) sb[0][BS::dst(ns, k)] = *BS::src(F, j0, ns, k);
        }
        __syncthreads();
    }
#pragma unroll 1
    for (int pass = 0; pass < 2; ++pass) {
        const int band = w + 4 * pass;
        const int64_t rowA = i0 + band * 32 + l32;
        float ni[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) ni[r] = F.nrm[i0 + band * 32 + 8 * (r >> 2) + 4 * h + (r & 3)];
        RowFrag<KIND, MP> fa;
        fa.load(F, rowA);
        double rs[4] = {0.0, 0.0, 0.0, 0.0};
        float rm[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 1
        for (int cb = 0; cb < TILE / 32; ++cb) {
            const int64_t colB = j0 + cb * 32 + l32;
            // the next block (the first again after the last of pass 0)
            const bool more = STG && !(pass == 1 && cb == TILE / 32 - 1);
            const int64_t nb0 = j0 + ((cb + 1) % (TILE / 32)) * 32;
            bf16x8 pre[PR];
            if constexpr (STG) {
                if (more) {
#pragma unroll
                    for (int i = 0; i < PR; ++i) {
                        const int k = tid + WG * i;
                        if (k < ch) pre[i] = *BS::src(F, nb0, ns, k);
                    }
                }
            }
            f32x16 acc = {};
            if constexpr (STG) BS::template mma<MP>(fa, sb[cur], ns, l, acc);
            else acc = fa.gram(F, rowA, F, colB);
            const float nj = F.nrm[colB];
            double cs = 0.0;
            float cm = 0.0f;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = 8 * (r >> 2) + 4 * h + (r & 3);
                const float kv = kernel_entry(ni[r], nj, acc[r], i0 + band * 32 + row, colB, kp);
                blk[w][row][l32] = kv;
                cs += (double)kv;
                cm = fmaxf(cm, kv);
            }
            // the column's 32 rows of this band: both lane halves
            cs = cs + __shfl_xor(cs, 32);
            cm = fmaxf(cm, __shfl_xor(cm, 32));
            const int col = cb * 32 + l32;
            if (h == 0) {
                if (pass == 0) { csum[w][col] = cs; cmax[w][col] = cm; }
                else { csum[w][col] += cs; cmax[w][col] = fmaxf(cmax[w][col], cm); }
            }
            wave_lds_sync();
            float* dst = Kp + tbase + (size_t)(band * 32 + rr) * TILE + cb * 32 + cq;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float* src = &blk[w][rr + 8 * k][cq];
                const f32x4v v = {src[0], src[1], src[2], src[3]};
                __builtin_nontemporal_store(v, reinterpret_cast<f32x4v*>(dst + (size_t)8 * k * TILE));
                rs[k] += ((double)v[0] + (double)v[1]) + ((double)v[2] + (double)v[3]);
                rm[k] = fmaxf(rm[k], fmaxf(fmaxf(v[0], v[1]), fmaxf(v[2], v[3])));
            }
            wave_lds_sync();
            if constexpr (STG) {
                if (more) {
#pragma unroll
                    for (int i = 0; i < PR; ++i) {
                        const int k = tid + WG * i;
                        if (k < ch) sb[cur ^ 1][BS::dst(ns, k)] = pre[i];
                    }
                }
                __syncthreads();
                cur ^= 1;
            }
        }
        // rows rr + 8 k: the eight lanes of each row add their column quads
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            double v = rs[k];
            v = v + dpp<0xB1>(v);
            v = v + dpp<0x4E>(v);
            v = v + dpp<0x141>(v);
            float mv = rm[k];
            mv = fmaxf(mv, dpp<0xB1>(mv));
            mv = fmaxf(mv, dpp<0x4E>(mv));
            mv = fmaxf(mv, dpp<0x141>(mv));
            if ((l & 7) == 0) {
                const size_t o = ((size_t)tc.I * (NB + 1) + tc.J) * TILE + band * 32 + rr + 8 * k;
                psum[o] = v;
                pmax[o] = (double)mv;
            }
        }
    }
    __syncthreads();
    const int slot = (tc.I < tc.J) ? tc.I : NB;
    const size_t cb = ((size_t)tc.J * (NB + 1) + slot) * TILE + tid;
    psum[cb] = (csum[0][tid] + csum[1][tid]) + (csum[2][tid] + csum[3][tid]);
    pmax[cb] = (double)fmaxf(fmaxf(cmax[0][tid], cmax[1][tid]), fmaxf(cmax[2][tid], cmax[3][tid]));
}

template <int KIND>
void gram_sums_kind(int mp, dim3 g, const Features& F, const KernelParams& kp, const uint32_t* tiles, float* Kp,
                    int NB, double* psum, double* pmax, hipStream_t s) {
    if (mp <= 32)
        hipLaunchKernelGGL((k_gram_sums<KIND, 32>), g, dim3(WG), 0, s, F, kp, tiles, Kp, NB, psum, pmax);
    else if (mp <= 64)
        hipLaunchKernelGGL((k_gram_sums<KIND, 64>), g, dim3(WG), 0, s, F, kp, tiles, Kp, NB, psum, pmax);
    else if (mp <= 128)
        hipLaunchKernelGGL((k_gram_sums<KIND, 128>), g, dim3(WG), 0, s, F, kp, tiles, Kp, NB, psum, pmax);
    else
        hipLaunchKernelGGL((k_gram_sums<KIND, 0>), g, dim3(WG), 0, s, F, kp, tiles, Kp, NB, psum, pmax);
}

// FP64 K' from direct differences (no Gram expansion, no centring).
__global__ __launch_bounds__(WG) void k_gram_f64(Features F, KernelParams kp,
                                                const uint32_t* __restrict__ tiles,
                                                double* __restrict__ Kp) {
    const TileCoord tc = tile_of(tiles);
    const size_t tbase = (size_t)blockIdx.x * TT;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, g = l >> 4, q = l & 15;
    const int col0 = w * 64 + q * 4;
    const int mp = F.m_pad;
    const double* xj = F.f64 + ((int64_t)tc.J * TILE + col0) * mp;
    for (int s = 0; s < TILE / 4; ++s) {
        const int r = 4 * s + g;
        const int64_t i = (int64_t)tc.I * TILE + r;
        const double* xi = F.f64 + i * mp;
        double d2[4] = {0.0, 0.0, 0.0, 0.0};
        for (int k = 0; k < mp; ++k) {
            const double a = xi[k];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double d = a - xj[c * mp + k];
                d2[c] = fma(d, d, d2[c]);
            }
        }
        V4<double> out;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int64_t j = (int64_t)tc.J * TILE + col0 + c;
            out.v[c] = (i < j && j < kp.N) ? exp(-kp.gamma * d2[c]) + kp.lam2 : 0.0;
        }
        st4(Kp + tbase + (size_t)r * TILE + col0, out);
    }
}

// K' taken from a caller-supplied dense N x N matrix (upper triangle).
template <class ST>
__global__ __launch_bounds__(WG) void k_gather_dense(const double* __restrict__ K, KernelParams kp,
                                                    const uint32_t* __restrict__ tiles,
                                                    ST* __restrict__ Kp) {
    const TileCoord tc = tile_of(tiles);
    const size_t tbase = (size_t)blockIdx.x * TT;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, g = l >> 4, q = l & 15;
    const int col0 = w * 64 + q * 4;
    for (int s = 0; s < TILE / 4; ++s) {
        const int r = 4 * s + g;
        const int64_t i = (int64_t)tc.I * TILE + r;
        V4<ST> out;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int64_t j = (int64_t)tc.J * TILE + col0 + c;
            out.v[c] = (i < j && j < kp.N) ? (ST)K[i * kp.N + j] : (ST)0;
        }
        st4(Kp + tbase + (size_t)r * TILE + col0, out);
    }
}

__global__ void k_dense_diag(const double* __restrict__ K, int64_t N, double* kdiag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) kdiag[i] = K[i * N + i];
}

__global__ void k_fill_value(double* dst, int64_t n, double v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = v;
}

// --------------------------------------------------- diagonal weighting --

// Partial sums r_i = sum_{j != i} |K'_ij| and maxima max_{j != i} |K'_ij| per
// tile slot (FP64), from the K' plane or from K' recomputed per band.
template <class ST, int KSRC, int GK>
__global__ __launch_bounds__(WG) void k_rowsum(const ST* __restrict__ Kp, Features F, KernelParams kp,
                                              const uint32_t* __restrict__ tiles, int NB,
                                              double* __restrict__ psum, double* __restrict__ pmax) {
    const TileCoord tc = tile_of(tiles);
    const size_t tbase = (size_t)blockIdx.x * TT;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, g = l >> 4, q = l & 15;
    const int col0 = w * 64 + q * 4;
    __shared__ double rows[4][TILE], rmax[4][TILE];
    __shared__ float kband[KSRC == KSRC_RECOMPUTE ? 4 : 1][KSRC == KSRC_RECOMPUTE ? 32 * 64 : 1];
    double cs[4] = {0.0, 0.0, 0.0, 0.0}, cm[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = 0; b < TILE / 32; ++b) {
        if constexpr (KSRC == KSRC_RECOMPUTE) {
            gram_band<GK>(F, kp, tc.I, tc.J, 32 * b, 64 * w, kband[w]);
            wave_lds_sync();
        }
        for (int s2 = 0; s2 < 8; ++s2) {
            const int r = 32 * b + 4 * s2 + g;
            V4<ST> k;
            if constexpr (KSRC == KSRC_RECOMPUTE) {
                const float4 kk = *reinterpret_cast<const float4*>(&kband[w][(4 * s2 + g) * 64 + 4 * q]);
                k = V4<ST>{{(ST)kk.x, (ST)kk.y, (ST)kk.z, (ST)kk.w}};
            } else {
                k = ld4(Kp + tbase + (size_t)r * TILE + col0);
            }
            double rs = 0.0, rm = 0.0;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double a = fabs((double)k.v[c]);
                cs[c] += a;
                rs += a;
                cm[c] = fmax(cm[c], a);
                rm = fmax(rm, a);
            }
            rs = sum16(rs);
            rm = fmax(rm, dpp<0xB1>(rm));
            rm = fmax(rm, dpp<0x4E>(rm));
            rm = fmax(rm, dpp<0x141>(rm));
            rm = fmax(rm, dpp<0x140>(rm));
            if (q == 0) { rows[w][r] = rs; rmax[w][r] = rm; }
        }
        if constexpr (KSRC == KSRC_RECOMPUTE) wave_lds_sync();
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        cs[c] = sum_groups(cs[c]);
        cm[c] = fmax(cm[c], __shfl_xor(cm[c], 16));
        cm[c] = fmax(cm[c], __shfl_xor(cm[c], 32));
    }
    __syncthreads();
    const size_t rs_ = ((size_t)tc.I * (NB + 1) + tc.J) * TILE + tid;
    psum[rs_] = (rows[0][tid] + rows[1][tid]) + (rows[2][tid] + rows[3][tid]);
    pmax[rs_] = fmax(fmax(rmax[0][tid], rmax[1][tid]), fmax(rmax[2][tid], rmax[3][tid]));
    if (g == 0) {
        const int slot = (tc.I < tc.J) ? tc.I : NB;
        const size_t cb = ((size_t)tc.J * (NB + 1) + slot) * TILE + col0;
#pragma unroll
        for (int c = 0; c < 4; ++c) { psum[cb + c] = cs[c]; pmax[cb + c] = cm[c]; }
    }
}

// Residual certificate of a finished solve: partial products
// sum_{j != i} K'_ij w_j (w_j = y_j alpha_j) per tile slot, in FP64, in the
// layout and lane order of k_rowsum (row part: slot J of block I; column
// part: slot I of block J, or slot NB for a diagonal tile).
template <class ST, int KSRC, int GK>
__global__ __launch_bounds__(WG) void k_apply(const ST* __restrict__ Kp, Features F, KernelParams kp,
                                             const uint32_t* __restrict__ tiles, int NB,
                                             const double* __restrict__ w, double* __restrict__ part) {
    const TileCoord tc = tile_of(tiles);
    const size_t tbase = (size_t)blockIdx.x * TT;
    const int tid = threadIdx.x, wv = tid >> 6, l = tid & 63, g = l >> 4, q = l & 15;
    const int col0 = wv * 64 + q * 4;
    __shared__ double rows[4][TILE];
    __shared__ float kband[KSRC == KSRC_RECOMPUTE ? 4 : 1][KSRC == KSRC_RECOMPUTE ? 32 * 64 : 1];
    const double* wI = w + (size_t)tc.I * TILE;
    const double* wJ = w + (size_t)tc.J * TILE;
    double wc[4], cs[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < 4; ++c) wc[c] = wJ[col0 + c];
    for (int b = 0; b < TILE / 32; ++b) {
        if constexpr (KSRC == KSRC_RECOMPUTE) {
            gram_band<GK>(F, kp, tc.I, tc.J, 32 * b, 64 * wv, kband[wv]);
            wave_lds_sync();
        }
        for (int s2 = 0; s2 < 8; ++s2) {
            const int r = 32 * b + 4 * s2 + g;
            V4<ST> k;
            if constexpr (KSRC == KSRC_RECOMPUTE) {
                const float4 kk = *reinterpret_cast<const float4*>(&kband[wv][(4 * s2 + g) * 64 + 4 * q]);
                k = V4<ST>{{(ST)kk.x, (ST)kk.y, (ST)kk.z, (ST)kk.w}};
            } else {
                k = ld4(Kp + tbase + (size_t)r * TILE + col0);
            }
            const double wr = wI[r];
            double rs = 0.0;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double a = (double)k.v[c];
                rs = fma(a, wc[c], rs);
                cs[c] = fma(a, wr, cs[c]);
            }
            rs = sum16(rs);
            if (q == 0) rows[wv][r] = rs;
        }
        if constexpr (KSRC == KSRC_RECOMPUTE) wave_lds_sync();
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) cs[c] = sum_groups(cs[c]);
    __syncthreads();
    part[((size_t)tc.I * (NB + 1) + tc.J) * TILE + tid] = (rows[0][tid] + rows[1][tid]) + (rows[2][tid] + rows[3][tid]);
    if (g == 0) {
        const int slot = (tc.I < tc.J) ? tc.I : NB;
        const size_t cb = ((size_t)tc.J * (NB + 1) + slot) * TILE + col0;
#pragma unroll
        for (int c = 0; c < 4; ++c) part[cb + c] = cs[c];
    }
}

// w_i = y_i alpha_i on [0, N), zero on the padded rows.
__global__ void k_weights(int64_t N, int64_t NPAD, const double* __restrict__ alpha,
                          const float* __restrict__ y, double* __restrict__ w) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < NPAD) w[i] = (i < N) ? (double)y[i] * alpha[i] : 0.0;
}

// Per node: (A alpha)_i = A_ii alpha_i + y_i sum_{j != i} K'_ij w_j from the
// slot partials in slot order; per block: max_i |1 - (A alpha)_i| (+inf for a
// non-finite value) and min_i (A_ii - r_i).
__global__ __launch_bounds__(WG) void k_residual_blocks(int64_t N, int NB, const double* __restrict__ part,
                                                        const double* __restrict__ Adiag,
                                                        const double* __restrict__ rsum,
                                                        const double* __restrict__ alpha,
                                                        const float* __restrict__ y, double* __restrict__ bres,
                                                        double* __restrict__ bgap) {
    __shared__ double sh4[4];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double res = 0.0, ngap = -INFINITY;
    if (i < N) {
        const int64_t B = i / TILE, t = i % TILE;
        double acc = 0.0;
        for (int sl = 0; sl <= NB; ++sl) acc += part[((size_t)B * (NB + 1) + sl) * TILE + t];
        const double r = 1.0 - (Adiag[i] * alpha[i] + (double)y[i] * acc);
        res = isfinite(r) ? fabs(r) : INFINITY;
        ngap = -(Adiag[i] - rsum[i]);
    }
    res = block_max(res, sh4);
    __syncthreads();
    ngap = block_max(ngap, sh4);
    if (threadIdx.x == 0) { bres[blockIdx.x] = res; bgap[blockIdx.x] = ngap; }
}

// out[0] = ||1 - A alpha||_inf, out[1] = min_i (A_ii - r_i), out[2] = Varah's
// bound out[0] / out[1] on ||alpha - A^-1 1||_inf (+inf unless out[1] > 0).
__global__ __launch_bounds__(WG) void k_residual_final(int nb, const double* __restrict__ bres,
                                                       const double* __restrict__ bgap, double* __restrict__ out) {
    __shared__ double sh4[4];
    double r = 0.0, ng = -INFINITY;
    for (int k = threadIdx.x; k < nb; k += blockDim.x) { r = fmax(r, bres[k]); ng = fmax(ng, bgap[k]); }
    r = block_max(r, sh4);
    __syncthreads();
    ng = block_max(ng, sh4);
    if (threadIdx.x == 0) {
        const double gap = -ng;
        out[0] = r;
        out[1] = gap;
        out[2] = (gap > 0.0) ? r / gap : INFINITY;
    }
}

// Weighted diagonal (subsection "GaBP Algorithm Convergence") and the row
// maxima of |K'|.  For the uniform rule this kernel leaves the per-block max
// of A_ii - K'_ii for k_diag_shift.
__global__ void k_diag(int64_t N, int NB, const double* __restrict__ psum,
                       const double* __restrict__ pmax, const double* __restrict__ kdiag, int mode,
                       double C, double delta, double* __restrict__ Adiag,
                       double* __restrict__ rowmax, double* __restrict__ rsum, double* __restrict__ blk) {
    __shared__ double sh4[4];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double wv = -INFINITY;
    if (i < N) {
        const int64_t B = i / TILE, t = i % TILE;
        double r = 0.0, mx = 0.0;
        for (int s = 0; s <= NB; ++s) {
            const size_t o = ((size_t)B * (NB + 1) + s) * TILE + t;
            r += psum[o];
            mx = fmax(mx, pmax[o]);
        }
        const double kii = kdiag[i];
        const double soft = kii + 1.0 / C, dom = (1.0 + delta) * r;
        double a;
        switch (mode) {
            case 0: a = kii; break;
            case 1: a = soft; break;
            default: a = fmax(soft, dom); break;
        }
        Adiag[i] = a;
        rowmax[i] = mx;
        rsum[i] = r;
        wv = a - kii;
    }
    if (mode == 3) {
        wv = block_max(wv, sh4);
        if (threadIdx.x == 0) blk[blockIdx.x] = wv;
    }
}

__global__ void k_max_reduce(int n, const double* __restrict__ in, double* out) {
    __shared__ double sh4[4];
    double v = -INFINITY;
    for (int k = threadIdx.x; k < n; k += blockDim.x) v = fmax(v, in[k]);
    v = block_max(v, sh4);
    if (threadIdx.x == 0) *out = v;
}

__global__ void k_diag_shift(int64_t N, const double* __restrict__ kdiag,
                             const double* __restrict__ shift, double* __restrict__ Adiag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) Adiag[i] = kdiag[i] + *shift;
}

__global__ void k_reset_status(DevStatus* st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->t = 0; st->done = 0; st->reason = R_NONE; st->since_best = 0; st->bad = 0; st->g = 0;
        st->delta = 0.0; st->amax = 0.0; st->best_delta = INFINITY;
    }
}

// Sweep 0: aggregates of all-zero messages, P~ = A_ii, S = b = y, in ring
// slot 0.  Padded nodes get P~ = 1, S = 0 so that their (zero) messages stay
// finite.
template <class AT>
__global__ void k_init(int64_t N, int64_t NPAD, int R, const double* __restrict__ Adiag,
                       const float* __restrict__ y, AT* __restrict__ Pt, AT* __restrict__ S,
                       double* __restrict__ alpha, DevStatus* st, double boxC) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NPAD) return;
    if (i < N) {
        const AT a = (AT)Adiag[i];
        AT b = (AT)y[i];
        double an = (double)(b / a) * (double)y[i];
        if (boxC > 0.0) {              // box projection of the initial means
            an = fmin(fmax(an, 0.0), boxC);
            b = a * (AT)(an * (double)y[i]);
        }
        Pt[i] = a;
        S[i] = b;
        alpha[i] = an;
        if (!(a > (AT)0) || !isfinite((double)a)) st->bad = 1;
        // slots of the sweeps before sweep 0 (stateless ring): P~ = +inf and
        // S = 0 make every message rebuilt from them exactly zero, which is
        // what the messages of sweep 0 are, so a fixed number of levels is
        // exact from sweep 1 on
        for (int r = 1; r < R; ++r) {
            Pt[(int64_t)r * NPAD + i] = (AT)INFINITY;
            S[(int64_t)r * NPAD + i] = (AT)0;
        }
    } else {
        // padding rows are never finalized: set them in every ring slot
        for (int r = 0; r < R; ++r) {
            Pt[(int64_t)r * NPAD + i] = (AT)1;
            S[(int64_t)r * NPAD + i] = (AT)0;
        }
    }
}

// Aggregates of the new sweep from the partial sums (fixed order) into ring
// slot `wslot`, the new alpha and the per-block change / magnitude maxima.
// boxC > 0: the belief mean is clipped to [0, boxC] (alpha space) and S is
// replaced by P~ times the clipped mean.
template <class AT, class PT>
__device__ inline void finalize_block(int64_t blk, int64_t N, int NB, const PT* __restrict__ partP,
                                      const PT* __restrict__ partE,
                                      const double* __restrict__ Adiag,
                                      const float* __restrict__ y, AT* __restrict__ Pt,
                                      AT* __restrict__ S, double* __restrict__ alpha,
                                      double* __restrict__ blk_delta,
                                      double* __restrict__ blk_amax, DevStatus* st, double boxC,
                                      AT* __restrict__ Inv, AT* __restrict__ Mean) {
    __shared__ double sh4[4];
    __shared__ AT shp[4][TILE], she[4][TILE];
    // the NB + 1 partial slots of the block, split into four contiguous
    // ranges, one per wave; each lane sums four nodes (64 apart) over its
    // wave's range, so every wave keeps eight independent loads in flight
    {
        const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
        const int S1 = NB + 1, qn = (S1 + 3) / 4;
        const int s0 = w * qn, s1 = (s0 + qn < S1) ? s0 + qn : S1;
        AT ap[4] = {0, 0, 0, 0}, ae[4] = {0, 0, 0, 0};
        for (int s = s0; s < s1; ++s) {
            const size_t o = ((size_t)blk * S1 + s) * TILE + l;
#pragma unroll
            for (int k = 0; k < 4; ++k) { ap[k] += (AT)partP[o + 64 * k]; ae[k] += (AT)partE[o + 64 * k]; }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) { shp[w][l + 64 * k] = ap[k]; she[w][l + 64 * k] = ae[k]; }
    }
    __syncthreads();
    const int64_t i = blk * blockDim.x + threadIdx.x;
    double d = 0.0, am = 0.0;
    bool bad = false;
    if (i < N) {
        const int t = threadIdx.x;
        AT p = (AT)Adiag[i] + ((shp[0][t] + shp[1][t]) + (shp[2][t] + shp[3][t]));
        AT e = (AT)y[i] + ((she[0][t] + she[1][t]) + (she[2][t] + she[3][t]));
        double an = (double)(e / p) * (double)y[i];
        bad = !(p > (AT)0) || !isfinite((double)p) || !isfinite((double)e);
        if (boxC > 0.0) {
            an = fmin(fmax(an, 0.0), boxC);
            e = p * (AT)(an * (double)y[i]);
        }
        Pt[i] = p;
        S[i] = e;
        if (Inv) { Inv[i] = (AT)1 / p; Mean[i] = e / p; }
        d = fabs(an - alpha[i]);
        am = fabs(an);
        alpha[i] = an;
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) st->bad = 1;
    d = block_max(d, sh4);
    am = block_max(am, sh4);
    if (threadIdx.x == 0) { blk_delta[blk] = d; blk_amax[blk] = am; }
}

template <class AT, class PT>
__global__ __launch_bounds__(WG) void k_finalize(int64_t N, int NB, const PT* __restrict__ partP,
                                                const PT* __restrict__ partE,
                                                const double* __restrict__ Adiag,
                                                const float* __restrict__ y, AT* __restrict__ Pt,
                                                AT* __restrict__ S, double* __restrict__ alpha,
                                                double* __restrict__ blk_delta,
                                                double* __restrict__ blk_amax, DevStatus* st, double boxC,
                                                AT* __restrict__ Inv, AT* __restrict__ Mean) {
    if (st->done) return;
    finalize_block<AT, PT>(blockIdx.x, N, NB, partP, partE, Adiag, y, Pt, S, alpha, blk_delta, blk_amax, st, boxC,
                           Inv, Mean);
}

// 1/P~ and S/P~ of every ring slot (series sweeps): P~ = +inf, S = 0 give 0
// and 0, the values a tile would form from them.
template <class AT>
__global__ void k_ring_recip(int64_t n, const AT* __restrict__ Pt, const AT* __restrict__ S,
                             AT* __restrict__ Inv, AT* __restrict__ Mean) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Inv[i] = (AT)1 / Pt[i];
    Mean[i] = S[i] / Pt[i];
}

// Grouped schedule: the node blocks [b0, b0 + gridDim.x) of one group.
template <class AT, class PT>
__global__ __launch_bounds__(WG) void k_finalize_range(int64_t b0, int64_t N, int NB, const PT* __restrict__ partP,
                                                      const PT* __restrict__ partE,
                                                      const double* __restrict__ Adiag,
                                                      const float* __restrict__ y, AT* __restrict__ Pt,
                                                      AT* __restrict__ S, double* __restrict__ alpha,
                                                      double* __restrict__ blk_delta,
                                                      double* __restrict__ blk_amax, DevStatus* st, double boxC,
                                                      AT* __restrict__ Inv, AT* __restrict__ Mean) {
    if (st->done) return;
    finalize_block<AT, PT>(b0 + blockIdx.x, N, NB, partP, partE, Adiag, y, Pt, S, alpha, blk_delta, blk_amax, st,
                           boxC, Inv, Mean);
}

// Served form: items are (request, block of 256 nodes).
template <class AT>
__global__ __launch_bounds__(WG) void k_finalize_batched(const ReqDesc* __restrict__ reqs,
                                                        const uint2* __restrict__ items, int nitems) {
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const uint2 w = items[it];
        const ReqDesc& rd = reqs[w.x];
        if (rd.sw.st->done) continue;
        const int64_t wslot = (int64_t)((rd.sw.st->t + 1) % rd.sw.R) * rd.sw.NPAD;
        AT* const Pt = static_cast<AT*>(const_cast<void*>(rd.sw.HP)) + wslot;
        AT* const S = static_cast<AT*>(const_cast<void*>(rd.sw.HS)) + wslot;
        // slots per block: NB + 1, or NBc + 1 after a sweep over chunks
        const int ns = (rd.sw.chunk > 1) ? (rd.sw.NB + rd.sw.chunk - 1) / rd.sw.chunk : rd.sw.NB;
        if (rd.sw.part32)
            finalize_block<AT, float>((int64_t)w.y, rd.N, ns, static_cast<const float*>(rd.sw.partP),
                                      static_cast<const float*>(rd.sw.partE), rd.Adiag, rd.y, Pt, S, rd.alpha,
                                      rd.blk_delta, rd.blk_amax, rd.sw.st, 0.0, nullptr, nullptr);
        else
            finalize_block<AT, AT>((int64_t)w.y, rd.N, ns, static_cast<const AT*>(rd.sw.partP),
                                   static_cast<const AT*>(rd.sw.partE), rd.Adiag, rd.y, Pt, S, rd.alpha,
                                   rd.blk_delta, rd.blk_amax, rd.sw.st, 0.0, nullptr, nullptr);
        __syncthreads();
    }
}

// Stop rule (Algorithm 2 step "Check", tested on alpha).
__device__ inline void status_update(int nblk, const double* __restrict__ bd,
                                     const double* __restrict__ ba, DevStatus* st,
                                     double* __restrict__ trace, const StopRule& rule) {
    __shared__ double sh4[4];
    double d = 0.0, a = 0.0;
    for (int k = threadIdx.x; k < nblk; k += blockDim.x) { d = fmax(d, bd[k]); a = fmax(a, ba[k]); }
    d = block_max(d, sh4);
    a = block_max(a, sh4);
    if (threadIdx.x == 0) {
        const int t = st->t + 1;
        st->t = t;
        st->delta = d;
        st->amax = a;
        trace[t - 1] = d;
        if (st->bad) {
            st->done = 1; st->reason = R_DIVERGED;
        } else if (d <= rule.tol_abs + rule.tol_rel * a) {
            st->done = 1; st->reason = R_CONVERGED;
        } else {
            if (d < st->best_delta) { st->best_delta = d; st->since_best = 0; }
            else st->since_best = st->since_best + 1;
            if (rule.stag_window > 0 && st->since_best >= rule.stag_window && d <= rule.stag_rel * a) {
                st->done = 1; st->reason = R_STAGNATED;
            } else if (t >= rule.max_sweeps) {
                st->done = 1; st->reason = R_MAX_SWEEPS;
            }
        }
    }
}

__global__ __launch_bounds__(WG) void k_status(int nblk, const double* __restrict__ bd,
                                              const double* __restrict__ ba, DevStatus* st,
                                              double* __restrict__ trace, StopRule rule) {
    if (st->done) return;
    status_update(nblk, bd, ba, st, trace, rule);
}

// Served form: one workgroup per active request; also copies the request's
// status into a packed array the host reads back in one transfer.
// Stop rule of served requests: a step visits one group of a grouped
// request (G groups; G = 1 for the synchronous schedule); after the visit of
// the last group the stop rule runs (one sweep done), and the group index
// advances for every request still running.
__global__ __launch_bounds__(WG) void k_status_grouped(const ReqDesc* __restrict__ reqs,
                                                      const int* __restrict__ slots, int n,
                                                      DevStatus* __restrict__ out) {
    const int k = blockIdx.x;
    if (k >= n) return;
    const ReqDesc& rd = reqs[slots[k]];
    DevStatus* st = rd.sw.st;
    const int done0 = st->done, g0 = st->g;
    __syncthreads();
    if (!done0) {
        if (g0 == rd.G - 1) status_update(rd.nblk, rd.blk_delta, rd.blk_amax, st, rd.trace, rd.rule);
        if (threadIdx.x == 0) st->g = (g0 + 1) % rd.G;
    }
    __syncthreads();
    if (threadIdx.x == 0) out[k] = *st;
}

// A-priori bound on the contraction of the message recursion.  With
// c_i = max_j |A_ij| * sum_{j != i} |A_ij|, every cavity precision satisfies
// Q_ij >= P~_i^(t-1) (messages are non-positive while Q > 0) and, by
// induction over sweeps, P~_i^t >= lo_i = A_ii - c_i / m* where
// m* = min_i (A_ii + sqrt(A_ii^2 - 4 c_i)) / 2 (the larger root of
// m^2 - A_ii m + c_i).  The induction needs every lo_i >= m* (then m* bounds
// every aggregate from below, P~^0 = A_ii included); lo_i equals m* at the
// node that defines it, so the comparison allows a 1e-12 relative rounding
// margin.  The reverse message enters the next one with a factor
// |A_ij| / Q_ij <= rowmax_i / lo_i, whose maximum is returned as rho (+inf if
// the bound does not exist).
__global__ void k_bound_root(int64_t N, const double* __restrict__ Adiag, const double* __restrict__ rowmax,
                             const double* __restrict__ rsum, double* __restrict__ blk) {
    __shared__ double sh4[4];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double v = -INFINITY;   // holds -root, so the block max is -(min root)
    if (i < N) {
        const double A = Adiag[i], c = rowmax[i] * rsum[i], disc = A * A - 4.0 * c;
        v = (disc >= 0.0 && A > 0.0) ? -0.5 * (A + sqrt(disc)) : INFINITY;
    }
    v = block_max(v, sh4);
    if (threadIdx.x == 0) blk[blockIdx.x] = v;
}

__global__ void k_bound_rho(int64_t N, const double* __restrict__ Adiag, const double* __restrict__ rowmax,
                            const double* __restrict__ rsum, const double* __restrict__ neg_mstar,
                            double* __restrict__ blk) {
    __shared__ double sh4[4];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double m = -*neg_mstar;
    double v = 0.0;
    if (i < N) {
        const double lo = Adiag[i] - rowmax[i] * rsum[i] / m;
        v = (m > 0.0 && lo >= m * (1.0 - 1e-12)) ? rowmax[i] / lo : INFINITY;
    }
    v = block_max(v, sh4);
    if (threadIdx.x == 0) blk[blockIdx.x] = v;
}

// ------------------------------------------------------------- queries --

template <class ST>
__global__ void k_entries(const ST* __restrict__ Kp, int NB, const int64_t* __restrict__ rows,
                          const int64_t* __restrict__ cols, int64_t n, double* __restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int64_t i = rows[k], j = cols[k];
    if (i > j) { const int64_t t = i; i = j; j = t; }
    const int I = (int)(i / TILE), J = (int)(j / TILE);
    out[k] = (double)Kp[(size_t)tile_index(I, J, NB) * TT + (size_t)(i % TILE) * TILE + (j % TILE)];
}

template <class AT>
__global__ void k_convert(const AT* __restrict__ src, double* __restrict__ dst, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (double)src[i];
}

// ----------------------------------------------------------- launchers --

static inline unsigned grid1(int64_t n) { return (unsigned)((n + WG - 1) / WG); }

hipError_t launch_fill_tiles(uint32_t* tiles, int NB, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_tiles, dim3(NB), dim3(WG), 0, s, tiles, NB);
    return hipGetLastError();
}

hipError_t launch_validate(const float* X, const float* y, int64_t N, int64_t m, int32_t* flag,
                           hipStream_t s) {
    int64_t n = std::max<int64_t>(N * m, N);
    unsigned g = (unsigned)std::min<int64_t>((n + WG - 1) / WG, 4096);
    if (g == 0) g = 1;
    hipLaunchKernelGGL(k_validate, dim3(g), dim3(WG), 0, s, X, y, N, m, flag);
    return hipGetLastError();
}

hipError_t launch_colmean(const float* X, int64_t N, int64_t m, double* mean, hipStream_t s) {
    hipLaunchKernelGGL(k_colmean, dim3((unsigned)m), dim3(WG), 0, s, X, N, m, mean);
    return hipGetLastError();
}

hipError_t launch_stage(const float* X, const double* mean, int64_t N, int64_t m, int64_t NPAD,
                        int m_pad, int kind, float* f32, uint16_t* hi, uint16_t* lo, uint16_t* lo2,
                        double* f64, float* nrm, hipStream_t s) {
    hipLaunchKernelGGL(k_stage, dim3(grid1(NPAD)), dim3(WG), 0, s, X, mean, N, m, NPAD, m_pad, kind,
                       f32, hi, lo, lo2, f64, nrm);
    return hipGetLastError();
}

hipError_t launch_gram(const Features& F, const KernelParams& kp, const uint32_t* tiles,
                       int64_t ntiles, void* Kp, hipStream_t s) {
    const dim3 g((unsigned)ntiles), b(WG);
    switch (F.kind) {
        case GRAM_F32: hipLaunchKernelGGL(k_gram_mfma<GRAM_F32>, g, b, 0, s, F, kp, tiles, (float*)Kp); break;
        case GRAM_BF16: hipLaunchKernelGGL(k_gram_mfma<GRAM_BF16>, g, b, 0, s, F, kp, tiles, (float*)Kp); break;
        case GRAM_BF16X3: hipLaunchKernelGGL(k_gram_mfma<GRAM_BF16X3>, g, b, 0, s, F, kp, tiles, (float*)Kp); break;
        case GRAM_BF16X6: hipLaunchKernelGGL(k_gram_mfma<GRAM_BF16X6>, g, b, 0, s, F, kp, tiles, (float*)Kp); break;
        case GRAM_F64: hipLaunchKernelGGL(k_gram_f64, g, b, 0, s, F, kp, tiles, (double*)Kp); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_gram_sums(const Features& F, const KernelParams& kp, const uint32_t* tiles, int64_t ntiles,
                            void* Kp, int NB, double* psum, double* pmax, hipStream_t s) {
    const dim3 g((unsigned)ntiles);
    float* K = (float*)Kp;
    switch (F.kind) {
        case GRAM_F32: gram_sums_kind<GRAM_F32>(F.m_pad, g, F, kp, tiles, K, NB, psum, pmax, s); break;
        case GRAM_BF16: gram_sums_kind<GRAM_BF16>(F.m_pad, g, F, kp, tiles, K, NB, psum, pmax, s); break;
        case GRAM_BF16X3: gram_sums_kind<GRAM_BF16X3>(F.m_pad, g, F, kp, tiles, K, NB, psum, pmax, s); break;
        case GRAM_BF16X6: gram_sums_kind<GRAM_BF16X6>(F.m_pad, g, F, kp, tiles, K, NB, psum, pmax, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_gather_dense(const double* K, const KernelParams& kp, const uint32_t* tiles,
                               int64_t ntiles, void* Kp, int prec, double* kdiag, hipStream_t s) {
    const dim3 g((unsigned)ntiles), b(WG);
    if (prec == PREC_FP64)
        hipLaunchKernelGGL(k_gather_dense<double>, g, b, 0, s, K, kp, tiles, (double*)Kp);
    else
        hipLaunchKernelGGL(k_gather_dense<float>, g, b, 0, s, K, kp, tiles, (float*)Kp);
    hipLaunchKernelGGL(k_dense_diag, dim3(grid1(kp.N)), dim3(WG), 0, s, K, kp.N, kdiag);
    return hipGetLastError();
}

hipError_t launch_fill_value(double* dst, int64_t n, double v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_value, dim3(grid1(n)), dim3(WG), 0, s, dst, n, v);
    return hipGetLastError();
}

hipError_t launch_rowsum(const void* Kp, int prec, int ksrc, const Features& F, const KernelParams& kp,
                         const uint32_t* tiles, int64_t ntiles, int NB, double* psum, double* pmax,
                         hipStream_t s) {
    const dim3 g((unsigned)ntiles), b(WG);
    if (ksrc == KSRC_PLANE) {
        if (prec == PREC_FP64)
            hipLaunchKernelGGL((k_rowsum<double, KSRC_PLANE, GRAM_F64>), g, b, 0, s, (const double*)Kp, F, kp, tiles, NB, psum, pmax);
        else
            hipLaunchKernelGGL((k_rowsum<float, KSRC_PLANE, GRAM_F32>), g, b, 0, s, (const float*)Kp, F, kp, tiles, NB, psum, pmax);
    } else {
        switch (F.kind) {
            case GRAM_F32: hipLaunchKernelGGL((k_rowsum<float, KSRC_RECOMPUTE, GRAM_F32>), g, b, 0, s, nullptr, F, kp, tiles, NB, psum, pmax); break;
            case GRAM_BF16: hipLaunchKernelGGL((k_rowsum<float, KSRC_RECOMPUTE, GRAM_BF16>), g, b, 0, s, nullptr, F, kp, tiles, NB, psum, pmax); break;
            case GRAM_BF16X3: hipLaunchKernelGGL((k_rowsum<float, KSRC_RECOMPUTE, GRAM_BF16X3>), g, b, 0, s, nullptr, F, kp, tiles, NB, psum, pmax); break;
            case GRAM_BF16X6: hipLaunchKernelGGL((k_rowsum<float, KSRC_RECOMPUTE, GRAM_BF16X6>), g, b, 0, s, nullptr, F, kp, tiles, NB, psum, pmax); break;
            default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

hipError_t launch_residual(const void* Kp, int prec, int ksrc, const Features& F, const KernelParams& kp,
                           const uint32_t* tiles, int64_t ntiles, int NB, int64_t N, int64_t NPAD,
                           const double* alpha, const float* y, const double* Adiag, const double* rsum,
                           double* w, double* part, double* blk1, double* blk2, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_weights, dim3(grid1(NPAD)), dim3(WG), 0, s, N, NPAD, alpha, y, w);
    const dim3 g((unsigned)ntiles), b(WG);
    if (ksrc == KSRC_PLANE) {
        if (prec == PREC_FP64)
            hipLaunchKernelGGL((k_apply<double, KSRC_PLANE, GRAM_F64>), g, b, 0, s, (const double*)Kp, F, kp, tiles, NB, w, part);
        else
            hipLaunchKernelGGL((k_apply<float, KSRC_PLANE, GRAM_F32>), g, b, 0, s, (const float*)Kp, F, kp, tiles, NB, w, part);
    } else {
        switch (F.kind) {
            case GRAM_F32: hipLaunchKernelGGL((k_apply<float, KSRC_RECOMPUTE, GRAM_F32>), g, b, 0, s, nullptr, F, kp, tiles, NB, w, part); break;
            case GRAM_BF16: hipLaunchKernelGGL((k_apply<float, KSRC_RECOMPUTE, GRAM_BF16>), g, b, 0, s, nullptr, F, kp, tiles, NB, w, part); break;
            case GRAM_BF16X3: hipLaunchKernelGGL((k_apply<float, KSRC_RECOMPUTE, GRAM_BF16X3>), g, b, 0, s, nullptr, F, kp, tiles, NB, w, part); break;
            case GRAM_BF16X6: hipLaunchKernelGGL((k_apply<float, KSRC_RECOMPUTE, GRAM_BF16X6>), g, b, 0, s, nullptr, F, kp, tiles, NB, w, part); break;
            default: return hipErrorInvalidValue;
        }
    }
    const unsigned nb = grid1(N);
    hipLaunchKernelGGL(k_residual_blocks, dim3(nb), dim3(WG), 0, s, N, NB, part, Adiag, rsum, alpha, y, blk1, blk2);
    hipLaunchKernelGGL(k_residual_final, dim3(1), dim3(WG), 0, s, (int)nb, blk1, blk2, out);
    return hipGetLastError();
}

hipError_t launch_diag(int64_t N, int NB, const double* psum, const double* pmax, const double* kdiag,
                       int mode, double C, double delta, double* Adiag, double* rowmax, double* rsum,
                       double* scratch_blk, double* scratch_one, hipStream_t s) {
    const unsigned nb = grid1(N);
    hipLaunchKernelGGL(k_diag, dim3(nb), dim3(WG), 0, s, N, NB, psum, pmax, kdiag, mode, C, delta, Adiag,
                       rowmax, rsum, scratch_blk);
    if (mode == 3) {
        hipLaunchKernelGGL(k_max_reduce, dim3(1), dim3(WG), 0, s, (int)nb, scratch_blk, scratch_one);
        hipLaunchKernelGGL(k_diag_shift, dim3(nb), dim3(WG), 0, s, N, kdiag, scratch_one, Adiag);
    }
    return hipGetLastError();
}

hipError_t launch_init(int prec, int64_t N, int64_t NPAD, int R, const double* Adiag, const float* y,
                       void* Pt, void* S, double* alpha, DevStatus* st, hipStream_t s, double boxC) {
    hipLaunchKernelGGL(k_reset_status, dim3(1), dim3(64), 0, s, st);
    if (prec == PREC_FP32)
        hipLaunchKernelGGL(k_init<float>, dim3(grid1(NPAD)), dim3(WG), 0, s, N, NPAD, R, Adiag, y,
                           (float*)Pt, (float*)S, alpha, st, boxC);
    else
        hipLaunchKernelGGL(k_init<double>, dim3(grid1(NPAD)), dim3(WG), 0, s, N, NPAD, R, Adiag, y,
                           (double*)Pt, (double*)S, alpha, st, boxC);
    return hipGetLastError();
}

// Per-precision sweep dispatch lives in gabp_sweep_{f32,mixed,f64}.hip.
hipError_t launch_sweep(int prec, int ksrc, int gram, int levels, bool first, int ser, const SweepArgs& a,
                        hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (levels == 0) ser = 0;
    switch (prec) {
        case PREC_FP32: return launch_sweep_f32(ksrc, gram, levels, first, ser, a, s, e0, e1);
        case PREC_MIXED: return launch_sweep_mixed(ksrc, gram, levels, first, ser, a, s, e0, e1);
        case PREC_FP64: return launch_sweep_f64(ksrc, gram, levels, first, ser, a, s, e0, e1);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep_grouped(int prec, int ksrc, int gram, int levels, int ser, const SweepArgs& a,
                                const uint32_t* within, int nwithin, const uint32_t* dir, int ndir, int t,
                                hipStream_t s) {
    if (levels == 0) ser = 0;
    switch (prec) {
        case PREC_FP32: return launch_sweep_grouped_f32(ksrc, gram, levels, ser, a, within, nwithin, dir, ndir, t, s);
        case PREC_MIXED: return launch_sweep_grouped_mixed(ksrc, gram, levels, ser, a, within, nwithin, dir, ndir, t, s);
        case PREC_FP64: return launch_sweep_grouped_f64(ksrc, gram, levels, ser, a, within, nwithin, dir, ndir, t, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_served_sweep(int prec, int levels, int ser, bool grouped, const ReqDesc* reqs, const uint2* items,
                               int n, hipStream_t s) {
    switch (prec) {
        case PREC_FP32: return launch_served_sweep_f32(levels, ser, grouped, reqs, items, n, s);
        case PREC_MIXED: return launch_served_sweep_mixed(levels, ser, grouped, reqs, items, n, s);
        case PREC_FP64: return launch_served_sweep_f64(levels, ser, grouped, reqs, items, n, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_served_finalize(bool agg_f32, const ReqDesc* reqs, const uint2* items, int n, hipStream_t s) {
    const int gf = std::max(1, std::min(n, 2048));
    if (agg_f32)
        hipLaunchKernelGGL(k_finalize_batched<float>, dim3(gf), dim3(WG), 0, s, reqs, items, n);
    else
        hipLaunchKernelGGL(k_finalize_batched<double>, dim3(gf), dim3(WG), 0, s, reqs, items, n);
    return hipGetLastError();
}

hipError_t launch_served_status(const ReqDesc* reqs, const int* slots, int nslots, DevStatus* status_out,
                                hipStream_t s) {
    hipLaunchKernelGGL(k_status_grouped, dim3(std::max(1, nslots)), dim3(WG), 0, s, reqs, slots, nslots, status_out);
    return hipGetLastError();
}

hipError_t launch_finalize(int prec, int64_t N, int NB, const void* partP, const void* partE,
                           const double* Adiag, const float* y, void* Pt, void* S, double* alpha,
                           double* blk_delta, double* blk_amax, DevStatus* st, hipStream_t s, double boxC,
                           void* Inv, void* Mean, int part32) {
    if ((Inv == nullptr) != (Mean == nullptr)) return hipErrorInvalidValue;
    const dim3 g(grid1(N)), b(WG);
    if (prec == PREC_FP32)
        hipLaunchKernelGGL((k_finalize<float, float>), g, b, 0, s, N, NB, (const float*)partP,
                           (const float*)partE, Adiag, y, (float*)Pt, (float*)S, alpha, blk_delta,
                           blk_amax, st, boxC, (float*)Inv, (float*)Mean);
    else if (part32)
        hipLaunchKernelGGL((k_finalize<double, float>), g, b, 0, s, N, NB, (const float*)partP,
                           (const float*)partE, Adiag, y, (double*)Pt, (double*)S, alpha,
                           blk_delta, blk_amax, st, boxC, (double*)Inv, (double*)Mean);
    else
        hipLaunchKernelGGL((k_finalize<double, double>), g, b, 0, s, N, NB, (const double*)partP,
                           (const double*)partE, Adiag, y, (double*)Pt, (double*)S, alpha,
                           blk_delta, blk_amax, st, boxC, (double*)Inv, (double*)Mean);
    return hipGetLastError();
}

hipError_t launch_ring_recip(int prec, int64_t NPAD, int R, const void* Pt, const void* S, void* Inv, void* Mean,
                             hipStream_t s) {
    const int64_t n = NPAD * (int64_t)R;
    if (prec == PREC_FP32)
        hipLaunchKernelGGL(k_ring_recip<float>, dim3(grid1(n)), dim3(WG), 0, s, n, (const float*)Pt,
                           (const float*)S, (float*)Inv, (float*)Mean);
    else
        hipLaunchKernelGGL(k_ring_recip<double>, dim3(grid1(n)), dim3(WG), 0, s, n, (const double*)Pt,
                           (const double*)S, (double*)Inv, (double*)Mean);
    return hipGetLastError();
}

hipError_t launch_finalize_range(int prec, int64_t b0, int64_t nb, int64_t N, int NB, const void* partP,
                                 const void* partE, const double* Adiag, const float* y, void* Pt, void* S,
                                 double* alpha, double* blk_delta, double* blk_amax, DevStatus* st,
                                 hipStream_t s, double boxC, void* Inv, void* Mean, int part32) {
    if (nb <= 0) return hipSuccess;
    if ((Inv == nullptr) != (Mean == nullptr)) return hipErrorInvalidValue;
    const dim3 g((unsigned)nb), b(WG);
    if (prec == PREC_FP32)
        hipLaunchKernelGGL((k_finalize_range<float, float>), g, b, 0, s, b0, N, NB, (const float*)partP,
                           (const float*)partE, Adiag, y, (float*)Pt, (float*)S, alpha, blk_delta, blk_amax, st,
                           boxC, (float*)Inv, (float*)Mean);
    else if (part32)
        hipLaunchKernelGGL((k_finalize_range<double, float>), g, b, 0, s, b0, N, NB, (const float*)partP,
                           (const float*)partE, Adiag, y, (double*)Pt, (double*)S, alpha, blk_delta, blk_amax,
                           st, boxC, (double*)Inv, (double*)Mean);
    else
        hipLaunchKernelGGL((k_finalize_range<double, double>), g, b, 0, s, b0, N, NB, (const double*)partP,
                           (const double*)partE, Adiag, y, (double*)Pt, (double*)S, alpha, blk_delta, blk_amax,
                           st, boxC, (double*)Inv, (double*)Mean);
    return hipGetLastError();
}

hipError_t launch_status(int nblk, const double* blk_delta, const double* blk_amax, DevStatus* st,
                         double* trace, StopRule rule, hipStream_t s) {
    hipLaunchKernelGGL(k_status, dim3(1), dim3(WG), 0, s, nblk, blk_delta, blk_amax, st, trace, rule);
    return hipGetLastError();
}

hipError_t launch_rho_bound(int64_t N, const double* Adiag, const double* rowmax, const double* rsum,
                            double* blk, double* one, hipStream_t s) {
    const unsigned nb = grid1(N);
    hipLaunchKernelGGL(k_bound_root, dim3(nb), dim3(WG), 0, s, N, Adiag, rowmax, rsum, blk);
    hipLaunchKernelGGL(k_max_reduce, dim3(1), dim3(WG), 0, s, (int)nb, blk, one);
    hipLaunchKernelGGL(k_bound_rho, dim3(nb), dim3(WG), 0, s, N, Adiag, rowmax, rsum, one, blk);
    hipLaunchKernelGGL(k_max_reduce, dim3(1), dim3(WG), 0, s, (int)nb, blk, one + 1);
    return hipGetLastError();
}

hipError_t launch_kernel_entries(const void* Kp, int prec, int NB, const int64_t* rows,
                                 const int64_t* cols, int64_t n, double* out, hipStream_t s) {
    if (prec == PREC_FP64)
        hipLaunchKernelGGL(k_entries<double>, dim3(grid1(n)), dim3(WG), 0, s, (const double*)Kp, NB,
                           rows, cols, n, out);
    else
        hipLaunchKernelGGL(k_entries<float>, dim3(grid1(n)), dim3(WG), 0, s, (const float*)Kp, NB,
                           rows, cols, n, out);
    return hipGetLastError();
}

hipError_t launch_convert_agg(int prec, const void* src, double* dst, int64_t n, hipStream_t s) {
    if (prec == PREC_FP32)
        hipLaunchKernelGGL(k_convert<float>, dim3(grid1(n)), dim3(WG), 0, s, (const float*)src, dst, n);
    else
        hipLaunchKernelGGL(k_convert<double>, dim3(grid1(n)), dim3(WG), 0, s, (const double*)src, dst, n);
    return hipGetLastError();
}

}  // namespace gabp

