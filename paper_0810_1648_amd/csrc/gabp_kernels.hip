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
#include "gabp_internal.h"

#include <math.h>

namespace gabp {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4v __attribute__((ext_vector_type(4)));

// ----------------------------------------------------------------- helpers

template <class T> struct V4 { T v[4]; };

__device__ inline V4<float> ld4(const float* p) {
    const float4 x = *reinterpret_cast<const float4*>(p);
    return {{x.x, x.y, x.z, x.w}};
}
__device__ inline V4<double> ld4(const double* p) {
    const double2 a = *reinterpret_cast<const double2*>(p);
    const double2 b = *reinterpret_cast<const double2*>(p + 2);
    return {{a.x, a.y, b.x, b.y}};
}
__device__ inline void st4(float* p, const V4<float>& v) {
    *reinterpret_cast<float4*>(p) = make_float4(v.v[0], v.v[1], v.v[2], v.v[3]);
}
__device__ inline void st4(double* p, const V4<double>& v) {
    *reinterpret_cast<double2*>(p) = make_double2(v.v[0], v.v[1]);
    *reinterpret_cast<double2*>(p + 2) = make_double2(v.v[2], v.v[3]);
}

template <int CTRL> __device__ inline int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL> __device__ inline float dpp(float v) {
    return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}
template <int CTRL> __device__ inline double dpp(double v) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const int lo = dpp_i<CTRL>((int)(unsigned)(u & 0xffffffffull));
    const int hi = dpp_i<CTRL>((int)(unsigned)(u >> 32));
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                            (unsigned long long)(unsigned)lo));
}
// Sum over the 16 lanes of a DPP row; every lane receives the same bits.
template <class T> __device__ inline T sum16(T v) {
    v = v + dpp<0xB1>(v);    // quad_perm(1,0,3,2): pairs
    v = v + dpp<0x4E>(v);    // quad_perm(2,3,0,1): quads
    v = v + dpp<0x141>(v);   // row_half_mirror: 8 lanes
    v = v + dpp<0x140>(v);   // row_mirror: 16 lanes
    return v;
}
// Sum over lanes q, q+16, q+32, q+48 in the fixed order (g0+g1)+(g2+g3).
template <class T> __device__ inline T sum_groups(T v) {
    v = v + __shfl_xor(v, 16);
    v = v + __shfl_xor(v, 32);
    return v;
}
__device__ inline double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}
// Block (256 threads) max; result valid in every thread.
__device__ inline double block_max(double v, double* sh4) {
    v = wave_max(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh4[w] = v;
    __syncthreads();
    v = fmax(fmax(sh4[0], sh4[1]), fmax(sh4[2], sh4[3]));
    __syncthreads();
    return v;
}

__device__ inline uint16_t f2bf(float f) {  // round to nearest even
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

struct TileCoord { int I, J; };
__device__ inline TileCoord tile_of(const uint32_t* tiles) {
    const uint32_t ij = tiles[blockIdx.x];
    return {(int)(ij >> 16), (int)(ij & 0xFFFFu)};
}

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

// ------------------------------------------------------------ K' build --

// Materialise K' = exp(-gamma d^2) + lambda^2 for one tile with MFMA Gram
// products: d^2 = n_i + n_j - 2 x_i.x_j.  Wave w computes the 32-row bands
// w and w + 4, one 32 x 32 sub-block at a time; operands come straight from
// the staged features (L2-resident).  The inner-product index k is split
// between the two lane halves so each lane reads contiguous features.
template <int KIND>
__global__ __launch_bounds__(WG) void k_gram_mfma(Features F, KernelParams kp,
                                                 const uint32_t* __restrict__ tiles,
                                                 float* __restrict__ Kp) {
    const TileCoord tc = tile_of(tiles);
    const size_t tbase = (size_t)blockIdx.x * TT;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, h = l >> 5, l32 = l & 31;
    const int mp = F.m_pad;
    const float lam2 = (float)kp.lam2;
    for (int band = w; band < TILE / 32; band += 4) {
        const int64_t rowA = (int64_t)tc.I * TILE + band * 32 + l32;
        float ni[16];
#pragma unroll
        for (int r = 0; r < 16; ++r)
            ni[r] = F.nrm[(int64_t)tc.I * TILE + band * 32 + 8 * (r >> 2) + 4 * h + (r & 3)];
        for (int cb = 0; cb < TILE / 32; ++cb) {
            const int64_t colB = (int64_t)tc.J * TILE + cb * 32 + l32;
            f32x16 acc = {};
            if constexpr (KIND == GRAM_F32) {
                const int half = mp >> 1;
                const float* pa = F.f32 + rowA * mp + h * half;
                const float* pb = F.f32 + colB * mp + h * half;
                for (int s = 0; s < half; s += 4) {
                    const f32x4v a4 = *reinterpret_cast<const f32x4v*>(pa + s);
                    const f32x4v b4 = *reinterpret_cast<const f32x4v*>(pb + s);
                    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a4[0], b4[0], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a4[1], b4[1], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a4[2], b4[2], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a4[3], b4[3], acc, 0, 0, 0);
                }
            } else {
                const uint16_t* pa = F.hi + rowA * mp + 8 * h;
                const uint16_t* pb = F.hi + colB * mp + 8 * h;
                for (int s = 0; s < mp; s += 16) {
                    const bf16x8 a = *reinterpret_cast<const bf16x8*>(pa + s);
                    const bf16x8 b = *reinterpret_cast<const bf16x8*>(pb + s);
                    if constexpr (KIND == GRAM_BF16X3 || KIND == GRAM_BF16X6) {
                        // correction terms first, then the leading product
                        const bf16x8 al = *reinterpret_cast<const bf16x8*>(F.lo + rowA * mp + 8 * h + s);
                        const bf16x8 bl = *reinterpret_cast<const bf16x8*>(F.lo + colB * mp + 8 * h + s);
                        if constexpr (KIND == GRAM_BF16X6) {
                            const bf16x8 a2 = *reinterpret_cast<const bf16x8*>(F.lo2 + rowA * mp + 8 * h + s);
                            const bf16x8 b2 = *reinterpret_cast<const bf16x8*>(F.lo2 + colB * mp + 8 * h + s);
                            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b2, acc, 0, 0, 0);
                            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a2, b, acc, 0, 0, 0);
                            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bl, acc, 0, 0, 0);
                        }
                        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bl, acc, 0, 0, 0);
                        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, b, acc, 0, 0, 0);
                    }
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
                }
            }
            const float nj = F.nrm[colB];
            const int col = cb * 32 + l32;
            const int64_t j = (int64_t)tc.J * TILE + col;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = band * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
                const int64_t i = (int64_t)tc.I * TILE + row;
                const float d2 = fmaxf(ni[r] + nj - 2.0f * acc[r], 0.0f);
                const float kv = exp2f(kp.neg_gamma_log2e * d2) + lam2;
                Kp[tbase + (size_t)row * TILE + col] = (i < j && j < kp.N) ? kv : 0.0f;
            }
        }
    }
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

// r_i = sum_{j != i} |K'_ij|, as per-tile partial sums (FP64).
template <class ST>
__global__ __launch_bounds__(WG) void k_rowsum(const ST* __restrict__ Kp,
                                              const uint32_t* __restrict__ tiles, int NB,
                                              double* __restrict__ part) {
    const TileCoord tc = tile_of(tiles);
    const size_t tbase = (size_t)blockIdx.x * TT;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, g = l >> 4, q = l & 15;
    const int col0 = w * 64 + q * 4;
    __shared__ double rows[4][TILE];
    double cs[4] = {0.0, 0.0, 0.0, 0.0};
    for (int s = 0; s < TILE / 4; ++s) {
        const int r = 4 * s + g;
        const V4<ST> k = ld4(Kp + tbase + (size_t)r * TILE + col0);
        double rs = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double a = fabs((double)k.v[c]);
            cs[c] += a;
            rs += a;
        }
        rs = sum16(rs);
        if (q == 0) rows[w][r] = rs;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) cs[c] = sum_groups(cs[c]);
    __syncthreads();
    part[((size_t)tc.I * (NB + 1) + tc.J) * TILE + tid] = (rows[0][tid] + rows[1][tid]) + (rows[2][tid] + rows[3][tid]);
    if (g == 0) {
        const int slot = (tc.I < tc.J) ? tc.I : NB;
        double* dst = part + ((size_t)tc.J * (NB + 1) + slot) * TILE + col0;
#pragma unroll
        for (int c = 0; c < 4; ++c) dst[c] = cs[c];
    }
}

// Weighted diagonal (subsection "GaBP Algorithm Convergence").  For the
// uniform rule this kernel leaves A_ii - K'_ii per node and a per-block max.
__global__ void k_diag(int64_t N, int NB, const double* __restrict__ part,
                       const double* __restrict__ kdiag, int mode, double C, double delta,
                       double* __restrict__ Adiag, double* __restrict__ blk) {
    __shared__ double sh4[4];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double wv = -INFINITY;
    if (i < N) {
        const int64_t B = i / TILE, t = i % TILE;
        double r = 0.0;
        for (int s = 0; s <= NB; ++s) r += part[((size_t)B * (NB + 1) + s) * TILE + t];
        const double kii = kdiag[i];
        const double soft = kii + 1.0 / C, dom = (1.0 + delta) * r;
        double a;
        switch (mode) {
            case 0: a = kii; break;
            case 1: a = soft; break;
            default: a = fmax(soft, dom); break;
        }
        Adiag[i] = a;
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

// Sweep 0: aggregates of all-zero messages, P~ = A_ii, S = b = y.  Padded
// nodes get P~ = 1, S = 0 so that their (zero) messages stay finite.
template <class AT>
__global__ void k_init(int64_t N, int64_t NPAD, const double* __restrict__ Adiag,
                       const float* __restrict__ y, AT* __restrict__ Pt, AT* __restrict__ S,
                       double* __restrict__ alpha, DevStatus* st) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NPAD) return;
    if (i < N) {
        const AT a = (AT)Adiag[i], b = (AT)y[i];
        Pt[i] = a;
        S[i] = b;
        alpha[i] = (double)(b / a) * (double)y[i];
        if (!(a > (AT)0) || !isfinite((double)a)) st->bad = 1;
    } else {
        Pt[i] = (AT)1;
        S[i] = (AT)0;
    }
}

__global__ void k_reset_status(DevStatus* st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->t = 0; st->done = 0; st->reason = R_NONE; st->since_best = 0; st->bad = 0; st->pad = 0;
        st->delta = 0.0; st->amax = 0.0; st->best_delta = INFINITY;
    }
}

// ------------------------------------------------------------------ sweep --

template <class ST, class MT, class AT, bool FIRST>
__global__ __launch_bounds__(WG) void k_sweep_stored(
    const uint32_t* __restrict__ tiles, int NB, const ST* __restrict__ Kp, ST* __restrict__ Pf,
    ST* __restrict__ Pb, ST* __restrict__ Ef, ST* __restrict__ Eb, const AT* __restrict__ Pt,
    const AT* __restrict__ S, AT* __restrict__ partP, AT* __restrict__ partE, DevStatus* st) {
    if (st->done) return;
    const TileCoord tc = tile_of(tiles);
    const size_t tbase = (size_t)blockIdx.x * TT;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, g = l >> 4, q = l & 15;
    const int col0 = w * 64 + q * 4;

    __shared__ AT sPt[TILE], sS[TILE];
    __shared__ AT rP[4][TILE], rE[4][TILE];
    sPt[tid] = Pt[(int64_t)tc.I * TILE + tid];
    sS[tid] = S[(int64_t)tc.I * TILE + tid];
    MT ptj[4], sj[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        ptj[c] = (MT)Pt[(int64_t)tc.J * TILE + col0 + c];
        sj[c] = (MT)S[(int64_t)tc.J * TILE + col0 + c];
    }
    AT cP[4] = {0, 0, 0, 0}, cE[4] = {0, 0, 0, 0};
    bool bad = false;
    __syncthreads();

    const ST* kp = Kp + tbase + (size_t)g * TILE + col0;
    size_t off = tbase + (size_t)g * TILE + col0;
    V4<ST> k = ld4(kp);
    V4<ST> pf{}, pb{}, ef{}, eb{};
    if (!FIRST) { pf = ld4(Pf + off); pb = ld4(Pb + off); ef = ld4(Ef + off); eb = ld4(Eb + off); }

    for (int s = 0; s < TILE / 4; ++s) {
        const int r = 4 * s + g;
        // prefetch the next row of this lane
        V4<ST> k2{}, pf2{}, pb2{}, ef2{}, eb2{};
        const size_t off2 = off + 4 * TILE;
        if (s + 1 < TILE / 4) {
            k2 = ld4(Kp + off2);
            if (!FIRST) { pf2 = ld4(Pf + off2); pb2 = ld4(Pb + off2); ef2 = ld4(Ef + off2); eb2 = ld4(Eb + off2); }
        }
        const MT pti = (MT)sPt[r], si = (MT)sS[r];
        AT rp = 0, re = 0;
        V4<ST> npf, npb, nef, neb;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const MT a = (MT)k.v[c];
            const MT a2 = a * a;
            const MT qf = pti - (MT)pb.v[c];       // P~_i - P_ji
            const MT qb = ptj[c] - (MT)pf.v[c];    // P~_j - P_ij
            bad |= !(qf > (MT)0) | !(qb > (MT)0);
            const MT rf = (MT)1 / qf, rb = (MT)1 / qb;
            const ST pij = (ST)(-a2 * rf);
            const ST eij = (ST)(-a * (si - (MT)eb.v[c]) * rf);
            const ST pji = (ST)(-a2 * rb);
            const ST eji = (ST)(-a * (sj[c] - (MT)ef.v[c]) * rb);
            npf.v[c] = pij; nef.v[c] = eij; npb.v[c] = pji; neb.v[c] = eji;
            cP[c] += (AT)pij; cE[c] += (AT)eij;     // received by column node j
            rp += (AT)pji; re += (AT)eji;            // received by row node i
        }
        st4(Pf + off, npf); st4(Pb + off, npb); st4(Ef + off, nef); st4(Eb + off, neb);
        rp = sum16(rp);
        re = sum16(re);
        if (q == 0) { rP[w][r] = rp; rE[w][r] = re; }
        k = k2; pf = pf2; pb = pb2; ef = ef2; eb = eb2;
        off = off2;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) { cP[c] = sum_groups(cP[c]); cE[c] = sum_groups(cE[c]); }
    __syncthreads();
    const size_t rowslot = ((size_t)tc.I * (NB + 1) + tc.J) * TILE + tid;
    partP[rowslot] = (rP[0][tid] + rP[1][tid]) + (rP[2][tid] + rP[3][tid]);
    partE[rowslot] = (rE[0][tid] + rE[1][tid]) + (rE[2][tid] + rE[3][tid]);
    if (g == 0) {
        const int slot = (tc.I < tc.J) ? tc.I : NB;
        const size_t cb = ((size_t)tc.J * (NB + 1) + slot) * TILE + col0;
#pragma unroll
        for (int c = 0; c < 4; ++c) { partP[cb + c] = cP[c]; partE[cb + c] = cE[c]; }
    }
    if (__any(bad) && l == 0) st->bad = 1;
}

// Aggregates of the new sweep from the partial sums (fixed order), the new
// alpha and the per-block change / magnitude maxima.
template <class AT>
__global__ __launch_bounds__(WG) void k_finalize(int64_t N, int NB, const AT* __restrict__ partP,
                                                const AT* __restrict__ partE,
                                                const double* __restrict__ Adiag,
                                                const float* __restrict__ y, AT* __restrict__ Pt,
                                                AT* __restrict__ S, double* __restrict__ alpha,
                                                double* __restrict__ blk_delta,
                                                double* __restrict__ blk_amax, DevStatus* st) {
    if (st->done) return;
    __shared__ double sh4[4];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double d = 0.0, am = 0.0;
    bool bad = false;
    if (i < N) {
        const int64_t B = i / TILE, t = i % TILE;
        AT p = (AT)Adiag[i], e = (AT)y[i];
        for (int s = 0; s <= NB; ++s) {
            const size_t o = ((size_t)B * (NB + 1) + s) * TILE + t;
            p += partP[o];
            e += partE[o];
        }
        Pt[i] = p;
        S[i] = e;
        const double an = (double)(e / p) * (double)y[i];
        bad = !(p > (AT)0) || !isfinite((double)p) || !isfinite((double)e);
        d = fabs(an - alpha[i]);
        am = fabs(an);
        alpha[i] = an;
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) st->bad = 1;
    d = block_max(d, sh4);
    am = block_max(am, sh4);
    if (threadIdx.x == 0) { blk_delta[blockIdx.x] = d; blk_amax[blockIdx.x] = am; }
}

// Stop rule (Algorithm 2 step "Check", tested on alpha).
__global__ __launch_bounds__(WG) void k_status(int nblk, const double* __restrict__ bd,
                                              const double* __restrict__ ba, DevStatus* st,
                                              double* __restrict__ trace, StopRule rule) {
    if (st->done) return;
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

// f(x_q) = sum_i alpha_i y_i (K(x_i, x_q) + lambda^2), one workgroup per query,
// direct differences; FP64 sum in a fixed order.
__global__ __launch_bounds__(WG) void k_predict(const float* __restrict__ Xtr,
                                               const float* __restrict__ y,
                                               const double* __restrict__ alpha, int64_t N,
                                               int64_t m, const float* __restrict__ Xq,
                                               double gamma, double lam2, int fp64,
                                               double* __restrict__ f) {
    __shared__ double sh[WG];
    const int64_t qi = blockIdx.x;
    const float* xq = Xq + qi * m;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < N; i += WG) {
        const float* xi = Xtr + i * m;
        double kv;
        if (fp64) {
            double d2 = 0.0;
            for (int64_t k = 0; k < m; ++k) { const double d = (double)xi[k] - (double)xq[k]; d2 = fma(d, d, d2); }
            kv = exp(-gamma * d2);
        } else {
            float d2 = 0.0f;
            for (int64_t k = 0; k < m; ++k) { const float d = xi[k] - xq[k]; d2 = fmaf(d, d, d2); }
            kv = (double)expf(-(float)gamma * d2);
        }
        acc += alpha[i] * (double)y[i] * (kv + lam2);
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = WG / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) f[qi] = sh[0];
}

// ----------------------------------------------------------- launchers --

static inline unsigned grid1(int64_t n) { return (unsigned)((n + WG - 1) / WG); }

hipError_t launch_fill_tiles(uint32_t* tiles, int NB, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_tiles, dim3(NB), dim3(WG), 0, s, tiles, NB);
    return hipGetLastError();
}

hipError_t launch_validate(const float* X, const float* y, int64_t N, int64_t m, int32_t* flag,
                           hipStream_t s) {
    int64_t n = N * m;
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
                       int64_t ntiles, void* Kp, int prec, hipStream_t s) {
    const dim3 g((unsigned)ntiles), b(WG);
    switch (F.kind) {
        case GRAM_F32: hipLaunchKernelGGL(k_gram_mfma<GRAM_F32>, g, b, 0, s, F, kp, tiles, (float*)Kp); break;
        case GRAM_BF16: hipLaunchKernelGGL(k_gram_mfma<GRAM_BF16>, g, b, 0, s, F, kp, tiles, (float*)Kp); break;
        case GRAM_BF16X3: hipLaunchKernelGGL(k_gram_mfma<GRAM_BF16X3>, g, b, 0, s, F, kp, tiles, (float*)Kp); break;
        case GRAM_BF16X6: hipLaunchKernelGGL(k_gram_mfma<GRAM_BF16X6>, g, b, 0, s, F, kp, tiles, (float*)Kp); break;
        case GRAM_F64: hipLaunchKernelGGL(k_gram_f64, g, b, 0, s, F, kp, tiles, (double*)Kp); break;
        default: return hipErrorInvalidValue;
    }
    (void)prec;
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

hipError_t launch_rowsum(const void* Kp, int prec, const uint32_t* tiles, int64_t ntiles, int NB,
                         double* partR, hipStream_t s) {
    const dim3 g((unsigned)ntiles), b(WG);
    if (prec == PREC_FP64)
        hipLaunchKernelGGL(k_rowsum<double>, g, b, 0, s, (const double*)Kp, tiles, NB, partR);
    else
        hipLaunchKernelGGL(k_rowsum<float>, g, b, 0, s, (const float*)Kp, tiles, NB, partR);
    return hipGetLastError();
}

hipError_t launch_diag(int64_t N, int NB, const double* partR, const double* kdiag, int mode,
                       double C, double delta, double* Adiag, double* scratch_blk,
                       double* scratch_one, hipStream_t s) {
    const unsigned nb = grid1(N);
    hipLaunchKernelGGL(k_diag, dim3(nb), dim3(WG), 0, s, N, NB, partR, kdiag, mode, C, delta, Adiag,
                       scratch_blk);
    if (mode == 3) {
        hipLaunchKernelGGL(k_max_reduce, dim3(1), dim3(WG), 0, s, (int)nb, scratch_blk, scratch_one);
        hipLaunchKernelGGL(k_diag_shift, dim3(nb), dim3(WG), 0, s, N, kdiag, scratch_one, Adiag);
    }
    return hipGetLastError();
}

hipError_t launch_init(int prec, int64_t N, int64_t NPAD, const double* Adiag, const float* y,
                       void* Pt, void* S, double* alpha, DevStatus* st, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_status, dim3(1), dim3(64), 0, s, st);
    if (prec == PREC_FP32)
        hipLaunchKernelGGL(k_init<float>, dim3(grid1(NPAD)), dim3(WG), 0, s, N, NPAD, Adiag, y,
                           (float*)Pt, (float*)S, alpha, st);
    else
        hipLaunchKernelGGL(k_init<double>, dim3(grid1(NPAD)), dim3(WG), 0, s, N, NPAD, Adiag, y,
                           (double*)Pt, (double*)S, alpha, st);
    return hipGetLastError();
}

template <class ST, class MT, class AT>
static void sweep_stored_t(bool first, const SweepBufs& b, hipStream_t s) {
    const dim3 g((unsigned)b.ntiles), blk(WG);
    if (first)
        hipLaunchKernelGGL((k_sweep_stored<ST, MT, AT, true>), g, blk, 0, s, b.tiles, b.NB,
                           (const ST*)b.Kp, (ST*)b.Pf, (ST*)b.Pb, (ST*)b.Ef, (ST*)b.Eb,
                           (const AT*)b.Pt, (const AT*)b.S, (AT*)b.partP, (AT*)b.partE, b.st);
    else
        hipLaunchKernelGGL((k_sweep_stored<ST, MT, AT, false>), g, blk, 0, s, b.tiles, b.NB,
                           (const ST*)b.Kp, (ST*)b.Pf, (ST*)b.Pb, (ST*)b.Ef, (ST*)b.Eb,
                           (const AT*)b.Pt, (const AT*)b.S, (AT*)b.partP, (AT*)b.partE, b.st);
}

hipError_t launch_sweep_stored(int prec, bool first, const SweepBufs& b, hipStream_t s) {
    switch (prec) {
        case PREC_FP32: sweep_stored_t<float, float, float>(first, b, s); break;
        case PREC_MIXED: sweep_stored_t<float, double, double>(first, b, s); break;
        case PREC_FP64: sweep_stored_t<double, double, double>(first, b, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_finalize(int prec, int64_t N, int NB, const void* partP, const void* partE,
                           const double* Adiag, const float* y, void* Pt, void* S, double* alpha,
                           double* blk_delta, double* blk_amax, DevStatus* st, hipStream_t s) {
    const dim3 g(grid1(N)), b(WG);
    if (prec == PREC_FP32)
        hipLaunchKernelGGL(k_finalize<float>, g, b, 0, s, N, NB, (const float*)partP,
                           (const float*)partE, Adiag, y, (float*)Pt, (float*)S, alpha, blk_delta,
                           blk_amax, st);
    else
        hipLaunchKernelGGL(k_finalize<double>, g, b, 0, s, N, NB, (const double*)partP,
                           (const double*)partE, Adiag, y, (double*)Pt, (double*)S, alpha,
                           blk_delta, blk_amax, st);
    return hipGetLastError();
}

hipError_t launch_status(int nblk, const double* blk_delta, const double* blk_amax, DevStatus* st,
                         double* trace, StopRule rule, hipStream_t s) {
    hipLaunchKernelGGL(k_status, dim3(1), dim3(WG), 0, s, nblk, blk_delta, blk_amax, st, trace, rule);
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

hipError_t launch_predict(const float* Xtr, const float* y, const double* alpha, int64_t N, int64_t m,
                          const float* Xq, int64_t nq, double gamma, double lam2, bool fp64,
                          double* f, hipStream_t s) {
    hipLaunchKernelGGL(k_predict, dim3((unsigned)nq), dim3(WG), 0, s, Xtr, y, alpha, N, m, Xq, gamma,
                       lam2, fp64 ? 1 : 0, f);
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
