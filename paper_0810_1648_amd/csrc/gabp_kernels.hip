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
#include "gabp_internal.h"

#include <math.h>

#include <algorithm>
#include <type_traits>

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

// Streaming accesses of the K' and pair-record planes: every element is used
// once per sweep, so loads and stores carry the non-temporal hint and leave
// the caches to the aggregates and partial sums.
__device__ inline V4<float> ld4nt(const float* p) {
    const f32x4v x = __builtin_nontemporal_load(reinterpret_cast<const f32x4v*>(p));
    return {{x[0], x[1], x[2], x[3]}};
}
__device__ inline void st4nt(float* p, const V4<float>& v) {
    const f32x4v x = {v.v[0], v.v[1], v.v[2], v.v[3]};
    __builtin_nontemporal_store(x, reinterpret_cast<f32x4v*>(p));
}
typedef double f64x2v __attribute__((ext_vector_type(2)));
__device__ inline V4<double> ld4nt(const double* p) {
    const f64x2v a = __builtin_nontemporal_load(reinterpret_cast<const f64x2v*>(p));
    const f64x2v b = __builtin_nontemporal_load(reinterpret_cast<const f64x2v*>(p + 2));
    return {{a[0], a[1], b[0], b[1]}};
}
__device__ inline void st4nt(double* p, const V4<double>& v) {
    const f64x2v a = {v.v[0], v.v[1]}, b = {v.v[2], v.v[3]};
    __builtin_nontemporal_store(a, reinterpret_cast<f64x2v*>(p));
    __builtin_nontemporal_store(b, reinterpret_cast<f64x2v*>(p + 2));
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

// Reciprocals: v_rcp_f32 (1 ulp) for FP32; for FP64, v_rcp_f64 refined by
// two Newton steps (the cavity precisions are far from the denormal range).
__device__ inline float rcp_fast(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double rcp_fast(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

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

// One 32 x 32 block of the Gram matrix x_a . x_b on MFMA, for A rows
// rowA = base_a + lane % 32 and B rows colB = base_b + lane % 32.  The
// inner-product index is split between the two lane halves so that each lane
// reads contiguous features.  Output layout of the 32x32 MFMAs: register r of
// lane l holds row 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32.
template <int KIND>
__device__ inline f32x16 mfma_gram_32x32(const Features& F, int64_t rowA, int64_t colB) {
    const int l = threadIdx.x & 63, h = l >> 5;
    const int mp = F.m_pad;
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
        const int64_t oa = rowA * mp + 8 * h, ob = colB * mp + 8 * h;
        for (int s = 0; s < mp; s += 16) {
            const bf16x8 a = *reinterpret_cast<const bf16x8*>(F.hi + oa + s);
            const bf16x8 b = *reinterpret_cast<const bf16x8*>(F.hi + ob + s);
            if constexpr (KIND == GRAM_BF16X3 || KIND == GRAM_BF16X6) {
                // correction terms first, then the leading product
                const bf16x8 al = *reinterpret_cast<const bf16x8*>(F.lo + oa + s);
                const bf16x8 bl = *reinterpret_cast<const bf16x8*>(F.lo + ob + s);
                if constexpr (KIND == GRAM_BF16X6) {
                    const bf16x8 a2 = *reinterpret_cast<const bf16x8*>(F.lo2 + oa + s);
                    const bf16x8 b2 = *reinterpret_cast<const bf16x8*>(F.lo2 + ob + s);
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
    return acc;
}

// K' = exp(-gamma d^2) + lambda^2 with d^2 = max(0, n_i + n_j - 2 G_ij), zero
// for pairs that are not strictly upper (i >= j) or are padding (j >= N).
__device__ inline float kernel_entry(float ni, float nj, float g, int64_t i, int64_t j,
                                     const KernelParams& kp) {
    const float d2 = fmaxf(ni + nj - 2.0f * g, 0.0f);
    const float kv = exp2f(kp.neg_gamma_log2e * d2) + (float)kp.lam2;
    return (i < j && j < kp.N) ? kv : 0.0f;
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

// K' for the 32 x 64 band [row0, row0 + 32) x [col0, col0 + 64) of tile
// (I, J), computed by one wave into its LDS buffer kb[32][64] (row-major).
template <int KIND>
__device__ inline void gram_band(const Features& F, const KernelParams& kp, int I, int J, int row0,
                                 int col0, float* kb) {
    const int l = threadIdx.x & 63, h = l >> 5, l32 = l & 31;
    const int64_t rowA = (int64_t)I * TILE + row0 + l32;
    float ni[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) ni[r] = F.nrm[(int64_t)I * TILE + row0 + 8 * (r >> 2) + 4 * h + (r & 3)];
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
        const int64_t colB = (int64_t)J * TILE + col0 + 32 * cb + l32;
        const f32x16 acc = mfma_gram_32x32<KIND>(F, rowA, colB);
        const float nj = F.nrm[colB];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = 8 * (r >> 2) + 4 * h + (r & 3);
            kb[row * 64 + 32 * cb + l32] =
                kernel_entry(ni[r], nj, acc[r], (int64_t)I * TILE + row0 + row, colB, kp);
        }
    }
}

__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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

// Weighted diagonal (subsection "GaBP Algorithm Convergence") and the row
// maxima of |K'|.  For the uniform rule this kernel leaves the per-block max
// of A_ii - K'_ii for k_diag_shift.
__global__ void k_diag(int64_t N, int NB, const double* __restrict__ psum,
                       const double* __restrict__ pmax, const double* __restrict__ kdiag, int mode,
                       double C, double delta, double* __restrict__ Adiag,
                       double* __restrict__ rowmax, double* __restrict__ blk) {
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
        st->t = 0; st->done = 0; st->reason = R_NONE; st->since_best = 0; st->bad = 0; st->pad = 0;
        st->delta = 0.0; st->amax = 0.0; st->best_delta = INFINITY;
    }
}

// Sweep 0: aggregates of all-zero messages, P~ = A_ii, S = b = y, in ring
// slot 0.  Padded nodes get P~ = 1, S = 0 so that their (zero) messages stay
// finite.
template <class AT>
__global__ void k_init(int64_t N, int64_t NPAD, int R, const double* __restrict__ Adiag,
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
        // padding rows are never finalized: set them in every ring slot
        for (int r = 0; r < R; ++r) {
            Pt[(int64_t)r * NPAD + i] = (AT)1;
            S[(int64_t)r * NPAD + i] = (AT)0;
        }
    }
}

// ------------------------------------------------------------------ sweep --

// One synchronous sweep over all tiles.  Template parameters:
//   ST storage type of K' and the message planes, MT type of the top-level
//   update (cavity denominators, reciprocals), AT aggregate type;
//   KSRC: K' from the materialised plane or recomputed per 32-row band;
//   GK: Gram kind of the recompute;
//   D: 0 = stored edge state (pair-record planes read and written);
//      D >= 1 = stateless: the messages of the previous sweep are rebuilt
//      from the aggregates of up to D earlier sweeps (runtime depth L <= D),
//      deeper levels in LT = float (FP32/MIXED) or double (FP64);
//   FIRST: the stored planes are all zero (sweep 1) and are not read.
// Work of one tile.  SER (stateless only): the reciprocals of the cavity
// precisions Q = P~ (1 - e), e = P_reverse / P~, are formed from the
// per-node 1/P~ by the series 1/Q = (1 + e + e^2 + ...) / P~ (one term at
// the lower levels, two at the top), valid because |e| <= rho^2 where rho is
// the contraction estimate; the host enables it only when the neglected terms
// are below the arithmetic's precision.  The deepest level starts from zero
// messages and costs four multiplications.
template <class ST, class MT, class AT, int KSRC, int GK, int D, bool FIRST, bool SER>
__device__ inline void sweep_tile(const SweepArgs& a, int64_t tile) {
    DevStatus* st = a.st;
    using LT = typename std::conditional<std::is_same<ST, double>::value, double, float>::type;
    constexpr bool STORED = (D == 0);
    constexpr int DL = (D > 1) ? D - 1 : 1;   // lower levels held per node
    constexpr int NL = STORED ? 1 : DL;
    constexpr int NT = STORED ? 1 : TILE;
    const uint32_t ij = a.tiles[tile];
    const TileCoord tc{(int)(ij >> 16), (int)(ij & 0xFFFFu)};
    const int NB = a.NB;
    const size_t tbase = (size_t)tile * TT;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, g = l >> 4, q = l & 15;
    const int col0 = w * 64 + q * 4;
    const int L = a.levels;
    const AT* HP = static_cast<const AT*>(a.HP);
    const AT* HS = static_cast<const AT*>(a.HS);
    const ST* Kp = static_cast<const ST*>(a.Kp);
    ST* Pf = static_cast<ST*>(a.Pf);
    ST* Pb = static_cast<ST*>(a.Pb);
    ST* Ef = static_cast<ST*>(a.Ef);
    ST* Eb = static_cast<ST*>(a.Eb);

    // row-node data: top level (P~ or, with SER, 1/P~) and lower levels
    __shared__ MT sPt[TILE], sS[TILE];
    __shared__ LT sPtL[NL][NT], sSL[NL][NT], sSIL[SER ? NL : 1][SER ? NT : 1];
    __shared__ AT rP[4][TILE], rE[4][TILE];
    __shared__ float kband[KSRC == KSRC_RECOMPUTE ? 4 : 1][KSRC == KSRC_RECOMPUTE ? 32 * 64 : 1];

    const int64_t top = (int64_t)a.slot_top * a.NPAD;
    {
        const MT p = (MT)HP[top + (int64_t)tc.I * TILE + tid];
        sPt[tid] = SER ? (MT)1 / p : p;
        sS[tid] = (MT)HS[top + (int64_t)tc.I * TILE + tid];
    }
    MT ptj[4], sj[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const MT p = (MT)HP[top + (int64_t)tc.J * TILE + col0 + c];
        ptj[c] = SER ? (MT)1 / p : p;
        sj[c] = (MT)HS[top + (int64_t)tc.J * TILE + col0 + c];
    }
    LT ptjL[DL][4], sjL[DL][4], sijL[SER ? DL : 1][4];
    if constexpr (!STORED) {
#pragma unroll
        for (int k = 1; k < D; ++k) {
            if (k < L) {
                const int64_t base = (int64_t)((a.slot_top - k + a.R) % a.R) * a.NPAD;
                const LT pr = (LT)HP[base + (int64_t)tc.I * TILE + tid];
                const LT sr = (LT)HS[base + (int64_t)tc.I * TILE + tid];
                sPtL[k - 1][tid] = SER ? (LT)1 / pr : pr;
                sSL[k - 1][tid] = sr;
                if constexpr (SER) sSIL[k - 1][tid] = sr / pr;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const LT pc = (LT)HP[base + (int64_t)tc.J * TILE + col0 + c];
                    const LT sc = (LT)HS[base + (int64_t)tc.J * TILE + col0 + c];
                    ptjL[k - 1][c] = SER ? (LT)1 / pc : pc;
                    sjL[k - 1][c] = sc;
                    if constexpr (SER) sijL[k - 1][c] = sc / pc;
                }
            }
        }
    }
    AT cP[4] = {0, 0, 0, 0}, cE[4] = {0, 0, 0, 0};
    bool bad = false;
    __syncthreads();

    size_t off = tbase + (size_t)g * TILE + col0;
    V4<ST> k{}, pf{}, pb{}, ef{}, eb{};
    if constexpr (KSRC == KSRC_PLANE) k = ld4nt(Kp + off);
    if constexpr (STORED && !FIRST) { pf = ld4nt(Pf + off); pb = ld4nt(Pb + off); ef = ld4nt(Ef + off); eb = ld4nt(Eb + off); }

    for (int b = 0; b < TILE / 32; ++b) {
        if constexpr (KSRC == KSRC_RECOMPUTE) {
            gram_band<GK>(a.F, a.kp, tc.I, tc.J, 32 * b, 64 * w, kband[w]);
            wave_lds_sync();
        }
        for (int s2 = 0; s2 < 8; ++s2) {
            const int r = 32 * b + 4 * s2 + g;
            const bool more = (b * 8 + s2 + 1) < TILE / 4;
            // prefetch the lane's next row
            V4<ST> k2{}, pf2{}, pb2{}, ef2{}, eb2{};
            const size_t off2 = off + 4 * TILE;
            if (more) {
                if constexpr (KSRC == KSRC_PLANE) k2 = ld4nt(Kp + off2);
                if constexpr (STORED && !FIRST) { pf2 = ld4nt(Pf + off2); pb2 = ld4nt(Pb + off2); ef2 = ld4nt(Ef + off2); eb2 = ld4nt(Eb + off2); }
            }
            if constexpr (KSRC == KSRC_RECOMPUTE) {
                const float4 kk = *reinterpret_cast<const float4*>(&kband[w][(4 * s2 + g) * 64 + 4 * q]);
                k = V4<ST>{{(ST)kk.x, (ST)kk.y, (ST)kk.z, (ST)kk.w}};
            }
            const MT pti = sPt[r], si = sS[r];
            AT rp = 0, re = 0;
            V4<ST> npf, npb, nef, neb;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const MT av = (MT)k.v[c];
                // messages of the previous sweep: stored, or rebuilt level by level
                MT opf, opb, oef, oeb;
                if constexpr (STORED) {
                    opf = (MT)pf.v[c]; opb = (MT)pb.v[c]; oef = (MT)ef.v[c]; oeb = (MT)eb.v[c];
                } else if constexpr (SER) {
                    const LT al = (LT)k.v[c], a2l = al * al;
                    LT lpf = 0, lpb = 0, lef = 0, leb = 0;
                    const int kd = L - 1;
#pragma unroll
                    for (int kk = D - 1; kk >= 1; --kk) {
                        if (kk == kd) {               // deepest level: reverse messages zero
                            lpf = -a2l * sPtL[kk - 1][r];
                            lpb = -a2l * ptjL[kk - 1][c];
                            lef = -al * sSIL[kk - 1][r];
                            leb = -al * sijL[kk - 1][c];
                        } else if (kk < kd) {
                            const LT ir = sPtL[kk - 1][r], ic = ptjL[kk - 1][c];
                            const LT e_f = lpb * ir, e_b = lpf * ic;
                            bad |= !(e_f > (LT)-0.5) | !(e_b > (LT)-0.5);
                            const LT tf = al * fma(ir, e_f, ir), tb = al * fma(ic, e_b, ic);
                            const LT npf_ = -al * tf, npb_ = -al * tb;
                            const LT nef_ = tf * (leb - sSL[kk - 1][r]);
                            const LT neb_ = tb * (lef - sjL[kk - 1][c]);
                            lpf = npf_; lpb = npb_; lef = nef_; leb = neb_;
                        }
                    }
                    opf = (MT)lpf; opb = (MT)lpb; oef = (MT)lef; oeb = (MT)leb;
                } else {
                    const LT al = (LT)k.v[c], a2l = al * al;
                    LT lpf = 0, lpb = 0, lef = 0, leb = 0;
#pragma unroll
                    for (int kk = D - 1; kk >= 1; --kk) {
                        if (kk < L) {
                            const LT qf = sPtL[kk - 1][r] - lpb, qb = ptjL[kk - 1][c] - lpf;
                            bad |= !(qf > (LT)0) | !(qb > (LT)0);
                            const LT rf = rcp_fast(qf), rb = rcp_fast(qb);
                            const LT npf_ = -a2l * rf, npb_ = -a2l * rb;
                            const LT nef_ = -al * (sSL[kk - 1][r] - leb) * rf;
                            const LT neb_ = -al * (sjL[kk - 1][c] - lef) * rb;
                            lpf = npf_; lpb = npb_; lef = nef_; leb = neb_;
                        }
                    }
                    opf = (MT)lpf; opb = (MT)lpb; oef = (MT)lef; oeb = (MT)leb;
                }
                MT pij_m, eij_m, pji_m, eji_m;
                if constexpr (SER) {
                    const MT e_f = opb * pti, e_b = opf * ptj[c];      // P_ji / P~_i, P_ij / P~_j
                    bad |= !(e_f > (MT)-0.5) | !(e_b > (MT)-0.5);
                    const MT tf = av * fma(pti, fma(e_f, e_f, e_f), pti);
                    const MT tb = av * fma(ptj[c], fma(e_b, e_b, e_b), ptj[c]);
                    pij_m = -av * tf;
                    pji_m = -av * tb;
                    eij_m = tf * (oeb - si);
                    eji_m = tb * (oef - sj[c]);
                } else {
                    const MT a2 = av * av;
                    const MT qf = pti - opb;        // P~_i - P_ji
                    const MT qb = ptj[c] - opf;     // P~_j - P_ij
                    bad |= !(qf > (MT)0) | !(qb > (MT)0);
                    const MT rf = rcp_fast(qf), rb = rcp_fast(qb);
                    pij_m = -a2 * rf;
                    eij_m = -av * (si - oeb) * rf;
                    pji_m = -a2 * rb;
                    eji_m = -av * (sj[c] - oef) * rb;
                }
                if constexpr (STORED) {
                    // the aggregates add the values as stored
                    const ST pij = (ST)pij_m, eij = (ST)eij_m, pji = (ST)pji_m, eji = (ST)eji_m;
                    npf.v[c] = pij; nef.v[c] = eij; npb.v[c] = pji; neb.v[c] = eji;
                    cP[c] += (AT)pij; cE[c] += (AT)eij;     // received by column node j
                    rp += (AT)pji; re += (AT)eji;            // received by row node i
                } else {
                    cP[c] += (AT)pij_m; cE[c] += (AT)eij_m;
                    rp += (AT)pji_m; re += (AT)eji_m;
                }
            }
            if constexpr (STORED) { st4nt(Pf + off, npf); st4nt(Pb + off, npb); st4nt(Ef + off, nef); st4nt(Eb + off, neb); }
            rp = sum16(rp);
            re = sum16(re);
            if (q == 0) { rP[w][r] = rp; rE[w][r] = re; }
            if constexpr (KSRC == KSRC_PLANE) k = k2;
            if constexpr (STORED && !FIRST) { pf = pf2; pb = pb2; ef = ef2; eb = eb2; }
            off = off2;
        }
        if constexpr (KSRC == KSRC_RECOMPUTE) wave_lds_sync();
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) { cP[c] = sum_groups(cP[c]); cE[c] = sum_groups(cE[c]); }
    __syncthreads();
    AT* partP = static_cast<AT*>(a.partP);
    AT* partE = static_cast<AT*>(a.partE);
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

template <class ST, class MT, class AT, int KSRC, int GK, int D, bool FIRST, bool SER>
__global__ __launch_bounds__(WG) void k_sweep(SweepArgs a) {
    if (a.st->done) return;
    sweep_tile<ST, MT, AT, KSRC, GK, D, FIRST, SER>(a, blockIdx.x);
}

// Served form: one persistent grid walks the union work list of (request,
// tile) items of every active request; each request keeps its own planes,
// partial sums and status, so its arithmetic does not depend on the mix.
template <class ST, class MT, class AT>
__global__ __launch_bounds__(WG) void k_sweep_batched(const ReqDesc* __restrict__ reqs,
                                                     const uint2* __restrict__ items, int nitems) {
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const uint2 w = items[it];
        const ReqDesc& rd = reqs[w.x];
        if (rd.sw.st->done) continue;
        sweep_tile<ST, MT, AT, KSRC_PLANE, GRAM_F32, 0, false, false>(rd.sw, (int64_t)w.y);
        __syncthreads();
    }
}

// Aggregates of the new sweep from the partial sums (fixed order) into ring
// slot `wslot`, the new alpha and the per-block change / magnitude maxima.
template <class AT>
__device__ inline void finalize_block(int64_t blk, int64_t N, int NB, const AT* __restrict__ partP,
                                      const AT* __restrict__ partE,
                                      const double* __restrict__ Adiag,
                                      const float* __restrict__ y, AT* __restrict__ Pt,
                                      AT* __restrict__ S, double* __restrict__ alpha,
                                      double* __restrict__ blk_delta,
                                      double* __restrict__ blk_amax, DevStatus* st) {
    __shared__ double sh4[4];
    const int64_t i = blk * blockDim.x + threadIdx.x;
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
    if (threadIdx.x == 0) { blk_delta[blk] = d; blk_amax[blk] = am; }
}

template <class AT>
__global__ __launch_bounds__(WG) void k_finalize(int64_t N, int NB, const AT* __restrict__ partP,
                                                const AT* __restrict__ partE,
                                                const double* __restrict__ Adiag,
                                                const float* __restrict__ y, AT* __restrict__ Pt,
                                                AT* __restrict__ S, double* __restrict__ alpha,
                                                double* __restrict__ blk_delta,
                                                double* __restrict__ blk_amax, DevStatus* st) {
    if (st->done) return;
    finalize_block<AT>(blockIdx.x, N, NB, partP, partE, Adiag, y, Pt, S, alpha, blk_delta, blk_amax, st);
}

// Served form: items are (request, block of 256 nodes).
template <class AT>
__global__ __launch_bounds__(WG) void k_finalize_batched(const ReqDesc* __restrict__ reqs,
                                                        const uint2* __restrict__ items, int nitems) {
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const uint2 w = items[it];
        const ReqDesc& rd = reqs[w.x];
        if (rd.sw.st->done) continue;
        finalize_block<AT>((int64_t)w.y, rd.N, rd.sw.NB, static_cast<const AT*>(rd.sw.partP),
                           static_cast<const AT*>(rd.sw.partE), rd.Adiag, rd.y,
                           static_cast<AT*>(const_cast<void*>(rd.sw.HP)),
                           static_cast<AT*>(const_cast<void*>(rd.sw.HS)), rd.alpha, rd.blk_delta,
                           rd.blk_amax, rd.sw.st);
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
__global__ __launch_bounds__(WG) void k_status_batched(const ReqDesc* __restrict__ reqs,
                                                      const int* __restrict__ slots, int n,
                                                      DevStatus* __restrict__ out) {
    const int k = blockIdx.x;
    if (k >= n) return;
    const ReqDesc& rd = reqs[slots[k]];
    DevStatus* st = rd.sw.st;
    if (!st->done) status_update(rd.nblk, rd.blk_delta, rd.blk_amax, st, rd.trace, rd.rule);
    __syncthreads();
    if (threadIdx.x == 0) out[k] = *st;
}

// Contraction estimate of the message recursion, max_i rowmax_i / P~_i,
// per block (the reverse message enters the next one with a factor A_ij / Q).
template <class AT>
__global__ void k_rho(int64_t N, const double* __restrict__ rowmax, const AT* __restrict__ Pt,
                      double* __restrict__ blk) {
    __shared__ double sh4[4];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double v = 0.0;
    if (i < N) v = rowmax[i] / (double)Pt[i];
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

hipError_t launch_diag(int64_t N, int NB, const double* psum, const double* pmax, const double* kdiag,
                       int mode, double C, double delta, double* Adiag, double* rowmax,
                       double* scratch_blk, double* scratch_one, hipStream_t s) {
    const unsigned nb = grid1(N);
    hipLaunchKernelGGL(k_diag, dim3(nb), dim3(WG), 0, s, N, NB, psum, pmax, kdiag, mode, C, delta, Adiag,
                       rowmax, scratch_blk);
    if (mode == 3) {
        hipLaunchKernelGGL(k_max_reduce, dim3(1), dim3(WG), 0, s, (int)nb, scratch_blk, scratch_one);
        hipLaunchKernelGGL(k_diag_shift, dim3(nb), dim3(WG), 0, s, N, kdiag, scratch_one, Adiag);
    }
    return hipGetLastError();
}

hipError_t launch_init(int prec, int64_t N, int64_t NPAD, int R, const double* Adiag, const float* y,
                       void* Pt, void* S, double* alpha, DevStatus* st, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_status, dim3(1), dim3(64), 0, s, st);
    if (prec == PREC_FP32)
        hipLaunchKernelGGL(k_init<float>, dim3(grid1(NPAD)), dim3(WG), 0, s, N, NPAD, R, Adiag, y,
                           (float*)Pt, (float*)S, alpha, st);
    else
        hipLaunchKernelGGL(k_init<double>, dim3(grid1(NPAD)), dim3(WG), 0, s, N, NPAD, R, Adiag, y,
                           (double*)Pt, (double*)S, alpha, st);
    return hipGetLastError();
}

// ---- sweep dispatch: precision x K' source x Gram kind x depth x first x series
template <class ST, class MT, class AT, int KSRC, int GK, int D, bool SER>
static void sweep_d(bool first, const SweepArgs& a, hipStream_t s) {
    const dim3 g((unsigned)a.ntiles), blk(WG);
    if constexpr (D == 0) {
        if (first) {
            hipLaunchKernelGGL((k_sweep<ST, MT, AT, KSRC, GK, D, true, false>), g, blk, 0, s, a);
            return;
        }
    }
    hipLaunchKernelGGL((k_sweep<ST, MT, AT, KSRC, GK, D, false, SER>), g, blk, 0, s, a);
}

template <class ST, class MT, class AT, int KSRC, int GK>
static hipError_t sweep_depth(int depth, bool first, bool ser, const SweepArgs& a, hipStream_t s) {
    if (ser) {
        switch (depth) {
            case 1: case 2: sweep_d<ST, MT, AT, KSRC, GK, 2, true>(first, a, s); break;
            case 3: case 4: sweep_d<ST, MT, AT, KSRC, GK, 4, true>(first, a, s); break;
            case 5: case 6: sweep_d<ST, MT, AT, KSRC, GK, 6, true>(first, a, s); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (depth) {
        case 0: sweep_d<ST, MT, AT, KSRC, GK, 0, false>(first, a, s); break;
        case 1: case 2: sweep_d<ST, MT, AT, KSRC, GK, 2, false>(first, a, s); break;
        case 3: case 4: sweep_d<ST, MT, AT, KSRC, GK, 4, false>(first, a, s); break;
        case 5: case 6: sweep_d<ST, MT, AT, KSRC, GK, 6, false>(first, a, s); break;
        case 7: case 8: sweep_d<ST, MT, AT, KSRC, GK, 8, false>(first, a, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_sweep(int prec, int ksrc, int gram, int depth, bool first, bool ser, const SweepArgs& a,
                        hipStream_t s) {
    if (depth == 0) ser = false;
    if (ksrc == KSRC_PLANE) {
        switch (prec) {
            case PREC_FP32: return sweep_depth<float, float, float, KSRC_PLANE, GRAM_F32>(depth, first, ser, a, s);
            case PREC_MIXED: return sweep_depth<float, double, double, KSRC_PLANE, GRAM_F32>(depth, first, ser, a, s);
            case PREC_FP64: return sweep_depth<double, double, double, KSRC_PLANE, GRAM_F64>(depth, first, ser, a, s);
            default: return hipErrorInvalidValue;
        }
    }
    if (prec == PREC_FP32 && gram == GRAM_F32)
        return sweep_depth<float, float, float, KSRC_RECOMPUTE, GRAM_F32>(depth, first, ser, a, s);
    if (prec == PREC_MIXED) {
        switch (gram) {
            case GRAM_BF16: return sweep_depth<float, double, double, KSRC_RECOMPUTE, GRAM_BF16>(depth, first, ser, a, s);
            case GRAM_BF16X3: return sweep_depth<float, double, double, KSRC_RECOMPUTE, GRAM_BF16X3>(depth, first, ser, a, s);
            case GRAM_BF16X6: return sweep_depth<float, double, double, KSRC_RECOMPUTE, GRAM_BF16X6>(depth, first, ser, a, s);
            default: break;
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_served_step(int prec, const ReqDesc* reqs, const uint2* tile_items, int ntile_items,
                              const uint2* node_items, int nnode_items, const int* slots, int nslots,
                              DevStatus* status_out, hipStream_t s) {
    const int gs = std::max(1, std::min(ntile_items, 2048));
    const int gf = std::max(1, std::min(nnode_items, 2048));
    switch (prec) {
        case PREC_FP32:
            hipLaunchKernelGGL((k_sweep_batched<float, float, float>), dim3(gs), dim3(WG), 0, s, reqs, tile_items, ntile_items);
            hipLaunchKernelGGL(k_finalize_batched<float>, dim3(gf), dim3(WG), 0, s, reqs, node_items, nnode_items);
            break;
        case PREC_MIXED:
            hipLaunchKernelGGL((k_sweep_batched<float, double, double>), dim3(gs), dim3(WG), 0, s, reqs, tile_items, ntile_items);
            hipLaunchKernelGGL(k_finalize_batched<double>, dim3(gf), dim3(WG), 0, s, reqs, node_items, nnode_items);
            break;
        case PREC_FP64:
            hipLaunchKernelGGL((k_sweep_batched<double, double, double>), dim3(gs), dim3(WG), 0, s, reqs, tile_items, ntile_items);
            hipLaunchKernelGGL(k_finalize_batched<double>, dim3(gf), dim3(WG), 0, s, reqs, node_items, nnode_items);
            break;
        default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_status_batched, dim3(std::max(1, nslots)), dim3(WG), 0, s, reqs, slots, nslots, status_out);
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

hipError_t launch_rho(int prec, int64_t N, const double* rowmax, const void* Pt, double* blk,
                      double* one, hipStream_t s) {
    const unsigned nb = grid1(N);
    if (prec == PREC_FP32)
        hipLaunchKernelGGL(k_rho<float>, dim3(nb), dim3(WG), 0, s, N, rowmax, (const float*)Pt, blk);
    else
        hipLaunchKernelGGL(k_rho<double>, dim3(nb), dim3(WG), 0, s, N, rowmax, (const double*)Pt, blk);
    hipLaunchKernelGGL(k_max_reduce, dim3(1), dim3(WG), 0, s, (int)nb, blk, one);
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
