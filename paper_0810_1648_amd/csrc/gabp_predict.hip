// Decision function of the trained machine on new points (section
// "Classification Using Support Vector Machines": the classifier is the sign
// of sum_i alpha_i y_i K(x_i, x) + b; with the bias absorbed by the constant
// feature lambda, b = lambda^2 sum_i alpha_i y_i, so that
//   f(x_q) = sum_i w_i K(x_i, x_q) + lambda^2 sum_i w_i,   w_i = alpha_i y_i.
//
// FP32 and MIXED handles form K(x_i, x_q) from the same staged features and
// Gram kind as the solve's K' (centred with the training column means, which
// leaves RBF distances unchanged): an MFMA 32 x 32 Gram block per wave step,
// then exp2 of the clamped distance, folded into per-query FP64 sums.  FP64
// handles take direct FP64 differences.  Partial sums per training chunk are
// reduced in a fixed order, so f does not depend on the launch shape's
// timing.
#include "gabp_device.h"

#include <mutex>

// Working memory of the allocation-free decision function: weights, partial
// sums and staged queries of one call.  Each device holds its own copy for
// the life of the process; host code reaches it only through the address
// that predict_scratch() looks up (the array's name is not a device address
// in host code).
static __device__ __align__(256) unsigned char scratch[gabp::PREDICT_SCRATCH_BYTES];

namespace gabp {

hipError_t predict_scratch(void** ptr) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

namespace {

constexpr int QB = 128;   // queries per workgroup: four waves of 32
constexpr int AUG_FR = 2;                // augmented form: 32-query A fragments per wave
constexpr int QBA = 4 * 32 * AUG_FR;      // augmented form: queries per workgroup

// w_i = alpha_i y_i (alpha clipped to [0, C] with the box option), zero on
// padded rows; per-block sums of w in a fixed tree order.
__global__ __launch_bounds__(WG) void k_predict_weights(const double* __restrict__ alpha,
                                                        const float* __restrict__ y, int64_t N,
                                                        int64_t NPAD, int box, double C,
                                                        double* __restrict__ w, double* __restrict__ blk) {
    __shared__ double sh[WG];
    const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
    double v = 0.0;
    if (i < N) {
        double a = alpha[i];
        if (box) a = fmin(fmax(a, 0.0), C);
        v = a * (double)y[i];
    }
    if (i < NPAD) w[i] = v;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = WG / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) blk[blockIdx.x] = sh[0];
}

// One workgroup: out[0] = sum of v[0 .. n) in a fixed order.
__global__ __launch_bounds__(WG) void k_sum_fixed(const double* __restrict__ v, int64_t n,
                                                  double* __restrict__ out) {
    __shared__ double sh[WG];
    double acc = 0.0;
    for (int64_t k = threadIdx.x; k < n; k += WG) acc += v[k];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = WG / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

// FP64: one workgroup per query, direct differences of the raw features.
__global__ __launch_bounds__(WG) void k_predict_direct(const float* __restrict__ Xtr,
                                                       const double* __restrict__ w, int64_t N,
                                                       int64_t m, const float* __restrict__ Xq,
                                                       double gamma, double* __restrict__ part) {
    __shared__ double sh[WG];
    const int64_t qi = blockIdx.x;
    const float* xq = Xq + qi * m;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < N; i += WG) {
        const float* xi = Xtr + i * m;
        double d2 = 0.0;
        for (int64_t k = 0; k < m; ++k) {
            const double d = (double)xi[k] - (double)xq[k];
            d2 = fma(d, d, d2);
        }
        acc = fma(w[i], exp(-gamma * d2), acc);
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = WG / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[qi] = sh[0];
}

// Workgroup (x, y): queries [128 x, 128 x + 128), training blocks of 32 rows
// [bpc y, bpc (y + 1)).  Wave v owns queries 32 v .. 32 v + 31; lane l's
// MFMA output register r is query row 8 (r / 4) + 4 (l / 32) + r % 4 and
// training row l % 32 of the block.  part[y][q] receives the chunk's sum.
template <int KIND, int MP>
__global__ __launch_bounds__(WG) void k_predict_mfma(Features Ft, Features Fq, const double* __restrict__ w,
                                                     int64_t nblk32, int bpc, float neg_gamma_log2e,
                                                     int64_t NQPAD, double* __restrict__ part) {
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63, h = l >> 5, l32 = l & 31;
    const int64_t q0 = (int64_t)blockIdx.x * QB + wv * 32;
    const int64_t rowA = q0 + l32;
    float ni[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) ni[r] = Fq.nrm[q0 + 8 * (r >> 2) + 4 * h + (r & 3)];
    RowFrag<KIND, MP> qa;
    qa.load(Fq, rowA);
    double acc[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0;
    const int64_t b0 = (int64_t)blockIdx.y * bpc;
    const int64_t b1 = (b0 + bpc < nblk32) ? b0 + bpc : nblk32;
    for (int64_t b = b0; b < b1; ++b) {
        const int64_t colB = b * 32 + l32;
        const f32x16 g = qa.gram(Fq, rowA, Ft, colB);
        const float nj = Ft.nrm[colB];
        const double wj = w[colB];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const float d2 = fmaxf(ni[r] + nj - 2.0f * g[r], 0.0f);
            acc[r] = fma((double)exp2f(neg_gamma_log2e * d2), wj, acc[r]);
        }
    }
    // sum over the 32 training rows held by lanes l % 32 of each half
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        double v = sum16(acc[r]);
        v = v + __shfl_xor(v, 16);
        acc[r] = v;
    }
    if (l32 == 0) {
        double* out = part + (int64_t)blockIdx.y * NQPAD + q0;
#pragma unroll
        for (int r = 0; r < 16; ++r) out[8 * (r >> 2) + 4 * h + (r & 3)] = acc[r];
    }
}

// BF16 Gram kinds with m_pad <= MP: the workgroup's four waves share every
// 32-row training block, so the block's B fragments (all split planes) are
// staged once in LDS, in fragment order (chunk (plane, step, lane) holds the
// 16 bytes lane `lane` feeds the MFMA at k-step `step`), together with the
// block's norms and weights.  The next block's chunks are loaded into
// registers while the current block is multiplied, then stored into the
// other buffer (one barrier per block).  A workgroup covers at most 32
// training blocks (the chunk): each lane sums its training points' terms in
// FP32 (at most 32 per query, an error below 32 ulp of the sum of their
// magnitudes), then the 32 training lanes are added in FP64.
template <int KIND, int MP>
__global__ __launch_bounds__(WG) void k_predict_lds(Features Ft, Features Fq, const double* __restrict__ w,
                                                    int64_t nblk32, int bpc, float neg_gamma_log2e,
                                                    int64_t NQPAD, double* __restrict__ part) {
    using BS = BStage<KIND>;
    constexpr int NP = BS::NP;                                                        // split planes
    constexpr int NS = MP / 16;                                                       // k-steps
    constexpr int CH = NP * NS * 64;                                                  // 16-byte chunks
    constexpr int PR = (CH + WG - 1) / WG;                                            // per thread
    __shared__ bf16x8 sb[2][CH];
    __shared__ float snj[2][32];
    __shared__ double swj[2][32];
    const int tid = threadIdx.x, wv = tid >> 6, l = tid & 63, h = l >> 5, l32 = l & 31;
    const int mp = Fq.m_pad, ns = mp / 16, ch = NP * ns * 64;
    const int64_t q0 = (int64_t)blockIdx.x * QB + wv * 32;
    const int64_t rowA = q0 + l32;
    float ni[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) ni[r] = Fq.nrm[q0 + 8 * (r >> 2) + 4 * h + (r & 3)];
    RowFrag<KIND, MP> qa;
    qa.load(Fq, rowA);
    float accf[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) accf[r] = 0.0f;
    const int64_t b0 = (int64_t)blockIdx.y * bpc;
    const int64_t b1 = (b0 + bpc < nblk32) ? b0 + bpc : nblk32;
    if (b0 < b1) {
#pragma unroll
        for (int i = 0; i < PR; ++i) {
            const int k = tid + WG * i;
            if (k < ch) sb[0][BS::dst(ns, k)] = *BS::src(Ft, b0 * 32, ns, k);
        }
        if (tid < 32) { snj[0][tid] = Ft.nrm[b0 * 32 + tid]; swj[0][tid] = w[b0 * 32 + tid]; }
    }
    __syncthreads();
    for (int64_t b = b0; b < b1; ++b) {
        const int cur = (int)((b - b0) & 1);
        const bool more = b + 1 < b1;
        bf16x8 pre[PR];
        float pn = 0.0f;
        double pw = 0.0;
        if (more) {
#pragma unroll
            for (int i = 0; i < PR; ++i) {
                const int k = tid + WG * i;
                if (k < ch) pre[i] = *BS::src(Ft, (b + 1) * 32, ns, k);
            }
            if (tid < 32) { pn = Ft.nrm[(b + 1) * 32 + tid]; pw = w[(b + 1) * 32 + tid]; }
        }
        f32x16 g = {};
        BS::template mma<MP>(qa, sb[cur], ns, l, g);
        const float nj = snj[cur][l32];
        const float wj = (float)swj[cur][l32];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const float d2 = fmaxf(ni[r] + nj - 2.0f * g[r], 0.0f);
            accf[r] = fmaf(__builtin_amdgcn_exp2f(neg_gamma_log2e * d2), wj, accf[r]);
        }
        if (more) {
#pragma unroll
            for (int i = 0; i < PR; ++i) {
                const int k = tid + WG * i;
                if (k < ch) sb[cur ^ 1][BS::dst(ns, k)] = pre[i];
            }
            if (tid < 32) { snj[cur ^ 1][tid] = pn; swj[cur ^ 1][tid] = pw; }
        }
        __syncthreads();
    }
    // sum over the 32 training rows held by lanes l % 32 of each half
    double acc[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        double v = sum16((double)accf[r]);
        v = v + __shfl_xor(v, 16);
        acc[r] = v;
    }
    if (l32 == 0) {
        double* out = part + (int64_t)blockIdx.y * NQPAD + q0;
#pragma unroll
        for (int r = 0; r < 16; ++r) out[8 * (r >> 2) + 4 * h + (r & 3)] = acc[r];
    }
}

// ---- augmented rows: the MFMA emits the scaled exponent itself ----------
//
// Rows are extended by two columns so that the Gram of a query row a and a
// training row b is the exponent of the kernel in base 2:
//   a = (x_q, n_q, 1),   b = c (x_t, -1/2, -n_t/2),   c = 2 gamma log2(e),
//   a . b = c (x_q . x_t - n_q/2 - n_t/2) = -gamma log2(e) ||x_q - x_t||^2,
// so K(x_t, x_q) = exp2(min(a . b, 0)) (the clamp keeps rounding from
// pushing K above 1).  Features are centred with the training column means
// (distances unchanged), and each entry is split into one, two or three
// BF16 terms (the Gram kind's planes); n is the squared norm of the split
// representation.  Columns past m + 1 and rows past n are zero.
__global__ void k_stage_aug(const float* __restrict__ X, const double* __restrict__ mean, int64_t n, int64_t m,
                            int64_t NPAD, int mp, int np, int side, float c, uint16_t* __restrict__ out,
                            int64_t plane) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NPAD) return;
    uint16_t* o0 = out + i * mp;
    uint16_t* o1 = o0 + plane;
    uint16_t* o2 = o1 + plane;
    auto put = [&](int k, float v) {
        uint16_t h, l, l2;
        split3(v, h, l, l2);
        o0[k] = h;
        if (np >= 2) o1[k] = l;
        if (np >= 3) o2[k] = l2;
    };
    float nrm = 0.0f;
    for (int k = 0; k < mp; ++k) {
        const bool in = (i < n) && (k < m);
        const float xc = in ? (float)((double)X[i * m + k] - mean[k]) : 0.0f;
        if (k < m) {
            uint16_t h, l, l2;
            split3(xc, h, l, l2);
            const float v = bf2f(h) + (np >= 2 ? bf2f(l) : 0.0f) + (np >= 3 ? bf2f(l2) : 0.0f);
            nrm = fmaf(v, v, nrm);
        }
        if (k < m || k >= m + 2) put(k, side == 0 ? xc : c * xc);
    }
    if (i >= n) nrm = 0.0f;
    const bool live = i < n;
    if (side == 0) {
        put((int)m, nrm);
        put((int)m + 1, live ? 1.0f : 0.0f);
    } else {
        put((int)m, live ? -0.5f * c : 0.0f);
        put((int)m + 1, -0.5f * c * nrm);
    }
}

// Workgroup (x, y): queries [256 x, 256 x + 256), training blocks of 32 rows
// [bpc y, bpc (y + 1)), with augmented rows (above).  Wave v owns queries
// 256 x + 64 v .. + 63 as two 32-row A fragments held in registers, so each
// B fragment read from LDS feeds two MFMA chains.  A block's B fragments
// (all split planes) are staged in LDS in fragment order: chunk
// (plane, step, lane) holds the 16 bytes lane `lane` feeds the MFMA at
// k-step `step` (training row lane % 32, columns 16 step + 8 (lane / 32)),
// and thread t loads chunks t, t + 256, ... so the LDS stores are
// contiguous; the next block's chunks are loaded into registers while the
// current block is multiplied, then stored into the other LDS buffer (one
// barrier per block).  MFMA output
// register r of lane l is query row 8 (r / 4) + 4 (l / 32) + r % 4 of its
// fragment and training row l % 32; each lane sums its training points'
// terms in FP32 (at most 32 per query and chunk), then the 32 training lanes
// are added in FP64 in a fixed order.  K = exp2 of the MFMA output, clamped
// to [0, 1] by the instruction's clamp modifier.
template <int KIND, int MP, int FR>
__global__ __launch_bounds__(WG) void k_predict_aug(const uint16_t* __restrict__ Bt, int64_t bplane,
                                                    const uint16_t* __restrict__ Aq, int64_t aplane,
                                                    const double* __restrict__ w, int64_t nblk32, int bpc,
                                                    int64_t NQPAD, double* __restrict__ part) {
    constexpr int NP = (KIND == GRAM_BF16X6) ? 3 : (KIND == GRAM_BF16X3) ? 2 : 1;
    constexpr int NS = MP / 16;
    constexpr int CH = NP * NS * 64;
    constexpr int PR = (CH + WG - 1) / WG;
    constexpr int QW = 32 * FR;                 // queries per wave
    __shared__ bf16x8 sb[2][CH];
    __shared__ float swj[2][32];
    const int tid = threadIdx.x, wv = tid >> 6, l = tid & 63, h = l >> 5, l32 = l & 31;
    const int64_t q0 = (int64_t)blockIdx.x * (4 * QW) + wv * QW;
    bf16x8 a[FR][NP][NS];
#pragma unroll
    for (int f = 0; f < FR; ++f)
#pragma unroll
        for (int pl = 0; pl < NP; ++pl)
#pragma unroll
            for (int st = 0; st < NS; ++st)
                a[f][pl][st] = *reinterpret_cast<const bf16x8*>(Aq + pl * aplane + (q0 + 32 * f + l32) * MP +
                                                                16 * st + 8 * h);
    // this thread's staging chunks: source offsets within a block
    int64_t so[PR];
#pragma unroll
    for (int i = 0; i < PR; ++i) {
        const int c = tid + WG * i, pl = c / (NS * 64), st = (c / 64) % NS, ll = c % 64;
        so[i] = pl * bplane + (ll & 31) * MP + 16 * st + 8 * (ll >> 5);
    }
    float accf[FR][16];
#pragma unroll
    for (int f = 0; f < FR; ++f)
#pragma unroll
        for (int r = 0; r < 16; ++r) accf[f][r] = 0.0f;
    const int64_t b0 = (int64_t)blockIdx.y * bpc;
    const int64_t b1 = (b0 + bpc < nblk32) ? b0 + bpc : nblk32;
    const int nb = (int)(b1 > b0 ? b1 - b0 : 0);

    auto load = [&](int k, bf16x8 (&pre)[PR], float& pw) {
        const int64_t off = (b0 + k) * 32 * MP;
#pragma unroll
        for (int i = 0; i < PR; ++i)
            if (tid + WG * i < CH) pre[i] = *reinterpret_cast<const bf16x8*>(Bt + so[i] + off);
        if (tid < 32) pw = (float)w[(b0 + k) * 32 + tid];
    };
    auto store = [&](int k, const bf16x8 (&pre)[PR], float pw) {
#pragma unroll
        for (int i = 0; i < PR; ++i)
            if (tid + WG * i < CH) sb[k & 1][tid + WG * i] = pre[i];
        if (tid < 32) swj[k & 1][tid] = pw;
    };
    // MFMAs of block k (LDS buffer k & 1) into g, the fragments' chains
    // interleaved (each B fragment read once for all of them)
    auto mma = [&](int k, f32x16 (&g)[FR]) {
#pragma unroll
        for (int f = 0; f < FR; ++f) g[f] = f32x16{};
        const bf16x8* sbc = sb[k & 1];
#pragma unroll
        for (int st = 0; st < NS; ++st) {
            const bf16x8 bh = sbc[st * 64 + l];
            if constexpr (NP >= 2) {
                const bf16x8 bl = sbc[(NS + st) * 64 + l];
                if constexpr (NP >= 3) {
                    const bf16x8 bl2 = sbc[(2 * NS + st) * 64 + l];
#pragma unroll
                    for (int f = 0; f < FR; ++f)
                        g[f] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[f][0][st], bl2, g[f], 0, 0, 0);
#pragma unroll
                    for (int f = 0; f < FR; ++f)
                        g[f] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[f][2][st], bh, g[f], 0, 0, 0);
#pragma unroll
                    for (int f = 0; f < FR; ++f)
                        g[f] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[f][1][st], bl, g[f], 0, 0, 0);
                }
#pragma unroll
                for (int f = 0; f < FR; ++f)
                    g[f] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[f][0][st], bl, g[f], 0, 0, 0);
#pragma unroll
                for (int f = 0; f < FR; ++f)
                    g[f] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[f][1][st], bh, g[f], 0, 0, 0);
            }
#pragma unroll
            for (int f = 0; f < FR; ++f)
                g[f] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[f][0][st], bh, g[f], 0, 0, 0);
        }
    };
    // exp2 and weighted sums of block k from its Gram g
    auto terms = [&](int k, const f32x16 (&g)[FR]) {
        const float wj = swj[k & 1][l32];
#pragma unroll
        for (int f = 0; f < FR; ++f)
#pragma unroll
            for (int r = 0; r < 16; ++r)
                accf[f][r] = fmaf(__builtin_amdgcn_fmed3f(__builtin_amdgcn_exp2f(g[f][r]), 0.0f, 1.0f), wj,
                                  accf[f][r]);
    };
    // one block per step: block k + 1 into registers, the MFMAs of block k
    // and its terms, block k + 1 into the other LDS buffer, one barrier
    if (nb > 0) {
        bf16x8 pre[PR];
        float pw = 0.0f;
        load(0, pre, pw);
        store(0, pre, pw);
        __syncthreads();
        for (int k = 0; k < nb; ++k) {
            const bool more = k + 1 < nb;
            if (more) load(k + 1, pre, pw);
            f32x16 g[FR];
            mma(k, g);
            terms(k, g);
            if (more) store(k + 1, pre, pw);
            __syncthreads();
        }
    }
#pragma unroll
    for (int f = 0; f < FR; ++f)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            double v = sum16((double)accf[f][r]);
            v = v + __shfl_xor(v, 16);
            if (l32 == 0) part[(int64_t)blockIdx.y * NQPAD + q0 + 32 * f + 8 * (r >> 2) + 4 * h + (r & 3)] = v;
        }
}

// f_q = sum over chunks (in order) of part[c][q] + lambda^2 sum_i w_i.
__global__ void k_predict_reduce(const double* __restrict__ part, int nchunk, int64_t stride, int64_t nq,
                                 const double* __restrict__ wsum, double lam2, double* __restrict__ f) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    double acc = 0.0;
    for (int c = 0; c < nchunk; ++c) acc += part[(int64_t)c * stride + q];
    f[q] = acc + lam2 * wsum[0];
}

template <int KIND>
void predict_kind(int mp, dim3 grid, const Features& Ft, const Features& Fq, const double* w, int64_t nblk32,
                  int bpc, float c, int64_t NQPAD, double* part, hipStream_t s) {
    if constexpr (KIND != GRAM_F32) {
        if (mp <= 32) {
            hipLaunchKernelGGL((k_predict_lds<KIND, 32>), grid, dim3(WG), 0, s, Ft, Fq, w, nblk32, bpc, c, NQPAD, part);
            return;
        }
        if (mp <= 64) {
            hipLaunchKernelGGL((k_predict_lds<KIND, 64>), grid, dim3(WG), 0, s, Ft, Fq, w, nblk32, bpc, c, NQPAD, part);
            return;
        }
    }
    if (mp <= 32)
        hipLaunchKernelGGL((k_predict_mfma<KIND, 32>), grid, dim3(WG), 0, s, Ft, Fq, w, nblk32, bpc, c, NQPAD, part);
    else if (mp <= 64)
        hipLaunchKernelGGL((k_predict_mfma<KIND, 64>), grid, dim3(WG), 0, s, Ft, Fq, w, nblk32, bpc, c, NQPAD, part);
    else if (mp <= 128)
        hipLaunchKernelGGL((k_predict_mfma<KIND, 128>), grid, dim3(WG), 0, s, Ft, Fq, w, nblk32, bpc, c, NQPAD, part);
    else
        hipLaunchKernelGGL((k_predict_mfma<KIND, 0>), grid, dim3(WG), 0, s, Ft, Fq, w, nblk32, bpc, c, NQPAD, part);
}

inline unsigned blocks_of(int64_t n) { return (unsigned)((n + WG - 1) / WG); }

}  // namespace

int64_t predict_query_pad(int64_t nq) { return (nq + QB - 1) / QB * QB; }

void predict_chunks(int64_t NPAD, int64_t NQPAD, int* nchunk, int* bpc) {
    const int64_t nblk32 = NPAD / 32, nqb = NQPAD / QB;
    // at most 32 training blocks per workgroup (the FP32 partial sums of the
    // staged kernel; longer chunks amortise the workgroup's query fragments
    // and first block: 10.2 ms with 8, 8.9 with 16, 7.9-8.2 with 32 at
    // 100k x 100k), and enough workgroups to fill the chip
    int64_t want = (4096 + nqb - 1) / nqb;
    want = std::max<int64_t>(want, (nblk32 + 31) / 32);
    want = std::max<int64_t>(1, std::min<int64_t>(want, nblk32));
    const int64_t per = (nblk32 + want - 1) / want;
    *bpc = (int)per;
    *nchunk = (int)((nblk32 + per - 1) / per);
}

hipError_t launch_predict_weights(const double* alpha, const float* y, int64_t N, int64_t NPAD, bool box,
                                  double C, double* w, double* blk, double* wsum, hipStream_t s) {
    const unsigned nb = blocks_of(NPAD);
    hipLaunchKernelGGL(k_predict_weights, dim3(nb), dim3(WG), 0, s, alpha, y, N, NPAD, box ? 1 : 0, C, w, blk);
    hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(WG), 0, s, blk, (int64_t)nb, wsum);
    return hipGetLastError();
}

hipError_t launch_predict_direct(const float* Xtr, const double* w, int64_t N, int64_t m, const float* Xq,
                                 int64_t nq, double gamma, double* part, hipStream_t s) {
    hipLaunchKernelGGL(k_predict_direct, dim3((unsigned)nq), dim3(WG), 0, s, Xtr, w, N, m, Xq, gamma, part);
    return hipGetLastError();
}

hipError_t launch_predict_mfma(const Features& Ft, const Features& Fq, const double* w, int64_t NPAD,
                               int64_t NQPAD, float neg_gamma_log2e, int nchunk, int bpc, double* part,
                               hipStream_t s) {
    if (NQPAD % QB != 0 || NPAD % 32 != 0 || Ft.m_pad != Fq.m_pad || Ft.kind != Fq.kind)
        return hipErrorInvalidValue;
    const dim3 grid((unsigned)(NQPAD / QB), (unsigned)nchunk);
    const int64_t nblk32 = NPAD / 32;
    switch (Ft.kind) {
        case GRAM_F32: predict_kind<GRAM_F32>(Ft.m_pad, grid, Ft, Fq, w, nblk32, bpc, neg_gamma_log2e, NQPAD, part, s); break;
        case GRAM_BF16: predict_kind<GRAM_BF16>(Ft.m_pad, grid, Ft, Fq, w, nblk32, bpc, neg_gamma_log2e, NQPAD, part, s); break;
        case GRAM_BF16X3: predict_kind<GRAM_BF16X3>(Ft.m_pad, grid, Ft, Fq, w, nblk32, bpc, neg_gamma_log2e, NQPAD, part, s); break;
        case GRAM_BF16X6: predict_kind<GRAM_BF16X6>(Ft.m_pad, grid, Ft, Fq, w, nblk32, bpc, neg_gamma_log2e, NQPAD, part, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int64_t predict_query_pad_aug(int64_t nq) { return (nq + QBA - 1) / QBA * QBA; }

void predict_chunks_aug(int64_t NPAD, int64_t NQPAD, int* nchunk, int* bpc) {
    const int64_t nblk32 = NPAD / 32, nqb = NQPAD / QBA;
    // at most 32 training blocks per workgroup (FP32 partial sums), and at
    // least 4096 workgroups when the training set allows
    int64_t want = (4096 + nqb - 1) / nqb;
    want = std::max<int64_t>(want, (nblk32 + 31) / 32);
    want = std::max<int64_t>(1, std::min<int64_t>(want, nblk32));
    const int64_t per = (nblk32 + want - 1) / want;
    *bpc = (int)per;
    *nchunk = (int)((nblk32 + per - 1) / per);
}

hipError_t launch_stage_aug(const float* X, const double* mean, int64_t n, int64_t m, int64_t NPAD, int mp, int kind,
                            int side, float c, uint16_t* out, hipStream_t s) {
    const int np = (kind == GRAM_BF16X6) ? 3 : (kind == GRAM_BF16X3) ? 2 : 1;
    if (m + 2 > mp || (mp != 32 && mp != 64) || (kind != GRAM_BF16 && kind != GRAM_BF16X3 && kind != GRAM_BF16X6))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_stage_aug, dim3(blocks_of(NPAD)), dim3(WG), 0, s, X, mean, n, m, NPAD, mp, np, side, c, out,
                       NPAD * mp);
    return hipGetLastError();
}

hipError_t launch_predict_aug(int kind, int mp, const uint16_t* Bt, int64_t NPAD, const uint16_t* Aq, int64_t NQPAD,
                              const double* w, int nchunk, int bpc, double* part, hipStream_t s, hipEvent_t e0,
                              hipEvent_t e1) {
    if (NQPAD % QBA != 0 || NPAD % 32 != 0) return hipErrorInvalidValue;
    const dim3 grid((unsigned)(NQPAD / QBA), (unsigned)nchunk);
    const int64_t nblk32 = NPAD / 32, bp = NPAD * mp, ap = NQPAD * mp;
#define GABP_AUG(K, M) launch_ev(k_predict_aug<K, M, AUG_FR>, grid, dim3(WG), s, e0, e1, Bt, bp, Aq, ap, w, nblk32, bpc, NQPAD, part)
    if (mp == 32) {
        switch (kind) {
            case GRAM_BF16: GABP_AUG(GRAM_BF16, 32); break;
            case GRAM_BF16X3: GABP_AUG(GRAM_BF16X3, 32); break;
            case GRAM_BF16X6: GABP_AUG(GRAM_BF16X6, 32); break;
            default: return hipErrorInvalidValue;
        }
    } else if (mp == 64) {
        switch (kind) {
            case GRAM_BF16: GABP_AUG(GRAM_BF16, 64); break;
            case GRAM_BF16X3: GABP_AUG(GRAM_BF16X3, 64); break;
            case GRAM_BF16X6: GABP_AUG(GRAM_BF16X6, 64); break;
            default: return hipErrorInvalidValue;
        }
    } else {
        return hipErrorInvalidValue;
    }
#undef GABP_AUG
    return hipGetLastError();
}

hipError_t launch_predict_reduce(const double* part, int nchunk, int64_t stride, int64_t nq, const double* wsum,
                                 double lam2, double* f, hipStream_t s) {
    hipLaunchKernelGGL(k_predict_reduce, dim3(blocks_of(nq)), dim3(WG), 0, s, part, nchunk, stride, nq, wsum,
                       lam2, f);
    return hipGetLastError();
}

}  // namespace gabp
