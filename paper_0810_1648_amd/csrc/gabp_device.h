// Device-side building blocks shared by the HIP translation units of the
// GaBP SVM solver: vector loads, wave reductions, MFMA Gram tiles, and the
// sweep of one tile (see gabp_kernels.hip for the data layout).
#pragma once

#include "gabp_internal.h"

#include <hip/hip_ext.h>

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

// K' row steps in flight per lane in the stateless sweep over an FP32 K'
// plane: each wave streams its row steps into an LDS ring by direct
// global-to-LDS loads, so the bytes in flight do not occupy registers.
#ifndef GABP_KRING
#define GABP_KRING 4
#endif
constexpr int KRING = GABP_KRING;

// LDS byte offset of a shared-memory pointer (wave-uniform here).
__device__ inline uint32_t lds_offset(const void* p) {
    return (uint32_t)reinterpret_cast<uintptr_t>((const __attribute__((address_space(3))) void*)p);
}

// One direct global-to-LDS load of 16 bytes per lane: lane l's bytes at
// base + voff land at LDS offset lds + 16 l, with the non-temporal hint.  The
// compiler's wait counting does not see this load: callers wait for it with
// wait_vm before reading the LDS it writes, and issue it only after their
// last read of that LDS has completed.
__device__ inline void dma16(const float* base, uint32_t voff, uint32_t lds) {
    // the base and the LDS offset are wave-uniform: scalar operands
    lds = __builtin_amdgcn_readfirstlane(lds);
    // (the builtin returns a signed int: each half goes through uint32_t so
    // that the low half is zero-extended, never sign-extended)
    const uint64_t b = reinterpret_cast<uint64_t>(base);
    const uint32_t bh = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
    const uint32_t bl = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
    base = reinterpret_cast<const float*>(((uint64_t)bh << 32) | (uint64_t)bl);
    asm volatile("s_mov_b32 m0, %2\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, %1 nt"
                 :: "v"(voff), "s"(base), "s"(lds) : "memory", "m0");
}
// Waits until at most N vector-memory operations of this wave are in flight.
template <int N> __device__ inline void wait_vm() {
    asm volatile("s_waitcnt vmcnt(%0)" :: "n"(N) : "memory");
}

// Address of a lane's element from a wave-uniform base (scalar registers)
// and a 32-bit lane offset: loads and stores then take the scalar-base form
// and the per-step address arithmetic stays off the vector ALU.
template <class T> __device__ inline T* lane_ptr(T* base, uint32_t elems) {
    using C = typename std::conditional<std::is_const<T>::value, const char, char>::type;
    return reinterpret_cast<T*>(reinterpret_cast<C*>(base) + elems * (uint32_t)sizeof(T));
}

template <int CTRL> __device__ inline int dpp_i(int v) {
    // every source lane of these patterns exists, so no fill value is needed
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
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
// v = h + l + l2 in BF16 (each the rounding of the remainder left by the
// terms before it): h alone carries about 2^-9 of v, h + l about 2^-18,
// h + l + l2 about 2^-27.
__device__ inline void split3(float v, uint16_t& h, uint16_t& l, uint16_t& l2) {
    h = f2bf(v);
    const float r = v - bf2f(h);
    l = f2bf(r);
    l2 = f2bf(r - bf2f(l));
}

// Reciprocals: v_rcp_f32 (1 ulp) for FP32; for FP64, v_rcp_f64 refined by
// two Newton steps (the cavity precisions are far from the denormal range).
__device__ inline float rcp_fast(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double rcp_fast(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    return __builtin_isinf(x) ? 0.0 : r;    // 1/inf = 0 (Newton would give NaN)
}

// Workgroups go to the eight XCDs in turn (workgroup b to XCD b mod 8).
// This index of workgroup b in [0, n) (n = the grid) gives every XCD one
// contiguous range instead, so that work items sharing data (neighbouring
// nodes and edges, tiles of one super-block) meet in the same L2.
__device__ inline int64_t xcd_contiguous(int64_t b, int64_t n) {
    const int64_t x = b & 7, q = b >> 3, base = n >> 3, rem = n & 7;
    return x * base + (x < rem ? x : rem) + q;
}

struct TileCoord { int I, J; };
__device__ inline TileCoord tile_of(const uint32_t* tiles) {
    const uint32_t ij = tiles[blockIdx.x];
    return {(int)(ij >> 16), (int)(ij & 0xFFFFu)};
}

// ------------------------------------------------------------ K' build --

// One 32 x 32 block of the Gram matrix x_a . x_b on MFMA, for A rows
// rowA = base_a + lane % 32 and B rows colB = base_b + lane % 32.  The
// inner-product index is split between the two lane halves so that each lane
// reads contiguous features.  Output layout of the 32x32 MFMAs: register r of
// lane l holds row 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32.
// The A rows come from FA and the B rows from FB (the same staging: m_pad
// and kind are taken from FA).
template <int KIND>
__device__ inline f32x16 mfma_gram_32x32(const Features& FA, int64_t rowA, const Features& FB, int64_t colB) {
    const int l = threadIdx.x & 63, h = l >> 5;
    const int mp = FA.m_pad;
    f32x16 acc = {};
    if constexpr (KIND == GRAM_F32) {
        const int half = mp >> 1;
        const float* pa = FA.f32 + rowA * mp + h * half;
        const float* pb = FB.f32 + colB * mp + h * half;
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
            const bf16x8 a = *reinterpret_cast<const bf16x8*>(FA.hi + oa + s);
            const bf16x8 b = *reinterpret_cast<const bf16x8*>(FB.hi + ob + s);
            if constexpr (KIND == GRAM_BF16X3 || KIND == GRAM_BF16X6) {
                // correction terms first, then the leading product
                const bf16x8 al = *reinterpret_cast<const bf16x8*>(FA.lo + oa + s);
                const bf16x8 bl = *reinterpret_cast<const bf16x8*>(FB.lo + ob + s);
                if constexpr (KIND == GRAM_BF16X6) {
                    const bf16x8 a2 = *reinterpret_cast<const bf16x8*>(FA.lo2 + oa + s);
                    const bf16x8 b2 = *reinterpret_cast<const bf16x8*>(FB.lo2 + ob + s);
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

template <int KIND>
__device__ inline f32x16 mfma_gram_32x32(const Features& F, int64_t rowA, int64_t colB) {
    return mfma_gram_32x32<KIND>(F, rowA, F, colB);
}

// A operand (32 rows) of the MFMA Gram, held in registers while a wave walks
// many 32-row B blocks, when m_pad <= MP; MP = 0 reloads it every block.
template <int KIND, int MP> struct RowFrag {
    static constexpr int NS = (KIND == GRAM_F32) ? MP / 8 : MP / 16;
    static constexpr int NSA = NS > 0 ? NS : 1;
    f32x4v f[KIND == GRAM_F32 ? NSA : 1];
    bf16x8 hi[KIND == GRAM_F32 ? 1 : NSA];
    bf16x8 lo[(KIND == GRAM_BF16X3 || KIND == GRAM_BF16X6) ? NSA : 1];
    bf16x8 lo2[KIND == GRAM_BF16X6 ? NSA : 1];

    __device__ void load(const Features& Fq, int64_t rowA) {
        if constexpr (MP > 0) {
            const int l = threadIdx.x & 63, h = l >> 5, mp = Fq.m_pad;
            if constexpr (KIND == GRAM_F32) {
                const int half = mp >> 1;
                const float* pa = Fq.f32 + rowA * mp + h * half;
#pragma unroll
                for (int s = 0; s < NS; ++s)
                    if (4 * s < half) f[s] = *reinterpret_cast<const f32x4v*>(pa + 4 * s);
            } else {
                const int64_t oa = rowA * mp + 8 * h;
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    if (16 * s >= mp) continue;
                    hi[s] = *reinterpret_cast<const bf16x8*>(Fq.hi + oa + 16 * s);
                    if constexpr (KIND == GRAM_BF16X3 || KIND == GRAM_BF16X6)
                        lo[s] = *reinterpret_cast<const bf16x8*>(Fq.lo + oa + 16 * s);
                    if constexpr (KIND == GRAM_BF16X6)
                        lo2[s] = *reinterpret_cast<const bf16x8*>(Fq.lo2 + oa + 16 * s);
                }
            }
        }
    }

    // Two A blocks (a0, a1) against the same B rows: each B fragment is
    // loaded once for both MFMA chains.
    __device__ static void gram2(const RowFrag& a0, const RowFrag& a1, const Features& Fq, int64_t rowA0,
                                 int64_t rowA1, const Features& Ft, int64_t colB, f32x16& acc0, f32x16& acc1) {
        if constexpr (MP == 0) {
            acc0 = mfma_gram_32x32<KIND>(Fq, rowA0, Ft, colB);
            acc1 = mfma_gram_32x32<KIND>(Fq, rowA1, Ft, colB);
        } else {
            const int l = threadIdx.x & 63, h = l >> 5, mp = Ft.m_pad;
            acc0 = f32x16{};
            acc1 = f32x16{};
            if constexpr (KIND == GRAM_F32) {
                const int half = mp >> 1;
                const float* pb = Ft.f32 + colB * mp + h * half;
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    if (4 * s >= half) continue;
                    const f32x4v b4 = *reinterpret_cast<const f32x4v*>(pb + 4 * s);
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0.f[s][e], b4[e], acc0, 0, 0, 0);
                        acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1.f[s][e], b4[e], acc1, 0, 0, 0);
                    }
                }
            } else {
                const int64_t ob = colB * mp + 8 * h;
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    if (16 * s >= mp) continue;
                    const bf16x8 b = *reinterpret_cast<const bf16x8*>(Ft.hi + ob + 16 * s);
                    if constexpr (KIND == GRAM_BF16X3 || KIND == GRAM_BF16X6) {
                        const bf16x8 bl = *reinterpret_cast<const bf16x8*>(Ft.lo + ob + 16 * s);
                        if constexpr (KIND == GRAM_BF16X6) {
                            const bf16x8 b2 = *reinterpret_cast<const bf16x8*>(Ft.lo2 + ob + 16 * s);
                            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0.hi[s], b2, acc0, 0, 0, 0);
                            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1.hi[s], b2, acc1, 0, 0, 0);
                            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0.lo2[s], b, acc0, 0, 0, 0);
                            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1.lo2[s], b, acc1, 0, 0, 0);
                            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0.lo[s], bl, acc0, 0, 0, 0);
                            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1.lo[s], bl, acc1, 0, 0, 0);
                        }
                        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0.hi[s], bl, acc0, 0, 0, 0);
                        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1.hi[s], bl, acc1, 0, 0, 0);
                        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0.lo[s], b, acc0, 0, 0, 0);
                        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1.lo[s], b, acc1, 0, 0, 0);
                    }
                    acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0.hi[s], b, acc0, 0, 0, 0);
                    acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1.hi[s], b, acc1, 0, 0, 0);
                }
            }
        }
    }

    // Gram block of the 32 A rows with the B rows colB (one per lane % 32).
    __device__ f32x16 gram(const Features& Fq, int64_t rowA, const Features& Ft, int64_t colB) const {
        if constexpr (MP == 0) {
            return mfma_gram_32x32<KIND>(Fq, rowA, Ft, colB);
        } else {
            const int l = threadIdx.x & 63, h = l >> 5, mp = Ft.m_pad;
            f32x16 acc = {};
            if constexpr (KIND == GRAM_F32) {
                const int half = mp >> 1;
                const float* pb = Ft.f32 + colB * mp + h * half;
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    if (4 * s >= half) continue;
                    const f32x4v b4 = *reinterpret_cast<const f32x4v*>(pb + 4 * s);
                    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(f[s][0], b4[0], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(f[s][1], b4[1], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(f[s][2], b4[2], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(f[s][3], b4[3], acc, 0, 0, 0);
                }
            } else {
                const int64_t ob = colB * mp + 8 * h;
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    if (16 * s >= mp) continue;
                    const bf16x8 b = *reinterpret_cast<const bf16x8*>(Ft.hi + ob + 16 * s);
                    if constexpr (KIND == GRAM_BF16X3 || KIND == GRAM_BF16X6) {
                        const bf16x8 bl = *reinterpret_cast<const bf16x8*>(Ft.lo + ob + 16 * s);
                        if constexpr (KIND == GRAM_BF16X6) {
                            const bf16x8 b2 = *reinterpret_cast<const bf16x8*>(Ft.lo2 + ob + 16 * s);
                            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(hi[s], b2, acc, 0, 0, 0);
                            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(lo2[s], b, acc, 0, 0, 0);
                            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(lo[s], bl, acc, 0, 0, 0);
                        }
                        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(hi[s], bl, acc, 0, 0, 0);
                        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(lo[s], b, acc, 0, 0, 0);
                    }
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(hi[s], b, acc, 0, 0, 0);
                }
            }
            return acc;
        }
    }
};

// acc += A B^T for register-held fragments of 32 A rows and 32 B rows (both
// loaded with RowFrag::load; MP > 0), in the products order of
// mfma_gram_32x32 (correction terms first).  Loading the next B fragment
// before this call hides its latency behind the MFMA chain.
template <int KIND, int MP>
__device__ inline void frag_mma(const RowFrag<KIND, MP>& a, const RowFrag<KIND, MP>& b, f32x16& acc, int mp) {
    static_assert(MP > 0, "register fragments only");
    constexpr int NS = RowFrag<KIND, MP>::NS;
    if constexpr (KIND == GRAM_F32) {
        const int half = mp >> 1;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (4 * s >= half) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.f[s][e], b.f[s][e], acc, 0, 0, 0);
        }
    } else {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (16 * s >= mp) continue;
            if constexpr (KIND == GRAM_BF16X3 || KIND == GRAM_BF16X6) {
                if constexpr (KIND == GRAM_BF16X6) {
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.hi[s], b.lo2[s], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.lo2[s], b.hi[s], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.lo[s], b.lo[s], acc, 0, 0, 0);
                }
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.hi[s], b.lo[s], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.lo[s], b.hi[s], acc, 0, 0, 0);
            }
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.hi[s], b.hi[s], acc, 0, 0, 0);
        }
    }
}

// B fragments of a 32-row block staged in LDS (BF16 splits), shared by the
// waves of a workgroup.  Chunk k of a block (k < planes x 64 x ns, ns =
// m_pad / 16) is 16 bytes of one staged row: plane k / (64 ns), row and
// 16-byte column of the row-major features, so that consecutive threads load
// consecutive bytes; its slot is the fragment order (plane, k-step, lane),
// lane = 32 (column / 2 parity) + row, so that a wave reads the operand of
// k-step s as 64 consecutive chunks.
template <int KIND> struct BStage {
    static constexpr int NP = (KIND == GRAM_BF16X6) ? 3 : (KIND == GRAM_BF16X3) ? 2 : 1;
    __device__ static const bf16x8* src(const Features& F, int64_t row0, int ns, int k) {
        const int pl = k / (64 * ns), rem = k - pl * 64 * ns, row = rem / (2 * ns), cc = rem - row * 2 * ns;
        const uint16_t* base = (pl == 0) ? F.hi : (pl == 1) ? F.lo : F.lo2;
        return reinterpret_cast<const bf16x8*>(base + (row0 + row) * F.m_pad + 8 * cc);
    }
    __device__ static int dst(int ns, int k) {
        const int pl = k / (64 * ns), rem = k - pl * 64 * ns, row = rem / (2 * ns), cc = rem - row * 2 * ns;
        return (pl * ns + (cc >> 1)) * 64 + (cc & 1) * 32 + row;
    }
    // acc += A B^T with A in registers and B staged at sb (the products of
    // frag_mma, in its order)
    template <int MP>
    __device__ static void mma(const RowFrag<KIND, MP>& a, const bf16x8* sb, int ns, int l, f32x16& acc) {
#pragma unroll
        for (int st = 0; st < MP / 16; ++st) {
            if (st >= ns) continue;
            const bf16x8 bh = sb[(0 * ns + st) * 64 + l];
            if constexpr (NP >= 2) {
                const bf16x8 bl = sb[(1 * ns + st) * 64 + l];
                if constexpr (NP >= 3) {
                    const bf16x8 bl2 = sb[(2 * ns + st) * 64 + l];
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.hi[st], bl2, acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.lo2[st], bh, acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.lo[st], bl, acc, 0, 0, 0);
                }
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.hi[st], bl, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.lo[st], bh, acc, 0, 0, 0);
            }
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.hi[st], bh, acc, 0, 0, 0);
        }
    }
};

// K' = exp(-gamma d^2) + lambda^2 with d^2 = max(0, n_i + n_j - 2 G_ij), zero
// for pairs that are not strictly upper (i >= j) or are padding (j >= N).
// K' from a Gram entry: exp2 of the scaled, clamped distance on the
// hardware exp2 (v_exp_f32; results below 2^-126 flush to zero, which the
// lambda^2 added next absorbs), plus lambda^2.
__device__ inline float kernel_value(float ni, float nj, float g, const KernelParams& kp) {
    const float d2 = fmaxf(ni + nj - 2.0f * g, 0.0f);
    return __builtin_amdgcn_exp2f(kp.neg_gamma_log2e * d2) + (float)kp.lam2;
}
// ... and zero outside the strict upper triangle and past N.
__device__ inline float kernel_entry(float ni, float nj, float g, int64_t i, int64_t j,
                                     const KernelParams& kp) {
    const float kv = kernel_value(ni, nj, g, kp);
    return (i < j && j < kp.N) ? kv : 0.0f;
}

// K' for the 32 x 64 band [row0, row0 + 32) x [col0, col0 + 64) of tile
// (I, J), computed by one wave into its LDS buffer kb[32][64] (row-major).
template <int KIND>
__device__ inline void gram_band(const Features& F, const KernelParams& kp, int I, int J, int row0,
                                 int col0, float* kb) {
    const int l = threadIdx.x & 63, h = l >> 5, l32 = l & 31;
    const int64_t rowA = (int64_t)I * TILE + row0 + l32;
    // the index test matters only on diagonal tiles and in the last column block
    const bool plain = (I < J) && ((int64_t)J * TILE + col0 + 64 <= kp.N);
    if constexpr (KIND != GRAM_F32) {
        if (F.aug0) {
            // augmented rows: the MFMA output is the exponent (clamped at 0,
            // the largest value of -gamma log2(e) d^2), K' = exp2 + lambda^2
            Features FA = F, FB = F;
            FA.hi = F.aug0; FA.lo = F.aug0 + F.aug_plane; FA.lo2 = F.aug0 + 2 * F.aug_plane;
            FB.hi = F.aug1; FB.lo = F.aug1 + F.aug_plane; FB.lo2 = F.aug1 + 2 * F.aug_plane;
            const float lam2 = (float)kp.lam2;
#pragma unroll 1
            for (int cb = 0; cb < 2; ++cb) {
                const int64_t colB = (int64_t)J * TILE + col0 + 32 * cb + l32;
                const f32x16 acc = mfma_gram_32x32<KIND>(FA, rowA, FB, colB);
                float* kl = kb + 4 * h * 64 + 32 * cb + l32;
                if (plain) {
#pragma unroll
                    for (int r = 0; r < 16; ++r)
                        kl[(8 * (r >> 2) + (r & 3)) * 64] = __builtin_amdgcn_exp2f(fminf(acc[r], 0.0f)) + lam2;
                } else {
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int64_t i = (int64_t)I * TILE + row0 + 8 * (r >> 2) + 4 * h + (r & 3);
                        const float kv = __builtin_amdgcn_exp2f(fminf(acc[r], 0.0f)) + lam2;
                        kl[(8 * (r >> 2) + (r & 3)) * 64] = (i < colB && colB < kp.N) ? kv : 0.0f;
                    }
                }
            }
            return;
        }
    }
    float ni[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) ni[r] = F.nrm[(int64_t)I * TILE + row0 + 8 * (r >> 2) + 4 * h + (r & 3)];
#pragma unroll 1
    for (int cb = 0; cb < 2; ++cb) {
        const int64_t colB = (int64_t)J * TILE + col0 + 32 * cb + l32;
        const f32x16 acc = mfma_gram_32x32<KIND>(F, rowA, colB);
        const float nj = F.nrm[colB];
        // the lane's column of its row half: the 16 rows sit at constant offsets
        float* kl = kb + 4 * h * 64 + 32 * cb + l32;
        if (plain) {
#pragma unroll
            for (int r = 0; r < 16; ++r)
                kl[(8 * (r >> 2) + (r & 3)) * 64] = kernel_value(ni[r], nj, acc[r], kp);
        } else {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = 8 * (r >> 2) + 4 * h + (r & 3);
                kl[(8 * (r >> 2) + (r & 3)) * 64] =
                    kernel_entry(ni[r], nj, acc[r], (int64_t)I * TILE + row0 + row, colB, kp);
            }
        }
    }
}

__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------------ sweep --

// Sums of one tile's messages: the row sums of node `threadIdx.x` of the row
// block, and the column sums of the lane's four columns (every row group of
// a wave holds the same values).
template <class AT>
struct TileSums {
    AT rp, re;
    AT cp[4], ce[4];
};

// Stores one partial sum of a tile: in FP32 when the plan keeps its partials
// in FP32 (the FP32-message form, whose tile sums are FP32 sums rounded once
// more here), else in the aggregate type.
template <class AT>
__device__ inline void put_part(void* base, size_t o, AT v, bool p32) {
    if (p32) static_cast<float*>(base)[o] = (float)v;
    else static_cast<AT*>(base)[o] = v;
}

// Type of the message arithmetic.  The MIXED path (FP32 storage, FP64
// aggregates) with series reciprocals computes its messages in FP32: the
// cavity denominator P~ - P_reverse is never formed (the series factor
// 1 + e + e^2 has |e| <= rho^2, bounded a priori, so nothing cancels), the
// per-node 1/P~ and S/P~ are rounded once from FP64, and FP32 sums of a few
// messages are added into the FP64 aggregates.  Every other path computes
// its messages in MT.
template <class ST, class MT, class AT, int SER>
struct MsgT {
    static constexpr bool F32 = SER && std::is_same<ST, float>::value && std::is_same<AT, double>::value;
    using T = typename std::conditional<F32, float, MT>::type;
};

// One synchronous sweep over all tiles.  Template parameters:
//   ST storage type of K' and the message planes, MT type of the top-level
//   update (cavity denominators, reciprocals), AT aggregate type;
//   KSRC: K' from the materialised plane or recomputed per 32-row band;
//   GK: Gram kind of the recompute;
//   D: 0 = stored edge state (pair-record planes read and written);
//      D >= 1 = stateless: the messages of the previous sweep are rebuilt
//      from the aggregates of the D - 1 earlier sweeps held in the ring (a
//      slot from before sweep 0 holds P~ = inf, S = 0 and yields exactly zero
//      messages), lower levels in LT (see below);
//   FIRST: the stored planes are all zero (sweep 1) and are not read.
// Work of one tile: its row and column sums go to the tile's partial slots,
// or, with `out`, to the caller (a chunk adds them up first).  SER (stateless
// only; 0 = exact reciprocals): the
// reciprocals of the cavity precisions Q = P~ (1 - e), e = P_reverse / P~,
// are formed from the per-node u = 1/P~ by the series
// 1/Q = (1 + e + e^2 + ...) u, one term at the lower levels and SER terms at
// the top (SER = 3: one term at the top, none at the lower levels).
// |e| <= rho^2 holds for every message by the a-priori contraction bound (no
// run-time check is needed); the host picks the series only when the
// neglected terms are below the arithmetic's precision.  The lower levels
// carry G = P / (-a^2) and F = E / a, which the one-term series turns into
// G_ij = u_i - a^2 u_i^2 G_ji and F_ij = G_ij (a F_ji - S_i): the deepest
// level (reverse messages zero) is G = u, F = -S/P~ of its source and costs
// nothing, a middle level costs four operations per direction (two with
// G = u).
template <class ST, class MT, class AT, int KSRC, int GK, int D, bool FIRST, int SER>
__device__ inline void sweep_tile(const SweepArgs& a, int64_t tile, int slot_top, TileSums<AT>* out = nullptr) {
    DevStatus* st = a.st;
    // lower levels: FP32 storage precision; with the series and up to three
    // levels they run in the top level's type (FP64 FMA issues at the FP32
    // rate on CDNA4, and no conversions are needed between levels; deeper
    // unrolls keep FP32 to bound the per-column register history)
    using XT = typename MsgT<ST, MT, AT, SER>::T;
    constexpr bool XF = MsgT<ST, MT, AT, SER>::F32;
    using LT = typename std::conditional<(SER && D <= 3) || std::is_same<ST, double>::value, XT, float>::type;
    constexpr bool STORED = (D == 0);
    constexpr bool LEAN = (SER == 3);         // lower levels: G = u (no series term)
    constexpr int DL = (D > 1) ? D - 1 : 1;   // lower levels held per node
    constexpr int NL = STORED ? 1 : DL;
    constexpr int NT = STORED ? 1 : TILE;
    // series: S and u^2 only at the middle levels 1 .. D - 2, S/P~ only at
    // the deepest level D - 1; exact reciprocals: S at every lower level
    constexpr int NSL = SER ? ((D > 2) ? D - 2 : 1) : NL;
    constexpr int NTS = (SER && D <= 2) ? 1 : NT;
    constexpr int NTQ = (SER && SER != 3 && D > 2) ? NT : 1;
    constexpr int NTD = (SER && D >= 2) ? NT : 1;
    const uint32_t ij = a.tiles[tile];
    const TileCoord tc{(int)(ij >> 16), (int)(ij & 0xFFFFu)};
    const int NB = a.NB;
    const size_t tbase = (size_t)tile * TT;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, g = l >> 4, q = l & 15;
    const int col0 = w * 64 + q * 4;
    constexpr int L = D;                      // stateless: levels unrolled in this launch
    const AT* HP = static_cast<const AT*>(a.HP);
    const AT* HS = static_cast<const AT*>(a.HS);
    // series: 1/P~ and S/P~ from the rings when the finalize formed them
    // (the same IEEE quotients as here)
    const AT* HI = static_cast<const AT*>(a.HI);
    const AT* HM = static_cast<const AT*>(a.HM);
    // branch-free around the loads (the ring pointers are uniform), so that
    // the node loads of the tile's prologue issue back to back
    const AT* HIs = HI ? HI : HP;
    const AT* HMs = HM ? HM : HS;
    auto inv_at = [&](int64_t o) -> AT {
        const AT v = HIs[o];
        return HI ? v : (AT)1 / v;
    };
    auto mean_at = [&](int64_t o) -> AT {
        const AT v = HMs[o], p = HP[o];
        return HM ? v : v / p;
    };
    const ST* Kp = static_cast<const ST*>(a.Kp);
    ST* Pf = static_cast<ST*>(a.Pf);
    ST* Pb = static_cast<ST*>(a.Pb);
    ST* Ef = static_cast<ST*>(a.Ef);
    ST* Eb = static_cast<ST*>(a.Eb);
    // the lane's offset inside a row group of a tile
    const uint32_t lo = (uint32_t)(g * TILE + col0);

    // stateless over an FP32 K' plane: row steps stream through a per-wave
    // LDS ring KR steps ahead (K' is the only stream; one register prefetch
    // per lane does not cover the HBM latency), the first KR issued before
    // the node data is loaded; other forms prefetch one row step ahead in
    // registers
    constexpr bool RING = (KSRC == KSRC_PLANE) && !STORED && std::is_same<ST, float>::value;
    constexpr int KR = RING ? KRING : 1;
    constexpr int SU = (RING && 8 % KR == 0) ? KR : 1;   // row steps unrolled (static ring slots)
    __shared__ __attribute__((aligned(16))) float kring[KR][4][RING ? 256 : 4];
    if constexpr (RING) {
#pragma unroll
        for (int u = 0; u < KR; ++u)
            dma16(reinterpret_cast<const float*>(Kp) + tbase + (size_t)u * 4 * TILE, lo * 4u,
                  lds_offset(&kring[u][w][0]));
    }

    // row-node data: top level (P~ or, with SER, 1/P~) and lower levels
    __shared__ XT sPt[TILE], sS[TILE];
    __shared__ LT sPtL[NL][NT], sSL[NSL][NTS], sUQL[NSL][NTQ], sSIL[NTD];
    // row partials per wave strip (XF: FP32 sums of 64 messages; exact in AT)
    using RT = typename std::conditional<XF, XT, AT>::type;
    __shared__ RT rP[4][TILE], rE[4][TILE];
    __shared__ float kband[KSRC == KSRC_RECOMPUTE ? 4 : 1][KSRC == KSRC_RECOMPUTE ? 32 * 64 : 1];
    // stateless: per-lane row partials of two row steps, reduced over the 16
    // column lanes through LDS once per two steps (a DPP tree per row step
    // costs 24 VALU slots in FP64; this costs about 5); XF reduces in FP32
    __shared__ RT red[STORED ? 1 : 4][2][2][64];

    const int64_t top = (int64_t)slot_top * a.NPAD;
    {
        const int64_t o = top + (int64_t)tc.I * TILE + tid;
        sPt[tid] = SER ? (XT)inv_at(o) : (XT)HP[o];
        sS[tid] = (XT)HS[o];
    }
    // one-term series: the top level forms 1/Q = u - a^2 u^2 G_rev from u and
    // u^2 (two operations per direction instead of three)
    constexpr bool SQ1 = (SER == 1 || SER == 3);
    __shared__ XT sPq[SQ1 ? TILE : 1];
    XT ptj[4], sj[4], pqj[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int64_t o = top + (int64_t)tc.J * TILE + col0 + c;
        ptj[c] = SER ? (XT)inv_at(o) : (XT)HP[o];
        sj[c] = (XT)HS[o];
        pqj[c] = ptj[c] * ptj[c];
    }
    if constexpr (SQ1) sPq[tid] = sPt[tid] * sPt[tid];
    // lower levels per node: P~ (exact) or u = 1/P~ (series) at every level;
    // exact: S at every level; series: S and u^2 at the middle levels, S/P~
    // at the deepest
    LT ptjL[DL][4], sjL[NSL][4], cuqL[NSL][4], sijL[4];
    if constexpr (!STORED) {
#pragma unroll
        for (int k = 1; k < D; ++k) {
            if (k < L) {
                const int64_t base = (int64_t)((slot_top - k + a.R) % a.R) * a.NPAD;
                const int64_t o = base + (int64_t)tc.I * TILE + tid;
                if constexpr (SER) {
                    // form 3: the deepest level's G (= u) is never read
                    if (!(LEAN && k == D - 1)) sPtL[k - 1][tid] = (LT)inv_at(o);
                    if (k == D - 1) {
                        sSIL[tid] = (LT)mean_at(o);
                    } else {
                        if constexpr (!LEAN) {
                            const AT u = inv_at(o);
                            sUQL[k - 1][tid] = (LT)(u * u);
                        }
                        sSL[k - 1][tid] = (LT)HS[o];
                    }
                } else {
                    sPtL[k - 1][tid] = (LT)HP[o];
                    sSL[k - 1][tid] = (LT)HS[o];
                }
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int64_t o = base + (int64_t)tc.J * TILE + col0 + c;
                    if constexpr (SER) {
                        const AT u = inv_at(o);
                        if (!(LEAN && k == D - 1)) ptjL[k - 1][c] = (LT)u;
                        if (k == D - 1) {
                            sijL[c] = (LT)mean_at(o);
                        } else {
                            if constexpr (!LEAN) cuqL[k - 1][c] = (LT)(u * u);
                            sjL[k - 1][c] = (LT)HS[o];
                        }
                    } else {
                        ptjL[k - 1][c] = (LT)HP[o];
                        sjL[k - 1][c] = (LT)HS[o];
                    }
                }
            }
        }
    }
    AT cP[4] = {0, 0, 0, 0}, cE[4] = {0, 0, 0, 0};
    XT cPm[4] = {0, 0, 0, 0}, cEm[4] = {0, 0, 0, 0};   // XF: FP32 column sums over the tile's 256 rows
    bool bad = false;
    __syncthreads();

    // row offset (wave-uniform: tile base plus 4 TILE per row step)
    size_t off = tbase;
    V4<ST> k{}, pf{}, pb{}, ef{}, eb{};
    if constexpr (!RING && KSRC == KSRC_PLANE) k = ld4nt(lane_ptr(Kp + off, lo));
    if constexpr (STORED && !FIRST) {
        pf = ld4nt(lane_ptr(Pf + off, lo)); pb = ld4nt(lane_ptr(Pb + off, lo));
        ef = ld4nt(lane_ptr(Ef + off, lo)); eb = ld4nt(lane_ptr(Eb + off, lo));
    }

    for (int b = 0; b < TILE / 32; ++b) {
        if constexpr (KSRC == KSRC_RECOMPUTE) {
            gram_band<GK>(a.F, a.kp, tc.I, tc.J, 32 * b, 64 * w, kband[w]);
            wave_lds_sync();
        }
#pragma unroll SU
        for (int s2 = 0; s2 < 8; ++s2) {
            const int r = 32 * b + 4 * s2 + g;
            // prefetch the lane's next row (the last row re-reads itself: the
            // offset stays inside the tile and no branch is needed)
            const bool more = (b * 8 + s2 + 1) < TILE / 4;
            const size_t off2 = more ? off + 4 * TILE : off;
            V4<ST> k2, pf2, pb2, ef2, eb2;
            const int u = b * 8 + s2;                 // row step
            if constexpr (RING) {
                // this step's slot has landed once at most KR - 1 loads are
                // in flight (every later step issued one), or all of them near
                // the tile's end
                if (u + KR <= TILE / 4) wait_vm<KR - 1>();
                else wait_vm<0>();
                const float4 kk = *reinterpret_cast<const float4*>(&kring[u % KR][w][4 * l]);
                k = V4<ST>{{(ST)kk.x, (ST)kk.y, (ST)kk.z, (ST)kk.w}};
            } else if constexpr (KSRC == KSRC_PLANE) {
                k2 = ld4nt(lane_ptr(Kp + off2, lo));
            }
            if constexpr (STORED && !FIRST) {
                pf2 = ld4nt(lane_ptr(Pf + off2, lo)); pb2 = ld4nt(lane_ptr(Pb + off2, lo));
                ef2 = ld4nt(lane_ptr(Ef + off2, lo)); eb2 = ld4nt(lane_ptr(Eb + off2, lo));
            }
            if constexpr (KSRC == KSRC_RECOMPUTE) {
                const float4 kk = *reinterpret_cast<const float4*>(&kband[w][(4 * s2 + g) * 64 + 4 * q]);
                k = V4<ST>{{(ST)kk.x, (ST)kk.y, (ST)kk.z, (ST)kk.w}};
            }
            const XT pti = sPt[r], si = sS[r];
            const XT pqi = SQ1 ? sPq[r] : (XT)0;
            AT rp = 0, re = 0;
            XT rpm = 0, rem = 0;                         // XF: FP32 row sums (4 columns, then 64 per wave)
            V4<ST> npf, npb, nef, neb;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const XT av = (XT)k.v[c];
                // messages of the previous sweep: stored, or rebuilt level by level
                XT opf, opb, oef, oeb;
                if constexpr (STORED) {
                    opf = (XT)pf.v[c]; opb = (XT)pb.v[c]; oef = (XT)ef.v[c]; oeb = (XT)eb.v[c];
                } else if constexpr (SER) {
                    // G = P / (-a^2), F = E / a of the previous sweep's messages,
                    // rebuilt from the deepest level up (XT = LT on this path)
                    const LT al = (LT)k.v[c], a2l = al * al;
                    LT gf = 0, gb = 0, ff = 0, fb = 0;
                    constexpr int kd = L - 1;
#pragma unroll
                    for (int kk = D - 1; kk >= 1; --kk) {
                        if (kk == kd) {               // deepest level: reverse messages zero
                            if constexpr (!LEAN) {    // (form 3 never reads this level's G)
                                gf = sPtL[kk - 1][r];
                                gb = ptjL[kk - 1][c];
                            }
                            ff = -sSIL[r];
                            fb = -sijL[c];
                        } else if (kk < kd) {
                            LT ngf, ngb;
                            if constexpr (LEAN) {
                                ngf = sPtL[kk - 1][r];
                                ngb = ptjL[kk - 1][c];
                            } else {
                                ngf = fma(-a2l * sUQL[kk - 1][r], gb, sPtL[kk - 1][r]);
                                ngb = fma(-a2l * cuqL[kk - 1][c], gf, ptjL[kk - 1][c]);
                            }
                            const LT nff = ngf * fma(al, fb, -sSL[kk - 1][r]);
                            const LT nfb = ngb * fma(al, ff, -sjL[kk - 1][c]);
                            gf = ngf; gb = ngb; ff = nff; fb = nfb;
                        }
                    }
                    opf = (XT)gf; opb = (XT)gb; oef = (XT)ff; oeb = (XT)fb;
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
                    opf = (XT)lpf; opb = (XT)lpb; oef = (XT)lef; oeb = (XT)leb;
                }
                XT pij_m, eij_m, pji_m, eji_m;
                if constexpr (SER) {
                    // opf, opb, oef, oeb hold G_ij, G_ji, F_ij, F_ji here
                    const XT a2 = av * av;
                    XT gt_f, gt_b;                                                  // (1 + e + ...) / P~
                    if constexpr (SER == 2) {
                        const XT e_f = -(a2 * opb) * pti, e_b = -(a2 * opf) * ptj[c];   // P_ji / P~_i, P_ij / P~_j
                        gt_f = fma(pti, fma(e_f, e_f, e_f), pti);
                        gt_b = fma(ptj[c], fma(e_b, e_b, e_b), ptj[c]);
                    } else {
                        gt_f = fma(-(a2 * pqi), opb, pti);                          // u (1 + e), e = -a^2 u G_rev
                        gt_b = fma(-(a2 * pqj[c]), opf, ptj[c]);
                    }
                    pij_m = -a2 * gt_f;
                    pji_m = -a2 * gt_b;
                    eij_m = (av * gt_f) * fma(av, oeb, -si);      // a G (E_ji - S_i)
                    eji_m = (av * gt_b) * fma(av, oef, -sj[c]);
                } else {
                    const XT a2 = av * av;
                    const XT qf = pti - opb;        // P~_i - P_ji
                    const XT qb = ptj[c] - opf;     // P~_j - P_ij
                    bad |= !(qf > (XT)0) | !(qb > (XT)0);
                    const XT rf = rcp_fast(qf), rb = rcp_fast(qb);
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
                } else if constexpr (XF) {
                    cPm[c] += pij_m; cEm[c] += eij_m;
                    rpm += pji_m; rem += eji_m;
                } else {
                    cP[c] += (AT)pij_m; cE[c] += (AT)eij_m;
                    rp += (AT)pji_m; re += (AT)eji_m;
                }
            }
            if constexpr (STORED) {
                st4nt(lane_ptr(Pf + off, lo), npf); st4nt(lane_ptr(Pb + off, lo), npb);
                st4nt(lane_ptr(Ef + off, lo), nef); st4nt(lane_ptr(Eb + off, lo), neb);
                rp = sum16(rp);
                re = sum16(re);
                if (q == 0) { rP[w][r] = rp; rE[w][r] = re; }
            } else {
                red[w][0][s2 & 1][l] = XF ? (RT)rpm : (RT)rp;
                red[w][1][s2 & 1][l] = XF ? (RT)rem : (RT)re;
                if (s2 & 1) {
                    // lane l sums quantity l / 32 of row step (l % 32) / 16 and
                    // row group ((l % 32) / 4) % 4 over the column lanes
                    // 4 (l % 4) .. +3; the quad then adds its four parts (the
                    // same sum in every lane: IEEE addition commutes)
                    wave_lds_sync();
                    const int qty = l >> 5, idx = l & 31, stp = idx >> 4, gg = (idx >> 2) & 3, pt = idx & 3;
                    const RT* src = &red[w][qty][stp][16 * gg + 4 * pt];
                    RT v = (src[0] + src[1]) + (src[2] + src[3]);
                    v = v + dpp<0xB1>(v);
                    v = v + dpp<0x4E>(v);
                    const int row = 32 * b + 4 * ((s2 & 6) + stp) + gg;
                    if (pt == 0) {
                        if (qty == 0) rP[w][row] = v;
                        else rE[w][row] = v;
                    }
                    wave_lds_sync();
                }
            }
            if constexpr (RING) {
                // the slot's next row step (k was read from it and used above)
                if (u + KR < TILE / 4)
                    dma16(reinterpret_cast<const float*>(Kp) + tbase + (size_t)(u + KR) * 4 * TILE, lo * 4u,
                          lds_offset(&kring[u % KR][w][0]));
            } else if constexpr (KSRC == KSRC_PLANE) {
                k = k2;
            }
            if constexpr (STORED && !FIRST) { pf = pf2; pb = pb2; ef = ef2; eb = eb2; }
            off = off2;
        }
        if constexpr (KSRC == KSRC_RECOMPUTE) wave_lds_sync();
    }
    if constexpr (XF) {
#pragma unroll
        for (int c = 0; c < 4; ++c) { cP[c] = (AT)cPm[c]; cE[c] = (AT)cEm[c]; }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) { cP[c] = sum_groups(cP[c]); cE[c] = sum_groups(cE[c]); }
    __syncthreads();
    if (__any(bad) && l == 0) st->bad = 1;
    const AT rowP = ((AT)rP[0][tid] + (AT)rP[1][tid]) + ((AT)rP[2][tid] + (AT)rP[3][tid]);
    const AT rowE = ((AT)rE[0][tid] + (AT)rE[1][tid]) + ((AT)rE[2][tid] + (AT)rE[3][tid]);
    if (out) {
        out->rp = rowP; out->re = rowE;
#pragma unroll
        for (int c = 0; c < 4; ++c) { out->cp[c] = cP[c]; out->ce[c] = cE[c]; }
        return;
    }
    const bool p32 = a.part32 != 0;
    const size_t rowslot = ((size_t)tc.I * (NB + 1) + tc.J) * TILE + tid;
    put_part(a.partP, rowslot, rowP, p32);
    put_part(a.partE, rowslot, rowE, p32);
    if (g == 0) {
        const int slot = (tc.I < tc.J) ? tc.I : NB;
        const size_t cb = ((size_t)tc.J * (NB + 1) + slot) * TILE + col0;
#pragma unroll
        for (int c = 0; c < 4; ++c) { put_part(a.partP, cb + c, cP[c], p32); put_part(a.partE, cb + c, cE[c], p32); }
    }
}

template <class ST, class MT, class AT, int KSRC, int GK, int D, bool FIRST, int SER>
__global__ __launch_bounds__(WG) void k_sweep(SweepArgs a) {
    if (a.st->done) return;
    sweep_tile<ST, MT, AT, KSRC, GK, D, FIRST, SER>(a, blockIdx.x, a.slot_top);
}

// The sweeps chunk_plan selects (a.chunk = 2, single solves and served
// alike) run over 2 x 2 chunks of tiles; every other sweep takes one tile per
// workgroup.
template <class ST, class MT, class AT, int KSRC, int D, int SER>
constexpr bool chunk_sweep_ok() {
    return KSRC == KSRC_PLANE && std::is_same<ST, float>::value &&
           chunk_plan(std::is_same<AT, float>::value || MsgT<ST, MT, AT, SER>::F32, D, SER);
}

// Synchronous sweep over chunks of C x C tiles (a.chunks: Ic << 16 | Jc,
// Ic <= Jc; the diagonal chunk holds its tiles with I <= J).  One workgroup
// per chunk adds each row's sums over the chunk's columns and each column's
// over its rows before storing them: a chunk stores one partial vector per
// row block and per column block, where single tiles store two per tile
// (C = 2 halves the partial-sum bytes, which reach HBM in small write bursts
// between the K' stream's reads).  The slots of block K (Kc = K / C, NBc =
// ceil(NB / C)) are those of the single-tile scheme with chunks in place of
// blocks: s < Kc the column sums of chunk (s, Kc), s = Kc the row sums of the
// diagonal chunk, Kc < s < NBc the row sums of chunk (Kc, s), s = NBc the
// column sums of the diagonal chunk.  Sums over a chunk are kept in CT: FP32
// where the partials are stored in FP32.
template <class ST, class MT, class AT, int GK, int D, int SER, int C>
__device__ inline void sweep_chunk(const SweepArgs& a, int Ic, int Jc, int slot_top) {
    using CT = typename std::conditional<MsgT<ST, MT, AT, SER>::F32, float, AT>::type;
    const int NB = a.NB, NBc = (NB + C - 1) / C;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, g = l >> 4, q = l & 15;
    const int col0 = w * 64 + q * 4;
    const bool p32 = a.part32 != 0;
    // row sums per row block of the chunk, in LDS (each thread its own row);
    // the column sums stay in registers
    __shared__ CT rs[C][2][TILE];
#pragma unroll
    for (int ii = 0; ii < C; ++ii) { rs[ii][0][tid] = 0; rs[ii][1][tid] = 0; }
    bool first = true;
    // one copy of the tile code (loops not unrolled)
#pragma unroll 1
    for (int jj = 0; jj < C; ++jj) {
        const int J = Jc * C + jj;
        if (J >= NB) break;
        CT csP[4] = {0, 0, 0, 0}, csE[4] = {0, 0, 0, 0};
#pragma unroll 1
        for (int ii = 0; ii < C; ++ii) {
            const int I = Ic * C + ii;
            if (I > J) break;          // (I >= NB implies I > J)
            if (!first) __syncthreads();
            first = false;
            TileSums<AT> o;
            sweep_tile<ST, MT, AT, KSRC_PLANE, GK, D, false, SER>(a, tile_index(I, J, NB), slot_top, &o);
            rs[ii][0][tid] += (CT)o.rp;
            rs[ii][1][tid] += (CT)o.re;
#pragma unroll
            for (int c = 0; c < 4; ++c) { csP[c] += (CT)o.cp[c]; csE[c] += (CT)o.ce[c]; }
        }
        if (g == 0) {
            const int slot = (Ic < Jc) ? Ic : NBc;
            const size_t cb = ((size_t)J * (NBc + 1) + slot) * TILE + col0;
#pragma unroll
            for (int c = 0; c < 4; ++c) { put_part(a.partP, cb + c, (AT)csP[c], p32); put_part(a.partE, cb + c, (AT)csE[c], p32); }
        }
    }
#pragma unroll
    for (int ii = 0; ii < C; ++ii) {
        const int I = Ic * C + ii;
        if (I >= NB) break;
        const size_t o = ((size_t)I * (NBc + 1) + Jc) * TILE + tid;
        put_part(a.partP, o, (AT)rs[ii][0][tid], p32);
        put_part(a.partE, o, (AT)rs[ii][1][tid], p32);
    }
}

template <class ST, class MT, class AT, int GK, int D, int SER, int C>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_sweep_chunk(SweepArgs a) {
    if (a.st->done) return;
    const uint32_t cc = a.chunks[blockIdx.x];
    sweep_chunk<ST, MT, AT, GK, D, SER, C>(a, (int)(cc >> 16), (int)(cc & 0xFFFFu), a.slot_top);
}

// Stateless sweep with K' recomputed per band: the Gram fragments, the
// band's K' (LDS) and the recursion's per-column state share the registers;
// at least three waves per SIMD keep the band computations of some waves
// overlapping the message steps of others.
template <class ST, class MT, class AT, int GK, int D, int SER>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_sweep_rc(SweepArgs a) {
    if (a.st->done) return;
    sweep_tile<ST, MT, AT, KSRC_RECOMPUTE, GK, D, false, SER>(a, blockIdx.x, a.slot_top);
}

// ------------------------------------------------ grouped (Gauss-Seidel) --
//
// Grouped schedule: the block rows are split into G ordered groups and a
// sweep visits them in order; the visit of group g recomputes every message
// INTO a node of g and then refreshes g's aggregates.  One launch per visit
// walks a list of (tile, direction) entries (GE_* bits): FWD = the messages
// i -> j into the column block J, BWD = j -> i into the row block I.

// Version of the source aggregates used at chain level k (k = 0: the message
// computed now; level k + 1: the reverse message it consumes) for a visit in
// sweep t, as an offset from t.  A message computed at a visit uses its
// source's aggregates as they stand then, and the reverse message as last
// computed, at the latest earlier visit of the source's group:
//   FWD across groups (row group earlier): row t+1, col t, row t, col t-1, ...
//   BWD across groups (column group later): col t, row t, col t-1, row t-1, ...
//   inside the group (Jacobi within g): t, t-1, t-2, ... as in the
//   synchronous schedule.
__device__ inline int level_version_offset(bool fwd, bool within, int k) {
    if (within) return -k;
    return fwd ? ((k & 1) ? -((k - 1) >> 1) : 1 - (k >> 1)) : -(k >> 1);
}
// Sweep of the visit that computed the level-k message, as an offset from t
// (FWD across: t, t, t-1, t-1, ...; BWD across: t, t-1, t-1, t-2, ...;
// inside: t - k).  A level whose visit precedes sweep 0 carries the zero
// start message; across groups its source version can still be 0, so the
// ring's pre-sweep slots alone do not make it zero.
__device__ inline int level_visit_offset(bool fwd, bool within, int k) {
    if (within) return -k;
    return fwd ? -(k >> 1) : -((k + 1) >> 1);
}

// LDS of one single-direction visit, declared by the kernel so that both
// directions share it.
template <class MT, class LT, class AT, class RT, int NRL, int RECOMP, int KRN = 0>
struct DirSmem {
    static constexpr int RING_STEPS = KRN;
    // K' ring (stateless visits over an FP32 plane): KRN row steps per wave
    __attribute__((aligned(16))) float kring[KRN > 0 ? KRN : 1][4][KRN > 0 ? 256 : 4];
    MT topP[TILE], topS[TILE];            // row source at level 0 (FWD)
    LT lowP[NRL][TILE], lowS[NRL][TILE];  // row source at lower levels
    LT lowSI[NRL][TILE];                  // series: S / P~
    LT lowUQ[NRL][TILE];                  // series: (1/P~)^2
    RT rP[4][TILE], rE[4][TILE];          // BWD row partials per wave strip (exact in AT)
    RT red[4][2][2][64];                  // BWD stateless: two row steps of lane partials
    float kband[RECOMP ? 4 : 1][RECOMP ? 32 * 64 : 1];
};

template <class ST, class MT, class AT, int D, int SER>
struct DirTypes {
    using XT = typename MsgT<ST, MT, AT, SER>::T;
    static constexpr bool XF = MsgT<ST, MT, AT, SER>::F32;
    using LT = typename std::conditional<(SER && D <= 3) || std::is_same<ST, double>::value, XT, float>::type;
    using RT = typename std::conditional<XF, XT, AT>::type;    // row reduction type
    static constexpr int NRL = (D / 2 > 0) ? D / 2 : 1;   // lower row-side levels
    static constexpr int NCL = (D / 2 > 0) ? D / 2 : 1;   // lower column-side levels
};

// One direction of one tile.  D = 0: stored pair records (the reverse
// message is read from its plane, the new one written to the other);
// D >= 1: the chain of D levels is rebuilt from the aggregate ring, the
// reverse message below the deepest level taken as zero.  The source's
// aggregates at version v sit in ring slot v mod R (R = 1 for stored
// records: every read is the node's latest value).
template <class ST, class MT, class AT, int KSRC, int GK, int D, int SER, bool FWD, class SM>
__device__ inline void sweep_tile_dir(const SweepArgs& a, int64_t tile, bool within, int t, SM& sm) {
    using DT = DirTypes<ST, MT, AT, D, SER>;
    using LT = typename DT::LT;
    using XT = typename DT::XT;
    constexpr bool XF = DT::XF;
    constexpr bool STORED = (D == 0);
    constexpr int L = STORED ? 1 : D;
    DevStatus* st = a.st;
    const uint32_t ij = a.tiles[tile];
    const TileCoord tc{(int)(ij >> 16), (int)(ij & 0xFFFFu)};
    const int NB = a.NB;
    const size_t tbase = (size_t)tile * TT;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, g = l >> 4, q = l & 15;
    const int col0 = w * 64 + q * 4;
    const AT* HP = static_cast<const AT*>(a.HP);
    const AT* HS = static_cast<const AT*>(a.HS);
    const AT* HI = static_cast<const AT*>(a.HI);
    const AT* HM = static_cast<const AT*>(a.HM);
    const ST* Kp = static_cast<const ST*>(a.Kp);
    const uint32_t lo = (uint32_t)(g * TILE + col0);      // lane offset inside a row group
    // stateless visits over an FP32 K' plane (single solves): row steps
    // stream through the per-wave LDS ring as in the synchronous sweep, the
    // first KR issued first.  The served form keeps the one-step register
    // prefetch: its many small launches run more workgroups per CU without
    // the ring's LDS.
    constexpr bool RING = (SM::RING_STEPS > 0) && (KSRC == KSRC_PLANE) && !STORED && std::is_same<ST, float>::value;
    constexpr int KR = RING ? SM::RING_STEPS : 1;
    constexpr int SU = (RING && 8 % KR == 0) ? KR : 1;   // row steps unrolled (static ring slots)
    if constexpr (RING) {
#pragma unroll
        for (int u = 0; u < KR; ++u)
            dma16(reinterpret_cast<const float*>(Kp) + tbase + (size_t)u * 4 * TILE, lo * 4u,
                  lds_offset(&sm.kring[u][w][0]));
    }
    auto slot_of = [&](int k) -> int64_t {
        if constexpr (STORED) return 0;
        const int v = t + level_version_offset(FWD, within, k);
        return (int64_t)(((v % a.R) + a.R) % a.R) * a.NPAD;
    };

    // source data per level: row side in LDS (per row), column side in
    // registers (the lane's four columns)
    XT ctP[4], ctS[4];                           // column source at level 0 (BWD)
    LT clP[DT::NCL][4], clS[DT::NCL][4], clSI[SER ? DT::NCL : 1][4], clUQ[SER ? DT::NCL : 1][4];
#pragma unroll
    for (int k = 0; k < L; ++k) {
        const bool row_side = FWD ? !(k & 1) : (k & 1);
        const int64_t base = slot_of(k);
        // levels computed before sweep 0: P~ = inf, S = 0 give exactly zero messages
        const bool live = STORED || t + level_visit_offset(FWD, within, k) >= 0;
        // per node: P~ (or, series, 1/P~), S and (series) S/P~; the rings'
        // 1/P~ and S/P~ when the finalize formed them (the same quotients)
        auto node = [&](int64_t o, AT& pv, AT& sv, AT& mv) {
            AT p = HP[o], s = HS[o];
            if (!live) { p = (AT)INFINITY; s = 0; }
            sv = s;
            if constexpr (SER) {
                pv = (HI && live) ? HI[o] : (AT)1 / p;
                mv = (HM && live) ? HM[o] : s / p;
            } else {
                pv = p;
                mv = 0;
            }
        };
        if (row_side) {
            AT pv, sv, mv;
            node(base + (int64_t)tc.I * TILE + tid, pv, sv, mv);
            if (k == 0) {
                sm.topP[tid] = (XT)pv;
                sm.topS[tid] = (XT)sv;
            } else {
                const int m = FWD ? (k >> 1) - 1 : (k >> 1);
                sm.lowP[m][tid] = (LT)pv;
                sm.lowS[m][tid] = (LT)sv;
                if constexpr (SER) { sm.lowSI[m][tid] = (LT)mv; sm.lowUQ[m][tid] = (LT)(pv * pv); }
            }
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                AT pv, sv, mv;
                node(base + (int64_t)tc.J * TILE + col0 + c, pv, sv, mv);
                if (k == 0) {
                    ctP[c] = (XT)pv;
                    ctS[c] = (XT)sv;
                } else {
                    const int m = FWD ? (k >> 1) : (k >> 1) - 1;
                    clP[m][c] = (LT)pv;
                    clS[m][c] = (LT)sv;
                    if constexpr (SER) { clSI[m][c] = (LT)mv; clUQ[m][c] = (LT)(pv * pv); }
                }
            }
        }
    }
    AT cP[4] = {0, 0, 0, 0}, cE[4] = {0, 0, 0, 0};
    XT cPm[4] = {0, 0, 0, 0}, cEm[4] = {0, 0, 0, 0};   // XF: FP32 column sums over the tile's 256 rows
    bool bad = false;
    __syncthreads();

    // stored records: FWD reads the reverse plane (P_ji, E_ji) and writes
    // the forward one; BWD the other way round
    ST* Prd = static_cast<ST*>(FWD ? a.Pb : a.Pf);
    ST* Erd = static_cast<ST*>(FWD ? a.Eb : a.Ef);
    ST* Pwr = static_cast<ST*>(FWD ? a.Pf : a.Pb);
    ST* Ewr = static_cast<ST*>(FWD ? a.Ef : a.Eb);

    size_t off = tbase;                                   // wave-uniform row offset
    V4<ST> k4{}, pr{}, er{};
    if constexpr (KSRC == KSRC_PLANE && !RING) k4 = ld4nt(lane_ptr(Kp + off, lo));
    if constexpr (STORED) { pr = ld4nt(lane_ptr(Prd + off, lo)); er = ld4nt(lane_ptr(Erd + off, lo)); }

    for (int b = 0; b < TILE / 32; ++b) {
        if constexpr (KSRC == KSRC_RECOMPUTE) {
            gram_band<GK>(a.F, a.kp, tc.I, tc.J, 32 * b, 64 * w, sm.kband[w]);
            wave_lds_sync();
        }
#pragma unroll SU
        for (int s2 = 0; s2 < 8; ++s2) {
            const int r = 32 * b + 4 * s2 + g;
            const bool more = (b * 8 + s2 + 1) < TILE / 4;
            const size_t off2 = more ? off + 4 * TILE : off;
            V4<ST> k2, pr2, er2;
            const int u = b * 8 + s2;                 // row step
            if constexpr (RING) {
                if (u + KR <= TILE / 4) wait_vm<KR - 1>();
                else wait_vm<0>();
                const float4 kk = *reinterpret_cast<const float4*>(&sm.kring[u % KR][w][4 * l]);
                k4 = V4<ST>{{(ST)kk.x, (ST)kk.y, (ST)kk.z, (ST)kk.w}};
            } else if constexpr (KSRC == KSRC_PLANE) {
                k2 = ld4nt(lane_ptr(Kp + off2, lo));
            }
            if constexpr (STORED) { pr2 = ld4nt(lane_ptr(Prd + off2, lo)); er2 = ld4nt(lane_ptr(Erd + off2, lo)); }
            if constexpr (KSRC == KSRC_RECOMPUTE) {
                const float4 kk = *reinterpret_cast<const float4*>(&sm.kband[w][(4 * s2 + g) * 64 + 4 * q]);
                k4 = V4<ST>{{(ST)kk.x, (ST)kk.y, (ST)kk.z, (ST)kk.w}};
            }
            AT rp = 0, re = 0;
            XT rpm = 0, rem = 0;                         // XF: FP32 row sums (4 columns, then 64 per wave)
            V4<ST> np, ne;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const XT av = (XT)k4.v[c];
                // reverse message consumed by the top level
                XT opr, oer;
                if constexpr (STORED) {
                    opr = (XT)pr.v[c]; oer = (XT)er.v[c];
                } else {
                    const LT al = (LT)k4.v[c], a2l = al * al;
                    LT lp = 0, le = 0;
#pragma unroll
                    for (int k = L - 1; k >= 1; --k) {
                        const bool row_side = FWD ? !(k & 1) : (k & 1);
                        const int mr = FWD ? (k >> 1) - 1 : (k >> 1);
                        const int mc = FWD ? (k >> 1) : (k >> 1) - 1;
                        const LT pv = row_side ? sm.lowP[mr][r] : clP[mc][c];
                        const LT sv = row_side ? sm.lowS[mr][r] : clS[mc][c];
                        if constexpr (SER) {
                            // G = P / (-a^2) and F = E / a (as in the synchronous sweep)
                            if (k == L - 1) {            // deepest: reverse message zero
                                const LT siv = row_side ? sm.lowSI[mr][r] : clSI[mc][c];
                                lp = pv;
                                le = -siv;
                            } else {
                                LT ng;
                                if constexpr (SER == 3) {       // G = u (no series term)
                                    ng = pv;
                                } else {
                                    const LT uq = row_side ? sm.lowUQ[mr][r] : clUQ[mc][c];
                                    ng = fma(-a2l * uq, lp, pv);
                                }
                                const LT nf = ng * fma(al, le, -sv);
                                lp = ng; le = nf;
                            }
                        } else {
                            const LT qv = pv - lp;
                            bad |= !(qv > (LT)0);
                            const LT rv = rcp_fast(qv);
                            const LT np_ = -a2l * rv;
                            const LT ne_ = -al * (sv - le) * rv;
                            lp = np_; le = ne_;
                        }
                    }
                    opr = (XT)lp; oer = (XT)le;
                }
                // top level: the message into the target, from the source at level 0
                const XT pt = FWD ? sm.topP[r] : ctP[c];
                const XT sv = FWD ? sm.topS[r] : ctS[c];
                XT pm, em;
                if constexpr (SER) {
                    // opr, oer hold G, F of the reverse message here
                    const XT a2 = av * av;
                    const XT e = -(a2 * opr) * pt;
                    XT gt;
                    if constexpr (SER == 2) gt = fma(pt, fma(e, e, e), pt);
                    else gt = fma(pt, e, pt);
                    pm = -a2 * gt;
                    em = (av * gt) * fma(av, oer, -sv);
                } else {
                    const XT qv = pt - opr;
                    bad |= !(qv > (XT)0);
                    const XT rv = rcp_fast(qv);
                    pm = -(av * av) * rv;
                    em = -av * (sv - oer) * rv;
                }
                if constexpr (STORED) {
                    const ST ps = (ST)pm, es = (ST)em;
                    np.v[c] = ps; ne.v[c] = es;
                    if constexpr (FWD) { cP[c] += (AT)ps; cE[c] += (AT)es; }
                    else { rp += (AT)ps; re += (AT)es; }
                } else if constexpr (XF) {
                    if constexpr (FWD) { cPm[c] += pm; cEm[c] += em; }
                    else { rpm += pm; rem += em; }
                } else {
                    if constexpr (FWD) { cP[c] += (AT)pm; cE[c] += (AT)em; }
                    else { rp += (AT)pm; re += (AT)em; }
                }
            }
            if constexpr (STORED) { st4nt(lane_ptr(Pwr + off, lo), np); st4nt(lane_ptr(Ewr + off, lo), ne); }
            if constexpr (!FWD && STORED) {
                rp = sum16(rp);
                re = sum16(re);
                if (q == 0) { sm.rP[w][r] = rp; sm.rE[w][r] = re; }
            } else if constexpr (!FWD) {
                // row sums over the 16 column lanes through LDS every two row
                // steps (same scheme as the synchronous stateless sweep)
                using RT = typename DT::RT;
                sm.red[w][0][s2 & 1][l] = XF ? (RT)rpm : (RT)rp;
                sm.red[w][1][s2 & 1][l] = XF ? (RT)rem : (RT)re;
                if (s2 & 1) {
                    wave_lds_sync();
                    const int qty = l >> 5, idx = l & 31, stp = idx >> 4, gg = (idx >> 2) & 3, pt = idx & 3;
                    const RT* src = &sm.red[w][qty][stp][16 * gg + 4 * pt];
                    RT v = (src[0] + src[1]) + (src[2] + src[3]);
                    v = v + dpp<0xB1>(v);
                    v = v + dpp<0x4E>(v);
                    const int row = 32 * b + 4 * ((s2 & 6) + stp) + gg;
                    if (pt == 0) {
                        if (qty == 0) sm.rP[w][row] = v;
                        else sm.rE[w][row] = v;
                    }
                    wave_lds_sync();
                }
            }
            if constexpr (RING) {
                // the slot's next row step (k4 was read from it and used above)
                if (u + KR < TILE / 4)
                    dma16(reinterpret_cast<const float*>(Kp) + tbase + (size_t)(u + KR) * 4 * TILE, lo * 4u,
                          lds_offset(&sm.kring[u % KR][w][0]));
            } else if constexpr (KSRC == KSRC_PLANE) {
                k4 = k2;
            }
            if constexpr (STORED) { pr = pr2; er = er2; }
            off = off2;
        }
        if constexpr (KSRC == KSRC_RECOMPUTE) wave_lds_sync();
    }
    const bool p32 = a.part32 != 0;
    if constexpr (FWD) {
        if constexpr (XF) {
#pragma unroll
            for (int c = 0; c < 4; ++c) { cP[c] = (AT)cPm[c]; cE[c] = (AT)cEm[c]; }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) { cP[c] = sum_groups(cP[c]); cE[c] = sum_groups(cE[c]); }
        if (g == 0) {
            const int slot = (tc.I < tc.J) ? tc.I : NB;
            const size_t cb = ((size_t)tc.J * (NB + 1) + slot) * TILE + col0;
#pragma unroll
            for (int c = 0; c < 4; ++c) { put_part(a.partP, cb + c, cP[c], p32); put_part(a.partE, cb + c, cE[c], p32); }
        }
    } else {
        __syncthreads();
        const size_t rowslot = ((size_t)tc.I * (NB + 1) + tc.J) * TILE + tid;
        put_part(a.partP, rowslot, ((AT)sm.rP[0][tid] + (AT)sm.rP[1][tid]) + ((AT)sm.rP[2][tid] + (AT)sm.rP[3][tid]), p32);
        put_part(a.partE, rowslot, ((AT)sm.rE[0][tid] + (AT)sm.rE[1][tid]) + ((AT)sm.rE[2][tid] + (AT)sm.rE[3][tid]), p32);
    }
    if (__any(bad) && l == 0) st->bad = 1;
}

// One visit of the grouped schedule over the entries list[0, n).
template <class ST, class MT, class AT, int KSRC, int GK, int D, int SER>
__global__ __launch_bounds__(WG) void k_sweep_dir(SweepArgs a, const uint32_t* __restrict__ list, int t) {
    using DT = DirTypes<ST, MT, AT, D, SER>;
    __shared__ DirSmem<typename DT::XT, typename DT::LT, AT, typename DT::RT, DT::NRL, KSRC == KSRC_RECOMPUTE,
                       (KSRC == KSRC_PLANE && D >= 1 && std::is_same<ST, float>::value) ? KRING : 0> sm;
    if (a.st->done) return;
    const uint32_t e = list[blockIdx.x];
    const int64_t tile = (int64_t)(e & GE_TILE);
    const bool within = (e & GE_WITHIN) != 0;
    if (e & GE_BWD) sweep_tile_dir<ST, MT, AT, KSRC, GK, D, SER, false>(a, tile, within, t, sm);
    else sweep_tile_dir<ST, MT, AT, KSRC, GK, D, SER, true>(a, tile, within, t, sm);
}

// Served grouped visit: items are (request, list entry) pairs of every
// request's current group, built by the host per step; the sweep index of a
// request is its own count of completed sweeps.
template <class ST, class MT, class AT, int D, int SER>
__global__ __launch_bounds__(WG) void k_sweep_dir_batched(const ReqDesc* __restrict__ reqs,
                                                         const uint2* __restrict__ items, int nitems) {
    using DT = DirTypes<ST, MT, AT, D, SER>;
    __shared__ DirSmem<typename DT::XT, typename DT::LT, AT, typename DT::RT, DT::NRL, 0> sm;
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const uint2 w = items[it];
        const ReqDesc& rd = reqs[w.x];
        const DevStatus* st = rd.sw.st;
        if (st->done) continue;
        const uint32_t e = w.y;
        const int64_t tile = (int64_t)(e & GE_TILE);
        const bool within = (e & GE_WITHIN) != 0;
        if (e & GE_BWD) sweep_tile_dir<ST, MT, AT, KSRC_PLANE, GRAM_F32, D, SER, false>(rd.sw, tile, within, st->t, sm);
        else sweep_tile_dir<ST, MT, AT, KSRC_PLANE, GRAM_F32, D, SER, true>(rd.sw, tile, within, st->t, sm);
        __syncthreads();
    }
}

// Stored records inside a group: both directions from the previous values
// (Jacobi within the group), over the listed tiles.
template <class ST, class MT, class AT, int KSRC, int GK>
__global__ __launch_bounds__(WG) void k_sweep_listed(SweepArgs a, const uint32_t* __restrict__ list) {
    if (a.st->done) return;
    sweep_tile<ST, MT, AT, KSRC, GK, 0, false, 0>(a, (int64_t)(list[blockIdx.x] & GE_TILE), 0);
}

// Served form: one persistent grid walks the union work list of (request,
// tile) items of the active requests of one group (same precision, edge
// state and level count).  Each request keeps its own planes or aggregate
// ring, partial sums and status, so its arithmetic does not depend on the
// mix; the ring slot of the previous sweep follows from the request's own
// sweep count (ring slots of the sweeps before sweep 0 hold P~ = inf, S = 0,
// so a fixed level count is exact from the first sweep).
template <class ST, class MT, class AT, int D, int SER>
__global__ __launch_bounds__(WG) void k_sweep_batched(const ReqDesc* __restrict__ reqs,
                                                     const uint2* __restrict__ items, int nitems) {
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const uint2 w = items[it];
        const ReqDesc& rd = reqs[w.x];
        const DevStatus* st = rd.sw.st;
        if (st->done) continue;
        sweep_tile<ST, MT, AT, KSRC_PLANE, GRAM_F32, D, false, SER>(rd.sw, (int64_t)w.y, st->t % rd.sw.R);
        __syncthreads();
    }
}

// Launch groups whose plan may run over 2 x 2 chunks of tiles: a request
// whose single solve takes chunks (sw.chunk = 2) takes the same chunks here
// (items (request, Ic << 16 | Jc)), so that both sum in the same order; the
// others take whole tiles (items (request, tile)).
template <class ST, class MT, class AT, int D, int SER>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_sweep_batched_chunk(
    const ReqDesc* __restrict__ reqs, const uint2* __restrict__ items, int nitems) {
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const uint2 w = items[it];
        const ReqDesc& rd = reqs[w.x];
        const DevStatus* st = rd.sw.st;
        if (st->done) continue;
        if (rd.sw.chunk > 1)
            sweep_chunk<ST, MT, AT, GRAM_F32, D, SER, 2>(rd.sw, (int)(w.y >> 16), (int)(w.y & 0xFFFFu), st->t % rd.sw.R);
        else
            sweep_tile<ST, MT, AT, KSRC_PLANE, GRAM_F32, D, false, SER>(rd.sw, (int64_t)w.y, st->t % rd.sw.R);
        __syncthreads();
    }
}

// Run-time (levels, reciprocal form) of a stateless launch to the
// compile-time pair (D, SER): exact reciprocals up to 8 levels, the series
// (one- or two-term top level) up to 6.  Every pair is its own
// instantiation, so the level loops are fully unrolled and branch-free.
template <class F>
inline hipError_t with_stateless(int levels, int ser, F&& f) {
    using std::integral_constant;
#define GABP_SL(S_, L_) \
    case S_ * 16 + L_: f(integral_constant<int, L_>{}, integral_constant<int, S_>{}); return hipSuccess;
    switch (ser * 16 + levels) {
        GABP_SL(0, 1) GABP_SL(0, 2) GABP_SL(0, 3) GABP_SL(0, 4) GABP_SL(0, 5) GABP_SL(0, 6) GABP_SL(0, 7) GABP_SL(0, 8)
        GABP_SL(1, 1) GABP_SL(1, 2) GABP_SL(1, 3) GABP_SL(1, 4) GABP_SL(1, 5) GABP_SL(1, 6)
        GABP_SL(2, 1) GABP_SL(2, 2) GABP_SL(2, 3) GABP_SL(2, 4) GABP_SL(2, 5) GABP_SL(2, 6)
        GABP_SL(3, 3) GABP_SL(3, 4) GABP_SL(3, 5) GABP_SL(3, 6)
        default: return hipErrorInvalidValue;
    }
#undef GABP_SL
}

template <class ST, class MT, class AT, int D, int SER>
inline void served_d(bool grouped, const ReqDesc* reqs, const uint2* items, int n, hipStream_t s) {
    const int g = std::max(1, std::min(n, 2048));
    if (grouped)
        hipLaunchKernelGGL((k_sweep_dir_batched<ST, MT, AT, D, SER>), dim3(g), dim3(WG), 0, s, reqs, items, n);
    else if constexpr (chunk_sweep_ok<ST, MT, AT, KSRC_PLANE, D, SER>())
        hipLaunchKernelGGL((k_sweep_batched_chunk<ST, MT, AT, D, SER>), dim3(g), dim3(WG), 0, s, reqs, items, n);
    else
        hipLaunchKernelGGL((k_sweep_batched<ST, MT, AT, D, SER>), dim3(g), dim3(WG), 0, s, reqs, items, n);
}

// levels 0: stored pair records; 1..8 stateless (1..6 with the series);
// grouped: the single-direction entries of one group visit (items
// (request, entry)); otherwise whole tiles (items (request, tile)).
template <class ST, class MT, class AT>
inline hipError_t served_sweep(int levels, int ser, bool grouped, const ReqDesc* reqs, const uint2* items, int n,
                               hipStream_t s) {
    if (levels == 0) {
        served_d<ST, MT, AT, 0, 0>(grouped, reqs, items, n, s);
        return hipGetLastError();
    }
    const hipError_t e = with_stateless(levels, ser, [&](auto L_, auto S_) {
        served_d<ST, MT, AT, decltype(L_)::value, decltype(S_)::value>(grouped, reqs, items, n, s);
    });
    return e != hipSuccess ? e : hipGetLastError();
}

// Launches `kern` on `s`. With an event pair the events take the dispatch's
// own begin and end timestamps (no marker packets around the kernel, so the
// span is the kernel's duration alone); without, a plain launch.
template <class K, class... Args>
inline void launch_ev(K kern, dim3 g, dim3 b, hipStream_t s, hipEvent_t e0, hipEvent_t e1, Args... args) {
    if (e0)
        hipExtLaunchKernelGGL(kern, g, b, 0, s, e0, e1, 0, args...);
    else
        hipLaunchKernelGGL(kern, g, b, 0, s, args...);
}

// ---- sweep dispatch: precision x K' source x Gram kind x depth x first x series

template <class ST, class MT, class AT, int KSRC, int GK, int D, int SER>
inline hipError_t sweep_d(bool first, const SweepArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    const dim3 g((unsigned)a.ntiles), blk(WG);
    if (a.chunk > 1) {
        if constexpr (chunk_sweep_ok<ST, MT, AT, KSRC, D, SER>()) {
            if (a.chunk != 2 || a.chunks == nullptr || a.nchunks <= 0) return hipErrorInvalidValue;
            launch_ev(k_sweep_chunk<ST, MT, AT, GK, D, SER, 2>, dim3((unsigned)a.nchunks), blk, s, e0, e1, a);
            return hipSuccess;
        } else {
            return hipErrorInvalidValue;
        }
    }
    if constexpr (D == 0) {
        if (first) {
            launch_ev(k_sweep<ST, MT, AT, KSRC, GK, D, true, 0>, g, blk, s, e0, e1, a);
            return hipSuccess;
        }
    }
    if constexpr (KSRC == KSRC_RECOMPUTE && D >= 1)
        launch_ev(k_sweep_rc<ST, MT, AT, GK, D, SER>, g, blk, s, e0, e1, a);
    else
        launch_ev(k_sweep<ST, MT, AT, KSRC, GK, D, false, SER>, g, blk, s, e0, e1, a);
    return hipSuccess;
}

// `levels` = 0: stored edge state; >= 1: stateless with exactly that many
// levels; `ser`: 0 exact reciprocals, 1 / 2 series with a one- / two-term
// top level. e0 / e1 (optional): timestamps of the launch.
template <class ST, class MT, class AT, int KSRC, int GK>
inline hipError_t sweep_depth(int levels, bool first, int ser, const SweepArgs& a, hipStream_t s, hipEvent_t e0,
                              hipEvent_t e1) {
    if (levels == 0) {
        const hipError_t e = sweep_d<ST, MT, AT, KSRC, GK, 0, 0>(first, a, s, e0, e1);
        return e != hipSuccess ? e : hipGetLastError();
    }
    hipError_t ed = hipSuccess;
    const hipError_t e = with_stateless(levels, ser, [&](auto L_, auto S_) {
        ed = sweep_d<ST, MT, AT, KSRC, GK, decltype(L_)::value, decltype(S_)::value>(first, a, s, e0, e1);
    });
    if (e != hipSuccess) return e;
    return ed != hipSuccess ? ed : hipGetLastError();
}

// ---- grouped schedule dispatch: one group visit
template <class ST, class MT, class AT, int KSRC, int GK, int D, int SER>
inline void grouped_d(const SweepArgs& a, const uint32_t* list, int n, int t, hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL((k_sweep_dir<ST, MT, AT, KSRC, GK, D, SER>), dim3((unsigned)n), dim3(WG), 0, s, a, list, t);
}

// Stored records (levels 0): the tiles inside the group in `within` (both
// directions), the others in `dir`; stateless: every entry in `dir`.
template <class ST, class MT, class AT, int KSRC, int GK>
inline hipError_t sweep_grouped(int levels, int ser, const SweepArgs& a, const uint32_t* within, int nwithin,
                                const uint32_t* dir, int ndir, int t, hipStream_t s) {
    if (levels == 0) {
        if (nwithin > 0)
            hipLaunchKernelGGL((k_sweep_listed<ST, MT, AT, KSRC, GK>), dim3((unsigned)nwithin), dim3(WG), 0, s, a,
                               within);
        grouped_d<ST, MT, AT, KSRC, GK, 0, 0>(a, dir, ndir, t, s);
        return hipGetLastError();
    }
    const hipError_t e = with_stateless(levels, ser, [&](auto L_, auto S_) {
        grouped_d<ST, MT, AT, KSRC, GK, decltype(L_)::value, decltype(S_)::value>(a, dir, ndir, t, s);
    });
    return e != hipSuccess ? e : hipGetLastError();
}

}  // namespace gabp
