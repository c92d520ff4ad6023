// Kernels and C ABI of the learned warm start's U-Net (declared in include/unet.h).
//
// Activations are NHWC bfloat16 (raw 16-bit patterns).  The 3x3 convolutions are
// implicit GEMMs on the gfx950 matrix cores (v_mfma_f32_16x16x32_bf16: FP32
// accumulation of bfloat16 products): rows are pixels, columns output channels,
// the reduction runs over (tap, input channel).  Operand layout of that instruction
// for lane l of a wavefront: A row l%16, reduction indices 8(l/16)..8(l/16)+7; B
// column l%16, the same reduction indices; result rows 4(l/16)..4(l/16)+3, column
// l%16.  With channels innermost, each lane's 8 reduction values are 8 consecutive
// channels of one pixel: one 16-byte load.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <mutex>
#include <string>

#include "../../include/unet.h"

namespace unet_dev {
namespace {

typedef uint16_t bf16_t;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

__device__ __forceinline__ float bf2f(uint32_t h) { return __uint_as_float(h << 16); }

// round to nearest even; NaN stays NaN
__device__ __forceinline__ uint32_t f2bf(float f) {
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (u >> 16) | ((u & 0xffffu) ? 0x40u : 0u);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

// round to nearest even with the gfx950 conversion instruction (same result as f2bf
// for every finite value)
__device__ __forceinline__ uint32_t f2bf_hw(float f) {
    return (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)f);
}

__device__ __forceinline__ uint4 ld16(const bf16_t* p) { return *reinterpret_cast<const uint4*>(p); }
__device__ __forceinline__ void st16(bf16_t* p, uint4 v) { *reinterpret_cast<uint4*>(p) = v; }

__device__ __forceinline__ float lo(uint32_t w) { return bf2f(w & 0xffffu); }
__device__ __forceinline__ float hi(uint32_t w) { return bf2f(w >> 16); }
__device__ __forceinline__ uint32_t pack(float a, float b) { return f2bf(a) | (f2bf(b) << 16); }

__device__ __forceinline__ void unpack8(uint4 v, float* f) {
    f[0] = lo(v.x); f[1] = hi(v.x); f[2] = lo(v.y); f[3] = hi(v.y);
    f[4] = lo(v.z); f[5] = hi(v.z); f[6] = lo(v.w); f[7] = hi(v.w);
}
__device__ __forceinline__ uint4 pack8(const float* f) {
    return make_uint4(pack(f[0], f[1]), pack(f[2], f[3]), pack(f[4], f[5]), pack(f[6], f[7]));
}

__device__ __forceinline__ bf16x8 as_frag(uint4 v) { return __builtin_bit_cast(bf16x8, v); }

// Logical index of workgroup b of nb: the hardware deals workgroups to the 8 XCDs
// round-robin (b mod 8), and this gives each XCD a contiguous range of logical
// indices, so workgroups that read the same rows (neighbouring pixel tiles, the
// tiles of one pixel slab) share that XCD's L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int q = nb >> 3, r = nb & 7, x = b & 7, slot = b >> 3;
    return x * q + min(x, r) + slot;
}
__device__ __forceinline__ uint4 sel(bool keep, uint4 v) {
    return keep ? v : make_uint4(0u, 0u, 0u, 0u);
}

// ---------------------------------------------------------------------------
// 3x3 convolution (forward; also the input gradient with flipped weights)
// ---------------------------------------------------------------------------
// The input may be the channel concatenation of two tensors and the output may go to
// two: input channels below `split` come from x (at half the size when `half`: the
// nearest-neighbour 2x upsampling), the rest from x2; output channels below `ysplit`
// go to y, the rest to y2.  One tensor each: split = C_in, ysplit = C_out.
struct ConvArgs {
    const bf16_t* x;      // offset applied
    const bf16_t* x2;     // offset applied (channels split ..)
    const bf16_t* w;      // [C_out][9 C_in]
    const float* bias;    // nullable
    void* y;              // offset applied (elements of the output type)
    void* y2;             // offset applied (channels ysplit ..)
    const bf16_t* mask;   // nullable, offset applied
    // 2x2 work on the output tile (k_conv_halo only): down = 1 also stores the 2x2 max
    // pooling of the stored output to yp (half size); down = 2 stores, for the output
    // channels below ysplit, the upsampling gradient (2x2 sums, zeroed where gate <= 0)
    // to y at half size instead of the full-size output
    void* yp;
    const bf16_t* gate;
    int ldx, ldx2, ldy, ldy2, ldm, ldyp, ldgt, down;
    int split, half, ysplit;
    int lh, lw;           // log2 H, log2 W
    int P;                // N H W
    int Cin, Cout, relu;
};

// Flat index at half the size of full-size pixel p: (y, x) of image n reads (y / 2, x / 2)
// of image n (nearest-neighbour 2x upsampling).
__device__ __forceinline__ int half_px(int p, int lh, int lw) {
    const int x = p & ((1 << lw) - 1), y = (p >> lw) & ((1 << lh) - 1), n = p >> (lh + lw);
    return (n << (lh + lw - 2)) + ((y >> 1) << (lw - 1)) + (x >> 1);
}

// Address of input channels ch .. ch + 7 of full-size pixel p (ch and split are
// multiples of 8, so a vector of 8 channels never straddles the two tensors).
template <class Args>
__device__ __forceinline__ const bf16_t* src_at(const Args& a, int p, int ch) {
    if (ch < a.split) return a.x + (size_t)(a.half ? half_px(p, a.lh, a.lw) : p) * a.ldx + ch;
    return a.x2 + (size_t)p * a.ldx2 + (ch - a.split);
}

// Source of the 32-channel block at c0 in the tiled kernels, uniform across a workgroup
// (there C_in % 32 == 0 and split % 32 == 0 when the input has two tensors), and the
// pixel it reads for full-size image offset img, row yy, column xx.
struct BlockSrc {
    const bf16_t* p;
    int ld;
    bool half;
};
template <class Args>
__device__ __forceinline__ BlockSrc block_src(const Args& a, int c0) {
    if (c0 < a.split) return BlockSrc{a.x + c0, a.ldx, a.half != 0};
    return BlockSrc{a.x2 + (c0 - a.split), a.ldx2, false};
}
__device__ __forceinline__ const bf16_t* block_at(const BlockSrc& b, int img, int yy, int xx, int lw) {
    const int q = b.half ? (img >> 2) + ((yy >> 1) << (lw - 1)) + (xx >> 1) : img + (yy << lw) + xx;
    return b.p + (size_t)q * b.ld;
}

// Address of output channel co (and the next 7 for vector stores) of pixel p.
template <class T>
__device__ __forceinline__ T* dst_at(const ConvArgs& a, size_t p, int co) {
    if (co < a.ysplit) return static_cast<T*>(a.y) + p * a.ldy + co;
    return static_cast<T*>(a.y2) + p * a.ldy2 + (co - a.ysplit);
}

// A wavefront computes (16 MT) pixels x (16 NT) output channels; a workgroup of four
// wavefronts covers 64 MT consecutive pixels.  kTapOuter (C_in % 32 == 0): each
// 32-wide reduction chunk lies inside one tap, so the tap loop is outside and the
// per-lane pixel addresses are computed once per tap.  Out-of-range pixels and
// channels load from a valid address and are zeroed by a select (no branches around
// the loads).
template <int MT, int NT, bool kTapOuter, bool kF32>
__global__ void __launch_bounds__(256) k_conv3x3(const ConvArgs a) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row = lane & 15, grp = lane >> 4;
    const int p0 = (blockIdx.x * 4 + wave) * (16 * MT);
    const int co0 = blockIdx.y * (16 * NT);
    const int Hm = (1 << a.lh) - 1, Wm = (1 << a.lw) - 1;
    const int K = 9 * a.Cin;
    int pimg[MT], py[MT], px[MT];
    bool pv[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        int p = p0 + 16 * m + row;
        pv[m] = p < a.P;
        if (!pv[m]) p = 0;
        px[m] = p & Wm;
        py[m] = (p >> a.lw) & Hm;
        pimg[m] = (p >> (a.lw + a.lh)) << (a.lw + a.lh);
    }
    const bf16_t* wrow[NT];
    bool cv[NT];
#pragma unroll
    for (int n = 0; n < NT; ++n) {
        const int co = co0 + 16 * n + row;
        cv[n] = co < a.Cout;
        wrow[n] = a.w + (size_t)(cv[n] ? co : 0) * K;
    }
    f32x4 acc[MT][NT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};

    if (kTapOuter) {
        for (int tap = 0; tap < 9; ++tap) {
            const int dy = tap / 3 - 1, dx = tap - 3 * (tap / 3) - 1;
            int pa[MT];
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                const int ys = (py[m] + dy) & Hm, xs = (px[m] + dx) & Wm;
                pa[m] = pimg[m] + (ys << a.lw) + xs;
            }
            const int kb = tap * a.Cin + 8 * grp;
            for (int c = 0; c < a.Cin; c += 32) {
                uint4 A[MT], B[NT];
#pragma unroll
                for (int m = 0; m < MT; ++m) A[m] = ld16(src_at(a, pa[m], c + 8 * grp));
#pragma unroll
                for (int n = 0; n < NT; ++n) B[n] = ld16(wrow[n] + kb + c);
#pragma unroll
                for (int m = 0; m < MT; ++m) A[m] = sel(pv[m], A[m]);
#pragma unroll
                for (int n = 0; n < NT; ++n) B[n] = sel(cv[n], B[n]);
#pragma unroll
                for (int m = 0; m < MT; ++m)
#pragma unroll
                    for (int n = 0; n < NT; ++n)
                        acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_frag(A[m]), as_frag(B[n]),
                                                                            acc[m][n], 0, 0, 0);
            }
        }
    } else {
        for (int kc = 0; kc < K; kc += 32) {
            const int k0 = kc + 8 * grp;
            const bool kv = k0 < K;
            const int tap = kv ? k0 / a.Cin : 0;
            const int ci = kv ? k0 - tap * a.Cin : 0;
            const int dy = tap / 3 - 1, dx = tap - 3 * (tap / 3) - 1;
            uint4 A[MT], B[NT];
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                const int ys = (py[m] + dy) & Hm, xs = (px[m] + dx) & Wm;
                A[m] = ld16(src_at(a, pimg[m] + (ys << a.lw) + xs, ci));
            }
#pragma unroll
            for (int n = 0; n < NT; ++n) B[n] = ld16(wrow[n] + (kv ? k0 : 0));
#pragma unroll
            for (int m = 0; m < MT; ++m) A[m] = sel(pv[m] && kv, A[m]);
#pragma unroll
            for (int n = 0; n < NT; ++n) B[n] = sel(cv[n] && kv, B[n]);
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int n = 0; n < NT; ++n)
                    acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_frag(A[m]), as_frag(B[n]), acc[m][n],
                                                                        0, 0, 0);
        }
    }

#pragma unroll
    for (int n = 0; n < NT; ++n) {
        const int co = co0 + 16 * n + row;
        if (co >= a.Cout) continue;
        const float b = a.bias ? a.bias[co] : 0.f;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int p = p0 + 16 * m + 4 * grp + r;
                if (p >= a.P) continue;
                float v = acc[m][n][r] + b;
                if (a.relu) v = fmaxf(v, 0.f);
                if (a.mask && !(bf2f(a.mask[(size_t)p * a.ldm + co]) > 0.f)) v = 0.f;
                if (kF32) *dst_at<float>(a, p, co) = v;
                else *dst_at<bf16_t>(a, p, co) = (bf16_t)f2bf(v);
            }
        }
    }
}

// LDS-staged form of the same convolution for C_in % 32 == 0, P % BM == 0 and
// C_out % BN == 0.  A workgroup owns BM pixels x BN output channels and walks the
// reduction in 32-wide chunks (one tap, 32 input channels).  Each chunk's pixel rows
// (periodically shifted for the tap) and weight rows are loaded once per workgroup
// with 16-byte loads, stored to LDS, and read back by the four wavefronts as MFMA
// fragments; the next chunk's global loads are in flight while the current chunk's
// MFMAs run (two LDS buffers, one barrier per chunk).  Wavefronts are arranged
// WM x WN over the tile.  An LDS row holds the 32 channels of one pixel (or weight
// row) as four 16-byte pieces, piece j stored at slot j ^ ((row >> 1) & 3): the
// 16-byte accesses of 8 consecutive lanes (8 rows of one piece for the fragment
// reads, 2 rows of 4 pieces for the stores) then fall in 8 distinct 16-byte bank
// groups.  The accumulation order per output is the chunk order (tap, channel
// block), as in k_conv3x3.
__device__ __forceinline__ int swz(int row, int piece) { return 8 * (piece ^ ((row >> 1) & 3)); }

template <int BM, int BN, int WM, int WN, bool kF32>
__global__ void __launch_bounds__(256) k_conv_lds(const ConvArgs a) {
    static_assert(WM * WN == 4, "four wavefronts");
    static_assert(BM % 64 == 0 && BN % 16 == 0, "the loader moves 64 rows of 4 vectors per pass");
    constexpr int WTM = BM / WM, WTN = BN / WN, MT = WTM / 16, NT = WTN / 16;
    constexpr int AV = BM / 64;              // 16-byte A vectors per thread per chunk
    constexpr int BV = (BN + 63) / 64;       // B vectors per thread (some threads idle for BN = 32)
    constexpr int AS = BM * 32, BS = BN * 32;
    constexpr int OP = BN + 8;               // pitch of the bf16 output tile staged at the end
    constexpr int SM = 2 * (AS + BS) > BM * OP ? 2 * (AS + BS) : BM * OP;
    __shared__ __attribute__((aligned(16))) bf16_t sm[SM];
    bf16_t(*As)[BM][32] = reinterpret_cast<bf16_t(*)[BM][32]>(sm);
    bf16_t(*Bs)[BN][32] = reinterpret_cast<bf16_t(*)[BN][32]>(sm + 2 * AS);
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    // flat grid: the column tiles of one pixel tile are adjacent, pixel tiles follow in order
    const int ctiles = a.Cout / BN, L = xcd_block(blockIdx.x, gridDim.x);
    const int p0 = (L / ctiles) * BM, co0 = (L % ctiles) * BN;
    const int Hm = (1 << a.lh) - 1, Wm = (1 << a.lw) - 1;
    const int K = 9 * a.Cin, cpt = a.Cin >> 5, nch = 9 * cpt;
    // loader roles: channels 8 lv .. 8 lv + 7 of the chunk, rows lr + 64 j
    const int lv = t & 3, lr = t >> 2;
    int pimg[AV], py[AV], px[AV];
#pragma unroll
    for (int j = 0; j < AV; ++j) {
        const int p = p0 + lr + 64 * j;
        px[j] = p & Wm;
        py[j] = (p >> a.lw) & Hm;
        pimg[j] = (p >> (a.lw + a.lh)) << (a.lw + a.lh);
    }
    const bf16_t* wrow[BV];
    bool bon[BV];
#pragma unroll
    for (int j = 0; j < BV; ++j) {
        const int r = lr + 64 * j;
        bon[j] = r < BN;
        wrow[j] = a.w + (size_t)(co0 + (bon[j] ? r : 0)) * K + 8 * lv;
    }
    uint4 ra[AV], rb[BV];
    auto load = [&](int ch) {
        const int tap = ch / cpt, c0 = (ch - tap * cpt) << 5;
        const int dy = tap / 3 - 1, dx = tap - 3 * (tap / 3) - 1;
        const BlockSrc src = block_src(a, c0);
#pragma unroll
        for (int j = 0; j < AV; ++j) {
            const int ys = (py[j] + dy) & Hm, xs = (px[j] + dx) & Wm;
            ra[j] = ld16(block_at(src, pimg[j], ys, xs, a.lw) + 8 * lv);
        }
#pragma unroll
        for (int j = 0; j < BV; ++j)
            if (bon[j]) rb[j] = ld16(wrow[j] + tap * a.Cin + c0);
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int j = 0; j < AV; ++j) {
            const int r = lr + 64 * j;
            *reinterpret_cast<uint4*>(&As[buf][r][swz(r, lv)]) = ra[j];
        }
#pragma unroll
        for (int j = 0; j < BV; ++j) {
            const int r = lr + 64 * j;
            if (bon[j]) *reinterpret_cast<uint4*>(&Bs[buf][r][swz(r, lv)]) = rb[j];
        }
    };
    f32x4 acc[MT][NT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int wm = (wave % WM) * WTM, wn = (wave / WM) * WTN;
    const int r16 = lane & 15, k4 = lane >> 4;
    load(0);
    store(0);
    __syncthreads();
    for (int ch = 0; ch < nch; ++ch) {
        const int buf = ch & 1;
        if (ch + 1 < nch) load(ch + 1);
        uint4 A[MT], B[NT];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const int r = wm + 16 * m + r16;
            A[m] = *reinterpret_cast<const uint4*>(&As[buf][r][swz(r, k4)]);
        }
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            const int r = wn + 16 * n + r16;
            B[n] = *reinterpret_cast<const uint4*>(&Bs[buf][r][swz(r, k4)]);
        }
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int n = 0; n < NT; ++n)
                acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_frag(A[m]), as_frag(B[n]), acc[m][n], 0, 0, 0);
        // the other buffer was last read before the previous barrier
        if (ch + 1 < nch) store(buf ^ 1);
        __syncthreads();
    }
    const int g4 = 4 * (lane >> 4);
    if constexpr (kF32) {
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            const int co = co0 + wn + 16 * n + r16;
            const float b = a.bias ? a.bias[co] : 0.f;
#pragma unroll
            for (int m = 0; m < MT; ++m) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int p = p0 + wm + 16 * m + g4 + r;
                    float v = acc[m][n][r] + b;
                    if (a.relu) v = fmaxf(v, 0.f);
                    if (a.mask && !(bf2f(a.mask[(size_t)p * a.ldm + co]) > 0.f)) v = 0.f;
                    *dst_at<float>(a, p, co) = v;
                }
            }
        }
    } else {
        // bf16 output: bias and ReLU into a tile in LDS (the staging buffers are free
        // after the last barrier), then 16-byte stores of 8 channels with the mask
        // applied per vector; zeroing after rounding equals rounding after zeroing
        bf16_t* Os = sm;
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            const int c = wn + 16 * n + r16;
            const float b = a.bias ? a.bias[co0 + c] : 0.f;
#pragma unroll
            for (int m = 0; m < MT; ++m) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    float v = acc[m][n][r] + b;
                    if (a.relu) v = fmaxf(v, 0.f);
                    Os[(wm + 16 * m + g4 + r) * OP + c] = (bf16_t)f2bf_hw(v);
                }
            }
        }
        __syncthreads();
        constexpr int VR = BN / 8;
        for (int v = t; v < BM * VR; v += 256) {
            const int row = v / VR, cv = v - row * VR;
            const size_t p = (size_t)(p0 + row);
            const int co = co0 + 8 * cv;
            uint4 o = *reinterpret_cast<const uint4*>(&Os[row * OP + 8 * cv]);
            if (a.mask) {
                const uint4 mk = ld16(a.mask + p * a.ldm + co);
                const uint32_t mw[4] = {mk.x, mk.y, mk.z, mk.w};
                uint32_t ow[4] = {o.x, o.y, o.z, o.w};
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const uint32_t keep = (lo(mw[j]) > 0.f ? 0xffffu : 0u) | (hi(mw[j]) > 0.f ? 0xffff0000u : 0u);
                    ow[j] &= keep;
                }
                o = make_uint4(ow[0], ow[1], ow[2], ow[3]);
            }
            st16(dst_at<bf16_t>(a, p, co), o);
        }
    }
}

// Epilogue of a 16 x 16 pixel tile x BN output channels (k_conv_halo, k_conv_halo8):
// bias, ReLU, mask, then FP32 stores, or bfloat16 through the staging tile Os (256 rows
// of BN + 8) as 16-byte stores, and with a.down the 2x2 work of ConvArgs on the staged
// tile (the tile holds whole 2x2 blocks: 16 x 16 tiles at even offsets).
template <bool kF32, int BN, int MT, int NT>
__device__ __forceinline__ void halo_epilogue(const ConvArgs& a, const f32x4 (&acc)[MT][NT], bf16_t* Os, int co0,
                                              int img, int ty0, int tx0, int wm, int lane, int t) {
    constexpr int BM = 256, OP = BN + 8;
    static_assert(NT * 16 == BN, "NT 16-wide blocks per BN");
    const int r16 = lane & 15;
    // image pixel of tile pixel q (row q >> 4, column q & 15)
    auto pixel = [&](int q) { return (size_t)(img + ((ty0 + (q >> 4)) << a.lw) + tx0 + (q & 15)); };
    const int g4 = 4 * (lane >> 4);
    if constexpr (kF32) {
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            const int co = co0 + 16 * n + r16;
            const float b = a.bias ? a.bias[co] : 0.f;
#pragma unroll
            for (int m = 0; m < MT; ++m) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const size_t p = pixel(wm + 16 * m + g4 + r);
                    float v = acc[m][n][r] + b;
                    if (a.relu) v = fmaxf(v, 0.f);
                    if (a.mask && !(bf2f(a.mask[p * a.ldm + co]) > 0.f)) v = 0.f;
                    *dst_at<float>(a, p, co) = v;
                }
            }
        }
    } else {
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            const int c = 16 * n + r16;
            const float b = a.bias ? a.bias[co0 + c] : 0.f;
#pragma unroll
            for (int m = 0; m < MT; ++m) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    float v = acc[m][n][r] + b;
                    if (a.relu) v = fmaxf(v, 0.f);
                    Os[(wm + 16 * m + g4 + r) * OP + c] = (bf16_t)f2bf_hw(v);
                }
            }
        }
        __syncthreads();
        constexpr int VR = BN / 8;
        // half-size pixel of 2x2 block q (row q >> 3, column q & 7) of the tile, whose tile
        // rows are r0, r0 + 1, r0 + 16, r0 + 17 with r0 = 32 (q >> 3) + 2 (q & 7)
        auto half_pixel = [&](int q) {
            return (size_t)((img >> 2) + (((ty0 >> 1) + (q >> 3)) << (a.lw - 1)) + (tx0 >> 1) + (q & 7));
        };
        if (a.down == 2 && co0 < a.ysplit) {
            // upsampling gradient: the 2x2 sums in block order, as k_up_bwd adds them
            for (int v = t; v < 64 * VR; v += 256) {
                const int q = v / VR, cv = v - q * VR, r0 = 32 * (q >> 3) + 2 * (q & 7);
                const int rows[4] = {r0, r0 + 1, r0 + 16, r0 + 17};
                float sum[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, e[8], gt[8];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    unpack8(*reinterpret_cast<const uint4*>(&Os[rows[k] * OP + 8 * cv]), e);
#pragma unroll
                    for (int c = 0; c < 8; ++c) sum[c] += e[c];
                }
                const size_t hp = half_pixel(q);
                const int co = co0 + 8 * cv;
                unpack8(ld16(a.gate + hp * a.ldgt + co), gt);
#pragma unroll
                for (int c = 0; c < 8; ++c)
                    if (!(gt[c] > 0.f)) sum[c] = 0.f;
                st16(static_cast<bf16_t*>(a.y) + hp * a.ldy + co, pack8(sum));
            }
            return;
        }
        for (int v = t; v < BM * VR; v += 256) {
            const int row = v / VR, cv = v - row * VR;
            const size_t p = pixel(row);
            const int co = co0 + 8 * cv;
            uint4 o = *reinterpret_cast<const uint4*>(&Os[row * OP + 8 * cv]);
            if (a.mask) {
                const uint4 mk = ld16(a.mask + p * a.ldm + co);
                const uint32_t mw[4] = {mk.x, mk.y, mk.z, mk.w};
                uint32_t ow[4] = {o.x, o.y, o.z, o.w};
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const uint32_t keep = (lo(mw[j]) > 0.f ? 0xffffu : 0u) | (hi(mw[j]) > 0.f ? 0xffff0000u : 0u);
                    ow[j] &= keep;
                }
                o = make_uint4(ow[0], ow[1], ow[2], ow[3]);
            }
            st16(dst_at<bf16_t>(a, p, co), o);
        }
        if (a.down == 1) {
            // 2x2 max pooling of the stored values, in k_pool_fwd's order
            for (int v = t; v < 64 * VR; v += 256) {
                const int q = v / VR, cv = v - q * VR, r0 = 32 * (q >> 3) + 2 * (q & 7);
                const int rows[3] = {r0 + 1, r0 + 16, r0 + 17};
                float m[8], e[8];
                unpack8(*reinterpret_cast<const uint4*>(&Os[r0 * OP + 8 * cv]), m);
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    unpack8(*reinterpret_cast<const uint4*>(&Os[rows[k] * OP + 8 * cv]), e);
#pragma unroll
                    for (int c = 0; c < 8; ++c) m[c] = e[c] > m[c] ? e[c] : m[c];
                }
                st16(static_cast<bf16_t*>(a.yp) + half_pixel(q) * a.ldyp + co0 + 8 * cv, pack8(m));
            }
        }
    }
}

// Halo-tile form for C_in % 32 == 0 (H, W multiples of 16): a workgroup owns a 16 x 16
// pixel tile and BN = 32 output channels.  Per block of 32 input channels it loads
// the 18 x 18 pixels of the tile and its one-pixel periodic halo and the weights of
// all nine taps, every load issued together, then runs the nine taps out of LDS: the
// A fragment of tile pixel (ty, tx) for tap (dy, dx) is halo pixel
// (ty + dy + 1) * 18 + (tx + dx + 1).  Pixels are reused across taps from LDS instead
// of being re-read from L2 per tap (324 pixels loaded per 256 computed).  One LDS
// buffer (39 KB); the next channel block's global loads are held in registers while
// the current block's MFMAs run, then stored to LDS after a barrier (the registers,
// not the LDS, set the occupancy: one workgroup per CU; forcing two, or keeping the
// tap loop rolled for three or four, was no faster).  LDS rows hold
// 4 x 16-byte pieces swizzled as in k_conv_lds (the 16 lanes of a fragment read 16
// consecutive halo pixels); the bf16 epilogue is the same.  Accumulation order: per
// output, channel block outer, taps inner.
//
// kOne: the layer has one channel block (C_in = 32).  Then there is no next block to
// prefetch, the loads' registers are free once the tile is in LDS, and the kernel asks
// for three wavefronts per SIMD (three workgroups per CU), so that more tiles' loads are
// in flight while others compute; the arithmetic is the same.
constexpr int kHalo = 18 * 18;

//
// BN = 64 (C_out a multiple of 64, several channel blocks): a workgroup owns 64 output
// channels, so each staged halo byte feeds twice the MFMAs (166 instead of 120 FLOP per
// byte staged in LDS); 57 KB of LDS, still two workgroups per CU.  The bfloat16 output
// tile is staged in the weight buffer, whose 9 x 64 x 32 elements are exactly 256 rows
// of 72.
template <bool kF32, bool kOne, int BN>
__global__ void __launch_bounds__(256, kOne ? 3 : 1) k_conv_halo(const ConvArgs a) {
    constexpr int BM = 256, WTM = 64, MT = 4, NT = BN / 16;
    constexpr int OP = BN + 8;
    static_assert(BN == 32 || BN == 64, "32 or 64 output channels per workgroup");
    static_assert(BM * OP <= (BN == 32 ? kHalo * 32 : 9 * BN * 32), "output tile fits its staging buffer");
    __shared__ __attribute__((aligned(16))) bf16_t Ah[kHalo * 32];
    __shared__ __attribute__((aligned(16))) bf16_t Bh[9 * BN * 32];
    const int t = threadIdx.x, lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int ctiles = a.Cout / BN, L = xcd_block(blockIdx.x, gridDim.x);
    const int tile = L / ctiles, co0 = (L % ctiles) * BN;
    const int W = 1 << a.lw, Hm = (1 << a.lh) - 1, Wm = W - 1;
    const int txs = a.lw - 4, tys = a.lh - 4;  // log2 of the tiles per row and per column
    const int tx0 = (tile & ((1 << txs) - 1)) << 4;
    const int ty0 = ((tile >> txs) & ((1 << tys) - 1)) << 4;
    const int img = (tile >> (txs + tys)) << (a.lw + a.lh);
    const int K = 9 * a.Cin;
    f32x4 acc[MT][NT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int wm = wave * WTM;
    const int r16 = lane & 15, k4 = lane >> 4;
    // the next channel block's global loads are in flight while this block's MFMAs run
    constexpr int HV = (kHalo * 4 + 255) / 256, WV = (9 * BN * 4 + 255) / 256;
    uint4 hv[HV], wv[WV];
    auto gload = [&](int c0) {
        const BlockSrc src = block_src(a, c0);
#pragma unroll
        for (int i = 0; i < HV; ++i) {
            const int v = t + 256 * i;
            if (v < kHalo * 4) {
                const int h = v >> 2, piece = v & 3;
                const int hr = h / 18, hc = h - 18 * hr;
                const int yy = (ty0 - 1 + hr) & Hm, xx = (tx0 - 1 + hc) & Wm;
                hv[i] = ld16(block_at(src, img, yy, xx, a.lw) + 8 * piece);
            }
        }
#pragma unroll
        for (int i = 0; i < WV; ++i) {
            const int v = t + 256 * i;
            if (v < 9 * BN * 4) {
                const int r = v >> 2, piece = v & 3;
                const int tap = r / BN, n = r - tap * BN;
                wv[i] = ld16(a.w + (size_t)(co0 + n) * K + tap * a.Cin + c0 + 8 * piece);
            }
        }
    };
    auto lstore = [&]() {
#pragma unroll
        for (int i = 0; i < HV; ++i) {
            const int v = t + 256 * i;
            if (v < kHalo * 4) {
                const int h = v >> 2, piece = v & 3;
                *reinterpret_cast<uint4*>(&Ah[h * 32 + swz(h, piece)]) = hv[i];
            }
        }
#pragma unroll
        for (int i = 0; i < WV; ++i) {
            const int v = t + 256 * i;
            if (v < 9 * BN * 4) {
                const int r = v >> 2, piece = v & 3;
                *reinterpret_cast<uint4*>(&Bh[r * 32 + swz(r, piece)]) = wv[i];
            }
        }
    };
    gload(0);
    for (int c0 = 0; c0 < a.Cin; c0 += 32) {
    if (c0 > 0) __syncthreads();  // the previous channel block's fragments have been read
    lstore();
    __syncthreads();
    if (!kOne && c0 + 32 < a.Cin) gload(c0 + 32);
    for (int tap = 0; tap < 9; ++tap) {
        const int dy = tap / 3, dx = tap - 3 * (tap / 3);  // offsets into the halo (0..2)
        uint4 A[MT], B[NT];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            // tile pixel wm + 16 m + r16: row (wm >> 4) + m, column r16
            const int h = ((wm >> 4) + m + dy) * 18 + r16 + dx;
            A[m] = *reinterpret_cast<const uint4*>(&Ah[h * 32 + swz(h, k4)]);
        }
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            const int r = tap * BN + 16 * n + r16;
            B[n] = *reinterpret_cast<const uint4*>(&Bh[r * 32 + swz(r, k4)]);
        }
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int n = 0; n < NT; ++n)
                acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_frag(A[m]), as_frag(B[n]), acc[m][n], 0, 0, 0);
    }
    }
    // the bfloat16 output tile is staged in the halo or weight buffer: every wavefront
    // must be done with them first
    if constexpr (!kF32) __syncthreads();
    halo_epilogue<kF32, BN, MT, NT>(a, acc, BN == 32 ? Ah : Bh, co0, img, ty0, tx0, wm, lane, t);
}

// Halo-tile form for C_in = 8 (the network's first layer; H, W multiples of 16).  As in
// k_conv_halo a workgroup owns a 16 x 16 pixel tile and 32 output channels, with the
// 18 x 18 halo pixels (one 16-byte piece each) and the weights in LDS, all loads issued
// together.  The 72-long reduction (9 taps x 8 channels) runs as three 32-wide MFMA
// chunks of four taps: the lane group k4 that supplies K elements 8 k4 .. 8 k4 + 7 of
// chunk j takes tap 4 j + k4, whose A fragment is one halo pixel.  Taps 9..11 of the
// last chunk are zero in A and in the weights: k_conv3x3's K order for C_in = 8, chunk
// by chunk, with the input read from L2 once per tile instead of once per tap.
template <bool kF32>
__global__ void __launch_bounds__(256) k_conv_halo8(const ConvArgs a) {
    constexpr int BM = 256, BN = 32, WTM = 64, MT = 4, NT = 2, OP = BN + 8;
    constexpr int KP = 12 * 8 + 8;  // weight row pitch: 12 taps of 8 channels, 8 elements of padding
    __shared__ __attribute__((aligned(16))) bf16_t Ah[kHalo * 8];
    __shared__ __attribute__((aligned(16))) bf16_t Bh[BN * KP];
    __shared__ __attribute__((aligned(16))) bf16_t Os[kF32 ? 8 : BM * OP];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int ctiles = a.Cout / BN, L = xcd_block(blockIdx.x, gridDim.x);
    const int tile = L / ctiles, co0 = (L % ctiles) * BN;
    const int W = 1 << a.lw, Hm = (1 << a.lh) - 1, Wm = W - 1;
    const int txs = a.lw - 4, tys = a.lh - 4;  // log2 of the tiles per row and per column
    const int tx0 = (tile & ((1 << txs) - 1)) << 4;
    const int ty0 = ((tile >> txs) & ((1 << tys) - 1)) << 4;
    const int img = (tile >> (txs + tys)) << (a.lw + a.lh);
    uint4 hv[2], wv[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int v = t + 256 * i;
        if (v < kHalo) {
            const int hr = v / 18, hc = v - 18 * hr;
            const int yy = (ty0 - 1 + hr) & Hm, xx = (tx0 - 1 + hc) & Wm;
            hv[i] = ld16(block_at(block_src(a, 0), img, yy, xx, a.lw));
        }
        if (v < BN * 12) {  // output channel v / 12, tap v % 12
            const int n = v / 12, tap = v - 12 * n;
            wv[i] = tap < 9 ? ld16(a.w + (size_t)(co0 + n) * 72 + 8 * tap) : make_uint4(0u, 0u, 0u, 0u);
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int v = t + 256 * i;
        if (v < kHalo) *reinterpret_cast<uint4*>(&Ah[v * 8]) = hv[i];
        if (v < BN * 12) {
            const int n = v / 12, tap = v - 12 * n;
            *reinterpret_cast<uint4*>(&Bh[n * KP + 8 * tap]) = wv[i];
        }
    }
    __syncthreads();
    f32x4 acc[MT][NT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int wm = wave * WTM, r16 = lane & 15, k4 = lane >> 4;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int tap = 4 * j + k4;
        const bool tv = tap < 9;
        const int dy = tv ? tap / 3 : 0, dx = tv ? tap - 3 * (tap / 3) : 0;  // offsets into the halo (0..2)
        uint4 A[MT], B[NT];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const int h = ((wm >> 4) + m + dy) * 18 + r16 + dx;
            A[m] = sel(tv, *reinterpret_cast<const uint4*>(&Ah[h * 8]));
        }
#pragma unroll
        for (int n = 0; n < NT; ++n) B[n] = *reinterpret_cast<const uint4*>(&Bh[(16 * n + r16) * KP + 32 * j + 8 * k4]);
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int n = 0; n < NT; ++n)
                acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_frag(A[m]), as_frag(B[n]), acc[m][n], 0, 0, 0);
    }
    halo_epilogue<kF32, 32, MT, NT>(a, acc, Os, co0, img, ty0, tx0, wm, lane, t);
}

// several layers in one launch: workgroup b works on the layer whose element range
// [first[l], first[l + 1]) (in units of 256) contains b
constexpr int kFlipMax = 64;
struct FlipSet {
    const bf16_t* w[kFlipMax];
    bf16_t* wf[kFlipMax];
    int cout[kFlipMax], cin[kFlipMax], first[kFlipMax + 1];
    int n;
};

__global__ void k_flip_many(const FlipSet f) {
    int l = 0;
    while (l + 1 < f.n && (int)blockIdx.x >= f.first[l + 1]) ++l;
    const int idx = (blockIdx.x - f.first[l]) * blockDim.x + threadIdx.x;
    const int Cout = f.cout[l], Cin = f.cin[l];
    if (idx >= Cout * 9 * Cin) return;
    const int o = idx % Cout, t = (idx / Cout) % 9, i = idx / (9 * Cout);
    f.wf[l][idx] = f.w[l][((size_t)o * 9 + (8 - t)) * Cin + i];
}

// wf[i][t][o] = w[o][8-t][i]
__global__ void k_flip(const bf16_t* __restrict__ w, bf16_t* __restrict__ wf, int Cout, int Cin) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = Cout * 9 * Cin;
    if (idx >= n) return;
    const int o = idx % Cout, t = (idx / Cout) % 9, i = idx / (9 * Cout);
    wf[idx] = w[((size_t)o * 9 + (8 - t)) * Cin + i];
}

// ---------------------------------------------------------------------------
// weight gradient: dw[o][k] = sum_p g[p][o] X[p][k], X[p][k] = x[p + off_tap(k)][ci(k)]
// ---------------------------------------------------------------------------
// MFMA with rows = k (im2col column), columns = output channel, reduction = pixels.
// The reduction runs over pixels, which are not contiguous in NHWC, so each
// 32-pixel chunk of X and g is staged through LDS transposed ([k][pixel],
// [o][pixel]).  Column K of X is the constant 1, which turns the same product
// into the bias gradient.  Workgroup tile: 64 k x CT output channels; the pixel
// range is split into slabs (grid z) whose partial sums are stored separately.
struct WgArgs {
    const bf16_t* x;
    const bf16_t* x2;     // input channels split .. (see ConvArgs)
    const bf16_t* g;
    float* part;          // [slabs][Cout][Kt]
    int ldx, ldx2, ldg;
    int split, half;
    int lh, lw, P, Cin, Cout, K, Kt, slab;
    int ktiles, ctiles;   // k_wgrad_tr's flat grid: ktiles x ctiles x slabs
};

constexpr int kLdsPad = 40;  // 32 pixels + 8: rows stay 16-byte aligned

template <int CT>
__global__ void __launch_bounds__(256) k_wgrad(const WgArgs a) {
    __shared__ __attribute__((aligned(16))) bf16_t Xs[64][kLdsPad];
    __shared__ __attribute__((aligned(16))) bf16_t Gs[CT][kLdsPad];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int kb = blockIdx.x * 64, cb = blockIdx.y * CT;
    const int pbeg = blockIdx.z * a.slab;
    const int pend = min(a.P, pbeg + a.slab);
    const int Hm = (1 << a.lh) - 1, Wm = (1 << a.lw) - 1;
    // loader roles: vector lg (8 consecutive k or channels) of pixel lp of the chunk
    const int lg = t & 7, lp = t >> 3;
    const int kx = kb + 8 * lg;
    const int mode = kx < a.K ? 0 : (kx == a.K ? 1 : 2);  // data, bias column, zero
    const int tap = mode == 0 ? kx / a.Cin : 0;
    const int ci = mode == 0 ? kx - tap * a.Cin : 0;
    const int dy = tap / 3 - 1, dx = tap - 3 * (tap / 3) - 1;
    const int cg = cb + 8 * lg;  // first output channel of this thread's g vector
    const bool gload = (CT == 64 || lg < 4) && cg < a.Cout;
    // MFMA roles: CT = 64: 2 x 2 wavefronts of 32 k x 32 channels; CT = 32: 4 x 1 of 16 k x 32
    constexpr int MI = CT == 64 ? 2 : 1;
    const int wk = CT == 64 ? (wave & 1) * 32 : wave * 16;
    const int wc = CT == 64 ? (wave >> 1) * 32 : 0;
    f32x4 acc[MI][2];
#pragma unroll
    for (int i = 0; i < MI; ++i) acc[i][0] = acc[i][1] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int p = pbeg; p < pend; p += 32) {
        const int pp = p + lp;
        const bool ok = pp < pend;
        const int q = ok ? pp : pbeg;
        uint4 xv = make_uint4(0u, 0u, 0u, 0u), gv = make_uint4(0u, 0u, 0u, 0u);
        if (mode == 0) {
            const int base = (q >> (a.lw + a.lh)) << (a.lw + a.lh);
            const int ys = ((q >> a.lw) + dy) & Hm, xs = ((q & Wm) + dx) & Wm;
            xv = ld16(src_at(a, base + (ys << a.lw) + xs, ci));
        } else if (mode == 1) {
            xv.x = 0x3f80u;  // bfloat16 1.0 in element 0 (k == K), zeros after it
        }
        if (gload) gv = ld16(a.g + (size_t)q * a.ldg + cg);
        xv = sel(ok, xv);
        gv = sel(ok, gv);
        __syncthreads();  // the previous chunk's fragments have been read
        const uint32_t xw[4] = {xv.x, xv.y, xv.z, xv.w};
        const uint32_t gw[4] = {gv.x, gv.y, gv.z, gv.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            Xs[8 * lg + 2 * j][lp] = (bf16_t)(xw[j] & 0xffffu);
            Xs[8 * lg + 2 * j + 1][lp] = (bf16_t)(xw[j] >> 16);
        }
        if (CT == 64 || lg < 4) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                Gs[8 * lg + 2 * j][lp] = (bf16_t)(gw[j] & 0xffffu);
                Gs[8 * lg + 2 * j + 1][lp] = (bf16_t)(gw[j] >> 16);
            }
        }
        __syncthreads();
        const int r16 = lane & 15, k8 = 8 * (lane >> 4);
        uint4 A[MI], B[2];
#pragma unroll
        for (int i = 0; i < MI; ++i) A[i] = *reinterpret_cast<const uint4*>(&Xs[wk + 16 * i + r16][k8]);
#pragma unroll
        for (int j = 0; j < 2; ++j) B[j] = *reinterpret_cast<const uint4*>(&Gs[wc + 16 * j + r16][k8]);
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_frag(A[i]), as_frag(B[j]), acc[i][j], 0, 0, 0);
    }
    float* part = a.part + (size_t)blockIdx.z * a.Cout * a.Kt;
    const int r16 = lane & 15, g4 = 4 * (lane >> 4);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int co = cb + wc + 16 * j + r16;
        if (co >= a.Cout) continue;
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) part[(size_t)co * a.Kt + kb + wk + 16 * i + g4 + r] = acc[i][j][r];
    }
}

// Weight gradient with the transposing LDS read of gfx950 (ds_read_b64_tr_b16), for
// C_out % 32 == 0.  MFMA rows are output channels, columns im2col columns k, the
// reduction runs over pixels.  Chunks of PC pixels of g ([pixel][channel]) and of the
// im2col rows X ([pixel][k]) are stored to LDS as loaded (16-byte vectors, no
// transposition on the way in).  An MFMA operand needs 8 consecutive pixels of one
// row: within each group of 16 lanes, the transposing read hands lane l element
// l mod 4 of the 8-byte chunk addressed by lane 4j + l/4 (j = 0..3), so when lane
// 4j + q addresses row p + j, columns c + 4q .. c + 4q + 3, lane l receives rows
// p .. p+3 of column c + l; two such reads give the 8 pixels of a fragment.  The row
// pitches (BO + 16 and BK + 16 elements) put the 4 rows of one read at distinct
// 32-byte bank groups.  Two LDS buffers, one barrier per chunk; WOW x (4 / WOW)
// wavefronts of (BO / WOW) x (BK / (4 / WOW)).  The partial sums per pixel slab are
// stored as by k_wgrad.
typedef short v4s __attribute__((ext_vector_type(4)));

template <int PITCH>
__device__ __forceinline__ bf16x8 tr_frag(const bf16_t (*T)[PITCH], int p0, int c0, int lane) {
    const int g = lane >> 4, i = lane & 15;
    const bf16_t* q = &T[p0 + 8 * g + (i >> 2)][c0 + 4 * (i & 3)];
    typedef __attribute__((address_space(3))) v4s lds_v4s;
    const v4s lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s*)(q));
    const v4s hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s*)(q + 4 * PITCH));
    uint4 u;
    u.x = (uint32_t)(uint16_t)lo[0] | ((uint32_t)(uint16_t)lo[1] << 16);
    u.y = (uint32_t)(uint16_t)lo[2] | ((uint32_t)(uint16_t)lo[3] << 16);
    u.z = (uint32_t)(uint16_t)hi[0] | ((uint32_t)(uint16_t)hi[1] << 16);
    u.w = (uint32_t)(uint16_t)hi[2] | ((uint32_t)(uint16_t)hi[3] << 16);
    return as_frag(u);
}

// The same fragment from a tile whose rows carry 32 extra elements after every 8 rows
// (row r at r * PITCH + (r >> 3) * 32), with the 32 pixels of step p0 (a multiple of
// 32) dealt as two rows of 16: lane group g takes pixels p0 + 16 (g & 1) + 8 (g >> 1)
// .. + 7.  The gfx950 LDS has 64 four-byte banks and serves a 64-bit read 32 lanes at
// a time; with this layout the two 16-lane groups of each half-wavefront fall on
// disjoint banks for row pitches of 48, 80 and 272 elements, where the unpadded tile
// with groups 8 rows apart puts them on the same banks (a 2-way conflict on every read).
__device__ __forceinline__ int pad_row(int r, int pitch) { return r * pitch + (r >> 3) * 32; }
__device__ __forceinline__ int frag_px(int p0, int g) { return p0 + 16 * (g & 1) + 8 * (g >> 1); }

template <int PITCH>
__device__ __forceinline__ bf16x8 tr_frag_pad(const bf16_t* T, int p0, int c0, int lane) {
    const int g = lane >> 4, i = lane & 15;
    const bf16_t* q = T + pad_row(frag_px(p0, g) + (i >> 2), PITCH) + c0 + 4 * (i & 3);
    typedef __attribute__((address_space(3))) v4s lds_v4s;
    const v4s lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s*)(q));
    const v4s hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s*)(q + 4 * PITCH));  // same 8-row block
    uint4 u;
    u.x = (uint32_t)(uint16_t)lo[0] | ((uint32_t)(uint16_t)lo[1] << 16);
    u.y = (uint32_t)(uint16_t)lo[2] | ((uint32_t)(uint16_t)lo[3] << 16);
    u.z = (uint32_t)(uint16_t)hi[0] | ((uint32_t)(uint16_t)hi[1] << 16);
    u.w = (uint32_t)(uint16_t)hi[2] | ((uint32_t)(uint16_t)hi[3] << 16);
    return as_frag(u);
}

template <int BO, int BK, int PC, int WOW>
__global__ void __launch_bounds__(256) k_wgrad_tr(const WgArgs a) {
    constexpr int PO = BO + 16, PK = BK + 16;
    constexpr int WKW = 4 / WOW;
    constexpr int WO = BO / WOW, WK = BK / WKW, MT = WO / 16, NT = WK / 16;
    constexpr int GVR = BO / 8, XVR = BK / 8;            // vectors per LDS row
    constexpr int GV = PC * GVR / 256, XV = PC * XVR / 256;  // vectors per thread per chunk
    static_assert(GV >= 1 && XV >= 1, "tile too small for the loader");
    static_assert(256 % GVR == 0 && 256 % XVR == 0 && PC % (256 / GVR) == 0 && PC % (256 / XVR) == 0,
                  "the loader steps rows by 256 / (vectors per row) and must tile the chunk exactly");
    __shared__ __attribute__((aligned(16))) bf16_t Gs[2][PC * PO + PC / 8 * 32];  // rows as pad_row
    __shared__ __attribute__((aligned(16))) bf16_t Xs[2][PC * PK + PC / 8 * 32];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    // flat grid: the k and channel tiles of one pixel slab are adjacent
    const int L = xcd_block(blockIdx.x, gridDim.x);
    const int kt = L % a.ktiles, rest = L / a.ktiles, ct = rest % a.ctiles, z = rest / a.ctiles;
    const int kb = kt * BK, cb = ct * BO;
    const int pbeg = z * a.slab;
    const int pend = min(a.P, pbeg + a.slab);
    const int Hm = (1 << a.lh) - 1, Wm = (1 << a.lw) - 1;
    // loaders: g rows t / GVR + j 256 / GVR, channels cb + 8 (t % GVR); X rows likewise,
    // columns kb + 8 (t % XVR)
    const int gcol = 8 * (t % GVR), grow = t / GVR;
    const int xcol = 8 * (t % XVR), xrow = t / XVR;
    const int kx = kb + xcol;
    const int mode = kx < a.K ? 0 : (kx == a.K ? 1 : 2);  // data, bias column, zero
    const int tap = mode == 0 ? kx / a.Cin : 0;
    const int ci = mode == 0 ? kx - tap * a.Cin : 0;
    const int dy = tap / 3 - 1, dx = tap - 3 * (tap / 3) - 1;
    uint4 gv[GV], xv[XV];
    auto load = [&](int pc) {
#pragma unroll
        for (int j = 0; j < GV; ++j) {
            const int pp = pc + grow + j * (256 / GVR);
            const bool ok = pp < pend;
            gv[j] = sel(ok, ld16(a.g + (size_t)(ok ? pp : pbeg) * a.ldg + cb + gcol));
        }
#pragma unroll
        for (int j = 0; j < XV; ++j) {
            const int pp = pc + xrow + j * (256 / XVR);
            const bool ok = pp < pend;
            const int q = ok ? pp : pbeg;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (mode == 0) {
                const int base = (q >> (a.lw + a.lh)) << (a.lw + a.lh);
                const int ys = ((q >> a.lw) + dy) & Hm, xs = ((q & Wm) + dx) & Wm;
                v = ld16(src_at(a, base + (ys << a.lw) + xs, ci));
            } else if (mode == 1) {
                v.x = 0x3f80u;  // bfloat16 1.0 in column K: the bias gradient
            }
            xv[j] = sel(ok, v);
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int j = 0; j < GV; ++j)
            *reinterpret_cast<uint4*>(&Gs[buf][pad_row(grow + j * (256 / GVR), PO) + gcol]) = gv[j];
#pragma unroll
        for (int j = 0; j < XV; ++j)
            *reinterpret_cast<uint4*>(&Xs[buf][pad_row(xrow + j * (256 / XVR), PK) + xcol]) = xv[j];
    };
    f32x4 acc[MT][NT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int wo = (wave % WOW) * WO, wk = (wave / WOW) * WK;
    load(pbeg);
    store(0);
    __syncthreads();
    int buf = 0;
    for (int pc = pbeg; pc < pend; pc += PC) {
        const bool more = pc + PC < pend;
        if (more) load(pc + PC);
#pragma unroll
        for (int ks = 0; ks < PC; ks += 32) {
            bf16x8 A[MT], B[NT];
#pragma unroll
            for (int m = 0; m < MT; ++m) A[m] = tr_frag_pad<PO>(Gs[buf], ks, wo + 16 * m, lane);
#pragma unroll
            for (int n = 0; n < NT; ++n) B[n] = tr_frag_pad<PK>(Xs[buf], ks, wk + 16 * n, lane);
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int n = 0; n < NT; ++n)
                    acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[m], B[n], acc[m][n], 0, 0, 0);
        }
        // the other buffer was last read before the previous barrier
        if (more) store(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
    float* part = a.part + (size_t)z * a.Cout * a.Kt;
    const int i16 = lane & 15, g4 = 4 * (lane >> 4);
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int n = 0; n < NT; ++n)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                part[(size_t)(cb + wo + 16 * m + g4 + r) * a.Kt + kb + wk + 16 * n + i16] = acc[m][n][r];
}

// Halo-tile weight gradient (C_in % 32 == 0, C_out = 32 or a multiple of 64, H and W
// multiples of 16: every layer of the network but the first).  A workgroup owns OC =
// 32 or 64 output channels and one block of 32 input channels and walks a slab of
// 16 x 16 pixel tiles.  Per tile it loads g (256 pixels x OC channels) and the 18 x 18
// pixels of the input tile with its periodic halo, once each, and forms the columns
// of all nine taps out of LDS: for 8 consecutive pixels of a tile row the tap-shifted
// halo pixels are consecutive rows, so the transposing read (as in k_wgrad_tr) yields
// the MFMA fragment directly.  Each input value is therefore read once per output
// tile, where the im2col form reads it once per tap.  LDS layout (bank conflicts): the
// g tile as in tr_frag_pad, and halo pixels at a pitch of 48 elements plus 96 after
// every halo row of 18, so that the eight 32-byte row pieces of every half-wavefront
// read fall on distinct banks for every tap, input-channel half and reduction step.
// The 18 column blocks (9 taps x 2 halves of the 32 input channels) are dealt to the
// four wavefronts round robin, each for all OC / 16 output blocks, so a halo fragment
// feeds OC / 16 MFMAs.  The next tile's loads are held in registers while the current
// tile's MFMAs run.  The bias gradient is summed per thread (FP32) over the g values
// it loads and combined in a fixed order.  The partial sums per slab go to the same
// [slab][C_out][Kt] layout as the other forms.
constexpr int kWgPitch = 48;                  // elements per halo pixel
constexpr int kWgHaloRow = 18 * kWgPitch + 96;  // elements per halo row of 18 pixels

// LDS element offset of halo pixel (hr, hc); g-tile pixel q (row-major 16 wide) sits at
// pad_row(q, GP), and reduction step ks covers pixels 32 ks .. + 31 dealt as frag_px
__device__ __forceinline__ int hs_at(int hr, int hc) { return hr * kWgHaloRow + hc * kWgPitch; }

__device__ __forceinline__ bf16x8 halo_frag(const bf16_t* Hs, int ks, int dy, int dx, int c0, int lane) {
    const int g = lane >> 4, i = lane & 15;
    const int px0 = frag_px(ks * 32, g);  // 8 consecutive tile pixels within one tile row
    const bf16_t* q = Hs + hs_at((px0 >> 4) + dy, (px0 & 15) + dx + (i >> 2)) + c0 + 4 * (i & 3);
    typedef __attribute__((address_space(3))) v4s lds_v4s;
    const v4s lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s*)(q));
    const v4s hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s*)(q + 4 * kWgPitch));
    uint4 u;
    u.x = (uint32_t)(uint16_t)lo[0] | ((uint32_t)(uint16_t)lo[1] << 16);
    u.y = (uint32_t)(uint16_t)lo[2] | ((uint32_t)(uint16_t)lo[3] << 16);
    u.z = (uint32_t)(uint16_t)hi[0] | ((uint32_t)(uint16_t)hi[1] << 16);
    u.w = (uint32_t)(uint16_t)hi[2] | ((uint32_t)(uint16_t)hi[3] << 16);
    return as_frag(u);
}

template <int OC>
__global__ void __launch_bounds__(256) k_wgrad_halo(const WgArgs a) {
    constexpr int NCB = 5;  // column blocks per wavefront (18 over 4: 5, 5, 4, 4)
    constexpr int GP = OC + 16;     // row pitch of the g tile (rows at pad_row(q, GP))
    constexpr int PPR = OC / 8;     // 16-byte pieces per pixel of g
    constexpr int RP = 256 / PPR;   // g pixels loaded per pass of the workgroup
    constexpr int MH = OC / 16;     // 16-row output blocks
    constexpr int KU = OC == 64 ? 1 : 2;
    __shared__ __attribute__((aligned(16))) bf16_t Gs[256 * GP + 32 * 32];
    __shared__ __attribute__((aligned(16))) bf16_t Hs[18 * kWgHaloRow];
    // the wavefront index is uniform: its column blocks, taps and LDS offsets are scalars
    const int t = threadIdx.x, lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);
    // flat grid: input-channel blocks, then output-channel blocks, then slabs
    const int L = xcd_block(blockIdx.x, gridDim.x);
    const int cc = L % a.ktiles, rest = L / a.ktiles, ob = rest % a.ctiles, z = rest / a.ctiles;
    const int c0 = cc * 32, o0 = ob * OC;
    const BlockSrc src = block_src(a, c0);
    const int tb = z * a.slab, te = min(a.P >> 8, tb + a.slab);
    const int Hm = (1 << a.lh) - 1, Wm = (1 << a.lw) - 1;
    const int txs = a.lw - 4, tys = a.lh - 4;
    const int gpiece = t % PPR;  // this thread's g channels: o0 + 8 gpiece .. + 7
    f32x4 acc[MH][NCB];
#pragma unroll
    for (int h = 0; h < MH; ++h)
#pragma unroll
        for (int i = 0; i < NCB; ++i) acc[h][i] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bsum[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    // the next tile's g and halo loads are in flight (in registers) while this tile's
    // MFMAs run; the registers cost no occupancy (the LDS tiles already allow two
    // workgroups per CU)
    constexpr int HV = (kHalo * 4 + 255) / 256;
    uint4 gv[PPR], hv[HV];
    auto gload = [&](int tile) {
        const int tx0 = (tile & ((1 << txs) - 1)) << 4;
        const int ty0 = ((tile >> txs) & ((1 << tys) - 1)) << 4;
        const int img = (tile >> (txs + tys)) << (a.lw + a.lh);
#pragma unroll
        for (int i = 0; i < PPR; ++i) {
            const int q = t / PPR + RP * i;  // tile pixel (row q >> 4, column q & 15)
            const size_t p = (size_t)(img + ((ty0 + (q >> 4)) << a.lw) + tx0 + (q & 15));
            gv[i] = ld16(a.g + p * a.ldg + o0 + 8 * gpiece);
        }
#pragma unroll
        for (int i = 0; i < HV; ++i) {
            const int v = t + 256 * i;
            if (v < kHalo * 4) {
                const int h = v >> 2, piece = v & 3;
                const int hr = h / 18, hc = h - 18 * hr;
                const int yy = (ty0 - 1 + hr) & Hm, xx = (tx0 - 1 + hc) & Wm;
                hv[i] = ld16(block_at(src, img, yy, xx, a.lw) + 8 * piece);
            }
        }
    };
    if (tb < te) gload(tb);
    for (int tile = tb; tile < te; ++tile) {
        if (tile != tb) __syncthreads();  // the previous tile's fragments have been read
#pragma unroll
        for (int i = 0; i < PPR; ++i) {
            const int q = t / PPR + RP * i;
            *reinterpret_cast<uint4*>(&Gs[pad_row(q, GP) + 8 * gpiece]) = gv[i];
            float f[8];
            unpack8(gv[i], f);
#pragma unroll
            for (int j = 0; j < 8; ++j) bsum[j] += f[j];
        }
#pragma unroll
        for (int i = 0; i < HV; ++i) {
            const int v = t + 256 * i;
            if (v < kHalo * 4) {
                const int h = v >> 2, piece = v & 3;
                const int hr = h / 18, hc = h - 18 * hr;
                *reinterpret_cast<uint4*>(&Hs[hs_at(hr, hc) + 8 * piece]) = hv[i];
            }
        }
        __syncthreads();
        if (tile + 1 < te) gload(tile + 1);
        // two reduction steps per iteration for 32 outputs; one for 64, whose second
        // set of A fragments would not fit two workgroups per CU
#pragma unroll KU
        for (int ks = 0; ks < 8; ++ks) {
            bf16x8 A[MH];
#pragma unroll
            for (int h = 0; h < MH; ++h)
                A[h] = tr_frag_pad<GP>(Gs, ks * 32, 16 * h, lane);
#pragma unroll
            for (int i = 0; i < NCB; ++i) {
                // no branch in the loop, so the LDS reads of later blocks overlap the MFMAs:
                // the fifth block of wavefronts 2 and 3 (blocks 18, 19) repeats block 17 and
                // is not stored; wavefronts 0 and 1 do five blocks anyway
                const int cb = min(wave + 4 * i, 17);
                const int tap = cb >> 1, dy = tap / 3, dx = tap - 3 * (tap / 3);
                const bf16x8 B = halo_frag(Hs, ks, dy, dx, 16 * (cb & 1), lane);
#pragma unroll
                for (int h = 0; h < MH; ++h)
                    acc[h][i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[h], B, acc[h][i], 0, 0, 0);
            }
        }
    }
    float* part = a.part + (size_t)z * a.Cout * a.Kt;
    const int i16 = lane & 15, g4 = 4 * (lane >> 4);
#pragma unroll
    for (int i = 0; i < NCB; ++i) {
        const int cb = wave + 4 * i;
        if (cb >= 18) continue;
        const int k = (cb >> 1) * a.Cin + c0 + 16 * (cb & 1) + i16;
#pragma unroll
        for (int h = 0; h < MH; ++h)
#pragma unroll
            for (int r = 0; r < 4; ++r) part[(size_t)(o0 + 16 * h + g4 + r) * a.Kt + k] = acc[h][i][r];
    }
    if (cc == 0) {
        // bias: the RP threads holding each 8-channel piece, combined in thread order
        __syncthreads();
        float* red = reinterpret_cast<float*>(Gs);
#pragma unroll
        for (int j = 0; j < 8; ++j) red[t * 8 + j] = bsum[j];
        __syncthreads();
        if (t < OC) {
            const int piece = t >> 3, j = t & 7;
            float s = 0.f;
            for (int u = 0; u < RP; ++u) s += red[(PPR * u + piece) * 8 + j];
            part[(size_t)(o0 + t) * a.Kt + a.K] = s;
        }
    }
}

// Halo-tile weight gradient for C_in = 8 (the network's first layer), the same scheme
// as k_wgrad_halo with one 16-byte piece per halo pixel.  The 72 columns (9 taps x 8
// channels) form five 16-column blocks of two taps: in the transposing read, lanes
// 4j + q with q < 2 address the first tap's halo row and q >= 2 the second's, so lane
// l receives column l = (tap 2 cb + l / 8, channel l % 8), k = 16 cb + l.  Tap 9 of the
// last block reads tap 8's rows (inside the halo) and its columns are not stored.
constexpr int kWg8Pitch = 16;  // halo row pitch: 8 channels + 8 elements of padding

__device__ __forceinline__ bf16x8 halo_frag8(const bf16_t* Hs, int ks, int cb, int lane) {
    const int g = lane >> 4, i = lane & 15;
    const int px0 = ks * 32 + 8 * g;  // 8 consecutive tile pixels within one tile row
    const int tap = min(2 * cb + ((i & 3) >> 1), 8);
    const int dy = tap / 3, dx = tap - 3 * (tap / 3);
    const int hb = ((px0 >> 4) + dy) * 18 + (px0 & 15) + dx;
    const bf16_t* q = Hs + (hb + (i >> 2)) * kWg8Pitch + 4 * (i & 1);
    typedef __attribute__((address_space(3))) v4s lds_v4s;
    const v4s lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s*)(q));
    const v4s hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s*)(q + 4 * kWg8Pitch));
    uint4 u;
    u.x = (uint32_t)(uint16_t)lo[0] | ((uint32_t)(uint16_t)lo[1] << 16);
    u.y = (uint32_t)(uint16_t)lo[2] | ((uint32_t)(uint16_t)lo[3] << 16);
    u.z = (uint32_t)(uint16_t)hi[0] | ((uint32_t)(uint16_t)hi[1] << 16);
    u.w = (uint32_t)(uint16_t)hi[2] | ((uint32_t)(uint16_t)hi[3] << 16);
    return as_frag(u);
}

template <int OC>
__global__ void __launch_bounds__(256) k_wgrad_halo8(const WgArgs a) {
    constexpr int NCB = 2;          // column blocks per wavefront (5 over 4: 2, 1, 1, 1)
    constexpr int GP = OC + 16;     // row pitch of the g tile
    constexpr int PPR = OC / 8;     // 16-byte pieces per pixel of g
    constexpr int RP = 256 / PPR;   // g pixels loaded per pass of the workgroup
    constexpr int MH = OC / 16;     // 16-row output blocks
    __shared__ __attribute__((aligned(16))) bf16_t Gs[256 * GP];
    __shared__ __attribute__((aligned(16))) bf16_t Hs[kHalo * kWg8Pitch];
    const int t = threadIdx.x, lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);
    // flat grid: output-channel blocks, then slabs (one input-channel block)
    const int L = xcd_block(blockIdx.x, gridDim.x);
    const int ob = L % a.ctiles, z = L / a.ctiles;
    const int o0 = ob * OC;
    const int tb = z * a.slab, te = min(a.P >> 8, tb + a.slab);
    const int Hm = (1 << a.lh) - 1, Wm = (1 << a.lw) - 1;
    const int txs = a.lw - 4, tys = a.lh - 4;
    const int gpiece = t % PPR;
    f32x4 acc[MH][NCB];
#pragma unroll
    for (int h = 0; h < MH; ++h)
#pragma unroll
        for (int i = 0; i < NCB; ++i) acc[h][i] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bsum[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    constexpr int HV = (kHalo + 255) / 256;
    uint4 gv[PPR], hv[HV];
    auto gload = [&](int tile) {
        const int tx0 = (tile & ((1 << txs) - 1)) << 4;
        const int ty0 = ((tile >> txs) & ((1 << tys) - 1)) << 4;
        const int img = (tile >> (txs + tys)) << (a.lw + a.lh);
#pragma unroll
        for (int i = 0; i < PPR; ++i) {
            const int q = t / PPR + RP * i;  // tile pixel (row q >> 4, column q & 15)
            const size_t p = (size_t)(img + ((ty0 + (q >> 4)) << a.lw) + tx0 + (q & 15));
            gv[i] = ld16(a.g + p * a.ldg + o0 + 8 * gpiece);
        }
#pragma unroll
        for (int i = 0; i < HV; ++i) {
            const int h = t + 256 * i;
            if (h < kHalo) {
                const int hr = h / 18, hc = h - 18 * hr;
                const int yy = (ty0 - 1 + hr) & Hm, xx = (tx0 - 1 + hc) & Wm;
                hv[i] = ld16(block_at(block_src(a, 0), img, yy, xx, a.lw));
            }
        }
    };
    if (tb < te) gload(tb);
    for (int tile = tb; tile < te; ++tile) {
        if (tile != tb) __syncthreads();  // the previous tile's fragments have been read
#pragma unroll
        for (int i = 0; i < PPR; ++i) {
            const int q = t / PPR + RP * i;
            *reinterpret_cast<uint4*>(&Gs[q * GP + 8 * gpiece]) = gv[i];
            float f[8];
            unpack8(gv[i], f);
#pragma unroll
            for (int j = 0; j < 8; ++j) bsum[j] += f[j];
        }
#pragma unroll
        for (int i = 0; i < HV; ++i) {
            const int h = t + 256 * i;
            if (h < kHalo) *reinterpret_cast<uint4*>(&Hs[h * kWg8Pitch]) = hv[i];
        }
        __syncthreads();
        if (tile + 1 < te) gload(tile + 1);
#pragma unroll 2
        for (int ks = 0; ks < 8; ++ks) {
            bf16x8 A[MH];
#pragma unroll
            for (int h = 0; h < MH; ++h)
                A[h] = tr_frag<GP>(reinterpret_cast<const bf16_t(*)[GP]>(Gs), ks * 32, 16 * h, lane);
#pragma unroll
            for (int i = 0; i < NCB; ++i) {
                // branch-free as in k_wgrad_halo: wavefronts 1 to 3 repeat block 4 as their
                // second block, which is not stored
                const int cb = min(wave + 4 * i, 4);
                const bf16x8 B = halo_frag8(Hs, ks, cb, lane);
#pragma unroll
                for (int h = 0; h < MH; ++h)
                    acc[h][i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[h], B, acc[h][i], 0, 0, 0);
            }
        }
    }
    float* part = a.part + (size_t)z * a.Cout * a.Kt;
    const int i16 = lane & 15, g4 = 4 * (lane >> 4);
#pragma unroll
    for (int i = 0; i < NCB; ++i) {
        const int cb = wave + 4 * i;
        const int k = 16 * cb + i16;
        if (cb >= 5 || k >= 72) continue;
#pragma unroll
        for (int h = 0; h < MH; ++h)
#pragma unroll
            for (int r = 0; r < 4; ++r) part[(size_t)(o0 + 16 * h + g4 + r) * a.Kt + k] = acc[h][i][r];
    }
    // bias: the RP threads holding each 8-channel piece, combined in thread order
    __syncthreads();
    float* red = reinterpret_cast<float*>(Gs);
#pragma unroll
    for (int j = 0; j < 8; ++j) red[t * 8 + j] = bsum[j];
    __syncthreads();
    if (t < OC) {
        const int piece = t >> 3, j = t & 7;
        float s = 0.f;
        for (int u = 0; u < RP; ++u) s += red[(PPR * u + piece) * 8 + j];
        part[(size_t)(o0 + t) * a.Kt + a.K] = s;
    }
}

// dw[o][k] = sum_s part[s][o][k] (k < K), db[o] = sum_s part[s][o][K].  A workgroup
// takes 64 consecutive outputs (one per lane) and its WV wavefronts take slabs
// w, w + WV, w + 2 WV, ... each with NA running sums (slab index mod NA WV), which are
// combined in a fixed order, then the wavefronts' sums in a fixed order: deterministic
// for a given slab count.  Long slab ranges take 16 wavefronts with eight loads in
// flight each (the 256^2 layers' 512 slabs: half the time of 4 x 4), short ones 4 x 4.
template <int WV, int NA>
__global__ void __launch_bounds__(64 * WV) k_wgrad_reduce(const float* __restrict__ part, float* __restrict__ dw,
                                                          float* __restrict__ db, int slabs, int Cout, int K,
                                                          int Kt) {
    static_assert((WV & (WV - 1)) == 0 && WV >= 2 && (NA == 4 || NA == 8), "power-of-two waves, 4 or 8 sums");
    __shared__ float sm[WV][64];
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int idx = blockIdx.x * 64 + lane;
    const bool on = idx < Cout * (K + 1);
    const int o = on ? idx / (K + 1) : 0, k = on ? idx - o * (K + 1) : 0;
    const size_t stride = (size_t)Cout * Kt;
    const float* q = part + (size_t)o * Kt + k;
    float a[NA];
#pragma unroll
    for (int j = 0; j < NA; ++j) a[j] = 0.f;
    if (on) {
        int z = wave;
        for (; z + (NA - 1) * WV < slabs; z += NA * WV) {
#pragma unroll
            for (int j = 0; j < NA; ++j) a[j] += q[(size_t)(z + j * WV) * stride];
        }
        for (; z < slabs; z += WV) a[0] += q[(size_t)z * stride];
    }
    float t = (a[0] + a[1]) + (a[2] + a[3]);
    if constexpr (NA == 8) t = t + ((a[4] + a[5]) + (a[6] + a[7]));
    sm[wave][lane] = t;
    __syncthreads();
    if (wave != 0 || !on) return;
    float r[WV / 2];
#pragma unroll
    for (int w = 0; w < WV / 2; ++w) r[w] = sm[2 * w][lane] + sm[2 * w + 1][lane];
#pragma unroll
    for (int h = WV / 4; h >= 1; h >>= 1)
#pragma unroll
        for (int w = 0; w < h; ++w) r[w] = r[2 * w] + r[2 * w + 1];
    if (k < K) dw[(size_t)o * K + k] = r[0];
    else if (db) db[o] = r[0];
}

// ---------------------------------------------------------------------------
// pooling, upsampling (16-byte vectors of 8 channels)
// ---------------------------------------------------------------------------
struct Geo {
    int N, lh, lw, C;  // lh, lw: log2 of the larger (unpooled) size
};

__device__ __forceinline__ void small_pixel(int idx, const Geo& g, int& cg, int& n, int& Y, int& X) {
    const int cgs = g.C >> 3;
    cg = idx % cgs;
    int r = idx / cgs;
    X = r & ((1 << (g.lw - 1)) - 1);
    r >>= g.lw - 1;
    Y = r & ((1 << (g.lh - 1)) - 1);
    n = r >> (g.lh - 1);
}

__global__ void k_pool_fwd(const bf16_t* x, int ldx, bf16_t* y, int ldy, Geo g, int total) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    int cg, n, Y, X;
    small_pixel(idx, g, cg, n, Y, X);
    const int W = 1 << g.lw, H = 1 << g.lh;
    const size_t p00 = ((size_t)n * H + 2 * Y) * W + 2 * X;
    float m[8], v[8];
    unpack8(ld16(x + p00 * ldx + 8 * cg), m);
    const size_t ps[3] = {p00 + 1, p00 + W, p00 + W + 1};
    for (int k = 0; k < 3; ++k) {
        unpack8(ld16(x + ps[k] * ldx + 8 * cg), v);
#pragma unroll
        for (int c = 0; c < 8; ++c) m[c] = v[c] > m[c] ? v[c] : m[c];
    }
    const size_t q = ((size_t)n * (H >> 1) + Y) * (W >> 1) + X;
    st16(y + q * ldy + 8 * cg, pack8(m));
}

__global__ void k_pool_bwd(const bf16_t* x, int ldx, const bf16_t* dy, int lddy, const bf16_t* add, int lda,
                           bf16_t* dx, int lddx, int gate, Geo g, int total) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    int cg, n, Y, X;
    small_pixel(idx, g, cg, n, Y, X);
    const int W = 1 << g.lw, H = 1 << g.lh;
    const size_t p00 = ((size_t)n * H + 2 * Y) * W + 2 * X;
    const size_t ps[4] = {p00, p00 + 1, p00 + W, p00 + W + 1};
    float xv[4][8], d[8];
    for (int k = 0; k < 4; ++k) unpack8(ld16(x + ps[k] * ldx + 8 * cg), xv[k]);
    const size_t q = ((size_t)n * (H >> 1) + Y) * (W >> 1) + X;
    unpack8(ld16(dy + q * lddy + 8 * cg), d);
    int arg[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        int best = 0;
        for (int k = 1; k < 4; ++k)
            if (xv[k][c] > xv[best][c]) best = k;
        arg[c] = best;
    }
    for (int k = 0; k < 4; ++k) {
        float o[8], ad[8];
        if (add) unpack8(ld16(add + ps[k] * lda + 8 * cg), ad);
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            float v = arg[c] == k ? d[c] : 0.f;
            if (add) v += ad[c];
            if (gate && !(xv[k][c] > 0.f)) v = 0.f;
            o[c] = v;
        }
        st16(dx + ps[k] * lddx + 8 * cg, pack8(o));
    }
}

// g describes the large (output) size
__global__ void k_up_fwd(const bf16_t* x, int ldx, bf16_t* y, int ldy, Geo g, int total) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    int cg, n, Y, X;
    small_pixel(idx, g, cg, n, Y, X);
    const int W = 1 << g.lw, H = 1 << g.lh;
    const size_t q = ((size_t)n * (H >> 1) + Y) * (W >> 1) + X;
    const uint4 v = ld16(x + q * ldx + 8 * cg);
    const size_t p00 = ((size_t)n * H + 2 * Y) * W + 2 * X;
    st16(y + p00 * ldy + 8 * cg, v);
    st16(y + (p00 + 1) * ldy + 8 * cg, v);
    st16(y + (p00 + W) * ldy + 8 * cg, v);
    st16(y + (p00 + W + 1) * ldy + 8 * cg, v);
}

__global__ void k_up_bwd(const bf16_t* dy, int lddy, const bf16_t* gate, int ldgt, bf16_t* dx, int lddx, Geo g,
                         int total) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    int cg, n, Y, X;
    small_pixel(idx, g, cg, n, Y, X);
    const int W = 1 << g.lw, H = 1 << g.lh;
    const size_t p00 = ((size_t)n * H + 2 * Y) * W + 2 * X;
    const size_t ps[4] = {p00, p00 + 1, p00 + W, p00 + W + 1};
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, v[8];
    for (int k = 0; k < 4; ++k) {
        unpack8(ld16(dy + ps[k] * lddy + 8 * cg), v);
#pragma unroll
        for (int c = 0; c < 8; ++c) s[c] += v[c];
    }
    const size_t q = ((size_t)n * (H >> 1) + Y) * (W >> 1) + X;
    if (gate) {
        float gt[8];
        unpack8(ld16(gate + q * ldgt + 8 * cg), gt);
#pragma unroll
        for (int c = 0; c < 8; ++c)
            if (!(gt[c] > 0.f)) s[c] = 0.f;
    }
    st16(dx + q * lddx + 8 * cg, pack8(s));
}

// ---------------------------------------------------------------------------
// input, head and loss, optimizer
// ---------------------------------------------------------------------------
// channels: 0 normalised density, 1 condition, 2 normalised temperature deviation, 3..7 zero
__global__ void k_prepare(const double* rho, const double* T, const double* rv, const double* rl, const double* T0,
                          const double* cond, double theta_scale, bf16_t* x, float* rin, int lhw, int total) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int n = idx >> lhw;
    const float v = (float)((rho[idx] - rv[n]) / (rl[n] - rv[n]));
    const float th = T ? (float)((T[idx] / T0[n] - 1.0) / theta_scale) : 0.f;
    if (rin) {
        rin[idx] = v;
        rin[(size_t)total + idx] = th;
    }
    if (x) st16(x + (size_t)idx * 8, make_uint4(f2bf(v) | (f2bf((float)cond[n]) << 16), f2bf(th), 0u, 0u));
}

__global__ void k_output(const float* out, int K, const double* rv, const double* rl, const double* T0,
                         double theta_scale, double* rho, double* T, int lhw, int total) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int n = idx >> lhw;
    rho[idx] = rv[n] + (rl[n] - rv[n]) * (double)out[idx];
    if (T) T[idx] = T0[n] * (1.0 + theta_scale * (K > 1 ? (double)out[(size_t)total + idx] : 0.0));
}

constexpr int kHeadBlock = 256;

// block sum of one float per thread (fixed tree order)
__device__ __forceinline__ float block_sum(float v, float* sm) {
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int s = kHeadBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
        __syncthreads();
    }
    const float r = sm[0];
    __syncthreads();
    return r;
}

// K output planes: out[k][p] = sum_c hw[k][c] d[p][c] + hb[k] + rin[k][p]
__global__ void __launch_bounds__(kHeadBlock) k_head_fwd(const bf16_t* d, int ldd, const float* hw, const float* hb,
                                                         const float* rin, const float* target, float* out,
                                                         float* dout, float* part, int C, int K, int P) {
    __shared__ float sm[kHeadBlock];
    const int p = blockIdx.x * kHeadBlock + threadIdx.x;
    float r2 = 0.f;
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    if (p < P) {
        for (int c = 0; c < C; c += 8) {
            float v[8];
            unpack8(ld16(d + (size_t)p * ldd + c), v);
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int j = 0; j < 8; ++j) acc[k] += hw[k * C + c + j] * v[j];
        }
        for (int k = 0; k < K; ++k) {
            const float s = acc[k] + hb[k] + rin[(size_t)k * P + p];
            out[(size_t)k * P + p] = s;
            if (target) {
                const float r = s - target[(size_t)k * P + p];
                dout[(size_t)k * P + p] = 2.f * r / (float)((size_t)K * P);
                r2 += r * r;
            }
        }
    }
    if (target) {
        const float b = block_sum(r2, sm);
        if (threadIdx.x == 0) part[blockIdx.x] = b;
    }
}

// wavefront sum (xor butterfly: the same association in every wavefront)
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// part: [blocks][K (C + 1)]: per-workgroup sums of dout_k d[., c] and of dout_k.  The
// C / 8 channel groups of a pixel sit on consecutive threads (16-byte accesses of whole
// pixel rows); thread t takes pixels t / G, t / G + (threads / G), ... (G = C / 8) and
// sums its products in registers; the workgroup then combines the threads' sums in
// thread order through LDS (deterministic).  C / 8 must divide the workgroup size.
constexpr int kHeadBwdBlocks = 2048;

__global__ void __launch_bounds__(kHeadBlock) k_head_bwd(const bf16_t* d, int ldd, const float* hw,
                                                         const float* dout, bf16_t* g, float* part, int C, int K,
                                                         int P) {
    __shared__ float red[kHeadBlock * 9];
    const int G = C >> 3, t = threadIdx.x;
    const int cg = t % G, c = 8 * cg;
    const int per_block = kHeadBlock / G;            // pixels per workgroup per sweep
    const int p0 = blockIdx.x * per_block + t / G, stride = gridDim.x * per_block;
    float w[4][8], acc[4][8], bs[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        bs[k] = 0.f;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            acc[k][j] = 0.f;
            w[k][j] = k < K ? hw[k * C + c + j] : 0.f;
        }
    }
    for (int p = p0; p < P; p += stride) {
        float dp[4], v[8], o[8];
#pragma unroll
        for (int k = 0; k < 4; ++k) dp[k] = k < K ? dout[(size_t)k * P + p] : 0.f;
        unpack8(ld16(d + (size_t)p * ldd + c), v);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            float s = 0.f;
#pragma unroll
            for (int k = 0; k < 4; ++k) s += dp[k] * w[k][j];
            o[j] = v[j] > 0.f ? s : 0.f;
#pragma unroll
            for (int k = 0; k < 4; ++k) acc[k][j] += dp[k] * v[j];
        }
        st16(g + (size_t)p * C + c, pack8(o));
#pragma unroll
        for (int k = 0; k < 4; ++k) bs[k] += dp[k];
    }
    // combine: for each k, entry (channel c + j) sums the threads of group cg, and the
    // bias entry sums the group-0 threads (one per pixel)
    const int m = K * (C + 1);
    float* row = part + (size_t)blockIdx.x * m;
    for (int k = 0; k < K; ++k) {
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 8; ++j) red[t * 9 + j] = acc[k][j];
        red[t * 9 + 8] = bs[k];
        __syncthreads();
        for (int e = t; e < C + 1; e += kHeadBlock) {
            float s = 0.f;
            if (e < C) {
                const int eg = e >> 3, ej = e & 7;
                for (int u = eg; u < kHeadBlock; u += G) s += red[u * 9 + ej];
            } else {
                for (int u = 0; u < kHeadBlock; u += G) s += red[u * 9 + 8];
            }
            row[k * (C + 1) + e] = s;
        }
    }
}

// Forward and backward of the head in one pass, for training.  Per pixel: the K outputs
// s_k = hw_k . d + hb_k + rin_k, dout_k = 2 (s_k - target_k) / (K P) and the gradient of d,
// g = sum_k dout_k hw_k where d > 0 (the ReLU of the last convolution).  Per workgroup:
// the sums of dout_k d and of dout_k (weight and bias gradients) combined as in
// k_head_bwd, in rows part[b][K (C + 1) + 1] whose last entry is the sum of
// (s_k - target_k)^2.  Thread layout of k_head_bwd: the C / 8 channel groups of a pixel on
// consecutive lanes, each with its 8 products per output, summed across the pixel's
// lanes by a fixed xor butterfly (C / 8 a power of two).  d is read once where the two
// separate passes read it twice, and dout is not read back.
template <int KK>
__global__ void __launch_bounds__(kHeadBlock) k_head_train(const bf16_t* d, int ldd, const float* hw, const float* hb,
                                                           const float* rin, const float* target, float* out,
                                                           float* dout, bf16_t* g, float* part, int C, int P) {
    constexpr int K = KK;
    __shared__ float red[kHeadBlock * 9];
    const int G = C >> 3, t = threadIdx.x;
    const int cg = t % G, c = 8 * cg;
    const int per_block = kHeadBlock / G;
    const int p0 = blockIdx.x * per_block + t / G, stride = gridDim.x * per_block;
    const float scale = 2.f / (float)((size_t)K * P);
    float w[KK][8], acc[KK][8], bs[KK], r2 = 0.f;
#pragma unroll
    for (int k = 0; k < KK; ++k) {
        bs[k] = 0.f;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            acc[k][j] = 0.f;
            w[k][j] = hw[k * C + c + j];
        }
    }
    // two pixels per iteration, every load of both issued before any arithmetic
    auto pixel = [&](int p, const float (&v)[8], const float (&ri)[KK], const float (&tg)[KK]) {
        float dp[KK], o[8];
#pragma unroll
        for (int k = 0; k < KK; ++k) {
            float sk = 0.f;
#pragma unroll
            for (int j = 0; j < 8; ++j) sk += w[k][j] * v[j];
            // the pixel's G lanes are consecutive and G-aligned: partners are in the group
            for (int m = 1; m < G; m <<= 1) sk += __shfl_xor(sk, m, 64);
            sk += hb[k] + ri[k];
            const float r = sk - tg[k];
            dp[k] = scale * r;
            if (cg == 0) {
                out[(size_t)k * P + p] = sk;
                dout[(size_t)k * P + p] = dp[k];
                r2 += r * r;
            }
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            float sg = 0.f;
#pragma unroll
            for (int k = 0; k < KK; ++k) sg += dp[k] * w[k][j];
            o[j] = v[j] > 0.f ? sg : 0.f;
#pragma unroll
            for (int k = 0; k < KK; ++k) acc[k][j] += dp[k] * v[j];
        }
        st16(g + (size_t)p * C + c, pack8(o));
#pragma unroll
        for (int k = 0; k < KK; ++k) bs[k] += dp[k];
    };
    for (int p = p0; p < P; p += 2 * stride) {
        const int pb = p + stride;
        const bool two = pb < P;  // the same for the pixel's G lanes
        float va[8], vb[8], ra[KK], ta[KK], rb[KK], tb[KK];
        unpack8(ld16(d + (size_t)p * ldd + c), va);
        unpack8(ld16(d + (size_t)(two ? pb : p) * ldd + c), vb);
#pragma unroll
        for (int k = 0; k < KK; ++k) {
            ra[k] = rin[(size_t)k * P + p];
            ta[k] = target[(size_t)k * P + p];
            rb[k] = two ? rin[(size_t)k * P + pb] : 0.f;
            tb[k] = two ? target[(size_t)k * P + pb] : 0.f;
        }
        pixel(p, va, ra, ta);
        if (two) pixel(pb, vb, rb, tb);
    }
    const int m = K * (C + 1);
    float* row = part + (size_t)blockIdx.x * (m + 1);  // weight sums, then the loss sum
    const float lb = block_sum(r2, red);
    if (t == 0) row[m] = lb;
    for (int k = 0; k < K; ++k) {
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 8; ++j) red[t * 9 + j] = acc[k][j];
        red[t * 9 + 8] = bs[k];
        __syncthreads();
        for (int e = t; e < C + 1; e += kHeadBlock) {
            float sm = 0.f;
            if (e < C) {
                const int eg = e >> 3, ej = e & 7;
                for (int u = eg; u < kHeadBlock; u += G) sm += red[u * 9 + ej];
            } else {
                for (int u = 0; u < kHeadBlock; u += G) sm += red[u * 9 + 8];
            }
            row[k * (C + 1) + e] = sm;
        }
    }
}

// out[j] = sum over blocks of part[b][j] (j < m) times scale, one workgroup per j (with
// `last`, column m - 1 goes to last[0] times last_scale instead):
// thread t sums rows t, t + 256, ... in order, then a fixed tree combines the 256
// partial sums (deterministic).  With stride > 0 the entries j % stride == stride - 1
// go to out1[j / stride] and the others to out0 with those entries skipped.
__global__ void __launch_bounds__(256) k_sum_partials(const float* part, int blocks, int m, float scale, float* out0,
                                                      float* out1, int stride, float* last, float last_scale) {
    __shared__ double sm[256];
    const int j = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < blocks; b += 256) s += part[(size_t)b * m + j];
    sm[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    if (last && j == m - 1) {  // an extra last column with a scale and destination of its own
        last[0] = (float)(sm[0] * last_scale);
        return;
    }
    const float v = (float)(sm[0] * scale);
    if (stride > 0 && j % stride == stride - 1) out1[j / stride] = v;
    else if (stride > 0) out0[(j / stride) * (stride - 1) + j % stride] = v;
    else out0[j] = v;
}

__global__ void k_adam(float* p, const float* g, float* m, float* v, bf16_t* p16, size_t n, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    if (p16) p16[i] = (bf16_t)f2bf(pi);
}

__global__ void k_to_bf16(const float* s, bf16_t* d, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = (bf16_t)f2bf(s[i]);
}
__global__ void k_to_f32(const bf16_t* s, float* d, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = bf2f(s[i]);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int launched(const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(UNET_EHIP, "%s: %s", what, hipGetErrorString(e));
    return UNET_OK;
}

int log2_exact(int v) {
    if (v < 2 || (v & (v - 1))) return -1;
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// tensor argument checks shared by every call: 16-byte aligned vectors of 8 channels
int check_tensor(const char* name, const void* p, int ld, int off, int C, bool nullable) {
    if (!p) return nullable ? UNET_OK : fail(UNET_EINVAL, "%s is NULL", name);
    if (!aligned16(p)) return fail(UNET_EINVAL, "%s must be 16-byte aligned", name);
    if (ld % 8 || off % 8 || off < 0 || ld < off + C)
        return fail(UNET_EINVAL, "%s: ld (%d) and off (%d) must be multiples of 8 with ld >= off + C (%d)", name, ld,
                    off, C);
    return UNET_OK;
}

int check_geo(int N, int H, int W, int* lh, int* lw) {
    *lh = log2_exact(H);
    *lw = log2_exact(W);
    if (N < 1 || *lh < 0 || *lw < 0) return fail(UNET_EINVAL, "N >= 1 and H, W powers of two >= 2 (got %d, %d, %d)", N, H, W);
    if ((int64_t)N * H * W >= ((int64_t)1 << 31)) return fail(UNET_EINVAL, "N H W must stay below 2^31");
    return UNET_OK;
}

// one thread per 8 channels of a full-resolution pixel must fit the int thread index
int check_threads(int N, int H, int W, int C) {
    if ((int64_t)N * H * W * (C / 8) >= ((int64_t)1 << 31))
        return fail(UNET_EINVAL, "N H W C/8 must stay below 2^31 (got %d, %d, %d, %d)", N, H, W, C);
    return UNET_OK;
}

template <int MT, int NT>
void launch_conv(const ConvArgs& a, bool tap_outer, bool f32, hipStream_t s) {
    const dim3 grid((a.P + 64 * MT - 1) / (64 * MT), (a.Cout + 16 * NT - 1) / (16 * NT));
    if (tap_outer) {
        if (f32) hipLaunchKernelGGL((k_conv3x3<MT, NT, true, true>), grid, dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_conv3x3<MT, NT, true, false>), grid, dim3(256), 0, s, a);
    } else {
        if (f32) hipLaunchKernelGGL((k_conv3x3<MT, NT, false, true>), grid, dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_conv3x3<MT, NT, false, false>), grid, dim3(256), 0, s, a);
    }
}

template <int BM, int BN, int WM, int WN>
void launch_lds(const ConvArgs& a, bool f32, hipStream_t s) {
    const dim3 grid((a.P / BM) * (a.Cout / BN));
    if (f32) hipLaunchKernelGGL((k_conv_lds<BM, BN, WM, WN, true>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_conv_lds<BM, BN, WM, WN, false>), grid, dim3(256), 0, s, a);
}

// The LDS-staged kernel where its shape conditions hold; false: use k_conv3x3.
// bf16 output is written in 16-byte vectors: it needs an aligned output and stride.
bool launch_conv_lds(const ConvArgs& a, bool f32, hipStream_t s) {
    if (!f32 && (!aligned16(a.y) || a.ldy % 8)) return false;
    if (!f32 && a.ysplit < a.Cout && (!aligned16(a.y2) || a.ldy2 % 8)) return false;
    if (a.Cin == 8 && a.lw >= 4 && a.lh >= 4 && a.Cout % 32 == 0) {
        const dim3 grid((a.P / 256) * (a.Cout / 32));
        if (f32) hipLaunchKernelGGL((k_conv_halo8<true>), grid, dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_conv_halo8<false>), grid, dim3(256), 0, s, a);
        return true;
    }
    if (a.Cin % 32) return false;
    // 16 x 16 pixel tiles: H and W multiples of 16
    if (a.lw >= 4 && a.lh >= 4 && a.Cout % 32 == 0) {
        const dim3 grid((a.P / 256) * (a.Cout / 32));
        if (a.Cin == 32) {
            if (f32) hipLaunchKernelGGL((k_conv_halo<true, true, 32>), grid, dim3(256), 0, s, a);
            else hipLaunchKernelGGL((k_conv_halo<false, true, 32>), grid, dim3(256), 0, s, a);
        } else if (a.Cout % 64 == 0) {
            const dim3 grid64((a.P / 256) * (a.Cout / 64));
            if (f32) hipLaunchKernelGGL((k_conv_halo<true, false, 64>), grid64, dim3(256), 0, s, a);
            else hipLaunchKernelGGL((k_conv_halo<false, false, 64>), grid64, dim3(256), 0, s, a);
        } else {
            if (f32) hipLaunchKernelGGL((k_conv_halo<true, false, 32>), grid, dim3(256), 0, s, a);
            else hipLaunchKernelGGL((k_conv_halo<false, false, 32>), grid, dim3(256), 0, s, a);
        }
        return true;
    }
    if (a.Cout % 128 == 0 && a.P % 128 == 0) {
        launch_lds<128, 128, 2, 2>(a, f32, s);
    } else if (a.Cout % 64 == 0 && a.P % 256 == 0) {
        launch_lds<256, 64, 4, 1>(a, f32, s);
    } else if (a.Cout % 32 == 0 && a.P % 128 == 0) {
        launch_lds<128, 32, 4, 1>(a, f32, s);
    } else {
        return false;
    }
    return true;
}

struct WgPlan {
    int ktiles, ctiles, CT, slabs, slab, Kt;
    bool tr;    // k_wgrad_tr (C_out % 32 == 0), else k_wgrad
    bool halo;  // k_wgrad_halo (or k_wgrad_halo8): ktiles = input-channel blocks, slab in 256-pixel tiles
    bool halo8; // C_in = 8: k_wgrad_halo8, one input-channel block
};

WgPlan wgrad_plan(int P, int lh, int lw, int Cin, int Cout) {
    WgPlan w;
    const int K = 9 * Cin;
    // the halo-tile form wherever its tiles fit: with the next tile prefetched it beats
    // the im2col form on every such layer of the network (measured, 256^2 x 16)
    w.halo8 = Cin == 8 && (Cout == 32 || Cout % 64 == 0) && lh >= 4 && lw >= 4;
    w.halo = w.halo8 || (Cin % 32 == 0 && (Cout == 32 || Cout % 64 == 0) && lh >= 4 && lw >= 4);
    if (w.halo) {
        w.tr = false;
        w.CT = Cout % 64 == 0 ? 64 : 32;
        w.ktiles = w.halo8 ? 1 : Cin / 32;
        w.ctiles = Cout / w.CT;
        w.Kt = (K + 1 + 31) / 32 * 32;
        const int tiles = P >> 8;
        int slabs = (512 + w.ktiles * w.ctiles - 1) / (w.ktiles * w.ctiles);
        if (slabs > tiles) slabs = tiles;
        if (slabs < 1) slabs = 1;
        w.slab = (tiles + slabs - 1) / slabs;
        w.slabs = (tiles + w.slab - 1) / w.slab;
        return w;
    }
    w.tr = Cout % 32 == 0;
    const int BK = w.tr ? (Cout % 64 == 0 ? 256 : 128) : 64;  // k columns per workgroup
    w.ktiles = (K + 1 + BK - 1) / BK;
    w.Kt = BK * w.ktiles;
    w.CT = Cout % 64 == 0 ? 64 : 32;
    w.ctiles = (Cout + w.CT - 1) / w.CT;
    // workgroups to aim for: fewer, longer slabs keep the FP32 partials (slabs x C_out x Kt)
    // and their reduction small
    const int want = w.tr ? 512 : 1024;
    int slabs = (want + w.ktiles * w.ctiles - 1) / (w.ktiles * w.ctiles);
    const int max_slabs = (P + 255) / 256;  // at least 256 pixels per slab
    if (slabs > max_slabs) slabs = max_slabs;
    if (slabs < 1) slabs = 1;
    w.slab = ((P + slabs - 1) / slabs + 63) / 64 * 64;  // whole 64-pixel chunks
    w.slabs = (P + w.slab - 1) / w.slab;
    return w;
}

}  // namespace
}  // namespace unet_dev

using namespace unet_dev;

extern "C" {

}  // extern "C"

namespace {

// Checks the arguments of the two-tensor convolution and fills *a (no 2x2 work).
int conv_cat_args(const void* x, int32_t ldx, int32_t offx, int32_t C_x, int32_t half, const void* x2, int32_t ldx2,
                  int32_t offx2, const void* w, const float* bias, void* y, int32_t ldy, int32_t offy, int32_t C_y,
                  void* y2, int32_t ldy2, int32_t offy2, const void* mask, int32_t ldm, int32_t offm, int32_t N,
                  int32_t H, int32_t W, int32_t C_in, int32_t C_out, int32_t flags, ConvArgs* out_args) {
    int lh, lw, r;
    if ((r = check_geo(N, H, W, &lh, &lw))) return r;
    if (C_in < 8 || C_in % 8 || C_out < 16 || C_out % 16)
        return fail(UNET_EINVAL, "C_in must be a multiple of 8 and C_out of 16 (got %d, %d)", C_in, C_out);
    if (flags & ~(UNET_RELU | UNET_OUT_F32)) return fail(UNET_EINVAL, "unknown flags %d", flags);
    if (C_x < 8 || C_x > C_in || C_x % 8 || (C_in % 32 == 0 && C_x % 32))
        return fail(UNET_EINVAL, "C_x must be a multiple of 8 in [8, C_in], of 32 when C_in is (got %d, C_in %d)",
                    C_x, C_in);
    if (C_y < 8 || C_y > C_out || C_y % 8)
        return fail(UNET_EINVAL, "C_y must be a multiple of 8 in [8, C_out] (got %d, C_out %d)", C_y, C_out);
    if ((r = check_tensor("x", x, ldx, offx, C_x, false))) return r;
    if (C_x < C_in) {
        if ((r = check_tensor("x2", x2, ldx2, offx2, C_in - C_x, false))) return r;
    } else if (x2) {
        return fail(UNET_EINVAL, "x2 must be NULL when C_x = C_in");
    }
    if ((r = check_tensor("mask", mask, ldm, offm, C_out, true))) return r;
    if (!w || !aligned16(w)) return fail(UNET_EINVAL, "w must be non-NULL and 16-byte aligned");
    if (!y || ldy < offy + C_y || offy < 0) return fail(UNET_EINVAL, "y: need ld >= off + C_y");
    if (C_y < C_out) {
        if (!y2 || ldy2 < offy2 + (C_out - C_y) || offy2 < 0)
            return fail(UNET_EINVAL, "y2: need ld >= off + C_out - C_y");
    } else if (y2) {
        return fail(UNET_EINVAL, "y2 must be NULL when C_y = C_out");
    }
    const bool f32 = flags & UNET_OUT_F32;
    auto out = [&](void* base, int off) -> void* {
        if (!base) return nullptr;
        return f32 ? (void*)(static_cast<float*>(base) + off) : (void*)(static_cast<bf16_t*>(base) + off);
    };
    ConvArgs& a = *out_args;
    a.x = static_cast<const bf16_t*>(x) + offx;
    a.x2 = x2 ? static_cast<const bf16_t*>(x2) + offx2 : nullptr;
    a.w = static_cast<const bf16_t*>(w);
    a.bias = bias;
    a.y = out(y, offy);
    a.y2 = out(y2, offy2);
    a.mask = mask ? static_cast<const bf16_t*>(mask) + offm : nullptr;
    a.ldx = ldx;
    a.ldx2 = ldx2;
    a.ldy = ldy;
    a.ldy2 = ldy2;
    a.ldm = ldm;
    a.split = C_x;
    a.half = half ? 1 : 0;
    a.ysplit = C_y;
    a.lh = lh;
    a.lw = lw;
    a.P = N * H * W;
    a.Cin = C_in;
    a.Cout = C_out;
    a.relu = (flags & UNET_RELU) ? 1 : 0;
    a.yp = nullptr;
    a.gate = nullptr;
    a.ldyp = a.ldgt = a.down = 0;
    return UNET_OK;
}

int conv_launch(const ConvArgs& a, bool f32, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool tap_outer = a.Cin % 32 == 0;
    if (!launch_conv_lds(a, f32, s)) {
        if (a.Cout % 64 == 0) launch_conv<2, 4>(a, tap_outer, f32, s);
        else launch_conv<4, 2>(a, tap_outer, f32, s);
    }
    return launched("conv3x3 launch");
}

// The 2x2 forms run in k_conv_halo only: bfloat16 output, 16 x 16 tiles, C_in % 32 == 0,
// C_out % 32 == 0, and (for the upsampling gradient) the split at a multiple of the
// workgroup's output width, so that each workgroup's channels are all on one side.
int halo_width(const ConvArgs& a) {
    if (a.lh < 4 || a.lw < 4 || a.Cin % 32 || a.Cout % 32) return 0;
    return (a.Cin != 32 && a.Cout % 64 == 0) ? 64 : 32;
}

}  // namespace

extern "C" {

int unet_conv3x3_fwd_cat(const void* x, int32_t ldx, int32_t offx, int32_t C_x, int32_t half, const void* x2,
                         int32_t ldx2, int32_t offx2, const void* w, const float* bias, void* y, int32_t ldy,
                         int32_t offy, int32_t C_y, void* y2, int32_t ldy2, int32_t offy2, const void* mask,
                         int32_t ldm, int32_t offm, int32_t N, int32_t H, int32_t W, int32_t C_in, int32_t C_out,
                         int32_t flags, void* stream) {
    ConvArgs a;
    const int r = conv_cat_args(x, ldx, offx, C_x, half, x2, ldx2, offx2, w, bias, y, ldy, offy, C_y, y2, ldy2, offy2,
                                mask, ldm, offm, N, H, W, C_in, C_out, flags, &a);
    return r ? r : conv_launch(a, flags & UNET_OUT_F32, stream);
}

int unet_conv3x3_fwd_pool(const void* x, int32_t ldx, int32_t offx, const void* w, const float* bias, void* y,
                          int32_t ldy, int32_t offy, void* yp, int32_t ldyp, int32_t offyp, int32_t N, int32_t H,
                          int32_t W, int32_t C_in, int32_t C_out, int32_t flags, void* stream) {
    if (flags & UNET_OUT_F32) return fail(UNET_EINVAL, "conv + pool: bfloat16 output only");
    ConvArgs a;
    int r = conv_cat_args(x, ldx, offx, C_in, 0, nullptr, 0, 0, w, bias, y, ldy, offy, C_out, nullptr, 0, 0, nullptr,
                          0, 0, N, H, W, C_in, C_out, flags, &a);
    if (r) return r;
    if ((r = check_tensor("y", y, ldy, offy, C_out, false)) || (r = check_tensor("yp", yp, ldyp, offyp, C_out, false)))
        return r;
    if (!halo_width(a)) return fail(UNET_ESHAPE, "conv + pool: needs H, W >= 16 and C_in, C_out multiples of 32");
    a.down = 1;
    a.yp = static_cast<bf16_t*>(yp) + offyp;
    a.ldyp = ldyp;
    return conv_launch(a, false, stream);
}

int unet_conv3x3_bwd_upcat(const void* g, int32_t ldg, int32_t offg, const void* wf, void* dlow, int32_t lddl,
                           int32_t offdl, const void* low, int32_t ldlow, int32_t offlow, int32_t C_low, void* dskip,
                           int32_t ldds, int32_t offds, int32_t N, int32_t H, int32_t W, int32_t C_g, int32_t C_in,
                           void* stream) {
    ConvArgs a;
    if (C_low < 8 || C_low >= C_in || C_low % 8)
        return fail(UNET_EINVAL, "bwd upcat: C_low must be a multiple of 8 below C_in (got %d, C_in %d)", C_low, C_in);
    // the full-size tensor of the upsampled branch is never written: y gets the split
    // only for the argument checks, the stores go to dlow at half size
    int r = conv_cat_args(g, ldg, offg, C_g, 0, nullptr, 0, 0, wf, nullptr, dlow, lddl, offdl, C_low, dskip, ldds,
                          offds, nullptr, 0, 0, N, H, W, C_g, C_in, 0, &a);
    if (r) return r;
    if ((r = check_tensor("dlow", dlow, lddl, offdl, C_low, false)) ||
        (r = check_tensor("low", low, ldlow, offlow, C_low, false)) ||
        (r = check_tensor("dskip", dskip, ldds, offds, C_in - C_low, false)))
        return r;
    const int bn = halo_width(a);
    if (!bn || C_low % bn)
        return fail(UNET_ESHAPE, "bwd upcat: needs H, W >= 16, C_g and C_in multiples of 32 and C_low of %d",
                    bn ? bn : 32);
    a.down = 2;
    a.gate = static_cast<const bf16_t*>(low) + offlow;
    a.ldgt = ldlow;
    return conv_launch(a, false, stream);
}

int unet_conv3x3_fwd(const void* x, int32_t ldx, int32_t offx, const void* w, const float* bias, void* y,
                     int32_t ldy, int32_t offy, const void* mask, int32_t ldm, int32_t offm, int32_t N, int32_t H,
                     int32_t W, int32_t C_in, int32_t C_out, int32_t flags, void* stream) {
    if (C_in < 8 || C_in % 8 || C_out < 16 || C_out % 16)
        return fail(UNET_EINVAL, "C_in must be a multiple of 8 and C_out of 16 (got %d, %d)", C_in, C_out);
    return unet_conv3x3_fwd_cat(x, ldx, offx, C_in, 0, nullptr, 0, 0, w, bias, y, ldy, offy, C_out, nullptr, 0, 0,
                                mask, ldm, offm, N, H, W, C_in, C_out, flags, stream);
}

int unet_flip_weights(const void* w, void* wf, int32_t C_out, int32_t C_in, void* stream) {
    if (!w || !wf || C_out < 1 || C_in < 1) return fail(UNET_EINVAL, "flip: bad arguments");
    const int n = C_out * 9 * C_in;
    hipLaunchKernelGGL(k_flip, dim3((n + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(stream),
                       static_cast<const bf16_t*>(w), static_cast<bf16_t*>(wf), C_out, C_in);
    return launched("flip launch");
}

int unet_flip_weights_many(const void* const* w, void* const* wf, const int32_t* C_out, const int32_t* C_in,
                           int32_t n, void* stream) {
    if (!w || !wf || !C_out || !C_in || n < 1 || n > kFlipMax) return fail(UNET_EINVAL, "flip many: bad arguments");
    FlipSet f;
    f.n = n;
    int blocks = 0;
    for (int l = 0; l < n; ++l) {
        if (!w[l] || !wf[l] || C_out[l] < 1 || C_in[l] < 1 || (int64_t)C_out[l] * 9 * C_in[l] >= (1 << 30))
            return fail(UNET_EINVAL, "flip many: bad entry %d", l);
        f.w[l] = static_cast<const bf16_t*>(w[l]);
        f.wf[l] = static_cast<bf16_t*>(wf[l]);
        f.cout[l] = C_out[l];
        f.cin[l] = C_in[l];
        f.first[l] = blocks;
        blocks += (C_out[l] * 9 * C_in[l] + 255) / 256;
    }
    f.first[n] = blocks;
    hipLaunchKernelGGL(k_flip_many, dim3(blocks), dim3(256), 0, static_cast<hipStream_t>(stream), f);
    return launched("flip many launch");
}

int unet_wgrad_partial_bytes(int32_t N, int32_t H, int32_t W, int32_t C_in, int32_t C_out, size_t* bytes) {
    int lh, lw, r;
    if ((r = check_geo(N, H, W, &lh, &lw))) return r;
    if (!bytes || C_in < 8 || C_in % 8 || C_out < 16 || C_out % 16) return fail(UNET_EINVAL, "wgrad: bad channels");
    const WgPlan p = wgrad_plan(N * H * W, lh, lw, C_in, C_out);
    *bytes = (size_t)p.slabs * C_out * p.Kt * sizeof(float);
    return UNET_OK;
}

}  // extern "C"

// Partial sums of unet_conv3x3_wgrad_noalloc.  In host code `scratch` names a host-side
// stand-in, not device memory: its device address is looked up once per device with
// hipGetSymbolAddress and only that address is ever handed to a kernel.
static __device__ __align__(256) float scratch[UNET_WGRAD_SCRATCH_BYTES / sizeof(float)];

namespace {

// Checks the arguments shared by both weight-gradient entry points; *need gets the
// partials size of this shape.
// The layer input of a weight gradient: channels [0, C_x) from x (at half the size when
// half), [C_x, C_in) from x2 (NULL when C_x = C_in); offsets not yet applied.
struct WgIn {
    const void* x;
    int32_t ldx, offx, C_x, half;
    const void* x2;
    int32_t ldx2, offx2;
};

int wgrad_check(const WgIn& in, const void* g, int32_t ldg, int32_t offg, const float* dw, int32_t N, int32_t H,
                int32_t W, int32_t C_in, int32_t C_out, size_t* need) {
    int r;
    if ((r = unet_wgrad_partial_bytes(N, H, W, C_in, C_out, need))) return r;
    if (in.C_x < 8 || in.C_x > C_in || in.C_x % 8 || (C_in % 32 == 0 && in.C_x % 32))
        return fail(UNET_EINVAL, "C_x must be a multiple of 8 in [8, C_in], of 32 when C_in is (got %d, C_in %d)",
                    in.C_x, C_in);
    if ((r = check_tensor("x", in.x, in.ldx, in.offx, in.C_x, false))) return r;
    if (in.C_x < C_in) {
        if ((r = check_tensor("x2", in.x2, in.ldx2, in.offx2, C_in - in.C_x, false))) return r;
    } else if (in.x2) {
        return fail(UNET_EINVAL, "x2 must be NULL when C_x = C_in");
    }
    if ((r = check_tensor("g", g, ldg, offg, C_out, false))) return r;
    if (!dw) return fail(UNET_EINVAL, "dw is NULL");
    return UNET_OK;
}

// Launches the split weight gradient with its partial sums in `partials` (device memory
// of at least the checked size) and the fixed-order reduction.
int wgrad_launch(const WgIn& in, const void* g, int32_t ldg, int32_t offg, float* dw, float* db, void* partials,
                 int32_t N, int32_t H, int32_t W, int32_t C_in, int32_t C_out, void* stream) {
    int r;
    int lh, lw;
    check_geo(N, H, W, &lh, &lw);
    const WgPlan p = wgrad_plan(N * H * W, lh, lw, C_in, C_out);
    WgArgs a;
    a.x = static_cast<const bf16_t*>(in.x) + in.offx;
    a.x2 = in.x2 ? static_cast<const bf16_t*>(in.x2) + in.offx2 : nullptr;
    a.g = static_cast<const bf16_t*>(g) + offg;
    a.part = static_cast<float*>(partials);
    a.ldx = in.ldx;
    a.ldx2 = in.ldx2;
    a.split = in.C_x;
    a.half = in.half ? 1 : 0;
    a.ldg = ldg;
    a.lh = lh;
    a.lw = lw;
    a.P = N * H * W;
    a.Cin = C_in;
    a.Cout = C_out;
    a.K = 9 * C_in;
    a.Kt = p.Kt;
    a.slab = p.slab;
    a.ktiles = p.ktiles;
    a.ctiles = p.ctiles;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const dim3 grid(p.ktiles, p.ctiles, p.slabs);
    if (p.halo8) {
        const dim3 flat(p.ctiles * p.slabs);
        if (p.CT == 64) hipLaunchKernelGGL((k_wgrad_halo8<64>), flat, dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_wgrad_halo8<32>), flat, dim3(256), 0, s, a);
    } else if (p.halo) {
        const dim3 flat(p.ktiles * p.ctiles * p.slabs);
        if (p.CT == 64) hipLaunchKernelGGL((k_wgrad_halo<64>), flat, dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_wgrad_halo<32>), flat, dim3(256), 0, s, a);
    } else if (p.tr) {
        const dim3 flat(p.ktiles * p.ctiles * p.slabs);
        if (p.CT == 64) hipLaunchKernelGGL((k_wgrad_tr<64, 256, 32, 2>), flat, dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_wgrad_tr<32, 128, 64, 1>), flat, dim3(256), 0, s, a);
    } else {
        if (p.CT == 64) hipLaunchKernelGGL((k_wgrad<64>), grid, dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_wgrad<32>), grid, dim3(256), 0, s, a);
    }
    if ((r = launched("wgrad launch"))) return r;
    const int n = C_out * (a.K + 1);
    if (p.slabs >= 256)
        hipLaunchKernelGGL((k_wgrad_reduce<16, 8>), dim3((n + 63) / 64), dim3(1024), 0, s, a.part, dw, db, p.slabs,
                           C_out, a.K, p.Kt);
    else
        hipLaunchKernelGGL((k_wgrad_reduce<4, 4>), dim3((n + 63) / 64), dim3(256), 0, s, a.part, dw, db, p.slabs,
                           C_out, a.K, p.Kt);
    return launched("wgrad reduce launch");
}

constexpr int kMaxDevices = 64;
std::mutex g_device_mutex;  // guards the per-device lookups below
float* g_scratch_ptr[kMaxDevices] = {};

// Workgroups of k_head_train<K> resident on the whole current device at once (the
// occupancy query times the CU count), looked up on the first call per device and K.
int g_head_round[kMaxDevices][4] = {};

int head_train_round(int K, int* out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(UNET_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(UNET_EINVAL, "device %d beyond the %d supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_device_mutex);
    int& slot = g_head_round[dev][K - 1];
    if (!slot) {
        int resident = 0, cus = 0;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess) {
            switch (K) {
                case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&resident, k_head_train<1>, kHeadBlock, 0); break;
                case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&resident, k_head_train<2>, kHeadBlock, 0); break;
                case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&resident, k_head_train<3>, kHeadBlock, 0); break;
                default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&resident, k_head_train<4>, kHeadBlock, 0);
            }
        }
        if (e != hipSuccess) return fail(UNET_EHIP, "head train: occupancy query: %s", hipGetErrorString(e));
        slot = std::max(resident, 1) * std::max(cus, 1);
    }
    *out = slot;
    return UNET_OK;
}

// Device address of `scratch` on the current device (looked up on the first call there).
int scratch_on_current_device(float** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(UNET_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(UNET_EINVAL, "device %d beyond the %d supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_device_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(UNET_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<float*>(p);
    }
    *out = g_scratch_ptr[dev];
    return UNET_OK;
}

}  // namespace

extern "C" {

int unet_conv3x3_wgrad_cat(const void* x, int32_t ldx, int32_t offx, int32_t C_x, int32_t half, const void* x2,
                           int32_t ldx2, int32_t offx2, const void* g, int32_t ldg, int32_t offg, float* dw, float* db,
                           void* partials, size_t partial_bytes, int32_t N, int32_t H, int32_t W, int32_t C_in,
                           int32_t C_out, void* stream) {
    const WgIn in{x, ldx, offx, C_x, half, x2, ldx2, offx2};
    size_t need = 0;
    int r;
    if ((r = wgrad_check(in, g, ldg, offg, dw, N, H, W, C_in, C_out, &need))) return r;
    if (!partials || partial_bytes < need) return fail(UNET_EINVAL, "partials: %zu bytes needed", need);
    return wgrad_launch(in, g, ldg, offg, dw, db, partials, N, H, W, C_in, C_out, stream);
}

int unet_conv3x3_wgrad(const void* x, int32_t ldx, int32_t offx, const void* g, int32_t ldg, int32_t offg, float* dw,
                       float* db, void* partials, size_t partial_bytes, int32_t N, int32_t H, int32_t W, int32_t C_in,
                       int32_t C_out, void* stream) {
    return unet_conv3x3_wgrad_cat(x, ldx, offx, C_in, 0, nullptr, 0, 0, g, ldg, offg, dw, db, partials,
                                  partial_bytes, N, H, W, C_in, C_out, stream);
}

int unet_conv3x3_wgrad_noalloc(const void* x, int32_t ldx, int32_t offx, const void* g, int32_t ldg, int32_t offg,
                               float* dw, float* db, int32_t N, int32_t H, int32_t W, int32_t C_in, int32_t C_out,
                               void* stream) {
    const WgIn in{x, ldx, offx, C_in, 0, nullptr, 0, 0};
    size_t need = 0;
    int r;
    if ((r = wgrad_check(in, g, ldg, offg, dw, N, H, W, C_in, C_out, &need))) return r;
    if (need > UNET_WGRAD_SCRATCH_BYTES)
        return fail(UNET_EINVAL, "wgrad_noalloc: this shape needs %zu bytes of partial sums, above the %zu-byte "
                                 "static scratch; use unet_conv3x3_wgrad with a caller workspace",
                    need, (size_t)UNET_WGRAD_SCRATCH_BYTES);
    float* part = nullptr;
    if ((r = scratch_on_current_device(&part))) return r;
    return wgrad_launch(in, g, ldg, offg, dw, db, part, N, H, W, C_in, C_out, stream);
}

int unet_maxpool2_fwd(const void* x, int32_t ldx, int32_t offx, void* y, int32_t ldy, int32_t offy, int32_t N,
                      int32_t H, int32_t W, int32_t C, void* stream) {
    int lh, lw, r;
    if ((r = check_geo(N, H, W, &lh, &lw))) return r;
    if (C < 8 || C % 8) return fail(UNET_EINVAL, "C must be a multiple of 8");
    if ((r = check_threads(N, H, W, C))) return r;
    if ((r = check_tensor("x", x, ldx, offx, C, false)) || (r = check_tensor("y", y, ldy, offy, C, false))) return r;
    const Geo g{N, lh, lw, C};
    const int total = N * (H / 2) * (W / 2) * (C / 8);
    hipLaunchKernelGGL(k_pool_fwd, dim3((total + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(stream),
                       static_cast<const bf16_t*>(x) + offx, ldx, static_cast<bf16_t*>(y) + offy, ldy, g, total);
    return launched("maxpool launch");
}

int unet_maxpool2_bwd(const void* x, int32_t ldx, int32_t offx, const void* dy, int32_t lddy, int32_t offdy,
                      const void* add, int32_t lda, int32_t offa, void* dx, int32_t lddx, int32_t offdx,
                      int32_t gate_relu, int32_t N, int32_t H, int32_t W, int32_t C, void* stream) {
    int lh, lw, r;
    if ((r = check_geo(N, H, W, &lh, &lw))) return r;
    if (C < 8 || C % 8) return fail(UNET_EINVAL, "C must be a multiple of 8");
    if ((r = check_threads(N, H, W, C))) return r;
    if ((r = check_tensor("x", x, ldx, offx, C, false)) || (r = check_tensor("dy", dy, lddy, offdy, C, false)) ||
        (r = check_tensor("add", add, lda, offa, C, true)) || (r = check_tensor("dx", dx, lddx, offdx, C, false)))
        return r;
    const Geo g{N, lh, lw, C};
    const int total = N * (H / 2) * (W / 2) * (C / 8);
    hipLaunchKernelGGL(k_pool_bwd, dim3((total + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(stream),
                       static_cast<const bf16_t*>(x) + offx, ldx, static_cast<const bf16_t*>(dy) + offdy, lddy,
                       add ? static_cast<const bf16_t*>(add) + offa : nullptr, lda,
                       static_cast<bf16_t*>(dx) + offdx, lddx, gate_relu ? 1 : 0, g, total);
    return launched("maxpool bwd launch");
}

int unet_upsample2_fwd(const void* x, int32_t ldx, int32_t offx, void* y, int32_t ldy, int32_t offy, int32_t N,
                       int32_t H, int32_t W, int32_t C, void* stream) {
    int lh, lw, r;
    if ((r = check_geo(N, 2 * H, 2 * W, &lh, &lw))) return r;
    if (C < 8 || C % 8) return fail(UNET_EINVAL, "C must be a multiple of 8");
    if ((r = check_threads(N, 2 * H, 2 * W, C))) return r;
    if ((r = check_tensor("x", x, ldx, offx, C, false)) || (r = check_tensor("y", y, ldy, offy, C, false))) return r;
    const Geo g{N, lh, lw, C};
    const int total = N * H * W * (C / 8);
    hipLaunchKernelGGL(k_up_fwd, dim3((total + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(stream),
                       static_cast<const bf16_t*>(x) + offx, ldx, static_cast<bf16_t*>(y) + offy, ldy, g, total);
    return launched("upsample launch");
}

int unet_upsample2_bwd(const void* dy, int32_t lddy, int32_t offdy, const void* gate, int32_t ldgt, int32_t offgt,
                       void* dx, int32_t lddx, int32_t offdx, int32_t N, int32_t H, int32_t W, int32_t C,
                       void* stream) {
    int lh, lw, r;
    if ((r = check_geo(N, 2 * H, 2 * W, &lh, &lw))) return r;
    if (C < 8 || C % 8) return fail(UNET_EINVAL, "C must be a multiple of 8");
    if ((r = check_threads(N, 2 * H, 2 * W, C))) return r;
    if ((r = check_tensor("dy", dy, lddy, offdy, C, false)) || (r = check_tensor("gate", gate, ldgt, offgt, C, true)) ||
        (r = check_tensor("dx", dx, lddx, offdx, C, false)))
        return r;
    const Geo g{N, lh, lw, C};
    const int total = N * H * W * (C / 8);
    hipLaunchKernelGGL(k_up_bwd, dim3((total + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(stream),
                       static_cast<const bf16_t*>(dy) + offdy, lddy,
                       gate ? static_cast<const bf16_t*>(gate) + offgt : nullptr, ldgt,
                       static_cast<bf16_t*>(dx) + offdx, lddx, g, total);
    return launched("upsample bwd launch");
}

int unet_prepare_input(const double* rho, const double* T, const double* rho_v, const double* rho_l,
                       const double* T0, const double* cond, double theta_scale, void* x, float* rin, int32_t N,
                       int32_t H, int32_t W, void* stream) {
    int lh, lw, r;
    if ((r = check_geo(N, H, W, &lh, &lw))) return r;
    if (!rho || !rho_v || !rho_l || !T0 || !cond || (!x && !rin) || (x && !aligned16(x)) || !(theta_scale > 0))
        return fail(UNET_EINVAL, "prepare: bad pointers or theta_scale");
    const int total = N * H * W;
    hipLaunchKernelGGL(k_prepare, dim3((total + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(stream), rho, T,
                       rho_v, rho_l, T0, cond, theta_scale, static_cast<bf16_t*>(x), rin, lh + lw, total);
    return launched("prepare launch");
}

int unet_output_fields(const float* out, int32_t K, const double* rho_v, const double* rho_l, const double* T0,
                       double theta_scale, double* rho, double* T, int32_t N, int32_t H, int32_t W, void* stream) {
    int lh, lw, r;
    if ((r = check_geo(N, H, W, &lh, &lw))) return r;
    if (!out || !rho_v || !rho_l || !rho || K < 1 || K > 4 || (T && !T0) || !(theta_scale > 0))
        return fail(UNET_EINVAL, "output: bad arguments");
    const int total = N * H * W;
    hipLaunchKernelGGL(k_output, dim3((total + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(stream), out, K, rho_v,
                       rho_l, T0, theta_scale, rho, T, lh + lw, total);
    return launched("output launch");
}

int unet_head_partial_bytes(int32_t N, int32_t H, int32_t W, int32_t C, int32_t K, size_t* bytes) {
    int lh, lw, r;
    if ((r = check_geo(N, H, W, &lh, &lw))) return r;
    if (!bytes || C < 8 || C % 8 || K < 1 || K > 4) return fail(UNET_EINVAL, "head: bad channels or outputs");
    const size_t blocks = ((size_t)N * H * W + kHeadBlock - 1) / kHeadBlock;
    *bytes = blocks * (kHeadBlock / 64) * K * (C + 1) * sizeof(float);  // one row per wavefront
    return UNET_OK;
}

int unet_head_fwd(const void* d, int32_t ldd, const float* hw, const float* hb, const float* rin, const float* target,
                  float* out, float* dout, float* loss, void* partials, size_t partial_bytes, int32_t N, int32_t H,
                  int32_t W, int32_t C, int32_t K, void* stream) {
    size_t need = 0;
    int r;
    if ((r = unet_head_partial_bytes(N, H, W, C, K, &need))) return r;
    if ((r = check_tensor("d", d, ldd, 0, C, false))) return r;
    if (!hw || !hb || !rin || !out) return fail(UNET_EINVAL, "head: NULL argument");
    if (target && (!dout || !loss || !partials || partial_bytes < need))
        return fail(UNET_EINVAL, "head with a target needs dout, loss and %zu bytes of partials", need);
    const int P = N * H * W, blocks = (P + kHeadBlock - 1) / kHeadBlock;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_head_fwd, dim3(blocks), dim3(kHeadBlock), 0, s, static_cast<const bf16_t*>(d), ldd, hw, hb,
                       rin, target, out, dout, static_cast<float*>(partials), C, K, P);
    if ((r = launched("head launch"))) return r;
    if (target) {
        hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, static_cast<const float*>(partials), blocks, 1,
                           1.0f / (float)((size_t)K * P), loss, (float*)nullptr, 0, (float*)nullptr, 0.f);
        return launched("loss reduce launch");
    }
    return UNET_OK;
}

int unet_head_bwd(const void* d, int32_t ldd, const float* hw, const float* dout, void* g, float* dhw, float* dhb,
                  void* partials, size_t partial_bytes, int32_t N, int32_t H, int32_t W, int32_t C, int32_t K,
                  void* stream) {
    size_t need = 0;
    int r;
    if ((r = unet_head_partial_bytes(N, H, W, C, K, &need))) return r;
    if ((r = check_tensor("d", d, ldd, 0, C, false)) || (r = check_tensor("g", g, C, 0, C, false))) return r;
    if (!hw || !dout || !dhw || !dhb || !partials || partial_bytes < need)
        return fail(UNET_EINVAL, "head bwd: NULL argument or partials below %zu bytes", need);
    if (kHeadBlock % (C / 8) != 0) return fail(UNET_EINVAL, "head bwd: C / 8 must divide %d (got C = %d)", kHeadBlock, C);
    const int P = N * H * W;
    // no more workgroups than the forward pass uses, so its partials buffer suffices
    const int blocks = std::min((P + kHeadBlock - 1) / kHeadBlock, kHeadBwdBlocks);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_head_bwd, dim3(blocks), dim3(kHeadBlock), 0, s, static_cast<const bf16_t*>(d), ldd, hw, dout,
                       static_cast<bf16_t*>(g), static_cast<float*>(partials), C, K, P);
    if ((r = launched("head bwd launch"))) return r;
    const int m = K * (C + 1);
    hipLaunchKernelGGL(k_sum_partials, dim3(m), dim3(256), 0, s, static_cast<const float*>(partials), blocks, m,
                       1.0f, dhw, dhb, C + 1, (float*)nullptr, 0.f);
    return launched("head reduce launch");
}

int unet_head_train(const void* d, int32_t ldd, const float* hw, const float* hb, const float* rin,
                    const float* target, float* out, float* dout, float* loss, void* g, float* dhw, float* dhb,
                    void* partials, size_t partial_bytes, int32_t N, int32_t H, int32_t W, int32_t C, int32_t K,
                    void* stream) {
    size_t need = 0;
    int r;
    if ((r = unet_head_partial_bytes(N, H, W, C, K, &need))) return r;
    if ((r = check_tensor("d", d, ldd, 0, C, false)) || (r = check_tensor("g", g, C, 0, C, false))) return r;
    if (!hw || !hb || !rin || !target || !out || !dout || !loss || !dhw || !dhb || !partials || partial_bytes < need)
        return fail(UNET_EINVAL, "head train: NULL argument or partials below %zu bytes", need);
    const int G = C / 8;
    if (kHeadBlock % G != 0 || (G & (G - 1)))
        return fail(UNET_EINVAL, "head train: C / 8 must be a power of two dividing %d (got C = %d)", kHeadBlock, C);
    const int P = N * H * W;
    // one full round of resident workgroups (a partial last round would run at a
    // fraction of the occupancy), at most one per 256 pixels; one row of K (C + 1) weight
    // sums and the loss sum per workgroup fits the partials size, which allows
    // (kHeadBlock / 64) rows of K (C + 1) per 256 pixels
    int round = 0;
    if ((r = head_train_round(K, &round))) return r;
    const int blocks = std::max(1, std::min((P + kHeadBlock - 1) / kHeadBlock, round));
    const int m = K * (C + 1);
    float* part = static_cast<float*>(partials);
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto* gb = static_cast<bf16_t*>(g);
    const auto* db = static_cast<const bf16_t*>(d);
    switch (K) {
        case 1: hipLaunchKernelGGL(k_head_train<1>, dim3(blocks), dim3(kHeadBlock), 0, s, db, ldd, hw, hb, rin, target,
                                   out, dout, gb, part, C, P); break;
        case 2: hipLaunchKernelGGL(k_head_train<2>, dim3(blocks), dim3(kHeadBlock), 0, s, db, ldd, hw, hb, rin, target,
                                   out, dout, gb, part, C, P); break;
        case 3: hipLaunchKernelGGL(k_head_train<3>, dim3(blocks), dim3(kHeadBlock), 0, s, db, ldd, hw, hb, rin, target,
                                   out, dout, gb, part, C, P); break;
        default: hipLaunchKernelGGL(k_head_train<4>, dim3(blocks), dim3(kHeadBlock), 0, s, db, ldd, hw, hb, rin, target,
                                    out, dout, gb, part, C, P); break;
    }
    if ((r = launched("head train launch"))) return r;
    // weight and bias gradients and the loss in one launch (the loss is the last column)
    hipLaunchKernelGGL(k_sum_partials, dim3(m + 1), dim3(256), 0, s, static_cast<const float*>(part), blocks, m + 1,
                       1.0f, dhw, dhb, C + 1, loss, 1.0f / (float)((size_t)K * P));
    return launched("head reduce launch");
}

int unet_adam(float* p, const float* g, float* m, float* v, void* p16, size_t n, float lr, float b1, float b2,
              float eps, int32_t t, void* stream) {
    if (!p || !g || !m || !v || t < 1 || !(lr >= 0) || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1) || !(eps > 0))
        return fail(UNET_EINVAL, "adam: bad arguments");
    if (n == 0) return UNET_OK;
    const float c1 = (float)(1.0 - std::pow((double)b1, t)), c2 = (float)(1.0 - std::pow((double)b2, t));
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, static_cast<hipStream_t>(stream), p, g,
                       m, v, static_cast<bf16_t*>(p16), n, lr, b1, b2, eps, c1, c2);
    return launched("adam launch");
}

int unet_to_bf16(const float* src, void* dst, size_t n, void* stream) {
    if (!src || !dst) return fail(UNET_EINVAL, "to_bf16: NULL");
    if (n == 0) return UNET_OK;
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, static_cast<hipStream_t>(stream), src,
                       static_cast<bf16_t*>(dst), n);
    return launched("to_bf16 launch");
}

int unet_to_f32(const void* src, float* dst, size_t n, void* stream) {
    if (!src || !dst) return fail(UNET_EINVAL, "to_f32: NULL");
    if (n == 0) return UNET_OK;
    hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, static_cast<hipStream_t>(stream),
                       static_cast<const bf16_t*>(src), dst, n);
    return launched("to_f32 launch");
}

const char* unet_last_error(void) { return g_err.c_str(); }

}  // extern "C"
