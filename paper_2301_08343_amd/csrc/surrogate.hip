// Training and inference kernels of the tactile surrogate (gfx950).
//
// Convolutions are implicit GEMMs on v_mfma_f32_16x16x32_bf16 (BF16 inputs,
// FP32 accumulation). The forward kernel puts the weights in the MFMA's A
// operand (rows = output channels) and the im2col patches in B (columns =
// pixels), so each lane ends with 4 consecutive channels of one pixel and
// stores them as one 8-byte write. Every operand fragment is a 16-byte load of
// 8 consecutive K values: 8 input channels of one tap of NHWC activations, or
// 8 entries of a packed weight row. The input gradient is the same kernel with
// the spatially flipped, transposed weights. The weight gradient reduces over
// pixels: pixel chunks are transposed through LDS, partial sums of pixel
// ranges go to scratch and are reduced in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>

#include "../../include/tsg.h"

namespace tsg {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

thread_local std::string g_err;

tsg_status fail(tsg_status st, const std::string &m)
{
    g_err = m;
    return st;
}

#define TSG_LAUNCHED()                                                                                  \
    do {                                                                                                \
        hipError_t e_ = hipGetLastError();                                                              \
        if (e_ != hipSuccess) return fail(-3, std::string("launch failed: ") + hipGetErrorString(e_)); \
    } while (0)

__device__ __forceinline__ float bf2f(uint16_t v) { return __uint_as_float((uint32_t)v << 16); }

// float -> bfloat16 with round-to-nearest-even (NaN kept quiet)
__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// erf(x) by Abramowitz & Stegun (1964), eq. 7.1.26 (Hastings' rational
// form): erf(|x|) = 1 - t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) exp(-x^2),
// t = 1 / (1 + p |x|), absolute error <= 1.5e-7 on the whole line (plus a
// few FP32 ulps of 1 from the hardware reciprocal and exp2), far below the
// bf16 rounding (2^-9 relative) of every value GELU and GELU' feed. e
// returns exp(-x^2), which GELU' needs as well. About 12 instructions.
__device__ __forceinline__ float erf_as(float x, float &e)
{
    const float ax = fabsf(x);
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, ax, 1.0f));
    const float poly =
        t * fmaf(t, fmaf(t, fmaf(t, fmaf(t, 1.061405429f, -1.453152027f), 1.421413741f), -0.284496736f), 0.254829592f);
    e = __builtin_amdgcn_exp2f(-(ax * ax) * 1.44269504088896341f);
    return copysignf(fmaf(-poly, e, 1.0f), x);
}

// GELU(z) = z Phi(z), Phi(z) = (1 + erf(z / sqrt 2)) / 2
__device__ __forceinline__ float gelu(float z)
{
    float e;
    return 0.5f * z * (1.0f + erf_as(z * 0.70710678118654752f, e));
}

// GELU'(z) = Phi(z) + z phi(z), phi(z) = exp(-z^2 / 2) / sqrt(2 pi)
__device__ __forceinline__ float dgelu(float z)
{
    float e;
    const float r = erf_as(z * 0.70710678118654752f, e);
    return 0.5f * (1.0f + r) + z * 0.39894228040143268f * e;
}

__device__ __forceinline__ bf16x8 load8(const uint16_t *p)
{
    return __builtin_bit_cast(bf16x8, *(const uint4 *)p);
}

__device__ __forceinline__ bf16x8 zero8() { return __builtin_bit_cast(bf16x8, uint4{0u, 0u, 0u, 0u}); }

// ------------------------------------------------------------------ weight packs

__global__ void k_pack(const float *w, int cout, int cin, int cin_p, int cout_p, int taps, int kf, int kt,
                       uint16_t *wf, uint16_t *wt)
{
    // one thread per (row, k) of the larger of the two packs
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (wf && idx < (int64_t)cout * kf) {
        const int co = (int)(idx / kf), k = (int)(idx % kf);
        const int tap = k / cin_p, ci = k % cin_p;
        float v = 0.0f;
        if (tap < taps && ci < cin) v = w[((int64_t)co * taps + tap) * cin + ci];
        wf[idx] = f2bf(v);
    }
    if (wt && idx < (int64_t)cin_p * kt) {
        const int ci = (int)(idx / kt), k = (int)(idx % kt);
        const int tap = k / cout_p, co = k % cout_p;
        float v = 0.0f;
        if (tap < taps && co < cout && ci < cin) v = w[((int64_t)co * taps + (taps - 1 - tap)) * cin + ci];
        wt[idx] = f2bf(v);
    }
}

// ------------------------------------------------------------------ convolution

struct ConvArgs {
    const uint16_t *in;
    int n, h, w, in_ld, in_off, cin_p;
    const uint16_t *wp;
    int kp;
    const float *bias;
    int cout;
    uint16_t *out;
    int out_ld, out_off;
    uint16_t *z;
    int z_ld, z_off;
    float *out32;
};

// Epilogue of both convolution kernels: lane holds acc[i][j][v] = out[pixel
// pix0 + 16 j + r16][channel co0 + 16 i + 4 (lane/16) + v].
template <int WCO, int WPX, int EPI>
__device__ __forceinline__ void conv_epilogue(const ConvArgs &a, const f32x4 (&acc)[WCO][WPX], int pix0, int co0,
                                              const bool (&pv)[WPX], int lane)
{
    const int r16 = lane & 15;
#pragma unroll
    for (int j = 0; j < WPX; ++j) {
        if (!pv[j]) continue;
        const int64_t p = pix0 + j * 16 + r16;
#pragma unroll
        for (int i = 0; i < WCO; ++i) {
            const int cb = co0 + i * 16 + (lane >> 4) * 4;
            if (EPI == TSG_EPI_F32) {
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    if (cb + v < a.cout) a.out32[p * a.cout + cb + v] = acc[i][j][v] + (a.bias ? a.bias[cb + v] : 0.0f);
                continue;
            }
            if (cb >= a.cout) continue;
            uint16_t o[4];
            if (EPI == TSG_EPI_BIAS_GELU) {
                uint16_t zz[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const float s = acc[i][j][v] + (a.bias ? a.bias[cb + v] : 0.0f);
                    zz[v] = f2bf(s);
                    o[v] = f2bf(gelu(s));
                }
                *(uint2 *)(a.z + p * a.z_ld + a.z_off + cb) =
                    uint2{(uint32_t)zz[0] | ((uint32_t)zz[1] << 16), (uint32_t)zz[2] | ((uint32_t)zz[3] << 16)};
            } else if (EPI == TSG_EPI_DGELU) {
                const uint2 zr = *(const uint2 *)(a.z + p * a.z_ld + a.z_off + cb);
                const uint16_t zz[4] = {(uint16_t)(zr.x & 0xffffu), (uint16_t)(zr.x >> 16), (uint16_t)(zr.y & 0xffffu),
                                        (uint16_t)(zr.y >> 16)};
#pragma unroll
                for (int v = 0; v < 4; ++v) o[v] = f2bf(acc[i][j][v] * dgelu(bf2f(zz[v])));
            } else {
#pragma unroll
                for (int v = 0; v < 4; ++v) o[v] = f2bf(acc[i][j][v] + (a.bias ? a.bias[cb + v] : 0.0f));
            }
            *(uint2 *)(a.out + p * a.out_ld + a.out_off + cb) =
                uint2{(uint32_t)o[0] | ((uint32_t)o[1] << 16), (uint32_t)o[2] | ((uint32_t)o[3] << 16)};
        }
    }
}

// One wave computes (WCO*16) output channels x (WPX*16) pixels; 4 waves per
// workgroup along the pixels.
template <int WCO, int WPX, int TAPS, int EPI>
__global__ void __launch_bounds__(256) k_conv(ConvArgs a)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int hw = a.h * a.w, npix = a.n * hw;
    const int co0 = blockIdx.y * (WCO * 16);
    const int pix0 = (blockIdx.x * 4 + wave) * (WPX * 16);
    if (pix0 >= npix) return;
    const int r16 = lane & 15, kg = (lane >> 4) * 8;
    int pn[WPX], ph[WPX], pw[WPX];
    bool pv[WPX];
#pragma unroll
    for (int j = 0; j < WPX; ++j) {
        const int p = pix0 + j * 16 + r16;
        pv[j] = p < npix;
        const int q = pv[j] ? p : 0;
        pn[j] = q / hw;
        const int rem = q - pn[j] * hw;
        ph[j] = rem / a.w;
        pw[j] = rem - ph[j] * a.w;
    }
    f32x4 acc[WCO][WPX];
#pragma unroll
    for (int i = 0; i < WCO; ++i)
#pragma unroll
        for (int j = 0; j < WPX; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = 0; k0 < a.kp; k0 += 32) {
        const int k = k0 + kg;
        const int tap = k / a.cin_p;
        const int ci = k - tap * a.cin_p;
        const int dh = TAPS == 9 ? tap / 3 - 1 : 0, dw = TAPS == 9 ? tap % 3 - 1 : 0;
        const bool tap_ok = tap < TAPS;
        bf16x8 av[WCO], bv[WPX];
#pragma unroll
        for (int i = 0; i < WCO; ++i) {
            const int co = co0 + i * 16 + r16;
            av[i] = co < a.cout ? load8(a.wp + (int64_t)co * a.kp + k) : zero8();
        }
#pragma unroll
        for (int j = 0; j < WPX; ++j) {
            const int hh = ph[j] + dh, ww = pw[j] + dw;
            const bool ok = tap_ok && pv[j] && (unsigned)hh < (unsigned)a.h && (unsigned)ww < (unsigned)a.w;
            bv[j] = ok ? load8(a.in + ((int64_t)(pn[j] * a.h + hh) * a.w + ww) * a.in_ld + a.in_off + ci) : zero8();
        }
#pragma unroll
        for (int i = 0; i < WCO; ++i)
#pragma unroll
            for (int j = 0; j < WPX; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    conv_epilogue<WCO, WPX, EPI>(a, acc, pix0, co0, pv, lane);
}

template <int WCO, int TAPS>
tsg_status launch_conv_epi(const ConvArgs &a, int epi, hipStream_t st)
{
    constexpr int WPX = 4;
    const int npix = a.n * a.h * a.w;
    const dim3 grid((npix + 4 * WPX * 16 - 1) / (4 * WPX * 16), (a.cout + WCO * 16 - 1) / (WCO * 16));
    switch (epi) {
    case TSG_EPI_BIAS: hipLaunchKernelGGL((k_conv<WCO, WPX, TAPS, TSG_EPI_BIAS>), grid, dim3(256), 0, st, a); break;
    case TSG_EPI_BIAS_GELU:
        hipLaunchKernelGGL((k_conv<WCO, WPX, TAPS, TSG_EPI_BIAS_GELU>), grid, dim3(256), 0, st, a);
        break;
    case TSG_EPI_DGELU: hipLaunchKernelGGL((k_conv<WCO, WPX, TAPS, TSG_EPI_DGELU>), grid, dim3(256), 0, st, a); break;
    default: hipLaunchKernelGGL((k_conv<WCO, WPX, TAPS, TSG_EPI_F32>), grid, dim3(256), 0, st, a); break;
    }
    TSG_LAUNCHED();
    return 0;
}

// 3x3 convolutions from an LDS copy of their input and weights. A tile is
// 256 consecutive output pixels, i.e. R = 256 / w whole image rows (w a power
// of two, 4..64), times 32 output channels; waves and lanes take a tile's
// pixels as in k_conv (wave q: pixels 64 q .. 64 q + 63). Per chunk of 32
// input channels a workgroup stages the global rows row0 - 1 .. row0 + R and
// the chunk's weights of all nine taps; every MFMA operand then comes from
// LDS, so the input is read from memory about (R + 2) / R times instead of
// nine times and no tap waits on a global load. A tap whose row leaves the
// output pixel's image (a staged row of another image, or past the batch)
// or whose column leaves the row reads zero instead: each lane keeps, per
// pixel, a mask of its valid taps. A staged pixel and a staged weight row
// take 40 bf16 (32 + 8): 16 consecutive pixels or rows then start 20 banks
// apart, and a fragment's 16 lanes read 64 distinct banks. The staged input
// is at most 6 w pixels (w = 64) and the LDS of a workgroup at most 52.5 KiB,
// so three workgroups share a CU at every width.
constexpr int kConvCC = 32, kConvCP = 40, kConvCo = 32;
constexpr int kConvWVec = 9 * kConvCo * 4;      // 16-byte weight vectors per chunk
constexpr int kConvXVecMax = 6 * 64 * 4;        // input vectors per chunk, largest: (R + 2) w 4 at w = 64

__host__ __device__ constexpr int conv_lds_weights() { return 9 * kConvCo * kConvCP; }

// A lane's four pixels of tile `tile` (local pixel lp = 64 wave + 16 j +
// lane % 16): the mask of its valid taps (bit 3 (dh + 1) + dw + 1; none for
// a pixel past the batch). Its centre tap is staged pixel lp + w, at LDS
// offset conv_tile_centre + 16 j kConvCP (plus the lane's K group).
__device__ __forceinline__ int conv_tile_centre(int w, int wave, int lane)
{
    return (wave * 64 + (lane & 15) + w) * kConvCP + (lane >> 4) * 8;
}

__device__ __forceinline__ void conv_tile_pixels(const ConvArgs &a, int tile, int lgw, int wave, int lane,
                                                 uint32_t (&tm)[4])
{
    const int R = 256 >> lgw, nrows = a.n * a.h;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int lp = wave * 64 + j * 16 + (lane & 15);
        const int lr = lp >> lgw, lc = lp & (a.w - 1), g = tile * R + lr;
        const int y = g % a.h;
        const uint32_t rows = 0x038u | (y > 0 ? 0x007u : 0u) | (y < a.h - 1 ? 0x1c0u : 0u);
        const uint32_t cols = 0x092u | (lc > 0 ? 0x049u : 0u) | (lc < a.w - 1 ? 0x124u : 0u);
        tm[j] = g < nrows ? rows & cols : 0u;
    }
}

// The nine taps of one staged chunk: acc += W x im2col, operands from LDS.
__device__ __forceinline__ void conv_tile_taps(const uint16_t *wst, const uint16_t *xst, int w, int wave, int lane,
                                               const uint32_t (&tm)[4], f32x4 (&acc)[2][4])
{
    const int r16 = lane & 15, kg = (lane >> 4) * 8, sb = conv_tile_centre(w, wave, lane);
#pragma unroll 3
    for (int tap = 0; tap < 9; ++tap) {
        const int dh = tap / 3 - 1, dw = tap - (tap / 3) * 3 - 1;
        const int soff = (dh * w + dw) * kConvCP;
        bf16x8 av[2], bv[4];
#pragma unroll
        for (int i = 0; i < 2; ++i)
            av[i] = __builtin_bit_cast(bf16x8, *(const uint4 *)(wst + (tap * kConvCo + i * 16 + r16) * kConvCP + kg));
#pragma unroll
        for (int j = 0; j < 4; ++j)
            bv[j] = (tm[j] >> tap) & 1u
                        ? __builtin_bit_cast(bf16x8, *(const uint4 *)(xst + sb + j * 16 * kConvCP + soff))
                        : zero8();
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
}

// A thread's share of staging one chunk: weight vectors t = thread + 256 q
// and input vectors u = thread + 256 q, with their LDS destinations (-1:
// none) and global element offsets (-1: stays zero) that depend on neither
// the tile nor the chunk; worked out once per workgroup. Weight vector t is
// (tap, co, v) = (t / 128, t / 4 % 32, t % 4): t + 256 is the same output
// channel two taps on, so one destination and one source offset serve every
// q. Input vector u is (staged pixel u / 4, v = u % 4): staged pixel pc is
// global pixel pc of the rows from row0 - 1 on; its LDS destination (below
// 2^15) and staged row share one register.
constexpr int kConvNW = (kConvWVec + 255) / 256, kConvNX = (kConvXVecMax + 255) / 256;

struct ConvStagePlan {
    int wdst, wsrc;          // weight vector q: wdst + q 64 kConvCP, wsrc + 2 q cin_p
    int xdr[kConvNX];        // LDS destination | staged row << 16, or -1
    int xsrc[kConvNX];       // element offset from the start of row row0 - 1
};

__device__ __forceinline__ void conv_stage_plan(const ConvArgs &a, int R, int lgw, int co0, ConvStagePlan &P)
{
    const int nin = (R + 2) * a.w * 4;
    const int t = threadIdx.x, v = t & 3, rc = t >> 2, co = co0 + (rc & 31);
    P.wdst = rc * kConvCP + v * 8;
    P.wsrc = co < a.cout ? co * a.kp + (rc >> 5) * a.cin_p + v * 8 : -1;
#pragma unroll
    for (int q = 0; q < kConvNX; ++q) {
        const int u = threadIdx.x + q * 256, pc = u >> 2;
        P.xdr[q] = u < nin ? (conv_lds_weights() + pc * kConvCP + (u & 3) * 8) | ((pc >> lgw) << 16) : -1;
        P.xsrc[q] = pc * a.in_ld + a.in_off + (u & 3) * 8;
    }
}

// Weight vector q of a thread exists (the last q covers half the threads).
__device__ __forceinline__ bool conv_stage_has_w(int q) { return q * 256 + (int)threadIdx.x < kConvWVec; }

// Input vector q of the chunk at channel offset c0 of the tile whose first
// row is row0 (zero outside the batch's rows).
__device__ __forceinline__ uint4 conv_stage_load_x(const ConvArgs &a, const ConvStagePlan &P, int q, int row0, int c0)
{
    const int g = row0 - 1 + (P.xdr[q] >> 16);
    if (P.xdr[q] < 0 || g < 0 || g >= a.n * a.h) return uint4{0u, 0u, 0u, 0u};
    return *(const uint4 *)(a.in + (int64_t)(row0 - 1) * a.w * a.in_ld + P.xsrc[q] + c0);
}

// A workgroup walks a contiguous run of tiles (the halo rows two
// neighbouring tiles share stay in its L2) and, per tile, the chunks of 32
// input channels. The weight and input vectors of the next (tile, chunk) are
// loaded into registers while the current one is computed, so a chunk waits
// for memory only when its compute is shorter than a round trip; with one
// chunk per tile the weights are staged once.
template <int EPI>
__global__ void __launch_bounds__(256, 3) k_conv_lds(ConvArgs a, int lgw, int tiles_per_wg)
{
    extern __shared__ __align__(16) uint16_t stage[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int R = 256 >> lgw;
    const int ntiles = (a.n * a.h + R - 1) / R;
    const int t_begin = blockIdx.x * tiles_per_wg, t_end = min(ntiles, t_begin + tiles_per_wg);
    if (t_begin >= t_end) return;
    const int co0 = blockIdx.y * kConvCo;
    const int nch = a.cin_p / kConvCC;
    ConvStagePlan P;
    conv_stage_plan(a, R, lgw, co0, P);
    uint4 wv[kConvNW], xv[kConvNX];
    auto fetch = [&](int tile, int c0, bool with_w) {
#pragma unroll
        for (int q = 0; q < kConvNW; ++q)
            wv[q] = with_w && P.wsrc >= 0 && conv_stage_has_w(q)
                        ? *(const uint4 *)(a.wp + P.wsrc + 2 * q * a.cin_p + c0)
                        : uint4{0u, 0u, 0u, 0u};
#pragma unroll
        for (int q = 0; q < kConvNX; ++q) xv[q] = conv_stage_load_x(a, P, q, tile * R, c0);
    };
    fetch(t_begin, 0, true);
    bool with_w = true;
    for (int tile = t_begin; tile < t_end; ++tile) {
        uint32_t tm[4];
        conv_tile_pixels(a, tile, lgw, wave, lane, tm);
        bool pv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) pv[j] = tm[j] != 0u;
        f32x4 acc[2][4];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        for (int ch = 0; ch < nch; ++ch) {
            __syncthreads();  // the previous chunk's LDS reads are done
            if (with_w) {
#pragma unroll
                for (int q = 0; q < kConvNW; ++q)
                    if (conv_stage_has_w(q)) *(uint4 *)(stage + P.wdst + q * 64 * kConvCP) = wv[q];
            }
#pragma unroll
            for (int q = 0; q < kConvNX; ++q)
                if (P.xdr[q] >= 0) *(uint4 *)(stage + (P.xdr[q] & 0xffff)) = xv[q];
            __syncthreads();
            with_w = nch > 1;
            const int nt = ch + 1 < nch ? tile : tile + 1, nc = ch + 1 < nch ? ch + 1 : 0;
            if (nt < t_end) fetch(nt, nc * kConvCC, with_w);
            conv_tile_taps(stage, stage + conv_lds_weights(), a.w, wave, lane, tm, acc);
        }
        conv_epilogue<2, 4, EPI>(a, acc, tile * 256 + wave * 64, co0, pv, lane);
    }
}

// bytes of the staged weights and input of k_conv_lds
size_t conv_lds_bytes(int w)
{
    const int R = 256 / w;
    return (size_t)(conv_lds_weights() + (R + 2) * w * kConvCP) * 2;
}

// Tiles per workgroup of a k_conv_lds launch: runs sized for about kConvWGs
// workgroups in all (three per CU at the LDS and register size, one round).
// Measured against one tile per workgroup: runs of four gain the 64 x 64
// layers 10-15 % and the 32 x 32 layers 10 %; layers with fewer tiles than
// that keep one tile per workgroup (runs of four there cost 2-3x: too few
// workgroups). Against 1024 and 1536 workgroups, 768 gains the 64 x 64 and
// 32 x 32 layers 5-12 % and leaves the 16 x 16 and 8 x 8 ones unchanged.
constexpr int kConvWGs = 768;

tsg_status launch_conv_lds(const ConvArgs &a, int epi, hipStream_t st)
{
    int lgw = 0;
    while ((1 << lgw) < a.w) ++lgw;
    const int R = 256 >> lgw;
    const int ntiles = (a.n * a.h + R - 1) / R, cot = (a.cout + kConvCo - 1) / kConvCo;
    const size_t lds = conv_lds_bytes(a.w);
    const int want = std::max(1, kConvWGs / cot);
    const int per = (ntiles + want - 1) / want;
    const dim3 grid((ntiles + per - 1) / per, cot);
    switch (epi) {
    case TSG_EPI_BIAS: hipLaunchKernelGGL((k_conv_lds<TSG_EPI_BIAS>), grid, dim3(256), lds, st, a, lgw, per); break;
    case TSG_EPI_BIAS_GELU:
        hipLaunchKernelGGL((k_conv_lds<TSG_EPI_BIAS_GELU>), grid, dim3(256), lds, st, a, lgw, per);
        break;
    default: hipLaunchKernelGGL((k_conv_lds<TSG_EPI_DGELU>), grid, dim3(256), lds, st, a, lgw, per); break;
    }
    TSG_LAUNCHED();
    return 0;
}

// k_conv_lds applies to 3x3 layers with BF16 outputs whose input channels
// come in multiples of 32 and whose rows are 4..64 pixels, a power of two
bool conv_lds_fits(int taps, int epi, int cin_p, int w)
{
    return taps == 9 && epi != TSG_EPI_F32 && cin_p % 32 == 0 && w >= 4 && w <= 64 && (w & (w - 1)) == 0;
}

// ------------------------------------------------------------------ weight gradient

// Partial dw over one pixel range for a tile of 32 output channels x 32
// input channels of one tap. Chunks of 128 pixels of dout and of the
// tap-shifted input are transposed into LDS (channel-major) so that each
// lane's MFMA fragment is 8 consecutive pixels of one channel; 4 waves each
// own one 16x16 quarter of the tile and issue 4 MFMAs per chunk. Blocks of
// the first (tap, input-channel) tile also sum the dout chunk per channel
// into bpart (the bias gradient's partials), when bpart is given.
constexpr int kWgChunk = 128;

__global__ void __launch_bounds__(256) k_wgrad(const uint16_t *in, int n, int h, int w, int in_ld, int in_off,
                                               int cin_p, const uint16_t *dout, int d_ld, int d_off, int cout,
                                               int taps, int pix_per_split, float *part, float *bpart)
{
    __shared__ __align__(16) uint16_t sA[32][kWgChunk + 8];  // [co][pixel], padded rows
    __shared__ __align__(16) uint16_t sB[32][kWgChunk + 8];  // [ci][pixel]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int hw = h * w, npix = n * hw;
    const int co0 = blockIdx.x * 32;
    const int tap = blockIdx.y / ((cin_p + 31) / 32);
    const int ci0 = (blockIdx.y % ((cin_p + 31) / 32)) * 32;
    const int split = blockIdx.z;
    const int dh = taps == 9 ? tap / 3 - 1 : 0, dw = taps == 9 ? tap % 3 - 1 : 0;
    const int pbeg = split * pix_per_split, pend = min(npix, pbeg + pix_per_split);
    const int wm = (wave >> 1) * 16, wn = (wave & 1) * 16;  // this wave's quarter
    const bool do_bias = bpart != nullptr && blockIdx.y == 0;
    f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    float bsum = 0.0f;
    // loader mapping: 256 threads = 32 pixels x 8 groups of 4 channels, 4 rounds
    const int lp = tid >> 3, lc = (tid & 7) * 4;
    for (int p0 = pbeg; p0 < pend; p0 += kWgChunk) {
        uint2 va[kWgChunk / 32], vb[kWgChunk / 32];
#pragma unroll
        for (int j = 0; j < kWgChunk / 32; ++j) {
            const int p = p0 + lp + 32 * j;
            va[j] = uint2{0u, 0u};
            vb[j] = uint2{0u, 0u};
            if (p < pend) {
                if (co0 + lc < cout) va[j] = *(const uint2 *)(dout + (int64_t)p * d_ld + d_off + co0 + lc);
                const int nn = p / hw, rem = p - nn * hw, hh = rem / w + dh, ww = rem % w + dw;
                if (ci0 + lc < cin_p && (unsigned)hh < (unsigned)h && (unsigned)ww < (unsigned)w)
                    vb[j] = *(const uint2 *)(in + ((int64_t)(nn * h + hh) * w + ww) * in_ld + in_off + ci0 + lc);
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kWgChunk / 32; ++j) {
            const int q = lp + 32 * j;
            sA[lc + 0][q] = (uint16_t)(va[j].x & 0xffffu);
            sA[lc + 1][q] = (uint16_t)(va[j].x >> 16);
            sA[lc + 2][q] = (uint16_t)(va[j].y & 0xffffu);
            sA[lc + 3][q] = (uint16_t)(va[j].y >> 16);
            sB[lc + 0][q] = (uint16_t)(vb[j].x & 0xffffu);
            sB[lc + 1][q] = (uint16_t)(vb[j].x >> 16);
            sB[lc + 2][q] = (uint16_t)(vb[j].y & 0xffffu);
            sB[lc + 3][q] = (uint16_t)(vb[j].y >> 16);
        }
        __syncthreads();
        const int r16 = lane & 15, kg = (lane >> 4) * 8;
#pragma unroll
        for (int j = 0; j < kWgChunk / 32; ++j) {
            const bf16x8 a8 = __builtin_bit_cast(bf16x8, *(const uint4 *)&sA[wm + r16][32 * j + kg]);
            const bf16x8 b8 = __builtin_bit_cast(bf16x8, *(const uint4 *)&sB[wn + r16][32 * j + kg]);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a8, b8, acc, 0, 0, 0);
        }
        if (do_bias && tid < 32) {
            // pixels past pend were loaded as zeros
            for (int q = 0; q < kWgChunk; ++q) bsum += bf2f(sA[tid][q]);
        }
    }
    // acc[v] = partial dw[co0 + wm + 4 (lane/16) + v][tap][ci0 + wn + lane%16]
    const int ci = ci0 + wn + (lane & 15);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int co = co0 + wm + (lane >> 4) * 4 + v;
        if (co < cout && ci < cin_p)
            part[(((int64_t)split * cout + co) * taps + tap) * cin_p + ci] = acc[v];
    }
    if (do_bias && tid < 32 && co0 + tid < cout) bpart[(int64_t)split * cout + co0 + tid] = bsum;
}

// All nine taps of a 3x3 weight gradient per workgroup (32 output x 32 input
// channels): the input rows a tap reads are the chunk's own rows shifted by
// dh rows and dw pixels, so the chunk plus one row above and below is staged
// once, in three copies pre-shifted by dw = -1, 0, +1 (zero where the shift
// leaves the row, and zero for rows of another image), and every tap reads
// its MFMA operand from a 16-byte aligned offset of one copy. The per-tap
// kernel reads the output gradient and the input once per tap. Requires
// chunks of CH pixels inside one image (h w % CH == 0, CH % w == 0) and
// 8 <= w <= 64, w % 8 == 0: CH = 128 for rows of 16..64 pixels, 64 for 8.
template <int CH>
constexpr int wgrad9_halo() { return CH + 2 * 64; }

// Channel c (0..3) of two 4-channel bf16 vectors lo and hi as one bf16 pair
// (lo's in the low half): one byte permute. v_perm_b32's selector bytes 0-3
// pick the bytes of its second operand, 4-7 those of its first.
__device__ __forceinline__ uint32_t pair_at(const uint2 &lo, const uint2 &hi, int c)
{
    const uint32_t l = c < 2 ? lo.x : lo.y, h = c < 2 ? hi.x : hi.y;
    return __builtin_amdgcn_perm(h, l, (c & 1) ? 0x07060302u : 0x05040100u);
}

// Channel c of each of v[0..7] as one 16-byte vector of eight bf16
__device__ __forceinline__ uint4 pack8_at(const uint2 *v, int c)
{
    return uint4{pair_at(v[0], v[1], c), pair_at(v[2], v[3], c), pair_at(v[4], v[5], c), pair_at(v[6], v[7], c)};
}

template <int CH>
__global__ void __launch_bounds__(256) k_wgrad9(const uint16_t *in, int n, int h, int w, int in_ld, int in_off,
                                                int cin_p, const uint16_t *dout, int d_ld, int d_off, int cout,
                                                int pix_per_split, float *part, float *bpart)
{
    __shared__ __align__(16) uint16_t sA[32][CH + 8];     // [co][pixel]
    __shared__ __align__(16) uint16_t sB[3][32][wgrad9_halo<CH>() + 8];   // [dw + 1][ci][haloed pixel]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int hw = h * w, npix = n * hw;
    const int co0 = blockIdx.x * 32, ci0 = blockIdx.y * 32, split = blockIdx.z;
    const int pbeg = split * pix_per_split, pend = min(npix, pbeg + pix_per_split);
    const int wm = (wave >> 1) * 16, wn = (wave & 1) * 16;
    const bool do_bias = bpart != nullptr && blockIdx.y == 0;
    const int halo = CH + 2 * w;
    f32x4 acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    float bsum = 0.0f;
    // staging item of this thread: an 8-pixel window `win` of 4 channels
    // lc .. lc+3, transposed in registers and stored as four 16-byte rows.
    // dout: windows 0..CH/8-1 of the chunk; input: windows
    // 0..halo/8-1 of the haloed chunk, read with one pixel on either side for
    // the copies shifted by dw = -1 and +1. The next chunk is loaded while
    // the current one computes.
    const int win = tid >> 3, lc = (tid & 7) * 4;
    const bool a_item = win < CH / 8, b_item = win * 8 < halo;
    uint2 va[8], vb[10];
    auto load = [&](int p0) {
        const int64_t ibeg = (int64_t)(p0 / hw) * hw, iend = ibeg + hw;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int p = p0 + win * 8 + k;
            va[k] = uint2{0u, 0u};
            if (a_item && p < pend && co0 + lc < cout) va[k] = *(const uint2 *)(dout + (int64_t)p * d_ld + d_off + co0 + lc);
        }
#pragma unroll
        for (int k = 0; k < 10; ++k) {
            const int i = win * 8 + k - 1;
            const int64_t r = (int64_t)p0 - w + i;
            vb[k] = uint2{0u, 0u};
            if (b_item && i >= 0 && i < halo && r >= ibeg && r < iend && ci0 + lc < cin_p)
                vb[k] = *(const uint2 *)(in + r * in_ld + in_off + ci0 + lc);
        }
    };
    // an empty split (none is launched, see tsg_conv_wgrad) writes zero
    // partials and reads nothing: its halo guard would name rows past the batch
    if (pbeg < pend) load(pbeg);
    for (int p0 = pbeg; p0 < pend; p0 += CH) {
        __syncthreads();  // the previous chunk's LDS reads are done
        if (a_item) {
#pragma unroll
            for (int c = 0; c < 4; ++c) *(uint4 *)&sA[lc + c][win * 8] = pack8_at(va, c);
        }
        if (b_item) {
            // entry e of copy dw + 1 holds pixel e + dw of the same row (zero
            // past the row's ends); an 8-entry window lies inside one row
            // (w % 8 == 0, and the haloed chunk starts at a row start)
            const bool row_first = (win * 8) % w == 0, row_last = (win * 8 + 8) % w == 0;
            // vb[0] feeds only entry 0 of copy 0, vb[9] only entry 7 of copy 2
            if (row_first) vb[0] = uint2{0u, 0u};
            if (row_last) vb[9] = uint2{0u, 0u};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                *(uint4 *)&sB[0][lc + c][win * 8] = pack8_at(vb, c);
                *(uint4 *)&sB[1][lc + c][win * 8] = pack8_at(vb + 1, c);
                *(uint4 *)&sB[2][lc + c][win * 8] = pack8_at(vb + 2, c);
            }
        }
        __syncthreads();
        if (p0 + CH < pend) load(p0 + CH);
        const int r16 = lane & 15, kg = (lane >> 4) * 8;
#pragma unroll
        for (int j = 0; j < CH / 32; ++j) {
            const bf16x8 a8 = __builtin_bit_cast(bf16x8, *(const uint4 *)&sA[wm + r16][32 * j + kg]);
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const int dh = t / 3 - 1, dwi = t % 3;
                const bf16x8 b8 = __builtin_bit_cast(
                    bf16x8, *(const uint4 *)&sB[dwi][wn + r16][w * (dh + 1) + 32 * j + kg]);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a8, b8, acc[t], 0, 0, 0);
            }
        }
        if (do_bias) {
            // output channel tid / 8, pixels (tid % 8) CH / 8 .. + CH / 8 of the chunk
            const uint4 *src = (const uint4 *)&sA[tid >> 3][(tid & 7) * (CH / 8)];
#pragma unroll
            for (int q = 0; q < CH / 64; ++q) {
                const uint4 v = src[q];
                const uint32_t e[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    bsum += __uint_as_float(e[k] << 16);
                    bsum += __uint_as_float(e[k] & 0xffff0000u);
                }
            }
        }
    }
    const int ci = ci0 + wn + (lane & 15);
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int co = co0 + wm + (lane >> 4) * 4 + v;
            if (co < cout && ci < cin_p) part[(((int64_t)split * cout + co) * 9 + t) * cin_p + ci] = acc[t][v];
        }
    if (do_bias) {
        // the eight partial sums of each output channel, added in order
        __syncthreads();  // the last chunk's reads of sA are done
        float *red = reinterpret_cast<float *>(&sA[0][0]);
        red[tid] = bsum;
        __syncthreads();
        if (tid < 32 && co0 + tid < cout) {
            float b = 0.0f;
#pragma unroll
            for (int g = 0; g < 8; ++g) b += red[tid * 8 + g];
            bpart[(int64_t)split * cout + co0 + tid] = b;
        }
    }
}

// dw[co][tap][ci] = sum over splits of the partials, ci < cin. 32 outputs
// per workgroup, 8 lanes per output: lane g sums splits g, g+8, ... and the
// eight lane sums are added in lane order, a fixed order (bit-reproducible).
// Workgroups from nw_blocks on sum the bias partials [splits][cout] into db
// the same way (one launch for both sums).
__global__ void __launch_bounds__(256) k_wgrad_reduce(const float *part, int splits, int cout, int taps, int cin,
                                                      int cin_p, float *dw, int nw_blocks, const float *bpart,
                                                      float *db)
{
    __shared__ float red[8][33];
    const int o = threadIdx.x & 31, g = threadIdx.x >> 5;
    const bool bias = (int)blockIdx.x >= nw_blocks;
    const int64_t idx = (int64_t)(bias ? blockIdx.x - nw_blocks : blockIdx.x) * 32 + o;
    const int64_t total = bias ? cout : (int64_t)cout * taps * cin;
    float s = 0.0f;
    if (idx < total) {
        // unrolled: eight loads in flight per thread, added in the same order
        if (bias) {
#pragma unroll 8
            for (int k = g; k < splits; k += 8) s += bpart[(int64_t)k * cout + idx];
        } else {
            const int ci = (int)(idx % cin);
            const int64_t ct = idx / cin;  // co * taps + tap
#pragma unroll 8
            for (int k = g; k < splits; k += 8) s += part[((int64_t)k * cout * taps + ct) * cin_p + ci];
        }
    }
    red[g][o] = s;
    __syncthreads();
    if (g == 0 && idx < total) {
        float t = 0.0f;
        for (int q = 0; q < 8; ++q) t += red[q][o];
        (bias ? db : dw)[idx] = t;
    }
}

// 1x1 head, FP32 output gradient: partial sums of dout^T in (cout x cin) and
// of dout (bias) per pixel range.
__global__ void k_head_wgrad(const uint16_t *in, int npix, int in_ld, int in_off, int cin, const float *dout,
                             int cout, int rows_per_split, float *part)
{
    const int split = blockIdx.x;
    const int t = threadIdx.x;  // one thread per (co, ci) pair or bias entry
    const int nval = cout * (cin + 1);
    if (t >= nval) return;
    const int co = t / (cin + 1), ci = t % (cin + 1);
    const int r0 = split * rows_per_split, r1 = min(npix, r0 + rows_per_split);
    float s = 0.0f;
    // eight rows' loads are issued before their (in-order) accumulation
    int r = r0;
    for (; r + 8 <= r1; r += 8) {
        float g[8], x[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            g[k] = dout[(int64_t)(r + k) * cout + co];
            x[k] = ci < cin ? bf2f(in[(int64_t)(r + k) * in_ld + in_off + ci]) : 1.0f;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) s += ci < cin ? g[k] * x[k] : g[k];
    }
    for (; r < r1; ++r) {
        const float g = dout[(int64_t)r * cout + co];
        s += ci < cin ? g * bf2f(in[(int64_t)r * in_ld + in_off + ci]) : g;
    }
    part[(int64_t)split * nval + t] = s;
}

constexpr int kHeadSplits = 4096;

__device__ __forceinline__ void unpack8(uint4 v, float f[8]);

// The same partial sums with 16-byte input loads, for inputs whose channels
// come in G groups of 8 (cin = 8 G) and CO <= 4 outputs: thread (rs, g)
// takes rows r0 + rs, r0 + rs + RS, ... (RS = 256 / G row slots) and sums,
// for its 8 channels and every output, the products (and, for g = 0, the
// output gradients: the bias), in row order; the RS slots of each value are
// then added in slot order through LDS. Same partial layout as k_head_wgrad.
template <int G, int CO>
__global__ void __launch_bounds__(256) k_head_wgrad_v8(const uint16_t *in, int npix, int in_ld, int in_off,
                                                       const float *dout, int rows_per_split, float *part)
{
    constexpr int RS = 256 / G, CIN = 8 * G, NV = CO * (CIN + 1);
    __shared__ float red[RS * NV];
    const int t = threadIdx.x, g = t % G, rs = t / G;
    const int split = blockIdx.x;
    const int r0 = split * rows_per_split, r1 = min(npix, r0 + rows_per_split);
    float acc[CO][8], bacc[CO];
#pragma unroll
    for (int co = 0; co < CO; ++co) {
        bacc[co] = 0.0f;
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[co][k] = 0.0f;
    }
    if (rs < RS) {
#pragma unroll 4
        for (int r = r0 + rs; r < r1; r += RS) {
            float x[8];
            unpack8(*(const uint4 *)(in + (int64_t)r * in_ld + in_off + g * 8), x);
#pragma unroll
            for (int co = 0; co < CO; ++co) {
                const float gg = dout[(int64_t)r * CO + co];
                bacc[co] += gg;
#pragma unroll
                for (int k = 0; k < 8; ++k) acc[co][k] += gg * x[k];
            }
        }
#pragma unroll
        for (int co = 0; co < CO; ++co) {
#pragma unroll
            for (int k = 0; k < 8; ++k) red[rs * NV + co * (CIN + 1) + g * 8 + k] = acc[co][k];
            if (g == 0) red[rs * NV + co * (CIN + 1) + CIN] = bacc[co];
        }
    }
    __syncthreads();
    for (int v = t; v < NV; v += 256) {
        float sum = 0.0f;
        for (int q = 0; q < RS; ++q) sum += red[q * NV + v];
        part[(int64_t)split * NV + v] = sum;
    }
}

// Fixed-order sum of the head partials into dw [cout][cin] and db [cout]:
// one workgroup per value, each thread a strided share of the splits, then a
// tree in LDS.
__global__ void __launch_bounds__(256) k_head_reduce(const float *part, int splits, int cout, int cin, float *dw,
                                                     float *db)
{
    __shared__ float red[256];
    const int t = blockIdx.x;
    const int nval = cout * (cin + 1);
    float s = 0.0f;
    for (int k = threadIdx.x; k < splits; k += 256) s += part[(int64_t)k * nval + t];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int co = t / (cin + 1), ci = t % (cin + 1);
        if (ci < cin)
            dw[co * cin + ci] = red[0];
        else
            db[co] = red[0];
    }
}

// Input gradient of the 1x1 head: din[p][ci] = sum_co dout[p][co] w[co][ci]
// (times GELU'(z) with z). One thread per (pixel, channel); npix * cin <
// 2^31 (checked by the caller), so the index splits in 32-bit arithmetic.
__global__ void k_head_dgrad(const float *dout, int npix, int cout, const float *w, int cin, uint16_t *din, int ld,
                             int off, const uint16_t *z, int z_ld, int z_off)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= npix * cin) return;
    const int p = idx / cin, ci = idx - p * cin;
    float s = 0.0f;
    for (int co = 0; co < cout; ++co) s += dout[(int64_t)p * cout + co] * w[co * cin + ci];
    if (z) s *= dgelu(bf2f(z[(int64_t)p * z_ld + z_off + ci]));
    din[(int64_t)p * ld + off + ci] = f2bf(s);
}

// The same for 8 channels of a pixel per thread (cin, ld, off, z_ld, z_off
// multiples of 8 and 16-byte aligned views): one 16-byte store.
__global__ void k_head_dgrad_v8(const float *dout, int npix, int cout, const float *w, int cin, uint16_t *din,
                                int ld, int off, const uint16_t *z, int z_ld, int z_off)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int g8 = cin >> 3;
    if (idx >= npix * g8) return;
    const int p = idx / g8, c0 = (idx - p * g8) * 8;
    float s[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    for (int co = 0; co < cout; ++co) {
        const float g = dout[(int64_t)p * cout + co];
#pragma unroll
        for (int k = 0; k < 8; ++k) s[k] += g * w[co * cin + c0 + k];
    }
    if (z) {
        const uint4 zr = *(const uint4 *)(z + (int64_t)p * z_ld + z_off + c0);
        const uint32_t zw[4] = {zr.x, zr.y, zr.z, zr.w};
#pragma unroll
        for (int k = 0; k < 8; ++k) s[k] *= dgelu(bf2f((uint16_t)(zw[k >> 1] >> ((k & 1) * 16))));
    }
    uint32_t o[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) o[k] = (uint32_t)f2bf(s[2 * k]) | ((uint32_t)f2bf(s[2 * k + 1]) << 16);
    *(uint4 *)(din + (int64_t)p * ld + off + c0) = uint4{o[0], o[1], o[2], o[3]};
}

// ------------------------------------------------------------------ pooling, upsampling, elementwise

__global__ void k_avgpool2(const uint16_t *in, int n, int h, int w, int c, int ld, int off, uint16_t *out, int old,
                           int ooff)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int ho = h / 2, wo = w / 2;
    if (idx >= (int64_t)n * ho * wo * c) return;
    const int ch = (int)(idx % c);
    const int64_t q = idx / c;
    const int x = (int)(q % wo), y = (int)((q / wo) % ho), nn = (int)(q / ((int64_t)wo * ho));
    float s = 0.0f;
    for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx)
            s += bf2f(in[((int64_t)(nn * h + 2 * y + dy) * w + 2 * x + dx) * ld + off + ch]);
    out[q * old + ooff + ch] = f2bf(0.25f * s);
}

__global__ void k_avgpool2_bwd(const uint16_t *dout, int n, int h, int w, int c, int dld, int doff, uint16_t *din,
                               int ild, int ioff, int accumulate)
{
    // h, w: input (fine) size; one thread per fine element
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * h * w * c) return;
    const int ch = (int)(idx % c);
    const int64_t q = idx / c;
    const int x = (int)(q % w), y = (int)((q / w) % h), nn = (int)(q / ((int64_t)w * h));
    const int ho = h / 2, wo = w / 2;
    float g = 0.25f * bf2f(dout[((int64_t)(nn * ho + y / 2) * wo + x / 2) * dld + doff + ch]);
    uint16_t *dst = din + q * ild + ioff + ch;
    if (accumulate) g += bf2f(*dst);
    *dst = f2bf(g);
}

__global__ void k_upsample2(const uint16_t *in, int n, int h, int w, int c, int ld, int off, uint16_t *out, int old,
                            int ooff)
{
    // h, w: input (coarse) size; one thread per fine element
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int H2 = 2 * h, W2 = 2 * w;
    if (idx >= (int64_t)n * H2 * W2 * c) return;
    const int ch = (int)(idx % c);
    const int64_t q = idx / c;
    const int x = (int)(q % W2), y = (int)((q / W2) % H2), nn = (int)(q / ((int64_t)W2 * H2));
    out[q * old + ooff + ch] = in[((int64_t)(nn * h + y / 2) * w + x / 2) * ld + off + ch];
}

__global__ void k_upsample2_bwd(const uint16_t *dout, int n, int h, int w, int c, int dld, int doff, uint16_t *din,
                                int ild, int ioff)
{
    // h, w: coarse size; one thread per coarse element
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * h * w * c) return;
    const int ch = (int)(idx % c);
    const int64_t q = idx / c;
    const int x = (int)(q % w), y = (int)((q / w) % h), nn = (int)(q / ((int64_t)w * h));
    const int W2 = 2 * w;
    float s = 0.0f;
    for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx)
            s += bf2f(dout[((int64_t)(nn * 2 * h + 2 * y + dy) * W2 + 2 * x + dx) * dld + doff + ch]);
    din[q * ild + ioff + ch] = f2bf(s);
}

// 8-channel vector forms of the pooling/upsampling kernels and their
// gradients (channel counts, row strides and offsets multiples of 8, 16-byte
// aligned rows): one thread per (pixel, group of 8 channels).
__device__ __forceinline__ void unpack8(uint4 v, float f[8])
{
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        f[2 * k] = bf2f((uint16_t)(w[k] & 0xffffu));
        f[2 * k + 1] = bf2f((uint16_t)(w[k] >> 16));
    }
}

__device__ __forceinline__ uint4 pack8(const float f[8])
{
    uint32_t w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = (uint32_t)f2bf(f[2 * k]) | ((uint32_t)f2bf(f[2 * k + 1]) << 16);
    return uint4{w[0], w[1], w[2], w[3]};
}

__global__ void k_avgpool2_v8(const uint16_t *in, int n, int h, int w, int c, int ld, int off, uint16_t *out, int old,
                              int ooff)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int ho = h / 2, wo = w / 2, g = c / 8;
    if (idx >= (int64_t)n * ho * wo * g) return;
    const int cg = (int)(idx % g) * 8;
    const int64_t q = idx / g;
    const int x = (int)(q % wo), y = (int)((q / wo) % ho), nn = (int)(q / ((int64_t)wo * ho));
    float acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) {
            float f[8];
            unpack8(*(const uint4 *)(in + ((int64_t)(nn * h + 2 * y + dy) * w + 2 * x + dx) * ld + off + cg), f);
#pragma unroll
            for (int k = 0; k < 8; ++k) acc[k] += f[k];
        }
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] *= 0.25f;
    *(uint4 *)(out + q * old + ooff + cg) = pack8(acc);
}

// z (optional, same layout as din with its own stride and offset): the
// result is multiplied by GELU'(z), the backward through the GELU that
// produced the pooled input, in the same pass.
__global__ void k_avgpool2_bwd_v8(const uint16_t *dout, int n, int h, int w, int c, int dld, int doff, uint16_t *din,
                                  int ild, int ioff, int accumulate, const uint16_t *z, int zld, int zoff)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int g = c / 8;
    if (idx >= (int64_t)n * h * w * g) return;
    const int cg = (int)(idx % g) * 8;
    const int64_t q = idx / g;
    const int x = (int)(q % w), y = (int)((q / w) % h), nn = (int)(q / ((int64_t)w * h));
    const int ho = h / 2, wo = w / 2;
    float f[8];
    unpack8(*(const uint4 *)(dout + ((int64_t)(nn * ho + y / 2) * wo + x / 2) * dld + doff + cg), f);
    uint4 *dst = (uint4 *)(din + q * ild + ioff + cg);
    float prev[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (accumulate) unpack8(*dst, prev);
#pragma unroll
    for (int k = 0; k < 8; ++k) f[k] = 0.25f * f[k] + prev[k];
    if (z) {
        float zz[8];
        unpack8(*(const uint4 *)(z + q * zld + zoff + cg), zz);
#pragma unroll
        for (int k = 0; k < 8; ++k) f[k] *= dgelu(zz[k]);
    }
    *dst = pack8(f);
}

__global__ void k_upsample2_v8(const uint16_t *in, int n, int h, int w, int c, int ld, int off, uint16_t *out, int old,
                               int ooff)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int H2 = 2 * h, W2 = 2 * w, g = c / 8;
    if (idx >= (int64_t)n * H2 * W2 * g) return;
    const int cg = (int)(idx % g) * 8;
    const int64_t q = idx / g;
    const int x = (int)(q % W2), y = (int)((q / W2) % H2), nn = (int)(q / ((int64_t)W2 * H2));
    *(uint4 *)(out + q * old + ooff + cg) =
        *(const uint4 *)(in + ((int64_t)(nn * h + y / 2) * w + x / 2) * ld + off + cg);
}

// z (optional, same layout as din): the sum is multiplied by GELU'(z).
__global__ void k_upsample2_bwd_v8(const uint16_t *dout, int n, int h, int w, int c, int dld, int doff, uint16_t *din,
                                   int ild, int ioff, const uint16_t *z, int zld, int zoff)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int g = c / 8;
    if (idx >= (int64_t)n * h * w * g) return;
    const int cg = (int)(idx % g) * 8;
    const int64_t q = idx / g;
    const int x = (int)(q % w), y = (int)((q / w) % h), nn = (int)(q / ((int64_t)w * h));
    const int W2 = 2 * w;
    float acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) {
            float f[8];
            unpack8(*(const uint4 *)(dout + ((int64_t)(nn * 2 * h + 2 * y + dy) * W2 + 2 * x + dx) * dld + doff + cg), f);
#pragma unroll
            for (int k = 0; k < 8; ++k) acc[k] += f[k];
        }
    if (z) {
        float zz[8];
        unpack8(*(const uint4 *)(z + q * zld + zoff + cg), zz);
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[k] *= dgelu(zz[k]);
    }
    *(uint4 *)(din + q * ild + ioff + cg) = pack8(acc);
}

__global__ void k_dgelu_v8(uint16_t *d, int dld, int doff, const uint16_t *z, int zld, int zoff, int npix, int c)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int g = c / 8;
    if (idx >= (int64_t)npix * g) return;
    const int cg = (int)(idx % g) * 8;
    const int64_t p = idx / g;
    uint4 *pd = (uint4 *)(d + p * dld + doff + cg);
    float f[8], zz[8];
    unpack8(*pd, f);
    unpack8(*(const uint4 *)(z + p * zld + zoff + cg), zz);
#pragma unroll
    for (int k = 0; k < 8; ++k) f[k] *= dgelu(zz[k]);
    *pd = pack8(f);
}

__global__ void k_add_inplace(uint16_t *a, int ald, int aoff, const uint16_t *b, int bld, int boff, int npix, int c)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)npix * c) return;
    const int64_t p = idx / c;
    const int ch = (int)(idx % c);
    uint16_t *pa = a + p * ald + aoff + ch;
    *pa = f2bf(bf2f(*pa) + bf2f(b[p * bld + boff + ch]));
}

__global__ void k_dgelu(uint16_t *d, int dld, int doff, const uint16_t *z, int zld, int zoff, int npix, int c)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)npix * c) return;
    const int64_t p = idx / c;
    const int ch = (int)(idx % c);
    uint16_t *pd = d + p * dld + doff + ch;
    *pd = f2bf(bf2f(*pd) * dgelu(bf2f(z[p * zld + zoff + ch])));
}

__global__ void k_to_bf16(const float *src, int npix, int c, uint16_t *dst, int cp)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)npix * cp) return;
    const int64_t p = idx / cp;
    const int ch = (int)(idx % cp);
    dst[idx] = ch < c ? f2bf(src[p * c + ch]) : (uint16_t)0;
}

// MSE: per-block partial sums of squared errors (fixed order), then one block
// adds the partials in order.
__global__ void __launch_bounds__(256) k_mse_partial(const float *pred, const float *target, int64_t count,
                                                     float *dpred, float scale, float *part)
{
    __shared__ float red[256];
    const int64_t per = (count + gridDim.x - 1) / gridDim.x;
    const int64_t b0 = blockIdx.x * per, b1 = min(count, b0 + per);
    float s = 0.0f;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += 256) {
        const float e = pred[i] - target[i];
        s += e * e;
        if (dpred) dpred[i] = 2.0f * e * scale;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// 64 lanes: lane l adds partial sums l, l + 64, ... in order (eight loads in
// flight), then lane 0 adds the 64 lane sums in lane order: a fixed order.
__global__ void __launch_bounds__(64) k_mse_final(const float *part, int nparts, float scale, float *loss)
{
    __shared__ float red[64];
    float s = 0.0f;
#pragma unroll 8
    for (int k = (int)threadIdx.x; k < nparts; k += 64) s += part[k];
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.0f;
        for (int l = 0; l < 64; ++l) t += red[l];
        *loss = t * scale;
    }
}

__global__ void k_adamw(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2,
                        float eps, float wd, float bc1, float bc2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / bc1, vh = vi / bc2;
    p[i] -= lr * (mh / (sqrtf(vh) + eps) + wd * p[i]);
}

// Nearest neighbour: one workgroup per query; the reference set is streamed.
__global__ void __launch_bounds__(256) k_nn(const float *q, int nq, const float *t, int nt, int d, float *dist2,
                                            int *index)
{
    __shared__ float best[256];
    __shared__ int bidx[256];
    const int i = blockIdx.x;
    if (i >= nq) return;
    float bd = INFINITY;
    int bi = 0x7fffffff;
    for (int j = threadIdx.x; j < nt; j += 256) {
        float s = 0.0f;
        for (int k = 0; k < d; ++k) {
            const float e = q[(int64_t)i * d + k] - t[(int64_t)j * d + k];
            s += e * e;
        }
        if (s < bd || (s == bd && j < bi)) {
            bd = s;
            bi = j;
        }
    }
    best[threadIdx.x] = bd;
    bidx[threadIdx.x] = bi;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            const float od = best[threadIdx.x + o];
            const int oi = bidx[threadIdx.x + o];
            if (od < best[threadIdx.x] || (od == best[threadIdx.x] && oi < bidx[threadIdx.x])) {
                best[threadIdx.x] = od;
                bidx[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        dist2[i] = best[0];
        index[i] = bidx[0];
    }
}

// Router features: the f x f box means of a gap field followed by the
// scaled depth; one thread per output value.
__global__ void k_features(const float *gap, int n, int h, int w, int f, const float *depth, float depth_scale,
                           float *out)
{
    const int ho = h / f, wo = w / f, row = ho * wo + 1;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * row) return;
    const int k = (int)(idx / row), t = (int)(idx - (int64_t)k * row);
    if (t == row - 1) {
        out[idx] = depth[k] * depth_scale;
        return;
    }
    const int y = t / wo, x = t - y * wo;
    float s = 0.0f;
    for (int dy = 0; dy < f; ++dy)
        for (int dx = 0; dx < f; ++dx) s += gap[((int64_t)k * h + y * f + dy) * w + x * f + dx];
    out[idx] = s / (float)(f * f);
}

// Per-sample mean squared difference of one channel: one workgroup per
// sample, fixed-order reduction.
__global__ void __launch_bounds__(256) k_channel_mse(const float *a, const float *b, int npix, int c, int ch,
                                                     float *out)
{
    __shared__ float red[256];
    const int k = blockIdx.x;
    const float *pa = a + (int64_t)k * npix * c + ch, *pb = b + (int64_t)k * npix * c + ch;
    float s = 0.0f;
    for (int p = threadIdx.x; p < npix; p += 256) {
        const float e = pa[(int64_t)p * c] - pb[(int64_t)p * c];
        s += e * e;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = red[0] / (float)npix;
}

// Symmetry copies of surrogate samples: op bit 2 transposes (x <-> y), bit 0
// mirrors x, bit 1 mirrors y, applied to the field in that order; vector
// channels (ux, uy) of the target turn with it. One thread per output pixel.
__global__ void k_augment(const float *x, const float *y, int n, int res, const int *ops, float *xo, float *yo)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * res * res) return;
    const int k = (int)(idx / ((int64_t)res * res));
    const int rem = (int)(idx - (int64_t)k * res * res);
    const int r = rem / res, c = rem - r * res;  // output row (y) and column (x)
    const int op = ops[k];
    int sx = c, sy = r;
    if (op & 2) sy = res - 1 - sy;
    if (op & 1) sx = res - 1 - sx;
    if (op & 4) {
        const int t = sx;
        sx = sy;
        sy = t;
    }
    const int64_t src = ((int64_t)k * res + sy) * res + sx;
    xo[idx * 2 + 0] = x[src * 2 + 0];
    xo[idx * 2 + 1] = x[src * 2 + 1];
    float ux = y[src * 3 + 0], uy = y[src * 3 + 1];
    if (op & 4) {
        const float t = ux;
        ux = uy;
        uy = t;
    }
    if (op & 1) ux = -ux;
    if (op & 2) uy = -uy;
    yo[idx * 3 + 0] = ux;
    yo[idx * 3 + 1] = uy;
    yo[idx * 3 + 2] = y[src * 3 + 2];
}

// out[p][2] += scale * min(x[p][0], 0): the contact term of the output,
// added in FP32 after the head.
__global__ void k_contact_residual(float *out, const float *x, int64_t npix, float scale)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npix) return;
    out[p * 3 + 2] += scale * fminf(x[p * 2], 0.0f);
}

unsigned blocks_for(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

// a view whose 8-channel groups are 16-byte aligned
bool v8_ok(const void *p, int c, int ld, int off) { return aligned16(p) && c % 8 == 0 && ld % 8 == 0 && off % 8 == 0; }

}  // namespace tsg

using namespace tsg;

extern "C" {

const char *tsg_last_error(void) { return g_err.c_str(); }

int32_t tsg_pack_k(int32_t taps, int32_t cin_p) { return ((taps * cin_p + 31) / 32) * 32; }

tsg_status tsg_pack_weights(const float *w, int32_t cout, int32_t cin, int32_t cin_p, int32_t cout_p, int32_t taps,
                            uint16_t *wf, uint16_t *wt, void *stream)
{
    if (!w || cout < 1 || cin < 1 || cin_p < cin || cout_p < cout || (taps != 1 && taps != 9) || cin_p % 8 ||
        (wt && cout_p % 8))
        return fail(-1, "tsg_pack_weights: bad arguments");
    const int kf = tsg_pack_k(taps, cin_p), kt = tsg_pack_k(taps, cout_p);
    const int64_t n = std::max<int64_t>(wf ? (int64_t)cout * kf : 0, wt ? (int64_t)cin_p * kt : 0);
    hipLaunchKernelGGL(k_pack, dim3(blocks_for(n)), dim3(256), 0, (hipStream_t)stream, w, cout, cin, cin_p, cout_p,
                       taps, kf, kt, wf, wt);
    TSG_LAUNCHED();
    return 0;
}

tsg_status tsg_conv(const uint16_t *in, int32_t n, int32_t h, int32_t w, int32_t in_ld, int32_t in_off, int32_t cin_p,
                    const uint16_t *wpack, const float *bias, int32_t cout, int32_t taps, int32_t epi, uint16_t *out,
                    int32_t out_ld, int32_t out_off, uint16_t *zbuf, int32_t z_ld, int32_t z_off, float *out32,
                    void *stream)
{
    if (!in || !wpack || n < 1 || h < 1 || w < 1 || cin_p < 8 || cin_p % 8 || in_ld % 8 || in_off % 8 ||
        in_off + cin_p > in_ld || cout < 1 || (taps != 1 && taps != 9) || epi < 0 || epi > 3 ||
        !aligned16(in) || !aligned16(wpack))
        return fail(-1, "tsg_conv: bad input view or weights");
    if (epi == TSG_EPI_F32) {
        if (!out32) return fail(-1, "tsg_conv: F32 epilogue needs out32");
    } else {
        if (!out || cout % 4 || out_ld % 4 || out_off % 4 || out_off + cout > out_ld || ((uintptr_t)out & 7))
            return fail(-1, "tsg_conv: bad output view");
        if ((epi == TSG_EPI_BIAS_GELU || epi == TSG_EPI_DGELU) &&
            (!zbuf || z_ld % 4 || z_off % 4 || z_off + cout > z_ld || ((uintptr_t)zbuf & 7)))
            return fail(-1, "tsg_conv: GELU epilogues need a pre-activation view");
    }
    ConvArgs a{in, n, h, w, in_ld, in_off, cin_p, wpack, tsg_pack_k(taps, cin_p), bias, cout, out, out_ld, out_off,
               zbuf, z_ld, z_off, out32};
    hipStream_t st = (hipStream_t)stream;
    const int wco = cout >= 64 ? 4 : (cout >= 32 ? 2 : 1);
    if (conv_lds_fits(taps, epi, cin_p, w)) return launch_conv_lds(a, epi, st);
    if (taps == 9) {
        if (wco == 4) return launch_conv_epi<4, 9>(a, epi, st);
        if (wco == 2) return launch_conv_epi<2, 9>(a, epi, st);
        return launch_conv_epi<1, 9>(a, epi, st);
    }
    if (wco == 4) return launch_conv_epi<4, 1>(a, epi, st);
    if (wco == 2) return launch_conv_epi<2, 1>(a, epi, st);
    return launch_conv_epi<1, 1>(a, epi, st);
}

// the all-taps kernel applies where its chunks stay inside one image and
// its shifted rows stay aligned
// Pixels per chunk of the all-taps weight gradient for this layer, 0 when
// the per-tap kernel runs instead.
static int wgrad9_chunk(int h, int w, int taps)
{
    if (taps != 9 || w < 8 || w > 64 || w % 8) return 0;
    const int64_t hw = (int64_t)h * w;
    if (w >= 16 && hw % 128 == 0) return 128;
    if (hw % 64 == 0 && 64 % w == 0) return 64;
    return 0;
}

static int wgrad_splits(int64_t npix, int h, int w, int cout, int cin_p, int taps)
{
    if (const int ch = wgrad9_chunk(h, w, taps)) {
        // ~2 workgroups per CU (the staged halo takes ~59 KB of LDS), each
        // over at least 4 chunks
        const int64_t tiles = (int64_t)((cout + 31) / 32) * ((cin_p + 31) / 32);
        int64_t s = std::max<int64_t>(1, 512 / tiles);
        s = std::min<int64_t>(s, std::max<int64_t>(1, npix / (4 * ch)));
        return (int)s;
    }
    const int64_t tiles = (int64_t)((cout + 31) / 32) * taps * ((cin_p + 31) / 32);
    int64_t s = std::max<int64_t>(1, 2048 / tiles);
    s = std::min<int64_t>(s, std::max<int64_t>(1, npix / 256));
    return (int)s;
}

size_t tsg_wgrad_scratch_bytes(int32_t n, int32_t h, int32_t w, int32_t cin_p, int32_t cout, int32_t taps)
{
    const int64_t npix = (int64_t)n * h * w;
    const int s = wgrad_splits(npix, h, w, cout, cin_p, taps);
    const size_t part = (size_t)s * cout * taps * cin_p * sizeof(float);
    const size_t bias = (size_t)s * cout * sizeof(float);
    return part + bias;
}

tsg_status tsg_conv_wgrad(const uint16_t *in, int32_t n, int32_t h, int32_t w, int32_t in_ld, int32_t in_off,
                          int32_t cin, int32_t cin_p, const uint16_t *dout, int32_t d_ld, int32_t d_off, int32_t cout,
                          int32_t taps, float *dw, float *db, float *scratch, size_t scratch_bytes, void *stream)
{
    if (!in || !dout || !dw || !scratch || cin < 1 || cin_p < cin || cin_p % 4 || cout % 4 || in_ld % 4 ||
        in_off % 4 || d_ld % 4 || d_off % 4 || (taps != 1 && taps != 9))
        return fail(-1, "tsg_conv_wgrad: bad arguments");
    if (scratch_bytes < tsg_wgrad_scratch_bytes(n, h, w, cin_p, cout, taps))
        return fail(-1, "tsg_conv_wgrad: scratch too small");
    hipStream_t st = (hipStream_t)stream;
    const int64_t npix = (int64_t)n * h * w;
    int splits = wgrad_splits(npix, h, w, cout, cin_p, taps);
    const int ch9 = wgrad9_chunk(h, w, taps), chunk = ch9 ? ch9 : kWgChunk;
    int pps = (int)((npix + splits - 1) / splits);
    pps = ((pps + chunk - 1) / chunk) * chunk;
    // rounding the splits up to whole chunks can leave the last ones empty:
    // only those holding pixels are launched and summed (never more than the
    // scratch was sized for)
    if (pps > 0) splits = (int)std::min<int64_t>(splits, (npix + pps - 1) / pps);
    float *bpart = db ? scratch + (size_t)splits * cout * taps * cin_p : nullptr;
    if (ch9) {
        const dim3 grid((cout + 31) / 32, (cin_p + 31) / 32, splits);
        if (ch9 == 128)
            hipLaunchKernelGGL(k_wgrad9<128>, grid, dim3(256), 0, st, in, n, h, w, in_ld, in_off, cin_p, dout, d_ld,
                               d_off, cout, pps, scratch, bpart);
        else
            hipLaunchKernelGGL(k_wgrad9<64>, grid, dim3(256), 0, st, in, n, h, w, in_ld, in_off, cin_p, dout, d_ld,
                               d_off, cout, pps, scratch, bpart);
    } else {
        const dim3 grid((cout + 31) / 32, taps * ((cin_p + 31) / 32), splits);
        hipLaunchKernelGGL(k_wgrad, grid, dim3(256), 0, st, in, n, h, w, in_ld, in_off, cin_p, dout, d_ld, d_off,
                           cout, taps, pps, scratch, bpart);
    }
    TSG_LAUNCHED();
    const int nw_blocks = (int)(((int64_t)cout * taps * cin + 31) / 32);
    const int nb_blocks = db ? (cout + 31) / 32 : 0;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((unsigned)(nw_blocks + nb_blocks)), dim3(256), 0, st, scratch, splits, cout,
                       taps, cin, cin_p, dw, nw_blocks, bpart, db);
    TSG_LAUNCHED();
    return 0;
}

size_t tsg_head_scratch_bytes(int32_t cout, int32_t cin)
{
    return (size_t)kHeadSplits * cout * (cin + 1) * sizeof(float);
}

tsg_status tsg_conv_wgrad_f32(const uint16_t *in, int32_t n, int32_t h, int32_t w, int32_t in_ld, int32_t in_off,
                              int32_t cin, int32_t cin_p, const float *dout, int32_t cout, float *dw, float *db,
                              float *scratch, size_t scratch_bytes, void *stream)
{
    const int64_t npix = (int64_t)n * h * w;
    if (!in || !dout || !dw || !db || !scratch || cout < 1 || cin < 1 || cout * (cin + 1) > 1024 || cin_p < cin ||
        in_off + cin > in_ld || npix < 1)
        return fail(-1, "tsg_conv_wgrad_f32: bad arguments");
    if (scratch_bytes < tsg_head_scratch_bytes(cout, cin)) return fail(-1, "tsg_conv_wgrad_f32: scratch too small");
    hipStream_t st = (hipStream_t)stream;
    const int nval = cout * (cin + 1);
    int splits = kHeadSplits;
    if (cin % 8 == 0 && cin <= 32 && cout <= 4 && v8_ok(in, cin, in_ld, in_off)) {
        // 16-byte loads; at least 16 rows per thread (fewer, larger splits)
        const int G = cin / 8, RS = 256 / G;
        splits = (int)std::max<int64_t>(1, std::min<int64_t>(kHeadSplits, npix / (16 * RS)));
        const int rps = (int)((npix + splits - 1) / splits);
        auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3(splits), dim3(256), 0, st, in, (int)npix, in_ld, in_off, dout, rps, scratch);
        };
#define TSG_HEAD_V8(GG)                                                      \
    case GG:                                                                 \
        if (cout == 1) go(k_head_wgrad_v8<GG, 1>);                           \
        else if (cout == 2) go(k_head_wgrad_v8<GG, 2>);                      \
        else if (cout == 3) go(k_head_wgrad_v8<GG, 3>);                      \
        else go(k_head_wgrad_v8<GG, 4>);                                     \
        break;
        switch (G) {
            TSG_HEAD_V8(1)
            TSG_HEAD_V8(2)
            TSG_HEAD_V8(3)
            default: TSG_HEAD_V8(4)
        }
#undef TSG_HEAD_V8
    } else {
        const int rps = (int)((npix + kHeadSplits - 1) / kHeadSplits);
        hipLaunchKernelGGL(k_head_wgrad, dim3(kHeadSplits), dim3(((nval + 63) / 64) * 64), 0, st, in, (int)npix, in_ld,
                           in_off, cin, dout, cout, rps, scratch);
    }
    TSG_LAUNCHED();
    hipLaunchKernelGGL(k_head_reduce, dim3(nval), dim3(256), 0, st, scratch, splits, cout, cin, dw, db);
    TSG_LAUNCHED();
    return 0;
}

tsg_status tsg_head_dgrad(const float *dout, int32_t npix, int32_t cout, const float *w, int32_t cin, uint16_t *din,
                          int32_t din_ld, int32_t din_off, const uint16_t *zbuf, int32_t z_ld, int32_t z_off,
                          void *stream)
{
    if (!dout || !w || !din || npix < 1 || cin < 1 || cout < 1 || (int64_t)npix * cin >= ((int64_t)1 << 31))
        return fail(-1, "tsg_head_dgrad: bad arguments");
    if (cin % 8 == 0 && v8_ok(din, cin, din_ld, din_off) && (!zbuf || v8_ok(zbuf, cin, z_ld, z_off)))
        hipLaunchKernelGGL(k_head_dgrad_v8, dim3(blocks_for((int64_t)npix * (cin / 8))), dim3(256), 0,
                           (hipStream_t)stream, dout, npix, cout, w, cin, din, din_ld, din_off, zbuf, z_ld, z_off);
    else
        hipLaunchKernelGGL(k_head_dgrad, dim3(blocks_for((int64_t)npix * cin)), dim3(256), 0, (hipStream_t)stream,
                           dout, npix, cout, w, cin, din, din_ld, din_off, zbuf, z_ld, z_off);
    TSG_LAUNCHED();
    return 0;
}

tsg_status tsg_avgpool2(const uint16_t *in, int32_t n, int32_t h, int32_t w, int32_t c, int32_t in_ld, int32_t in_off,
                        uint16_t *out, int32_t out_ld, int32_t out_off, void *stream)
{
    if (!in || !out || h % 2 || w % 2) return fail(-1, "tsg_avgpool2: bad arguments");
    if (v8_ok(in, c, in_ld, in_off) && v8_ok(out, c, out_ld, out_off)) {
        hipLaunchKernelGGL(k_avgpool2_v8, dim3(blocks_for((int64_t)n * (h / 2) * (w / 2) * (c / 8))), dim3(256), 0,
                           (hipStream_t)stream, in, n, h, w, c, in_ld, in_off, out, out_ld, out_off);
        TSG_LAUNCHED();
        return 0;
    }
    hipLaunchKernelGGL(k_avgpool2, dim3(blocks_for((int64_t)n * (h / 2) * (w / 2) * c)), dim3(256), 0,
                       (hipStream_t)stream, in, n, h, w, c, in_ld, in_off, out, out_ld, out_off);
    TSG_LAUNCHED();
    return 0;
}

tsg_status tsg_avgpool2_bwd(const uint16_t *dout, int32_t n, int32_t h, int32_t w, int32_t c, int32_t d_ld,
                            int32_t d_off, uint16_t *din, int32_t din_ld, int32_t din_off, int32_t accumulate,
                            void *stream)
{
    if (!dout || !din || h % 2 || w % 2) return fail(-1, "tsg_avgpool2_bwd: bad arguments");
    if (v8_ok(dout, c, d_ld, d_off) && v8_ok(din, c, din_ld, din_off)) {
        hipLaunchKernelGGL(k_avgpool2_bwd_v8, dim3(blocks_for((int64_t)n * h * w * (c / 8))), dim3(256), 0,
                           (hipStream_t)stream, dout, n, h, w, c, d_ld, d_off, din, din_ld, din_off, accumulate,
                           nullptr, 0, 0);
        TSG_LAUNCHED();
        return 0;
    }
    hipLaunchKernelGGL(k_avgpool2_bwd, dim3(blocks_for((int64_t)n * h * w * c)), dim3(256), 0, (hipStream_t)stream,
                       dout, n, h, w, c, d_ld, d_off, din, din_ld, din_off, accumulate);
    TSG_LAUNCHED();
    return 0;
}

tsg_status tsg_upsample2(const uint16_t *in, int32_t n, int32_t h, int32_t w, int32_t c, int32_t in_ld,
                         int32_t in_off, uint16_t *out, int32_t out_ld, int32_t out_off, void *stream)
{
    if (!in || !out) return fail(-1, "tsg_upsample2: bad arguments");
    if (v8_ok(in, c, in_ld, in_off) && v8_ok(out, c, out_ld, out_off)) {
        hipLaunchKernelGGL(k_upsample2_v8, dim3(blocks_for((int64_t)n * 4 * h * w * (c / 8))), dim3(256), 0,
                           (hipStream_t)stream, in, n, h, w, c, in_ld, in_off, out, out_ld, out_off);
        TSG_LAUNCHED();
        return 0;
    }
    hipLaunchKernelGGL(k_upsample2, dim3(blocks_for((int64_t)n * 4 * h * w * c)), dim3(256), 0, (hipStream_t)stream,
                       in, n, h, w, c, in_ld, in_off, out, out_ld, out_off);
    TSG_LAUNCHED();
    return 0;
}

tsg_status tsg_upsample2_bwd(const uint16_t *dout, int32_t n, int32_t h, int32_t w, int32_t c, int32_t d_ld,
                             int32_t d_off, uint16_t *din, int32_t din_ld, int32_t din_off, void *stream)
{
    if (!dout || !din) return fail(-1, "tsg_upsample2_bwd: bad arguments");
    if (v8_ok(dout, c, d_ld, d_off) && v8_ok(din, c, din_ld, din_off)) {
        hipLaunchKernelGGL(k_upsample2_bwd_v8, dim3(blocks_for((int64_t)n * h * w * (c / 8))), dim3(256), 0,
                           (hipStream_t)stream, dout, n, h, w, c, d_ld, d_off, din, din_ld, din_off, nullptr, 0, 0);
        TSG_LAUNCHED();
        return 0;
    }
    hipLaunchKernelGGL(k_upsample2_bwd, dim3(blocks_for((int64_t)n * h * w * c)), dim3(256), 0, (hipStream_t)stream,
                       dout, n, h, w, c, d_ld, d_off, din, din_ld, din_off);
    TSG_LAUNCHED();
    return 0;
}

tsg_status tsg_add_inplace(uint16_t *a, int32_t a_ld, int32_t a_off, const uint16_t *b, int32_t b_ld, int32_t b_off,
                           int32_t npix, int32_t c, void *stream)
{
    if (!a || !b) return fail(-1, "tsg_add_inplace: bad arguments");
    hipLaunchKernelGGL(k_add_inplace, dim3(blocks_for((int64_t)npix * c)), dim3(256), 0, (hipStream_t)stream, a, a_ld,
                       a_off, b, b_ld, b_off, npix, c);
    TSG_LAUNCHED();
    return 0;
}

tsg_status tsg_dgelu(uint16_t *d, int32_t d_ld, int32_t d_off, const uint16_t *z, int32_t z_ld, int32_t z_off,
                     int32_t npix, int32_t c, void *stream)
{
    if (!d || !z) return fail(-1, "tsg_dgelu: bad arguments");
    if (v8_ok(d, c, d_ld, d_off) && v8_ok(z, c, z_ld, z_off)) {
        hipLaunchKernelGGL(k_dgelu_v8, dim3(blocks_for((int64_t)npix * (c / 8))), dim3(256), 0, (hipStream_t)stream, d,
                           d_ld, d_off, z, z_ld, z_off, npix, c);
        TSG_LAUNCHED();
        return 0;
    }
    hipLaunchKernelGGL(k_dgelu, dim3(blocks_for((int64_t)npix * c)), dim3(256), 0, (hipStream_t)stream, d, d_ld, d_off,
                       z, z_ld, z_off, npix, c);
    TSG_LAUNCHED();
    return 0;
}

tsg_status tsg_avgpool2_bwd_dgelu(const uint16_t *dout, int32_t n, int32_t h, int32_t w, int32_t c, int32_t d_ld,
                                  int32_t d_off, uint16_t *din, int32_t din_ld, int32_t din_off, int32_t accumulate,
                                  const uint16_t *z, int32_t z_ld, int32_t z_off, void *stream)
{
    if (!dout || !din || !z || h % 2 || w % 2) return fail(-1, "tsg_avgpool2_bwd_dgelu: bad arguments");
    if (v8_ok(dout, c, d_ld, d_off) && v8_ok(din, c, din_ld, din_off) && v8_ok(z, c, z_ld, z_off)) {
        hipLaunchKernelGGL(k_avgpool2_bwd_v8, dim3(blocks_for((int64_t)n * h * w * (c / 8))), dim3(256), 0,
                           (hipStream_t)stream, dout, n, h, w, c, d_ld, d_off, din, din_ld, din_off, accumulate, z,
                           z_ld, z_off);
        TSG_LAUNCHED();
        return 0;
    }
    // layouts the 8-channel kernels do not take: the two passes
    if (const tsg_status e = tsg_avgpool2_bwd(dout, n, h, w, c, d_ld, d_off, din, din_ld, din_off, accumulate, stream))
        return e;
    return tsg_dgelu(din, din_ld, din_off, z, z_ld, z_off, n * h * w, c, stream);
}

tsg_status tsg_upsample2_bwd_dgelu(const uint16_t *dout, int32_t n, int32_t h, int32_t w, int32_t c, int32_t d_ld,
                                   int32_t d_off, uint16_t *din, int32_t din_ld, int32_t din_off, const uint16_t *z,
                                   int32_t z_ld, int32_t z_off, void *stream)
{
    if (!dout || !din || !z) return fail(-1, "tsg_upsample2_bwd_dgelu: bad arguments");
    if (v8_ok(dout, c, d_ld, d_off) && v8_ok(din, c, din_ld, din_off) && v8_ok(z, c, z_ld, z_off)) {
        hipLaunchKernelGGL(k_upsample2_bwd_v8, dim3(blocks_for((int64_t)n * h * w * (c / 8))), dim3(256), 0,
                           (hipStream_t)stream, dout, n, h, w, c, d_ld, d_off, din, din_ld, din_off, z, z_ld, z_off);
        TSG_LAUNCHED();
        return 0;
    }
    if (const tsg_status e = tsg_upsample2_bwd(dout, n, h, w, c, d_ld, d_off, din, din_ld, din_off, stream)) return e;
    return tsg_dgelu(din, din_ld, din_off, z, z_ld, z_off, n * h * w, c, stream);
}

tsg_status tsg_mse(const float *pred, const float *target, int64_t count, float *loss, float *dpred, float *scratch,
                   void *stream)
{
    if (!pred || !target || !loss || !scratch || count < 1) return fail(-1, "tsg_mse: bad arguments");
    const int parts = 1024;
    hipLaunchKernelGGL(k_mse_partial, dim3(parts), dim3(256), 0, (hipStream_t)stream, pred, target, count, dpred,
                       1.0f / (float)count, scratch);
    TSG_LAUNCHED();
    hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(64), 0, (hipStream_t)stream, scratch, parts, 1.0f / (float)count,
                       loss);
    TSG_LAUNCHED();
    return 0;
}

tsg_status tsg_adamw(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2, float eps,
                     float wd, int32_t step, void *stream)
{
    if (!p || !g || !m || !v || n < 1 || step < 1) return fail(-1, "tsg_adamw: bad arguments");
    // 1 - b^t in FP64 before rounding: b2^t is close to 1 for small t
    const float bc1 = (float)(1.0 - std::pow((double)b1, (double)step));
    const float bc2 = (float)(1.0 - std::pow((double)b2, (double)step));
    hipLaunchKernelGGL(k_adamw, dim3(blocks_for(n)), dim3(256), 0, (hipStream_t)stream, p, g, m, v, n, lr, b1, b2, eps,
                       wd, bc1, bc2);
    TSG_LAUNCHED();
    return 0;
}

tsg_status tsg_to_bf16(const float *src, int32_t npix, int32_t c, uint16_t *dst, int32_t cp, void *stream)
{
    if (!src || !dst || cp < c) return fail(-1, "tsg_to_bf16: bad arguments");
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks_for((int64_t)npix * cp)), dim3(256), 0, (hipStream_t)stream, src, npix, c,
                       dst, cp);
    TSG_LAUNCHED();
    return 0;
}

tsg_status tsg_nn_dist(const float *q, int32_t nq, const float *t, int32_t nt, int32_t d, float *dist2, int32_t *index,
                       void *stream)
{
    if (!q || !t || !dist2 || !index || nq < 1 || nt < 1 || d < 1) return fail(-1, "tsg_nn_dist: bad arguments");
    hipLaunchKernelGGL(k_nn, dim3(nq), dim3(256), 0, (hipStream_t)stream, q, nq, t, nt, d, dist2, index);
    TSG_LAUNCHED();
    return 0;
}

tsg_status tsg_features(const float *gap, int32_t n, int32_t h, int32_t w, int32_t f, const float *depth,
                        float depth_scale, float *out, void *stream)
{
    if (!gap || !depth || !out || n < 1 || f < 1 || h % f || w % f) return fail(-1, "tsg_features: bad arguments");
    const int64_t total = (int64_t)n * ((h / f) * (w / f) + 1);
    hipLaunchKernelGGL(k_features, dim3(blocks_for(total)), dim3(256), 0, (hipStream_t)stream, gap, n, h, w, f, depth,
                       depth_scale, out);
    TSG_LAUNCHED();
    return 0;
}

tsg_status tsg_channel_mse(const float *a, const float *b, int32_t n, int32_t npix, int32_t c, int32_t ch, float *out,
                           void *stream)
{
    if (!a || !b || !out || n < 1 || npix < 1 || c < 1 || ch < 0 || ch >= c)
        return fail(-1, "tsg_channel_mse: bad arguments");
    hipLaunchKernelGGL(k_channel_mse, dim3(n), dim3(256), 0, (hipStream_t)stream, a, b, npix, c, ch, out);
    TSG_LAUNCHED();
    return 0;
}

tsg_status tsg_augment(const float *x, const float *y, int32_t n, int32_t res, const int32_t *ops, float *x_out,
                       float *y_out, void *stream)
{
    if (!x || !y || !ops || !x_out || !y_out || n < 1 || res < 1 || x == x_out || y == y_out)
        return fail(-1, "tsg_augment: bad arguments");
    hipLaunchKernelGGL(k_augment, dim3(blocks_for((int64_t)n * res * res)), dim3(256), 0, (hipStream_t)stream, x, y, n,
                       res, ops, x_out, y_out);
    TSG_LAUNCHED();
    return 0;
}

tsg_status tsg_contact_residual(float *out, const float *x, int64_t npix, float scale, void *stream)
{
    if (!out || !x || npix < 1) return fail(-1, "tsg_contact_residual: bad arguments");
    hipLaunchKernelGGL(k_contact_residual, dim3(blocks_for(npix)), dim3(256), 0, (hipStream_t)stream, out, x, npix,
                       scale);
    TSG_LAUNCHED();
    return 0;
}

}  // extern "C"
