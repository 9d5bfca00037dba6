// The dose denoiser: a fixed 4-level 3D U-Net trained and run by this
// library's own kernels.
//
// Tensors are channels-last (N, D, H, W, C) bf16 with C a multiple of 8.
// The 3x3x3 convolutions (zero padding 1) are implicit GEMMs on the gfx950
// MFMA unit (mfma_f32_16x16x32_bf16, fp32 accumulation): a wave computes 16
// consecutive voxels x all output channels; the K dimension runs over
// (offset, input channel) in chunks of 32, each lane loading 8 contiguous
// input channels of one neighbour (16 bytes) and 8 contiguous weights.
//   forward  y = act(conv(x, W) + b)               (k_conv3)
//   dgrad    dx = conv(dy, W') * (x > 0)            (k_conv3 with W' the
//            offset-flipped, channel-transposed weights and a ReLU mask)
//   wgrad    dW[co][o][ci] = sum_v dy[v][co] x[v+o][ci]  (k_conv3_wgrad:
//            dy and shifted x tiles staged in LDS, MFMA over voxels,
//            fp32 atomics per tile)
// Average pooling, nearest up-sampling, channel concatenation, the 1x1
// residual head, the MSE loss and Adam are plain streaming kernels.
#include "common.hpp"

#include <hip/hip_bf16.h>

#include <atomic>
#include <cmath>
#include <vector>

namespace psl {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef uint16_t bf16_t;   // storage type

__device__ __forceinline__ float bf2f(bf16_t v) {
    return __uint_as_float((uint32_t)v << 16);
}
// round to nearest even
__device__ __forceinline__ bf16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (bf16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (bf16_t)(u >> 16);
}

struct Vol {
    int n, d, h, w;
    __host__ __device__ int64_t voxels() const {
        return (int64_t)n * d * h * w;
    }
};

constexpr int kMaxCout = 128;

// ------------------------------------------------------------ conv 3x3x3 --
// y[v][co] = epilogue(sum_{o,ci} x[v + o][ci] W[co][o*Cin + ci]),
// W rows padded to Kp = roundup(27 Cin, 32) with zeros.  A wave computes MT
// tiles of 16 consecutive voxels x 16 NB output channels (channel blocks
// blockIdx.y NB .. blockIdx.y NB + NB - 1), so every weight fragment it
// loads feeds MT matrix instructions and every input fragment NB of them.
template <int NB, int MT>   // output channel blocks of 16, voxel tiles of 16
__global__ void __launch_bounds__(256)
k_conv3(const bf16_t *__restrict__ x, Vol V, int Cin,
        const bf16_t *__restrict__ W, int Kp, const float *__restrict__ bias,
        int relu, const bf16_t *__restrict__ mask, int mask_c,
        bf16_t *__restrict__ y, int Cout) {
    const int lane = __lane_id();
    const int64_t tile0 =
        ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * (16 * MT);
    const int64_t nvox = V.voxels();
    if (tile0 >= nvox) return;
    // the A row of this lane in tile t: voxel tile0 + 16 t + lane % 16
    int vw[MT], vh[MT], vd[MT];
    int64_t vn[MT];
    bool vok[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) {
        const int64_t v = tile0 + 16 * t + (lane & 15);
        vok[t] = v < nvox;
        int64_t q = vok[t] ? v : 0;
        vw[t] = (int)(q % V.w); q /= V.w;
        vh[t] = (int)(q % V.h); q /= V.h;
        vd[t] = (int)(q % V.d); vn[t] = q / V.d;
    }
    f32x4 acc[MT][NB];
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[t][b] = f32x4{0, 0, 0, 0};
    const int kq = 8 * (lane >> 4);
    const int cb0 = blockIdx.y * NB;   // first channel block of the wave
    for (int k0 = 0; k0 < Kp; k0 += 32) {
        const int k = k0 + kq;
        const int o = k / Cin, ci = k - o * Cin;
        const int dz = o / 9 - 1, dy = (o / 3) % 3 - 1, dx = o % 3 - 1;
        bf16x8 a[MT];
#pragma unroll
        for (int t = 0; t < MT; ++t) {
            const int zz = vd[t] + dz, yy = vh[t] + dy, xx = vw[t] + dx;
            const bool ok = vok[t] && o < 27 &&
                            (unsigned)zz < (unsigned)V.d &&
                            (unsigned)yy < (unsigned)V.h &&
                            (unsigned)xx < (unsigned)V.w;
            if (ok) {
                const int64_t nb = ((vn[t] * V.d + zz) * V.h + yy) * V.w + xx;
                a[t] = *reinterpret_cast<const bf16x8 *>(x + nb * Cin + ci);
            } else {
                a[t] = bf16x8{};
            }
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int co = (cb0 + b) * 16 + (lane & 15);
            const bf16x8 wv = *reinterpret_cast<const bf16x8 *>(
                W + (int64_t)co * Kp + k);
#pragma unroll
            for (int t = 0; t < MT; ++t)
                acc[t][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    a[t], wv, acc[t][b], 0, 0, 0);
        }
    }
    // acc[t][b][r] is (voxel tile0 + 16 t + 4 (lane/16) + r,
    //                  channel 16 b + lane % 16)
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int co = (cb0 + b) * 16 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t vv = tile0 + 16 * t + 4 * (lane >> 4) + r;
                if (vv >= nvox || co >= Cout) continue;
                float val = acc[t][b][r] + (bias ? bias[co] : 0.0f);
                if (relu) val = fmaxf(val, 0.0f);
                if (mask && !(bf2f(mask[vv * mask_c + co]) > 0.0f))
                    val = 0.0f;
                y[vv * Cout + co] = f2bf(val);
            }
        }
}

// bf16 pair (x in the low half) by the hardware's round-to-nearest-even
// conversion; equal to f2bf for every non-NaN value
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
    const f32x2 v = {lo, hi};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}

constexpr int kBZ = 4, kBY = 4;

// The output head fused into the last convolution (inference): out[v] =
// dose[v] scale[sample] + bh + sum_c f[v][c] wh[c], in k_head's order.
struct HeadArgs {
    const float *wh, *bh, *dose, *scale;
    float *out;                 // nullptr: no head
};

// The epilogue of the brick kernels.  acc[t][c][r] is voxel x = 4 (lane/16)
// + r of brick row wid ROWS + t, channel (cb0 + c) 16 + lane % 16.  Bias and
// ReLU are applied per value and the results packed to bf16; the wave's
// tile then goes through LDS (s_out, ROWS x 16 x (16 NB + 8) elements per
// wave, free for reuse by the caller) so that each lane stores 16 bytes: 8
// consecutive channels of one voxel.  The data-gradient mask is applied to
// those 16 bytes (a value is kept where the mask is > 0).  With yp given
// (no mask), the brick's 2x2x2 averages go to yp on the half-resolution
// grid as well, summed in the order and precision of k_pool.  breg, when
// given, holds the lane's bias value per channel block (read beforehand).
template <int ROWS, int NB>
__device__ __forceinline__ void store_tiles(
    const f32x4 (&acc)[ROWS][NB], bf16_t *s_out, int wid, int lane,
    int64_t bn, int z0, int y0, int x0, Vol V, int cb0,
    const float *__restrict__ bias, int relu, const bf16_t *__restrict__ mask,
    bf16_t *__restrict__ y, int Cout, bf16_t *__restrict__ yp = nullptr,
    HeadArgs hd = HeadArgs{}, const float *breg = nullptr) {
    constexpr int OP = 16 * NB + 8;            // LDS pitch per voxel
    const int q = lane >> 4, l16 = lane & 15;
    bf16_t *tile = s_out + wid * ROWS * 16 * OP;
#pragma unroll
    for (int c = 0; c < NB; ++c) {
        const int ch = c * 16 + l16;
        const float bv = breg ? breg[c] : bias ? bias[cb0 * 16 + ch] : 0.0f;
#pragma unroll
        for (int t = 0; t < ROWS; ++t)
#pragma unroll
            for (int r = 0; r < 4; r += 2) {
                float v0 = acc[t][c][r] + bv, v1 = acc[t][c][r + 1] + bv;
                if (relu) { v0 = fmaxf(v0, 0.0f); v1 = fmaxf(v1, 0.0f); }
                const uint32_t pk = pack_bf16x2(v0, v1);
                bf16_t *dst = tile + (t * 16 + 4 * q + r) * OP + ch;
                dst[0] = (bf16_t)(pk & 0xffffu);
                dst[OP] = (bf16_t)(pk >> 16);
            }
    }
    __syncthreads();
    if (NB == 1 && hd.out) {
        // one voxel per lane: its 16 channels from the tile, the head's
        // products in channel order, the residual input added last
        static_assert(ROWS * 16 == 64, "a wave's tile is 64 voxels");
        const int t = lane / 16, xv = lane % 16;
        const int row = wid * ROWS + t;
        const int rz = row / kBY, ry = row % kBY;
        const int64_t v =
            ((bn * V.d + z0 + rz) * V.h + (y0 + ry)) * V.w + x0 + xv;
        float sacc = hd.bh[0];
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            const uint4 u =
                *reinterpret_cast<const uint4 *>(tile + lane * OP + 8 * g);
            const uint32_t w4[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                sacc += __uint_as_float(w4[m] << 16) * hd.wh[8 * g + 2 * m];
                sacc += __uint_as_float(w4[m] & 0xffff0000u) *
                        hd.wh[8 * g + 2 * m + 1];
            }
        }
        hd.out[v] = hd.dose[v] * hd.scale[bn] + sacc;
        return;
    }
    constexpr int PER = ROWS * 16 * 2 * NB / 64;   // 16-byte stores per lane
#pragma unroll
    for (int h = 0; h < PER; ++h) {
        const int idx = lane + 64 * h;
        const int p = idx / (2 * NB), k = idx % (2 * NB);
        const int t = p / 16, xv = p % 16;
        const int row = wid * ROWS + t;
        const int rz = row / kBY, ry = row % kBY;
        uint4 val = *reinterpret_cast<const uint4 *>(tile + p * OP + 8 * k);
        const int64_t off =
            (((bn * V.d + z0 + rz) * V.h + (y0 + ry)) * V.w + x0 + xv) * Cout +
            cb0 * 16 + 8 * k;
        if (mask) {
            const uint4 m = *reinterpret_cast<const uint4 *>(mask + off);
            const uint32_t mw[4] = {m.x, m.y, m.z, m.w};
            uint32_t vw[4] = {val.x, val.y, val.z, val.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const bool klo = __uint_as_float(mw[e] << 16) > 0.0f;
                const bool khi = __uint_as_float(mw[e] & 0xffff0000u) > 0.0f;
                vw[e] &= (klo ? 0x0000ffffu : 0u) | (khi ? 0xffff0000u : 0u);
            }
            val = make_uint4(vw[0], vw[1], vw[2], vw[3]);
        }
        *reinterpret_cast<uint4 *>(y + off) = val;
    }
    if (yp) {
        // one thread per pooled voxel of the brick and 8 channels: wave w
        // holds brick z-slice w, row t holds y-row t (4 x 4 bricks)
        static_assert(ROWS == kBY && kBZ == 4, "pooling assumes 4x4 bricks");
        __syncthreads();
        const int i = threadIdx.x;
        if (i < 64 * NB) {
            const int k = i % (2 * NB), pv = i / (2 * NB);
            const int px = pv % 8, py = (pv / 8) % 2, pz = pv / 16;
            float sum[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            for (int a = 0; a < 8; ++a) {
                const int zz = 2 * pz + (a >> 2), yy = 2 * py + ((a >> 1) & 1),
                          xx = 2 * px + (a & 1);
                const uint4 u = *reinterpret_cast<const uint4 *>(
                    s_out + zz * ROWS * 16 * OP + (yy * 16 + xx) * OP + 8 * k);
                const uint32_t uw[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    sum[2 * e] += __uint_as_float(uw[e] << 16);
                    sum[2 * e + 1] += __uint_as_float(uw[e] & 0xffff0000u);
                }
            }
            const Vol U{V.n, V.d / 2, V.h / 2, V.w / 2};
            const int64_t pofs =
                (((bn * U.d + z0 / 2 + pz) * U.h + (y0 / 2 + py)) * U.w +
                 x0 / 2 + px) * Cout + cb0 * 16 + 8 * k;
            *reinterpret_cast<uint4 *>(yp + pofs) = make_uint4(
                pack_bf16x2(0.125f * sum[0], 0.125f * sum[1]),
                pack_bf16x2(0.125f * sum[2], 0.125f * sum[3]),
                pack_bf16x2(0.125f * sum[4], 0.125f * sum[5]),
                pack_bf16x2(0.125f * sum[6], 0.125f * sum[7]));
        }
    }
}

// The same convolution with the input staged in LDS.  A block computes a
// brick of kBZ x kBY rows of 16 consecutive x-voxels for NB blocks of 16
// output channels (channel group blockIdx.y); each wave owns kBZ*kBY/4 rows.
// The zero-padded halo of the brick ((kBZ+2) x (kBY+2) x 18 voxels) is
// staged CC input channels at a time with 16-byte loads, at a voxel pitch of
// CC + 8 elements so that the 16 lanes reading one A fragment row hit
// distinct LDS banks.  Within a chunk the reduction runs over slots
// (tap o, 8-channel group g), four per matrix instruction (one per lane
// quarter); A and B take the same slot, so any slot order sums the same
// products.  A per-block table holds each slot's LDS and weight offsets, so
// the steps do no index arithmetic.  Requires W % 16 == 0, H % kBY == 0,
// D % kBZ == 0 and Cin % CC == 0.
// With xc given, the input is the decoder's concatenation read in place:
// channels [0, cc) are xc (half resolution, nearest up-sampling) and
// [cc, Cin) are x (cc and Cin - cc multiples of CC).  With yp given, the
// 2x2x2 average pool of the output is written there too.  With hd.out
// given (16 output channels), the output head is applied and y is not
// written.
template <int CC, int NB>
__global__ void __launch_bounds__(256)
k_conv3_bk(const bf16_t *__restrict__ x, Vol V, int Cin,
           const bf16_t *W, int Kp,
           const float *__restrict__ bias, int relu,
           const bf16_t *__restrict__ mask, bf16_t *__restrict__ y,
           int Cout, const bf16_t *__restrict__ xc, int cc,
           bf16_t *__restrict__ yp, HeadArgs hd) {
    constexpr int HZ = kBZ + 2, HY = kBY + 2, HX = 18;
    constexpr int HVOX = HZ * HY * HX;
    constexpr int G = CC / 8;                  // 16-byte groups per voxel
    constexpr int PITCH = CC + 8;              // LDS voxel pitch (elements)
    // The reduction runs over slots (dz, dx, g): for each, the three taps
    // dy = 0, 1, 2 of the wave's four consecutive output rows t read halo
    // rows t + dy, so six A fragments (halo rows 0..5) feed twelve matrix
    // instructions, tap dy taking weight fragment dy.  Four slots per step,
    // one per lane quarter.
    constexpr int SLOTS = 9 * G;
    constexpr int STEPS = (SLOTS + 3) / 4;
    constexpr int ROWS = kBZ * kBY / 4;        // rows (tiles) per wave
    static_assert(ROWS == 4, "a wave owns four consecutive y rows");
    static_assert(HVOX * PITCH >= 4 * ROWS * 16 * (16 * NB + 8),
                  "the epilogue reuses the halo buffer");
    __shared__ __attribute__((aligned(16))) bf16_t s_in[HVOX * PITCH];
    __shared__ int2 s_tab[STEPS * 4];
    // 16-channel input, one output block: the chunk's weights are staged
    // in LDS beside the halo (rows of 27 CC + 8 elements, so the 16 lanes
    // of a fragment row hit distinct banks), read there at every step
    constexpr bool WL = CC == 16 && NB == 1;
    constexpr int WP = 27 * CC + 8;
    __shared__ __attribute__((aligned(16))) bf16_t s_w[WL ? 16 * WP : 8];
    const int lane = __lane_id(), wid = threadIdx.x >> 6;
    const int nxb = V.w / 16, nyb = V.h / kBY, nzb = V.d / kBZ;
    int64_t b = blockIdx.x;
    const int bx = (int)(b % nxb); b /= nxb;
    const int by = (int)(b % nyb); b /= nyb;
    const int bz = (int)(b % nzb);
    const int64_t bn = b / nzb;
    const int x0 = bx * 16, y0 = by * kBY, z0 = bz * kBZ;
    const int cb0 = blockIdx.y * NB;
    const int q = lane >> 4, vx = lane & 15;
    // slot -> (LDS offset of (dz, dx, g) at dy = 0 relative to the lane's
    // first row, weight offset of tap (dz, 0, dx) and group g); slots past
    // the last point at slot 0 and are zeroed in the last step
    for (int sl = threadIdx.x; sl < STEPS * 4; sl += 256) {
        const int u = sl < SLOTS ? sl / G : 0, g = sl < SLOTS ? sl % G : 0;
        const int dz = u / 3, dx = u % 3;
        s_tab[sl] = make_int2((dz * HY * HX + dx) * PITCH + 8 * g,
                              (dz * 9 + dx) * (WL ? CC : Cin) + 8 * g);
    }
    // the lane's A row in the halo: brick row wid ROWS (rz = wid, ry = 0),
    // voxel vx; halo row r adds r HX PITCH
    const int a_base = ((wid * ROWS / kBY) * HY + (wid * ROWS) % kBY) * HX *
                           PITCH + vx * PITCH;
    const int dyw = 3 * (WL ? CC : Cin);       // weight offset of dy + 1
    const bf16_t *wrow[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c)
        wrow[c] = W + (int64_t)((cb0 + c) * 16 + vx) * Kp;
    f32x4 acc[ROWS][NB];
#pragma unroll
    for (int t = 0; t < ROWS; ++t)
#pragma unroll
        for (int c = 0; c < NB; ++c) acc[t][c] = f32x4{0, 0, 0, 0};
    constexpr int NIT = (HVOX * G + 255) / 256;  // halo loads per thread
    for (int c0 = 0; c0 < Cin; c0 += CC) {
        if (c0) __syncthreads();               // the last chunk's reads
        // the chunk's source: x, or with xc the coarse or the skip part
        const bool up = xc && c0 < cc;
        const bf16_t *src = up ? xc : x;
        const int sC = xc ? (up ? cc : Cin - cc) : Cin;
        const int sc0 = (xc && !up) ? c0 - cc : c0;
        const int sh = up ? 1 : 0;
        const int sd = V.d >> sh, shh = V.h >> sh, sw = V.w >> sh;
        // halo: voxel (hz, hy, hx) = input (z0+hz-1, y0+hy-1, x0+hx-1); all
        // of a thread's loads are issued before its LDS stores, so their
        // latencies overlap
        constexpr int NWI = WL ? (16 * 27 * G + 255) / 256 : 1;
        uint4 wval[NWI];
        if constexpr (WL) {
#pragma unroll
            for (int it = 0; it < NWI; ++it) {
                const int i = threadIdx.x + 256 * it;
                const int row = i / (27 * G), o = (i / G) % 27, g = i % G;
                wval[it] = make_uint4(0, 0, 0, 0);
                if (i < 16 * 27 * G)
                    wval[it] = *reinterpret_cast<const uint4 *>(
                        W + (int64_t)(cb0 * 16 + row) * Kp + o * Cin + c0 +
                        8 * g);
            }
        }
        uint4 hval[NIT];
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int i = threadIdx.x + 256 * it;
            const int g = i % G, hv = i / G;
            const int hx = hv % HX, hy = (hv / HX) % HY, hz = hv / (HX * HY);
            const int zz = z0 + hz - 1, yy = y0 + hy - 1, xx = x0 + hx - 1;
            hval[it] = make_uint4(0, 0, 0, 0);
            if (i < HVOX * G && (unsigned)zz < (unsigned)V.d &&
                (unsigned)yy < (unsigned)V.h && (unsigned)xx < (unsigned)V.w)
                hval[it] = *reinterpret_cast<const uint4 *>(
                    src + (((bn * sd + (zz >> sh)) * shh + (yy >> sh)) * sw +
                           (xx >> sh)) * sC + sc0 + g * 8);
        }
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int i = threadIdx.x + 256 * it;
            if (i < HVOX * G)
                *reinterpret_cast<uint4 *>(s_in + (i / G) * PITCH +
                                           (i % G) * 8) = hval[it];
        }
        if constexpr (WL) {
#pragma unroll
            for (int it = 0; it < NWI; ++it) {
                const int i = threadIdx.x + 256 * it;
                const int row = i / (27 * G), o = (i / G) % 27, g = i % G;
                if (i < 16 * 27 * G)
                    *reinterpret_cast<uint4 *>(s_w + row * WP + o * CC +
                                               8 * g) = wval[it];
            }
        }
        __syncthreads();
        // Weights of step j + 1 (three taps dy per channel block) are
        // loaded while step j computes (two buffers in turn; the empty asm
        // statements keep each prefetch ahead of the step that does not use
        // it).  Each buffer carries its step's LDS offset.
        auto wload = [&](int j, bf16x8 (*wv)[NB], int &aoff) {
            const int2 tb = s_tab[4 * j + q];
            aoff = a_base + tb.x;
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                for (int c = 0; c < NB; ++c)
                    wv[dy][c] = WL
                        ? *reinterpret_cast<const bf16x8 *>(
                              s_w + vx * WP + tb.y + dy * dyw)
                        : *reinterpret_cast<const bf16x8 *>(
                              wrow[c] + c0 + tb.y + dy * dyw);
        };
        auto step = [&](bf16x8 (*wv)[NB], int aoff, bool ok) {
            bf16x8 a[ROWS + 2];
#pragma unroll
            for (int r = 0; r < ROWS + 2; ++r) {
                const bf16x8 v = *reinterpret_cast<const bf16x8 *>(
                    s_in + aoff + r * HX * PITCH);
                a[r] = ok ? v : bf16x8{};
            }
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                for (int t = 0; t < ROWS; ++t)
#pragma unroll
                    for (int c = 0; c < NB; ++c)
                        acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            a[t + dy], wv[dy][c], acc[t][c], 0, 0, 0);
        };
        bf16x8 wa[3][NB], wb[3][NB];
        int oa, ob;
        wload(0, wa, oa);
        int j = 0;
#pragma unroll 1
        for (; j + 2 < STEPS; j += 2) {        // pairs before the last step
            wload(j + 1, wb, ob);
            asm volatile("" ::: "memory");
            step(wa, oa, true);
            wload(j + 2, wa, oa);
            asm volatile("" ::: "memory");
            step(wb, ob, true);
        }
        // the last one or two steps; only the last can hold padding slots
        const bool ok_last = (SLOTS % 4 == 0) || 4 * (STEPS - 1) + q < SLOTS;
        if (j + 1 < STEPS) {
            wload(j + 1, wb, ob);
            asm volatile("" ::: "memory");
            step(wa, oa, true);
            step(wb, ob, ok_last);
        } else {
            step(wa, oa, ok_last);
        }
    }
    __syncthreads();                           // the halo is free
    store_tiles<ROWS, NB>(acc, s_in, wid, lane, bn, z0, y0, x0, V, cb0, bias,
                          relu, mask, y, Cout, yp, hd);
}

// k_conv3_bk for 16 input channels per chunk and one block of 16 output
// channels per block (blockIdx.y; the finest level), as a loop over bricks: each block walks its share of the
// bricks (grid = the blocks resident at once) and loads the halo of its next
// (brick, chunk) into registers while the current one computes, so the
// latency of those loads hides behind the matrix instructions instead of
// behind other blocks.  With more bricks than blocks, the blocks of one XCD
// (blockIdx % 8) take one contiguous eighth of the bricks, so that the
// halos of neighbouring bricks meet in the same L2.  The weights of a chunk
// are staged in LDS beside the halo (once when Cin = 16, the case it is
// launched for).  Same arguments, requirements and sums as
// k_conv3_bk<16, 1>.
__global__ void __launch_bounds__(256)
k_conv3_bk16p(const bf16_t *__restrict__ x, Vol V, int Cin,
              const bf16_t *W, int Kp,
              const float *__restrict__ bias, int relu,
              const bf16_t *__restrict__ mask, bf16_t *__restrict__ y,
              int Cout, const bf16_t *__restrict__ xc, int cc,
              bf16_t *__restrict__ yp, HeadArgs hd) {
    constexpr int CC = 16, G = 2, PITCH = CC + 8;
    constexpr int HZ = kBZ + 2, HY = kBY + 2, HX = 18;
    constexpr int HVOX = HZ * HY * HX;
    constexpr int SLOTS = 9 * G, STEPS = (SLOTS + 3) / 4;
    constexpr int ROWS = kBZ * kBY / 4;
    constexpr int WP = 27 * CC + 8;            // LDS weight row (elements)
    static_assert(ROWS == 4, "a wave owns four consecutive y rows");
    static_assert(HVOX * PITCH >= 4 * ROWS * 16 * 24,
                  "the epilogue reuses the halo buffer");
    __shared__ __attribute__((aligned(16))) bf16_t s_in[HVOX * PITCH];
    __shared__ __attribute__((aligned(16))) bf16_t s_w[16 * WP];
    __shared__ int2 s_tab[STEPS * 4];
    const int lane = __lane_id(), wid = threadIdx.x >> 6;
    const int nxb = V.w / 16, nyb = V.h / kBY, nzb = V.d / kBZ;
    const int nbr = nxb * nyb * nzb * V.n;     // < 2^31 (grid limit)
    int br = blockIdx.x, br_end = nbr, br_step = gridDim.x;
    if (nbr > (int)gridDim.x && gridDim.x >= 8) {
        const int k = blockIdx.x & 7, per = (nbr + 7) / 8;
        br = k * per + (blockIdx.x >> 3);
        br_end = min(nbr, (k + 1) * per);
        br_step = ((int)gridDim.x - k + 7) / 8;
    }
    if (br >= br_end) return;
    const int q = lane >> 4, vx = lane & 15;
    for (int sl = threadIdx.x; sl < STEPS * 4; sl += 256) {
        const int u = sl < SLOTS ? sl / G : 0, g = sl < SLOTS ? sl % G : 0;
        const int dz = u / 3, dx = u % 3;
        s_tab[sl] = make_int2((dz * HY * HX + dx) * PITCH + 8 * g,
                              (dz * 9 + dx) * CC + 8 * g);
    }
    const int a_base = ((wid * ROWS / kBY) * HY + (wid * ROWS) % kBY) * HX *
                           PITCH + vx * PITCH;
    const int cb0 = blockIdx.y;                // output channel block
    const float bv = bias ? bias[cb0 * 16 + vx] : 0.0f;
    constexpr int NIT = (HVOX * G + 255) / 256;
    constexpr int NWI = (16 * 27 * G + 255) / 256;
    uint4 hval[NIT];
    auto fetch = [&](int bb, int c0) {
        const int bx = bb % nxb; bb /= nxb;
        const int by = bb % nyb; bb /= nyb;
        const int bz = bb % nzb;
        const int64_t bn = bb / nzb;
        const int x0 = bx * 16, y0 = by * kBY, z0 = bz * kBZ;
        const bool up = xc && c0 < cc;
        const bf16_t *src = up ? xc : x;
        const int sC = xc ? (up ? cc : Cin - cc) : Cin;
        const int sc0 = (xc && !up) ? c0 - cc : c0;
        const int sh = up ? 1 : 0;
        const int sd = V.d >> sh, shh = V.h >> sh, sw = V.w >> sh;
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int i = threadIdx.x + 256 * it;
            const int g = i % G, hv = i / G;
            const int hx = hv % HX, hy = (hv / HX) % HY, hz = hv / (HX * HY);
            const int zz = z0 + hz - 1, yy = y0 + hy - 1, xx = x0 + hx - 1;
            hval[it] = make_uint4(0, 0, 0, 0);
            if (i < HVOX * G && (unsigned)zz < (unsigned)V.d &&
                (unsigned)yy < (unsigned)V.h && (unsigned)xx < (unsigned)V.w)
                hval[it] = *reinterpret_cast<const uint4 *>(
                    src + (((bn * sd + (zz >> sh)) * shh + (yy >> sh)) * sw +
                           (xx >> sh)) * sC + sc0 + g * 8);
        }
    };
    f32x4 acc[ROWS];
    int c0 = 0, wc0 = -1;
    fetch(br, 0);
    for (;;) {
        if (c0 != wc0) {
            // the chunk's weights: through registers into LDS after the
            // barrier below
            uint4 wval[NWI];
#pragma unroll
            for (int it = 0; it < NWI; ++it) {
                const int i = threadIdx.x + 256 * it;
                const int row = i / (27 * G), o = (i / G) % 27, g = i % G;
                wval[it] = make_uint4(0, 0, 0, 0);
                if (i < 16 * 27 * G)
                    wval[it] = *reinterpret_cast<const uint4 *>(
                        W + (int64_t)(cb0 * 16 + row) * Kp + o * Cin + c0 +
                        8 * g);
            }
            __syncthreads();   // the last unit's reads of s_in / s_w
#pragma unroll
            for (int it = 0; it < NWI; ++it) {
                const int i = threadIdx.x + 256 * it;
                const int row = i / (27 * G), o = (i / G) % 27, g = i % G;
                if (i < 16 * 27 * G)
                    *reinterpret_cast<uint4 *>(s_w + row * WP + o * CC +
                                               8 * g) = wval[it];
            }
            wc0 = c0;
        } else {
            __syncthreads();   // the last unit's reads of s_in
        }
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int i = threadIdx.x + 256 * it;
            if (i < HVOX * G)
                *reinterpret_cast<uint4 *>(s_in + (i / G) * PITCH +
                                           (i % G) * 8) = hval[it];
        }
        __syncthreads();
        int nb2 = br, nc0 = c0 + CC;
        if (nc0 >= Cin) { nc0 = 0; nb2 = br + br_step; }
        const bool more = nb2 < br_end;
        if (more) fetch(nb2, nc0);             // in flight during the steps
        if (c0 == 0) {
#pragma unroll
            for (int t = 0; t < ROWS; ++t) acc[t] = f32x4{0, 0, 0, 0};
        }
        auto wload = [&](int j, bf16x8 (&wv)[3], int &aoff) {
            const int2 tb = s_tab[4 * j + q];
            aoff = a_base + tb.x;
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
                wv[dy] = *reinterpret_cast<const bf16x8 *>(
                    s_w + vx * WP + tb.y + dy * 3 * CC);
        };
        auto step = [&](const bf16x8 (&wv)[3], int aoff, bool ok) {
            bf16x8 a[ROWS + 2];
#pragma unroll
            for (int r = 0; r < ROWS + 2; ++r) {
                const bf16x8 v = *reinterpret_cast<const bf16x8 *>(
                    s_in + aoff + r * HX * PITCH);
                a[r] = ok ? v : bf16x8{};
            }
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                for (int t = 0; t < ROWS; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        a[t + dy], wv[dy], acc[t], 0, 0, 0);
        };
        bf16x8 wa[3], wb[3];
        int oa, ob;
        wload(0, wa, oa);
        int j = 0;
#pragma unroll 1
        for (; j + 2 < STEPS; j += 2) {
            wload(j + 1, wb, ob);
            step(wa, oa, true);
            wload(j + 2, wa, oa);
            step(wb, ob, true);
        }
        const bool ok_last = (SLOTS % 4 == 0) || 4 * (STEPS - 1) + q < SLOTS;
        if (j + 1 < STEPS) {
            wload(j + 1, wb, ob);
            step(wa, oa, true);
            step(wb, ob, ok_last);
        } else {
            step(wa, oa, ok_last);
        }
        if (nc0 == 0) {
            __syncthreads();                   // the halo is free
            int bb = br;
            const int x0 = (bb % nxb) * 16; bb /= nxb;
            const int y0 = (bb % nyb) * kBY; bb /= nyb;
            const int z0 = (bb % nzb) * kBZ;
            const int64_t bn = bb / nzb;
            f32x4 out[ROWS][1];
#pragma unroll
            for (int t = 0; t < ROWS; ++t) out[t][0] = acc[t];
            store_tiles<ROWS, 1>(out, s_in, wid, lane, bn, z0, y0, x0, V,
                                 cb0, bias, relu, mask, y, Cout, yp, hd, &bv);
        }
        if (!more) break;
        br = nb2;
        c0 = nc0;
    }
}

// The first layer: of the 16 padded input channels only the first two
// (dose, density) are non-zero, so the reduction runs over 27 offsets x 2
// channels, padded to 64 (two matrix instructions) instead of 27 x 16.
// Slot k holds offset k / 2, channel k % 2; a lane's 8 slots are 4 offsets
// with both channels, i.e. 4 32-bit halo words.  16 output channels; same
// bricks as k_conv3_bk, the halo staged as one 32-bit word per voxel.
// DIRECT: the words are made here from the fp32 dose (times the sample's
// scale) and density, rounded exactly as k_pack_input rounds them, so the
// padded input need not be written at all (inference); otherwise they are
// read from the padded input x.  Each block walks bricks as k_conv3_bk16p
// does (the blocks of one XCD on one contiguous share of them), with the
// next brick's halo loaded into registers while the current one computes.
template <bool DIRECT>
__global__ void __launch_bounds__(256)
k_conv3_first(const bf16_t *__restrict__ x, const float *__restrict__ dose,
              const float *__restrict__ rho, const float *__restrict__ scale,
              Vol V, int Cin, const bf16_t *__restrict__ W, int Kp,
              const float *__restrict__ bias, bf16_t *__restrict__ y) {
    constexpr int HZ = kBZ + 2, HY = kBY + 2, HX = 18;
    constexpr int HVOX = HZ * HY * HX;
    constexpr int ROWS = kBZ * kBY / 4;
    constexpr int C = 16, KS = 64;
    __shared__ uint32_t s_in[HVOX];
    __shared__ __attribute__((aligned(16))) bf16_t s_w[C * KS];
    __shared__ __attribute__((aligned(16))) bf16_t s_out[4 * ROWS * 16 * 24];
    const int lane = __lane_id(), wid = threadIdx.x >> 6;
    const int nxb = V.w / 16, nyb = V.h / kBY, nzb = V.d / kBZ;
    const int nbr = nxb * nyb * nzb * V.n;     // < 2^31 (grid limit)
    int br = blockIdx.x, br_end = nbr, br_step = gridDim.x;
    if (nbr > (int)gridDim.x && gridDim.x >= 8) {
        const int k = blockIdx.x & 7, per = (nbr + 7) / 8;
        br = k * per + (blockIdx.x >> 3);
        br_end = min(nbr, (k + 1) * per);
        br_step = ((int)gridDim.x - k + 7) / 8;
    }
    if (br >= br_end) return;
    const int q = lane >> 4, vx = lane & 15;
    for (int i = threadIdx.x; i < C * KS; i += 256) {
        const int co = i / KS, k = i % KS;
        s_w[i] = k < 54 ? W[(int64_t)co * Kp + (k >> 1) * Cin + (k & 1)]
                        : (bf16_t)0;
    }
    constexpr int NIT = (HVOX + 255) / 256;
    // the prefetched halo as loaded (DIRECT: dose and density, rounded
    // when staged, so that no conversion waits for the loads in flight)
    uint32_t hval[NIT];
    float hdose[NIT], hrho[NIT], hsc = 0.0f;
    auto fetch = [&](int bb) {
        const int bx = bb % nxb; bb /= nxb;
        const int by = bb % nyb; bb /= nyb;
        const int bz = bb % nzb;
        const int64_t bn = bb / nzb;
        const int x0 = bx * 16, y0 = by * kBY, z0 = bz * kBZ;
        if (DIRECT) hsc = scale[bn];
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int i = threadIdx.x + 256 * it;
            const int hx = i % HX, hy = (i / HX) % HY, hz = i / (HX * HY);
            const int zz = z0 + hz - 1, yy = y0 + hy - 1, xx = x0 + hx - 1;
            hval[it] = 0u;
            hdose[it] = 0.0f;
            hrho[it] = 0.0f;
            if (i < HVOX && (unsigned)zz < (unsigned)V.d &&
                (unsigned)yy < (unsigned)V.h && (unsigned)xx < (unsigned)V.w) {
                const int64_t v = ((bn * V.d + zz) * V.h + yy) * V.w + xx;
                if (DIRECT) {
                    hdose[it] = dose[v];
                    hrho[it] = rho[v];
                } else {
                    hval[it] =
                        *reinterpret_cast<const uint32_t *>(x + v * Cin);
                }
            }
        }
    };
    fetch(br);
    for (;;) {
        __syncthreads();   // the last brick's reads of s_in are done
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int i = threadIdx.x + 256 * it;
            if (i < HVOX)
                s_in[i] = DIRECT ? (uint32_t)f2bf(hdose[it] * hsc) |
                                       ((uint32_t)f2bf(hrho[it]) << 16)
                                 : hval[it];
        }
        __syncthreads();
        const int nb2 = br + br_step;
        const bool more = nb2 < br_end;
        if (more) fetch(nb2);                  // in flight during the steps
        f32x4 acc[ROWS][1];
#pragma unroll
        for (int t = 0; t < ROWS; ++t) acc[t][0] = f32x4{0, 0, 0, 0};
#pragma unroll
        for (int st = 0; st < 2; ++st) {
            const bf16x8 wv = *reinterpret_cast<const bf16x8 *>(
                s_w + vx * KS + 32 * st + 8 * q);
#pragma unroll
            for (int t = 0; t < ROWS; ++t) {
                const int row = wid * ROWS + t;
                const int rz = row / kBY, ry = row % kBY;
                uint32_t w4[4];
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const int o = 16 * st + 4 * q + jj;
                    const int oc = o < 27 ? o : 0;
                    const int dz = oc / 9, dy = (oc / 3) % 3, dx = oc % 3;
                    const uint32_t v =
                        s_in[((rz + dz) * HY + (ry + dy)) * HX + (vx + dx)];
                    w4[jj] = o < 27 ? v : 0u;
                }
                const bf16x8 a = __builtin_bit_cast(
                    bf16x8, make_uint4(w4[0], w4[1], w4[2], w4[3]));
                acc[t][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    a, wv, acc[t][0], 0, 0, 0);
            }
        }
        int bb = br;
        const int x0 = (bb % nxb) * 16; bb /= nxb;
        const int y0 = (bb % nyb) * kBY; bb /= nyb;
        const int z0 = (bb % nzb) * kBZ;
        const int64_t bn = bb / nzb;
        store_tiles<ROWS, 1>(acc, s_out, wid, lane, bn, z0, y0, x0, V, 0,
                             bias, 1, nullptr, y, C);
        if (!more) break;
        br = nb2;
    }
}

// W'[ci][o'][co] = W[co][26 - o'][ci]: the weights of the transposed
// convolution (data gradient), padded to Kp2 = roundup(27 Cout, 32).
__global__ void k_flip_weights(const bf16_t *__restrict__ W, int Cin,
                               int Cout, int Kp, bf16_t *__restrict__ Wt,
                               int Kp2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)Cin * Kp2) return;
    const int ci = (int)(i / Kp2), k = (int)(i % Kp2);
    bf16_t v = 0;
    if (k < 27 * Cout) {
        const int o2 = k / Cout, co = k % Cout;
        v = W[(int64_t)co * Kp + (26 - o2) * Cin + ci];
    }
    Wt[i] = v;
}

// dW[co][o][ci] += sum over a voxel chunk of dy[v][co] x[v + o][ci].  One
// block per (offset, voxel chunk).  32 voxels at a time are staged in LDS
// transposed (channel-major, 16-byte global loads), so that each lane reads
// its 8 consecutive voxels of one channel -- an MFMA operand -- with one
// 16-byte LDS read; the neighbour index of each voxel is computed once.
// Each wave owns up to 16 of the (Cout/16) x (Cin/16) output tiles; the
// partial sums go out with one fp32 atomic per weight per block.
constexpr int kWgVox = 32;
constexpr int kWgPitch = kWgVox + 8;   // LDS row pitch (elements)

// The 8 bf16 values packed in q (channel c8 + j in bits 16 j of the 128)
// written down a column of a row-pitch-kWgPitch LDS tile.  The halves are
// split with 32-bit shifts: extracting elements of a bf16 vector type was
// lowered incorrectly by this toolchain (every element read as element 0).
__device__ __forceinline__ void put8_transposed(bf16_t *col, uint4 q) {
    const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        col[(2 * m) * kWgPitch] = (bf16_t)(w[m] & 0xffffu);
        col[(2 * m + 1) * kWgPitch] = (bf16_t)(w[m] >> 16);
    }
}
__global__ void __launch_bounds__(256)
k_conv3_wgrad(const bf16_t *__restrict__ x, Vol V, int Cin,
              const bf16_t *__restrict__ dy, int Cout, int64_t chunk,
              float *__restrict__ dW, int Kp) {
    __shared__ __attribute__((aligned(16))) bf16_t s_dy[kMaxCout * kWgPitch];
    __shared__ __attribute__((aligned(16))) bf16_t s_x[2 * kMaxCout * kWgPitch];
    __shared__ int64_t s_nb[kWgVox];
    const int o = blockIdx.y;
    const int lane = __lane_id(), wid = threadIdx.x >> 6;
    const int dz = o / 9 - 1, dyo = (o / 3) % 3 - 1, dx = o % 3 - 1;
    const int64_t nvox = V.voxels();
    const int64_t v0 = (int64_t)blockIdx.x * chunk;
    const int64_t v1 = v0 + chunk < nvox ? v0 + chunk : nvox;
    const int mt = Cout / 16, nt = Cin / 16;
    const int n_tiles = mt * nt;
    const int gy = Cout / 8, gx = Cin / 8;   // 16-byte groups per voxel
    f32x4 acc[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) acc[t] = f32x4{0, 0, 0, 0};
    for (int64_t vb = v0; vb < v1; vb += kWgVox) {
        __syncthreads();
        if (threadIdx.x < kWgVox) {
            const int64_t v = vb + threadIdx.x;
            int64_t nb = -1;
            if (v < v1) {
                int64_t t = v;
                const int w = (int)(t % V.w); t /= V.w;
                const int h = (int)(t % V.h); t /= V.h;
                const int d = (int)(t % V.d);
                const int64_t n = t / V.d;
                const int zz = d + dz, yy = h + dyo, xx = w + dx;
                if ((unsigned)zz < (unsigned)V.d &&
                    (unsigned)yy < (unsigned)V.h &&
                    (unsigned)xx < (unsigned)V.w)
                    nb = ((n * V.d + zz) * V.h + yy) * V.w + xx;
            }
            s_nb[threadIdx.x] = nb;
        }
        // dy rows of the 32 voxels (contiguous in memory), transposed
        // (consecutive threads take consecutive voxels: the transposed LDS
        // writes of a wave then fall on consecutive addresses)
        for (int i = threadIdx.x; i < kWgVox * gy; i += 256) {
            const int vi = i % kWgVox, c8 = (i / kWgVox) * 8;
            const int64_t v = vb + vi;
            uint4 q = make_uint4(0, 0, 0, 0);
            if (v < v1) q = *reinterpret_cast<const uint4 *>(dy + v * Cout + c8);
            put8_transposed(s_dy + c8 * kWgPitch + vi, q);
        }
        __syncthreads();
        // shifted x rows, transposed
        for (int i = threadIdx.x; i < kWgVox * gx; i += 256) {
            const int vi = i % kWgVox, c8 = (i / kWgVox) * 8;
            const int64_t nb = s_nb[vi];
            uint4 q = make_uint4(0, 0, 0, 0);
            if (nb >= 0) q = *reinterpret_cast<const uint4 *>(x + nb * Cin + c8);
            put8_transposed(s_x + c8 * kWgPitch + vi, q);
        }
        __syncthreads();
        // A[i = co][k = voxel], B[k = voxel][j = ci]
        const int kk = 8 * (lane >> 4);
#pragma unroll
        for (int slot = 0; slot < 16; ++slot) {
            const int t = wid + 4 * slot;
            if (t >= n_tiles) break;
            const int cb = t / nt, ib = t % nt;
            const int co = cb * 16 + (lane & 15);
            const int ci = ib * 16 + (lane & 15);
            const bf16x8 a =
                *reinterpret_cast<const bf16x8 *>(&s_dy[co * kWgPitch + kk]);
            const bf16x8 b =
                *reinterpret_cast<const bf16x8 *>(&s_x[ci * kWgPitch + kk]);
            acc[slot] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                a, b, acc[slot], 0, 0, 0);
        }
    }
    // acc[slot][r] is (co = 16 cb + 4 (lane/16) + r, ci = 16 ib + lane%16)
#pragma unroll
    for (int slot = 0; slot < 16; ++slot) {
        const int t = wid + 4 * slot;
        if (t >= n_tiles) break;
        const int cb = t / nt, ib = t % nt;
        const int ci = ib * 16 + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int co = cb * 16 + 4 * (lane >> 4) + r;
            unsafeAtomicAdd(&dW[(int64_t)co * Kp + o * Cin + ci],
                            acc[slot][r]);
        }
    }
}

// The weight gradient on LDS-staged bricks.  A block runs over bricks of
// 16 x kBY x kBZ voxels (grid-stride over blockIdx.x) for one chunk of 16
// input channels (blockIdx.y) and 16 MTP output channels (blockIdx.z).  Per
// brick, dy is staged transposed (channel rows of the brick's 256 voxels)
// and x likewise, one x-shift dx at a time ((kBZ+2) x (kBY+2) rows of 16
// voxels, zero outside the volume), so that the 8 consecutive voxels of an
// MFMA operand are one aligned 16-byte LDS read for every offset.  The
// transposes pair two channels per 32-bit load.  The reduction dimension
// of the matrix instruction is the voxel: K step s covers brick rows 2s and
// 2s + 1.  Wave w accumulates all 27 offsets of output tile w % MTP over
// the K steps congruent to w / MTP; the waves of a tile are summed through
// LDS at the end and the block writes its partial sums (no atomics) to
// part[blockIdx.x][o][co][ci], which k_wgrad_reduce adds into dW in a fixed
// order.
constexpr int kWgDyPitch = 16 * kBY * kBZ + 8;          // 264
constexpr int kWgXRows = (kBZ + 2) * (kBY + 2);          // 36
constexpr int kWgXPitch = kWgXRows * 16 + 8;             // 584
constexpr int64_t kWgPartFloats = int64_t(8) << 20;      // 32 MB
// One byte permute per output word: 0x05040100 takes the low halves of
// (p[2m], p[2m+1]), 0x07060302 the high halves.
__device__ __forceinline__ void put_pair_rows(bf16_t *row0, bf16_t *row1,
                                              const uint32_t p[8]) {
    uint4 lo, hi;
    lo.x = __builtin_amdgcn_perm(p[1], p[0], 0x05040100u);
    lo.y = __builtin_amdgcn_perm(p[3], p[2], 0x05040100u);
    lo.z = __builtin_amdgcn_perm(p[5], p[4], 0x05040100u);
    lo.w = __builtin_amdgcn_perm(p[7], p[6], 0x05040100u);
    hi.x = __builtin_amdgcn_perm(p[1], p[0], 0x07060302u);
    hi.y = __builtin_amdgcn_perm(p[3], p[2], 0x07060302u);
    hi.z = __builtin_amdgcn_perm(p[5], p[4], 0x07060302u);
    hi.w = __builtin_amdgcn_perm(p[7], p[6], 0x07060302u);
    *reinterpret_cast<uint4 *>(row0) = lo;
    *reinterpret_cast<uint4 *>(row1) = hi;
}
template <int MTP>
__global__ void __launch_bounds__(256)
k_conv3_wgrad_bk(const bf16_t *__restrict__ x, Vol V, int Cin,
                 const bf16_t *__restrict__ dy, int Cout,
                 float *__restrict__ part) {
    constexpr int NKG = 4 / MTP;               // waves per output tile
    constexpr int NKS = 8 / NKG;               // K steps per wave and brick
    __shared__ __attribute__((aligned(16))) bf16_t s_dy[16 * MTP * kWgDyPitch];
    __shared__ __attribute__((aligned(16))) bf16_t s_x[16 * kWgXPitch];
    __shared__ __attribute__((aligned(16))) f32x4 s_red[(NKG - 1) * MTP * 64 + 1];
    const int lane = __lane_id(), wid = threadIdx.x >> 6;
    const int tw = wid % MTP, kg = wid / MTP;
    const int q = lane >> 4, l16 = lane & 15;
    const int ci0 = blockIdx.y * 16, co0 = blockIdx.z * 16 * MTP;
    const int nxb = V.w / 16, nyb = V.h / kBY, nzb = V.d / kBZ;
    const int64_t bricks = (int64_t)V.n * nzb * nyb * nxb;
    f32x4 acc[27];
#pragma unroll
    for (int o = 0; o < 27; ++o) acc[o] = f32x4{0, 0, 0, 0};
    for (int64_t br = blockIdx.x; br < bricks; br += gridDim.x) {
        int64_t b = br;
        const int bx = (int)(b % nxb); b /= nxb;
        const int by = (int)(b % nyb); b /= nyb;
        const int bz = (int)(b % nzb);
        const int64_t bn = b / nzb;
        const int x0 = bx * 16, y0 = by * kBY, z0 = bz * kBZ;
        __syncthreads();                       // the last brick's reads
        // dy, transposed: item = (voxel octet, channel pair); MTP items
        // per thread, all loads issued before the LDS stores
        uint32_t pd[MTP][8];
#pragma unroll
        for (int it = 0; it < MTP; ++it) {
            const int i = threadIdx.x + 256 * it;
            const int cp = i % (8 * MTP), oc = i / (8 * MTP);
            const int row = oc >> 1, xo = 8 * (oc & 1);
            const int rz = row / kBY, ry = row % kBY;
            const int64_t v =
                ((bn * V.d + z0 + rz) * V.h + (y0 + ry)) * V.w + x0 + xo;
            const bf16_t *src = dy + v * Cout + co0 + 2 * cp;
#pragma unroll
            for (int j = 0; j < 8; ++j)
                pd[it][j] = *reinterpret_cast<const uint32_t *>(src + j * Cout);
        }
#pragma unroll
        for (int it = 0; it < MTP; ++it) {
            const int i = threadIdx.x + 256 * it;
            const int cp = i % (8 * MTP), oc = i / (8 * MTP);
            const int row = oc >> 1, xo = 8 * (oc & 1);
            put_pair_rows(s_dy + (2 * cp) * kWgDyPitch + row * 16 + xo,
                          s_dy + (2 * cp + 1) * kWgDyPitch + row * 16 + xo,
                          pd[it]);
        }
        __syncthreads();
        bf16x8 a[NKS];
#pragma unroll
        for (int m = 0; m < NKS; ++m) {
            const int st = kg + NKG * m;
            const int row = 2 * st + (q >> 1), xo = 8 * (q & 1);
            a[m] = *reinterpret_cast<const bf16x8 *>(
                s_dy + (tw * 16 + l16) * kWgDyPitch + row * 16 + xo);
        }
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
            if (dx) __syncthreads();           // the last shift's reads
            // x shifted by dx - 1, transposed: item = (row octet, pair);
            // all of a thread's loads are issued before its LDS stores
            // item i = threadIdx.x + 256 it: channel pair i % 8, octet
            // (i / 8) % 2, halo row i / 16 (the first two do not depend on
            // it)
            constexpr int NXI = 8 * kWgXRows * 2, NIT = (NXI + 255) / 256;
            const int cp = threadIdx.x % 8, oct = (threadIdx.x / 8) & 1;
            const int xb = x0 + 8 * oct + dx - 1;
            uint32_t px[NIT][8];
#pragma unroll
            for (int it = 0; it < NIT; ++it) {
                const int hr = threadIdx.x / 16 + 16 * it;
                const int hz = hr / (kBY + 2), hy = hr % (kBY + 2);
                const int zz = z0 + hz - 1, yy = y0 + hy - 1;
                const bool zy = hr < kWgXRows &&
                                (unsigned)zz < (unsigned)V.d &&
                                (unsigned)yy < (unsigned)V.h;
                const int64_t vrow = ((bn * V.d + zz) * V.h + yy) * V.w;
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int xx = xb + j;
                    px[it][j] = 0u;
                    if (zy && (unsigned)xx < (unsigned)V.w)
                        px[it][j] = *reinterpret_cast<const uint32_t *>(
                            x + (vrow + xx) * Cin + ci0 + 2 * cp);
                }
            }
#pragma unroll
            for (int it = 0; it < NIT; ++it) {
                const int hr = threadIdx.x / 16 + 16 * it;
                if (hr < kWgXRows)
                    put_pair_rows(
                        s_x + (2 * cp) * kWgXPitch + hr * 16 + 8 * oct,
                        s_x + (2 * cp + 1) * kWgXPitch + hr * 16 + 8 * oct,
                        px[it]);
            }
            __syncthreads();
#pragma unroll
            for (int dz = 0; dz < 3; ++dz)
#pragma unroll
                for (int dyo = 0; dyo < 3; ++dyo) {
                    const int o = dz * 9 + dyo * 3 + dx;
#pragma unroll
                    for (int m = 0; m < NKS; ++m) {
                        const int st = kg + NKG * m;
                        const int row = 2 * st + (q >> 1), xo = 8 * (q & 1);
                        const int rz = row / kBY, ry = row % kBY;
                        const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(
                            s_x + l16 * kWgXPitch +
                            ((rz + dz) * (kBY + 2) + (ry + dyo)) * 16 + xo);
                        acc[o] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            a[m], bv, acc[o], 0, 0, 0);
                    }
                }
        }
    }
    // sum the waves of each tile, then write this block's partial sums:
    // acc[o][r] is (co = 16 tw + 4 (lane/16) + r, ci = lane % 16)
    float *dst = part + (int64_t)blockIdx.x * 27 * Cout * Cin;
#pragma unroll
    for (int o = 0; o < 27; ++o) {
        if (NKG > 1) {
            __syncthreads();
            if (kg > 0) s_red[((kg - 1) * MTP + tw) * 64 + lane] = acc[o];
            __syncthreads();
            if (kg == 0)
                for (int g = 1; g < NKG; ++g) {
                    const f32x4 t = s_red[((g - 1) * MTP + tw) * 64 + lane];
                    acc[o] += t;
                }
        }
        if (kg == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int co = co0 + tw * 16 + 4 * q + r;
                dst[((int64_t)o * Cout + co) * Cin + ci0 + l16] = acc[o][r];
            }
        }
    }
}

// dW[co][o Cin + ci] += sum over b < nb of part[b][o][co][ci].  A block
// takes 16 entries; its 16 thread groups sum the partials b = g mod 16,
// eight at a time into independent sums (so that eight loads are in flight),
// and the groups are added in order: a fixed order for a given nb.
__global__ void __launch_bounds__(256)
k_wgrad_reduce(const float *__restrict__ part, int nb, int Cout, int Cin,
               float *__restrict__ dW, int Kp) {
    __shared__ float s_sum[16][17];
    const int64_t slab = (int64_t)27 * Cout * Cin;
    const int e = threadIdx.x & 15, g = threadIdx.x >> 4;
    const int64_t i = (int64_t)blockIdx.x * 16 + e;
    float acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (i < slab) {
        int b = g;
        for (; b + 16 * 7 < nb; b += 16 * 8)
#pragma unroll
            for (int k = 0; k < 8; ++k)
                acc[k] += part[(int64_t)(b + 16 * k) * slab + i];
        for (; b < nb; b += 16) acc[0] += part[(int64_t)b * slab + i];
    }
    s_sum[g][e] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) +
                  ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    __syncthreads();
    if (g == 0 && i < slab) {
        float t = 0.0f;
        for (int k = 0; k < 16; ++k) t += s_sum[k][e];
        const int ci = (int)(i % Cin);
        const int co = (int)((i / Cin) % Cout);
        const int o = (int)(i / ((int64_t)Cin * Cout));
        dW[(int64_t)co * Kp + o * Cin + ci] += t;
    }
}

// dbias[co] += sum_v dy[v][co].  A thread sums 8 channels (one 16-byte
// load per voxel) over a strided set of voxels; the block adds its rows in
// LDS and issues one atomic per channel.
__global__ void __launch_bounds__(256)
k_bias_grad(const bf16_t *__restrict__ dy, int64_t nvox, int C,
            float *__restrict__ db) {
    __shared__ float s[256 * 8];
    const int groups = C / 8;
    const int rows = 256 / groups;
    const int cg = threadIdx.x % groups, r0 = threadIdx.x / groups;
    float acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (r0 < rows)
        for (int64_t v = (int64_t)blockIdx.x * rows + r0; v < nvox;
             v += (int64_t)gridDim.x * rows) {
            const uint4 q =
                *reinterpret_cast<const uint4 *>(dy + v * C + cg * 8);
            const uint32_t w4[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                acc[2 * m] += __uint_as_float(w4[m] << 16);
                acc[2 * m + 1] += __uint_as_float(w4[m] & 0xffff0000u);
            }
        }
#pragma unroll
    for (int k = 0; k < 8; ++k) s[threadIdx.x * 8 + k] = acc[k];
    __syncthreads();
    if (threadIdx.x < C) {
        const int c = threadIdx.x, g = c / 8, k = c % 8;
        float t = 0.0f;
        for (int r = 0; r < rows; ++r) t += s[(r * groups + g) * 8 + k];
        unsafeAtomicAdd(&db[c], t);
    }
}

// ------------------------------------------------------ pooling and such --
// average of 2x2x2 children
__global__ void k_pool(const bf16_t *__restrict__ x, Vol V, int C,
                       bf16_t *__restrict__ y) {
    const Vol U{V.n, V.d / 2, V.h / 2, V.w / 2};
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= U.voxels() * C) return;
    const int c = (int)(i % C);
    int64_t t = i / C;
    const int w = (int)(t % U.w); t /= U.w;
    const int h = (int)(t % U.h); t /= U.h;
    const int d = (int)(t % U.d);
    const int64_t n = t / U.d;
    float s = 0.0f;
    for (int a = 0; a < 8; ++a) {
        const int zz = 2 * d + (a >> 2), yy = 2 * h + ((a >> 1) & 1),
                  xx = 2 * w + (a & 1);
        s += bf2f(x[(((n * V.d + zz) * V.h + yy) * V.w + xx) * C + c]);
    }
    y[i] = f2bf(0.125f * s);
}

// gradient of the average pool: each child gets dy / 8
__global__ void k_pool_back(const bf16_t *__restrict__ dy, Vol V, int C,
                            bf16_t *__restrict__ dx) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= V.voxels() * C) return;
    const int c = (int)(i % C);
    int64_t t = i / C;
    const int w = (int)(t % V.w); t /= V.w;
    const int h = (int)(t % V.h); t /= V.h;
    const int d = (int)(t % V.d);
    const int64_t n = t / V.d;
    const Vol U{V.n, V.d / 2, V.h / 2, V.w / 2};
    const int64_t u = ((n * U.d + d / 2) * U.h + h / 2) * U.w + w / 2;
    dx[i] = f2bf(0.125f * bf2f(dy[u * C + c]));
}

// out = concat(nearest-upsampled a [coarse, Ca], b [fine, Cb]) on the fine
// grid V
// One thread per voxel and 8-channel group (16 bytes); Ca, Cb multiples
// of 8.
__global__ void k_up_concat(const bf16_t *__restrict__ a, int Ca,
                            const bf16_t *__restrict__ b, int Cb, Vol V,
                            bf16_t *__restrict__ out) {
    const int G = (Ca + Cb) / 8;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= V.voxels() * G) return;
    const int g = (int)(i % G);
    const int64_t v = i / G;
    uint4 val;
    if (g * 8 >= Ca) {
        val = *reinterpret_cast<const uint4 *>(b + v * Cb + (g * 8 - Ca));
    } else {
        int64_t t = v;
        const int w = (int)(t % V.w); t /= V.w;
        const int h = (int)(t % V.h); t /= V.h;
        const int d = (int)(t % V.d);
        const int64_t n = t / V.d;
        const Vol U{V.n, V.d / 2, V.h / 2, V.w / 2};
        const int64_t u = ((n * U.d + d / 2) * U.h + h / 2) * U.w + w / 2;
        val = *reinterpret_cast<const uint4 *>(a + u * Ca + g * 8);
    }
    *reinterpret_cast<uint4 *>(out + v * (Ca + Cb) + g * 8) = val;
}

// split the gradient of concat: the up-sampling part summed over the 8
// children into da (coarse), the skip part added into db (fine, times the
// ReLU mask of the skip activation)
__global__ void k_up_concat_back_a(const bf16_t *__restrict__ g, int Ca,
                                   int Cb, Vol V, const bf16_t *__restrict__ am,
                                   bf16_t *__restrict__ da) {
    const Vol U{V.n, V.d / 2, V.h / 2, V.w / 2};
    const int C = Ca + Cb;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= U.voxels() * Ca) return;
    const int c = (int)(i % Ca);
    int64_t t = i / Ca;
    const int w = (int)(t % U.w); t /= U.w;
    const int h = (int)(t % U.h); t /= U.h;
    const int d = (int)(t % U.d);
    const int64_t n = t / U.d;
    float s = 0.0f;
    for (int k = 0; k < 8; ++k) {
        const int zz = 2 * d + (k >> 2), yy = 2 * h + ((k >> 1) & 1),
                  xx = 2 * w + (k & 1);
        s += bf2f(g[((((n * V.d + zz) * V.h + yy) * V.w + xx)) * C + c]);
    }
    if (am && !(bf2f(am[i]) > 0.0f)) s = 0.0f;
    da[i] = f2bf(s);
}

__global__ void k_up_concat_back_b(const bf16_t *__restrict__ g, int Ca,
                                   int Cb, Vol V, bf16_t *__restrict__ db) {
    const int C = Ca + Cb;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= V.voxels() * Cb) return;
    const int c = (int)(i % Cb);
    const int64_t v = i / Cb;
    db[i] = g[v * C + Ca + c];
}

// out = (a + b) * (mask > 0)
__global__ void k_add_mask(const bf16_t *__restrict__ a,
                           const bf16_t *__restrict__ b,
                           const bf16_t *__restrict__ mask, int64_t n,
                           bf16_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float s = bf2f(a[i]) + (b ? bf2f(b[i]) : 0.0f);
    out[i] = f2bf(bf2f(mask[i]) > 0.0f ? s : 0.0f);
}

constexpr int kInC = 16;   // input channels: dose, density, 14 zeros

// per-sample normalisation: scale[n] = 1 / max(dose of sample n), or 1 when
// that maximum is not positive.  kMaxBlocks blocks per sample each reduce a
// slice and merge with an integer atomicMax on the bits of max(m, 0): for
// non-negative floats the bit patterns order like the values.
constexpr int kMaxBlocks = 256;
__global__ void __launch_bounds__(256)
k_sample_max(const float *__restrict__ dose, int64_t per_sample,
             unsigned int *__restrict__ mbits) {
    __shared__ float s[256];
    const float *d = dose + (int64_t)blockIdx.y * per_sample;
    // four independent maxima, so that four loads are in flight (the
    // maximum does not depend on the order)
    const int64_t stride = (int64_t)gridDim.x * 256;
    float m0 = 0.0f, m1 = 0.0f, m2 = 0.0f, m3 = 0.0f;
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    for (; i + 3 * stride < per_sample; i += 4 * stride) {
        m0 = fmaxf(m0, d[i]);
        m1 = fmaxf(m1, d[i + stride]);
        m2 = fmaxf(m2, d[i + 2 * stride]);
        m3 = fmaxf(m3, d[i + 3 * stride]);
    }
    for (; i < per_sample; i += stride) m0 = fmaxf(m0, d[i]);
    s[threadIdx.x] = fmaxf(fmaxf(m0, m1), fmaxf(m2, m3));
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) s[threadIdx.x] = fmaxf(s[threadIdx.x],
                                                    s[threadIdx.x + h]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(&mbits[blockIdx.y], __float_as_uint(s[0]));
}

__global__ void k_scale_from_max(const unsigned int *__restrict__ mbits,
                                 int n, float *__restrict__ scale) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float m = __uint_as_float(mbits[i]);
    scale[i] = m > 0.0f ? 1.0f / m : 1.0f;
}

__global__ void k_fill_u32(unsigned int *p, int64_t n, unsigned int v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// input tensor: channels (dose * scale, density, 0 ...)
// One thread per voxel: its 16 channels as two 16-byte stores.
__global__ void k_pack_input(const float *__restrict__ dose,
                             const float *__restrict__ rho, int64_t nvox,
                             int64_t per_sample, const float *__restrict__ scale,
                             bf16_t *__restrict__ x) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nvox) return;
    const uint32_t d = f2bf(dose[v] * scale[v / per_sample]);
    const uint32_t r = f2bf(rho[v]);
    uint4 *o = reinterpret_cast<uint4 *>(x + v * kInC);
    o[0] = make_uint4(d | (r << 16), 0u, 0u, 0u);
    o[1] = make_uint4(0u, 0u, 0u, 0u);
}

// out[v] = dose[v] * scale + sum_c f[v][c] wh[c] + bh  (normalised units)
__global__ void k_head(const bf16_t *__restrict__ f, int C,
                       const float *__restrict__ wh, const float *__restrict__ bh,
                       const float *__restrict__ dose, int64_t per_sample,
                       const float *__restrict__ scale, int64_t nvox,
                       float *__restrict__ out) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nvox) return;
    float s = bh[0];
    // 16-byte loads; bf16 halves split by shifts
    const uint4 *fv = reinterpret_cast<const uint4 *>(f + v * C);
    for (int g = 0; g < C / 8; ++g) {
        const uint4 q = fv[g];
        const uint32_t w4[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            s += __uint_as_float(w4[m] << 16) * wh[8 * g + 2 * m];
            s += __uint_as_float(w4[m] & 0xffff0000u) * wh[8 * g + 2 * m + 1];
        }
    }
    out[v] = dose[v] * scale[v / per_sample] + s;
}

// loss = mean over voxels of (out - target * scale)^2; g = dL/dout; head
// gradients; df = g wh masked by the ReLU of f.  Each block writes its sums
// of the squared error, of g and of g f[c] (kLossParts values) to
// part[blockIdx.x]; k_loss_head_sum adds them up in block order.
constexpr int kLossParts = 18;
constexpr int kLossBlocks = 1024;
__global__ void __launch_bounds__(256)
k_loss_head_back(const float *__restrict__ out, const float *__restrict__ tgt,
                 int64_t per_sample, const float *__restrict__ scale,
                 int64_t nvox, const bf16_t *__restrict__ f,
                 const float *__restrict__ wh, bf16_t *__restrict__ df,
                 float *__restrict__ part) {
    constexpr int C = 16;
    __shared__ float s_r[4][kLossParts];
    const float inv_n = 1.0f / (float)nvox;
    float l = 0.0f, gb = 0.0f;
    float gw[C];
#pragma unroll
    for (int c = 0; c < C; ++c) gw[c] = 0.0f;
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < nvox;
         v += (int64_t)gridDim.x * 256) {
        const float e = out[v] - tgt[v] * scale[v / per_sample];
        l += e * e;
        const float g = 2.0f * e * inv_n;
        gb += g;
        // the 16 channels as two 16-byte loads and stores (bf16 halves
        // split by shifts)
        const uint4 *fv4 = reinterpret_cast<const uint4 *>(f + v * C);
        uint4 *dv4 = reinterpret_cast<uint4 *>(df + v * C);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint4 q4 = fv4[h];
            const uint32_t w4[4] = {q4.x, q4.y, q4.z, q4.w};
            uint32_t o4[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int c = 8 * h + 2 * m;
                const float f0 = __uint_as_float(w4[m] << 16);
                const float f1 = __uint_as_float(w4[m] & 0xffff0000u);
                gw[c] += g * f0;
                gw[c + 1] += g * f1;
                o4[m] = (uint32_t)f2bf(f0 > 0.0f ? g * wh[c] : 0.0f) |
                        ((uint32_t)f2bf(f1 > 0.0f ? g * wh[c + 1] : 0.0f)
                         << 16);
            }
            dv4[h] = make_uint4(o4[0], o4[1], o4[2], o4[3]);
        }
    }
    // block sums of l, gb and gw[0..15]: wave sums, then the four waves
    float vals[kLossParts];
    vals[0] = l;
    vals[1] = gb;
#pragma unroll
    for (int c = 0; c < C; ++c) vals[2 + c] = gw[c];
    const int lane = __lane_id(), wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kLossParts; ++k) {
        float v = vals[k];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (lane == 0) s_r[wid][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < kLossParts) {
        const int k = threadIdx.x;
        part[(int64_t)blockIdx.x * kLossParts + k] =
            (s_r[0][k] + s_r[1][k]) + (s_r[2][k] + s_r[3][k]);
    }
}

// loss += sum of the blocks' squared errors / nvox; dbh, dwh += their sums.
// One block: thread t takes blocks t, t + 256, ...; the threads' sums are
// then added in a fixed order (wave butterflies, then the four waves).
__global__ void __launch_bounds__(256)
k_loss_head_sum(const float *__restrict__ part, int nblocks, int64_t nvox,
                double *__restrict__ loss, float *__restrict__ dbh,
                float *__restrict__ dwh) {
    __shared__ double s_w[4][kLossParts];
    double t[kLossParts];
#pragma unroll
    for (int k = 0; k < kLossParts; ++k) t[k] = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256)
#pragma unroll
        for (int k = 0; k < kLossParts; ++k)
            t[k] += part[(int64_t)b * kLossParts + k];
    const int lane = __lane_id(), wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kLossParts; ++k) {
        double v = t[k];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (lane == 0) s_w[wid][k] = v;
    }
    __syncthreads();
    const int k = threadIdx.x;
    if (k >= kLossParts) return;
    const double sum = (s_w[0][k] + s_w[1][k]) + (s_w[2][k] + s_w[3][k]);
    if (k == 0) loss[0] += sum / (double)nvox;
    else if (k == 1) dbh[0] += (float)sum;
    else dwh[k - 2] += (float)sum;
}

// de-normalise: y = o / scale of the sample
__global__ void k_out_scale(const float *__restrict__ o, int64_t n,
                            int64_t per_sample, const float *__restrict__ scale,
                            float *__restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = o[i] / scale[i / per_sample];
}

// Adam on the fp32 master parameters, then the bf16 copies of the conv
// weights (layout: per layer W [Cout][Kp] then b [Cout]).
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g,
                       float *__restrict__ m, float *__restrict__ v,
                       int64_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

__global__ void k_to_bf16(const float *__restrict__ p, int64_t n,
                          bf16_t *__restrict__ q) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) q[i] = f2bf(p[i]);
}

__global__ void k_fill_f32(float *p, int64_t n, float v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// He-normal initialisation from a counter-based generator (Philox,
// Box-Muller); biases zero.
__global__ void k_init_layer(float *__restrict__ W, int Cout, int Kp,
                             int K, float stdv, uint64_t seed,
                             uint32_t layer) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)Cout * Kp) return;
    const int k = (int)(i % Kp);
    if (k >= K) {
        W[i] = 0.0f;
        return;
    }
    u32x4 r = philox4x32_10(u32x4{(uint32_t)i, layer, 0x5eedu, 0u},
                            (uint32_t)seed, (uint32_t)(seed >> 32));
    const float u1 = u01(r.x), u2 = u01(r.y);
    W[i] = stdv * sqrtf(-2.0f * __logf(u1)) * __cosf(6.2831853f * u2);
}

}  // namespace
}  // namespace psl

// ============================================================== host side ==
namespace psl {
namespace {

struct ConvL {
    int cin, cout, kp;
    int64_t w_off, b_off;
};

// The fixed architecture: 4 levels of 16/32/64/128 channels.
struct Net {
    std::vector<ConvL> L;
    int64_t head_w = 0, head_b = 0, n_params = 0;
};

enum {
    E0A, E0B, E1A, E1B, E2A, E2B, E3A, E3B, D2A, D2B, D1A, D1B, D0A, D0B,
    N_CONV
};

Net make_net(int base) {
    Net n;
    const int c0 = base, c1 = 2 * base, c2 = 4 * base, c3 = 8 * base;
    const int io[N_CONV][2] = {{kInC, c0}, {c0, c0},      {c0, c1},
                               {c1, c1},   {c1, c2},      {c2, c2},
                               {c2, c3},   {c3, c3},      {c3 + c2, c2},
                               {c2, c2},   {c2 + c1, c1}, {c1, c1},
                               {c1 + c0, c0}, {c0, c0}};
    int64_t off = 0;
    for (int i = 0; i < N_CONV; ++i) {
        ConvL l;
        l.cin = io[i][0];
        l.cout = io[i][1];
        l.kp = (27 * l.cin + 31) / 32 * 32;
        l.w_off = off;
        off += (int64_t)l.cout * l.kp;
        l.b_off = off;
        off += l.cout;
        n.L.push_back(l);
    }
    n.head_w = off;
    off += c0;
    n.head_b = off;
    off += 8;   // keeps the blob a multiple of 8 floats
    n.n_params = off;
    return n;
}

struct Acts {
    Vol V[4];
    bf16_t *xin, *e0a, *e0b, *p1, *e1a, *e1b, *p2, *e2a, *e2b, *p3, *e3a,
        *e3b, *cat2, *d2a, *d2b, *cat1, *d1a, *d1b, *cat0, *d0a, *d0b;
    float *out, *scale;
    unsigned int *maxbits;
    // backward
    bf16_t *gA, *gB, *gC, *sk0, *sk1, *sk2, *wt;
    float *wpart;         // weight-gradient partial sums per block
    float *lpart;         // loss and head-gradient sums per block
    size_t bytes;
};

Acts carve_acts(void *base, int n, int d, int h, int w, int b, bool train) {
    Carver c(base);
    Acts a;
    for (int l = 0; l < 4; ++l) a.V[l] = Vol{n, d >> l, h >> l, w >> l};
    const int64_t v0 = a.V[0].voxels(), v1 = a.V[1].voxels(),
                  v2 = a.V[2].voxels(), v3 = a.V[3].voxels();
    const int c0 = b, c1 = 2 * b, c2 = 4 * b, c3 = 8 * b;
    a.xin = c.take<bf16_t>(v0 * kInC);
    a.e0a = c.take<bf16_t>(v0 * c0);
    a.e0b = c.take<bf16_t>(v0 * c0);
    a.p1 = c.take<bf16_t>(v1 * c0);
    a.e1a = c.take<bf16_t>(v1 * c1);
    a.e1b = c.take<bf16_t>(v1 * c1);
    a.p2 = c.take<bf16_t>(v2 * c1);
    a.e2a = c.take<bf16_t>(v2 * c2);
    a.e2b = c.take<bf16_t>(v2 * c2);
    a.p3 = c.take<bf16_t>(v3 * c2);
    a.e3a = c.take<bf16_t>(v3 * c3);
    a.e3b = c.take<bf16_t>(v3 * c3);
    a.cat2 = c.take<bf16_t>(v2 * (c3 + c2));
    a.d2a = c.take<bf16_t>(v2 * c2);
    a.d2b = c.take<bf16_t>(v2 * c2);
    a.cat1 = c.take<bf16_t>(v1 * (c2 + c1));
    a.d1a = c.take<bf16_t>(v1 * c1);
    a.d1b = c.take<bf16_t>(v1 * c1);
    a.cat0 = c.take<bf16_t>(v0 * (c1 + c0));
    a.d0a = c.take<bf16_t>(v0 * c0);
    a.d0b = c.take<bf16_t>(v0 * c0);
    a.out = c.take<float>(v0);
    a.scale = c.take<float>(n);
    a.maxbits = c.take<unsigned int>(n);
    a.gA = a.gB = a.gC = a.sk0 = a.sk1 = a.sk2 = a.wt = nullptr;
    a.wpart = a.lpart = nullptr;
    if (train) {
        const int64_t big = std::max({v0 * (c1 + c0), v1 * (c2 + c1),
                                      v2 * (c3 + c2)});
        a.gA = c.take<bf16_t>(big);
        a.gB = c.take<bf16_t>(big);
        a.gC = c.take<bf16_t>(big);
        a.sk0 = c.take<bf16_t>(v0 * c0);
        a.sk1 = c.take<bf16_t>(v1 * c1);
        a.sk2 = c.take<bf16_t>(v2 * c2);
        a.wt = c.take<bf16_t>((int64_t)(c3 + c2) * ((27 * c3 + 31) / 32 * 32));
        a.wpart = c.take<float>(kWgPartFloats);
        a.lpart = c.take<float>((int64_t)kLossBlocks * kLossParts);
    }
    a.bytes = c.used;
    return a;
}

unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

template <int NB, int MT>
void launch_conv(const bf16_t *x, Vol V, int cin, const bf16_t *W, int kp,
                 const float *bias, int relu, const bf16_t *mask, int mask_c,
                 bf16_t *y, int cout, hipStream_t st) {
    hipLaunchKernelGGL((k_conv3<NB, MT>),
                       dim3(nblk(V.voxels(), 64 * MT),
                            (unsigned)(cout / (16 * NB))),
                       dim3(256), 0, st, x, V, cin, W, kp, bias, relu, mask,
                       mask_c, y, cout);
}

// Tile shape per layer: the most output channels per wave (reuse of each
// input fragment) that still gives kConvWaves waves, with voxel tiles per
// wave such that the accumulators (4 MT NB registers) stay at 64 or fewer.
// Small volumes (the coarse levels) thus split the output channels across
// waves instead of leaving most of the chip idle.
constexpr int64_t kConvWaves = 2048;

// xc, cc: see k_conv3_bk (brick volumes only; brick_ok tells)
// unet_set_brick_blocks: 0 = as many blocks as are resident at once
std::atomic<int> g_brick_blocks{0};

bool brick_ok(Vol V, int cin) {
    return cin % 16 == 0 && V.w % 16 == 0 && V.h % kBY == 0 &&
           V.d % kBZ == 0;
}

psl_status conv(const bf16_t *x, Vol V, int cin, const bf16_t *W, int kp,
                const float *bias, int relu, const bf16_t *mask, bf16_t *y,
                int cout, hipStream_t st, const bf16_t *xc = nullptr,
                int cc = 0, bf16_t *yp = nullptr,
                HeadArgs hd = HeadArgs{}) {
    if (cout % 16 != 0 || cout > 16 * 12) {
        set_error("unsupported channel count %d", cout);
        return PSL_EINVAL;
    }
    const int nc = cout / 16;
    const int64_t nv = V.voxels();
    // LDS-staged bricks wherever the volume tiles into them: two output
    // channel blocks per wave up to 32 channels (the fine levels, where the
    // volume gives blocks enough), one above (the coarse levels, small
    // volumes: more blocks)
    if ((hd.out && (cout != 16 || mask || yp || !brick_ok(V, cin))) ||
        (yp && (mask || !brick_ok(V, cin))) ||
        (xc && !(brick_ok(V, cin) && cc % (cin % 32 == 0 ? 32 : 16) == 0 &&
                (cin - cc) % (cin % 32 == 0 ? 32 : 16) == 0))) {
        set_error("fused concatenation, pooling or head needs brick "
                  "volumes");
        return PSL_EINVAL;
    }
    if (brick_ok(V, cin)) {
        const unsigned bricks = (unsigned)(nv / (16 * kBY * kBZ));
        const int nbk = (cout == 32) ? 2 : 1;
        const dim3 grid(bricks, (unsigned)(nc / nbk));
#define PSL_CONV_BK(CC, NBV)                                                  \
    hipLaunchKernelGGL((k_conv3_bk<CC, NBV>), grid, dim3(256), 0, st, x, V,  \
                       cin, W, kp, bias, relu, mask, y, cout, xc, cc, yp, \
                       hd)
        if (cin % 32 == 0) {
            if (nbk == 2) PSL_CONV_BK(32, 2);
            else PSL_CONV_BK(32, 1);
        } else if (nbk == 2) {
            PSL_CONV_BK(16, 2);
        } else if (cin != 16) {
            // several chunks: their weights would be staged once per brick
            // and chunk, in series with the steps
            PSL_CONV_BK(16, 1);
        } else {
            // as many blocks as are resident at once, each walking bricks
            static const int per_cu = [] {
                int n = 0;
                if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                        &n, k_conv3_bk16p, 256, 0) != hipSuccess || n < 1)
                    n = 1;
                return n;
            }();
            int64_t cap = (int64_t)per_cu * device_cu_count();
            const int lim = g_brick_blocks.load(std::memory_order_relaxed);
            if (lim > 0) cap = std::min<int64_t>(cap, lim);
            const dim3 g2((unsigned)std::min<int64_t>(bricks, cap), grid.y);
            hipLaunchKernelGGL(k_conv3_bk16p, g2, dim3(256), 0, st, x, V, cin,
                               W, kp, bias, relu, mask, y, cout, xc, cc, yp,
                               hd);
        }
#undef PSL_CONV_BK
        PSL_LAUNCHED();
        return PSL_OK;
    }
    auto waves = [&](int nb, int mt) {
        return (nv + 16 * mt - 1) / (16 * mt) * (nc / nb);
    };
    static const int kNB[] = {12, 8, 6, 4, 3, 2, 1};
    int nb = 1, mt = 1;
    for (int cand : kNB) {
        if (nc % cand) continue;
        const int m = cand <= 4 ? 4 : (cand <= 8 ? 2 : 1);
        if (waves(cand, m) >= kConvWaves) { nb = cand; mt = m; break; }
    }
    if (nb == 1 && waves(1, 4) >= kConvWaves) mt = 4;
    switch (nb * 8 + mt) {
    case 12 * 8 + 1: launch_conv<12, 1>(x, V, cin, W, kp, bias, relu, mask, cout, y, cout, st); break;
    case 8 * 8 + 2: launch_conv<8, 2>(x, V, cin, W, kp, bias, relu, mask, cout, y, cout, st); break;
    case 6 * 8 + 2: launch_conv<6, 2>(x, V, cin, W, kp, bias, relu, mask, cout, y, cout, st); break;
    case 4 * 8 + 4: launch_conv<4, 4>(x, V, cin, W, kp, bias, relu, mask, cout, y, cout, st); break;
    case 3 * 8 + 4: launch_conv<3, 4>(x, V, cin, W, kp, bias, relu, mask, cout, y, cout, st); break;
    case 2 * 8 + 4: launch_conv<2, 4>(x, V, cin, W, kp, bias, relu, mask, cout, y, cout, st); break;
    case 1 * 8 + 4: launch_conv<1, 4>(x, V, cin, W, kp, bias, relu, mask, cout, y, cout, st); break;
    default: launch_conv<1, 1>(x, V, cin, W, kp, bias, relu, mask, cout, y, cout, st); break;
    }
    PSL_LAUNCHED();
    return PSL_OK;
}

struct Ctx {
    Net net;
    const float *p;       // fp32 master
    const bf16_t *pb;     // bf16 copy
    hipStream_t st;
};

// train: the backward pass follows and needs the padded input written
psl_status forward(const Ctx &c, const Acts &a, const float *dose,
                   const float *rho, bool train) {
    psl_status s;
    const auto &L = c.net.L;
    auto W = [&](int i) { return c.pb + L[i].w_off; };
    auto B = [&](int i) { return c.p + L[i].b_off; };
    const Vol *V = a.V;
    const int64_t per = V[0].voxels() / V[0].n;
    hipLaunchKernelGGL(k_fill_u32, dim3(nblk(V[0].n)), dim3(256), 0, c.st,
                       a.maxbits, (int64_t)V[0].n, 0u);
    hipLaunchKernelGGL(k_sample_max,
                       dim3((unsigned)std::min<int64_t>(kMaxBlocks,
                                                        nblk(per)),
                            V[0].n),
                       dim3(256), 0, c.st, dose, per, a.maxbits);
    hipLaunchKernelGGL(k_scale_from_max, dim3(nblk(V[0].n)), dim3(256), 0,
                       c.st, a.maxbits, V[0].n, a.scale);
    const bool first_bk = L[0].cout == 16 && V[0].w % 16 == 0 &&
                          V[0].h % kBY == 0 && V[0].d % kBZ == 0;
    if (train || !first_bk)
        hipLaunchKernelGGL(k_pack_input, dim3(nblk(V[0].voxels())),
                           dim3(256), 0, c.st, dose, rho, V[0].voxels(), per,
                           a.scale, a.xin);
    // encoder
    bf16_t *ins[4] = {a.xin, a.p1, a.p2, a.p3};
    bf16_t *ea[4] = {a.e0a, a.e1a, a.e2a, a.e3a};
    bf16_t *eb[4] = {a.e0b, a.e1b, a.e2b, a.e3b};
    bf16_t *pools[3] = {a.p1, a.p2, a.p3};
    for (int l = 0; l < 4; ++l) {
        const ConvL &la = L[2 * l], &lb = L[2 * l + 1];
        if (l == 0 && first_bk) {
            // the input's two real channels only; as many blocks as are
            // resident at once, each walking bricks
            static const int per_cu = [] {
                int n = 0;
                if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                        &n, k_conv3_first<true>, 256, 0) != hipSuccess ||
                    n < 1)
                    n = 1;
                return n;
            }();
            int64_t cap = (int64_t)per_cu * device_cu_count();
            const int lim = g_brick_blocks.load(std::memory_order_relaxed);
            if (lim > 0) cap = std::min<int64_t>(cap, lim);
            const dim3 grid((unsigned)std::min<int64_t>(
                V[0].voxels() / (16 * kBY * kBZ), cap));
            if (train)
                hipLaunchKernelGGL(k_conv3_first<false>, grid, dim3(256), 0,
                                   c.st, ins[0], dose, rho, a.scale, V[0],
                                   la.cin, W(0), la.kp, B(0), ea[0]);
            else
                hipLaunchKernelGGL(k_conv3_first<true>, grid, dim3(256), 0,
                                   c.st, ins[0], dose, rho, a.scale, V[0],
                                   la.cin, W(0), la.kp, B(0), ea[0]);
        } else if ((s = conv(ins[l], V[l], la.cin, W(2 * l), la.kp,
                             B(2 * l), 1, nullptr, ea[l], la.cout, c.st)))
            return s;
        // the pooled features come out of the convolution's epilogue where
        // the volume tiles into bricks
        const bool fuse_pool = l < 3 && brick_ok(V[l], lb.cin);
        if ((s = conv(ea[l], V[l], lb.cin, W(2 * l + 1), lb.kp, B(2 * l + 1),
                      1, nullptr, eb[l], lb.cout, c.st, nullptr, 0,
                      fuse_pool ? pools[l] : nullptr)))
            return s;
        if (l < 3 && !fuse_pool)
            hipLaunchKernelGGL(k_pool, dim3(nblk(V[l + 1].voxels() * lb.cout)),
                               dim3(256), 0, c.st, eb[l], V[l], lb.cout,
                               pools[l]);
    }
    // decoder
    bf16_t *cats[3] = {a.cat0, a.cat1, a.cat2};
    bf16_t *da[3] = {a.d0a, a.d1a, a.d2a};
    bf16_t *db[3] = {a.d0b, a.d1b, a.d2b};
    const bf16_t *coarse = a.e3b;
    int cc = L[E3B].cout;
    for (int l = 2; l >= 0; --l) {
        const int ia = (l == 2) ? D2A : (l == 1 ? D1A : D0A);
        const ConvL &la = L[ia], &lb = L[ia + 1];
        const int cf = L[2 * l + 1].cout;
        const int ccs = la.cin % 32 == 0 ? 32 : 16;
        if (!train && brick_ok(V[l], la.cin) && cc % ccs == 0 &&
            cf % ccs == 0) {
            // inference: the convolution reads the concatenation in place
            if ((s = conv(eb[l], V[l], la.cin, W(ia), la.kp, B(ia), 1,
                          nullptr, da[l], la.cout, c.st, coarse, cc)))
                return s;
        } else {
            hipLaunchKernelGGL(k_up_concat,
                               dim3(nblk(V[l].voxels() * ((cc + cf) / 8))),
                               dim3(256), 0, c.st, coarse, cc, eb[l], cf,
                               V[l], cats[l]);
            if ((s = conv(cats[l], V[l], la.cin, W(ia), la.kp, B(ia), 1,
                          nullptr, da[l], la.cout, c.st)))
                return s;
        }
        // inference: the head comes out of the last convolution's epilogue
        HeadArgs hd{};
        if (l == 0 && !train && lb.cout == 16 && brick_ok(V[0], lb.cin))
            hd = HeadArgs{c.p + c.net.head_w, c.p + c.net.head_b, dose,
                          a.scale, a.out};
        if ((s = conv(da[l], V[l], lb.cin, W(ia + 1), lb.kp, B(ia + 1), 1,
                      nullptr, db[l], lb.cout, c.st, nullptr, 0, nullptr,
                      hd)))
            return s;
        coarse = db[l];
        cc = lb.cout;
        if (l == 0 && !hd.out)
            hipLaunchKernelGGL(k_head, dim3(nblk(V[0].voxels())), dim3(256),
                               0, c.st, a.d0b, L[D0B].cout,
                               c.p + c.net.head_w, c.p + c.net.head_b, dose,
                               per, a.scale, V[0].voxels(), a.out);
    }
    PSL_LAUNCHED();
    return PSL_OK;
}

// weight and bias gradients of layer i, then (if dx) its data gradient
psl_status layer_back(const Ctx &c, const Acts &a, int i, const bf16_t *x,
                      Vol V, const bf16_t *dy, float *grads, bf16_t *dx,
                      const bf16_t *dx_mask) {
    const ConvL &l = c.net.L[i];
    const int64_t nv = V.voxels();
    if (V.w % 16 == 0 && V.h % kBY == 0 && V.d % kBZ == 0 &&
        l.cin % 16 == 0 && l.cout % 16 == 0) {
        // bricks: partial sums per block, then an ordered reduction.  Up to
        // about 2048 blocks in all, at most the partial buffer's worth.
        const int64_t bricks = nv / (16 * kBY * kBZ);
        const int nt = l.cout / 16;
        const int mtp = nt % 2 == 0 ? 2 : 1;
        const int64_t chunks = (int64_t)(l.cin / 16) * (nt / mtp);
        const int64_t slab = (int64_t)27 * l.cout * l.cin;
        if (slab > kWgPartFloats) {
            set_error("layer %d: %lld weights exceed the partial-sum buffer",
                      i, (long long)slab);
            return PSL_EINVAL;
        }
        const int64_t nb = std::max<int64_t>(1, std::min<int64_t>(
            {bricks, kWgPartFloats / slab, (2048 + chunks - 1) / chunks}));
        const dim3 grid((unsigned)nb, (unsigned)(l.cin / 16),
                        (unsigned)(nt / mtp));
        if (mtp == 2)
            hipLaunchKernelGGL(k_conv3_wgrad_bk<2>, grid, dim3(256), 0, c.st,
                               x, V, l.cin, dy, l.cout, a.wpart);
        else
            hipLaunchKernelGGL(k_conv3_wgrad_bk<1>, grid, dim3(256), 0, c.st,
                               x, V, l.cin, dy, l.cout, a.wpart);
        hipLaunchKernelGGL(k_wgrad_reduce, dim3(nblk(slab, 16)), dim3(256), 0,
                           c.st, a.wpart, (int)nb, l.cout, l.cin,
                           grads + l.w_off, l.kp);
    } else {
        // about 64 chunks per offset (27 x 64 blocks): enough blocks to
        // fill the chip, few enough that the per-block atomics stay small
        int64_t chunk = std::max<int64_t>(256, (nv / 64 + 31) / 32 * 32);
        const unsigned nch = (unsigned)((nv + chunk - 1) / chunk);
        hipLaunchKernelGGL(k_conv3_wgrad, dim3(nch, 27), dim3(256), 0, c.st,
                           x, V, l.cin, dy, l.cout, chunk, grads + l.w_off,
                           l.kp);
    }
    hipLaunchKernelGGL(k_bias_grad, dim3(256), dim3(256), 0, c.st, dy, nv,
                       l.cout, grads + l.b_off);
    if (dx) {
        const int kp2 = (27 * l.cout + 31) / 32 * 32;
        hipLaunchKernelGGL(k_flip_weights, dim3(nblk((int64_t)l.cin * kp2)),
                           dim3(256), 0, c.st, c.pb + l.w_off, l.cin, l.cout,
                           l.kp, a.wt, kp2);
        psl_status s = conv(dy, V, l.cout, a.wt, kp2, nullptr, 0, dx_mask, dx,
                            l.cin, c.st);
        if (s) return s;
    }
    PSL_LAUNCHED();
    return PSL_OK;
}

psl_status backward(const Ctx &c, const Acts &a, const float *tgt,
                    float *grads, double *loss) {
    psl_status s;
    const auto &L = c.net.L;
    const Vol *V = a.V;
    const int64_t per = V[0].voxels() / V[0].n;
    bf16_t *g = a.gA, *g2 = a.gB, *t = a.gC;
    hipLaunchKernelGGL(k_loss_head_back, dim3(kLossBlocks), dim3(256), 0,
                       c.st, a.out, tgt, per, a.scale, V[0].voxels(), a.d0b,
                       c.p + c.net.head_w, g, a.lpart);
    hipLaunchKernelGGL(k_loss_head_sum, dim3(1), dim3(256), 0, c.st, a.lpart,
                       kLossBlocks, V[0].voxels(), loss, grads + c.net.head_b,
                       grads + c.net.head_w);
    // decoder, level 0 .. 2 (gradient g of the level's output d_lb)
    bf16_t *cats[3] = {a.cat0, a.cat1, a.cat2};
    bf16_t *da[3] = {a.d0a, a.d1a, a.d2a};
    bf16_t *db[3] = {a.d0b, a.d1b, a.d2b};
    bf16_t *sk[3] = {a.sk0, a.sk1, a.sk2};
    const int ia_of[3] = {D0A, D1A, D2A};
    for (int l = 0; l < 3; ++l) {
        const int ia = ia_of[l];
        // d_lb = relu(conv(d_la)); g is its masked gradient
        if ((s = layer_back(c, a, ia + 1, da[l], V[l], g, grads, g2, da[l])))
            return s;
        // d_la = relu(conv(cat)); g2 its masked gradient -> gradient of cat
        if ((s = layer_back(c, a, ia, cats[l], V[l], g2, grads, t, nullptr)))
            return s;
        const int cf = L[2 * l + 1].cout;          // skip channels
        const int cc = L[ia].cin - cf;             // up-sampled channels
        const bf16_t *coarse_act = (l == 2) ? a.e3b : db[l + 1];
        hipLaunchKernelGGL(k_up_concat_back_a, dim3(nblk(V[l + 1].voxels() * cc)),
                           dim3(256), 0, c.st, t, cc, cf, V[l], coarse_act, g);
        hipLaunchKernelGGL(k_up_concat_back_b, dim3(nblk(V[l].voxels() * cf)),
                           dim3(256), 0, c.st, t, cc, cf, V[l], sk[l]);
    }
    // encoder, level 3 .. 0 (g: masked gradient of e_lb)
    bf16_t *ins[4] = {a.xin, a.p1, a.p2, a.p3};
    bf16_t *ea[4] = {a.e0a, a.e1a, a.e2a, a.e3a};
    bf16_t *eb[4] = {a.e0b, a.e1b, a.e2b, a.e3b};
    for (int l = 3; l >= 0; --l) {
        if ((s = layer_back(c, a, 2 * l + 1, ea[l], V[l], g, grads, g2,
                            ea[l])))
            return s;
        if ((s = layer_back(c, a, 2 * l, ins[l], V[l], g2, grads,
                            l > 0 ? t : nullptr, nullptr)))
            return s;
        if (l > 0) {
            // gradient of p_l -> e_(l-1)b: pool back, add the skip part,
            // ReLU mask of e_(l-1)b
            const int C = L[2 * l - 1].cout;
            const int64_t n = V[l - 1].voxels() * C;
            hipLaunchKernelGGL(k_pool_back, dim3(nblk(n)), dim3(256), 0, c.st,
                               t, V[l - 1], C, g2);
            hipLaunchKernelGGL(k_add_mask, dim3(nblk(n)), dim3(256), 0, c.st,
                               g2, sk[l - 1], eb[l - 1], n, g);
        }
    }
    PSL_LAUNCHED();
    return PSL_OK;
}

psl_status check_net(const psl_unet *u, int n, int d, int h, int w) {
    PSL_REQUIRE(u && u->params && u->params_bf16, "NULL network");
    PSL_REQUIRE(u->levels == 4 && u->base == 16,
                "this build has the 4-level, 16-channel network only");
    PSL_REQUIRE(u->n_params == make_net(u->base).n_params,
                "n_params %lld does not match the architecture",
                (long long)u->n_params);
    PSL_REQUIRE(n >= 1 && d >= 8 && h >= 8 && w >= 8 && d % 8 == 0 &&
                    h % 8 == 0 && w % 8 == 0,
                "volume must be at least 8 voxels and divisible by 8 per "
                "axis");
    return PSL_OK;
}

}  // namespace
}  // namespace psl

using namespace psl;

extern "C" int64_t unet_param_count(int32_t levels, int32_t base) {
    if (levels != 4 || base != 16) return 0;
    return make_net(base).n_params;
}

extern "C" size_t unet_workspace_bytes(const psl_unet *u, int32_t n,
                                       int32_t nz, int32_t ny, int32_t nx,
                                       int32_t training) {
    if (!u || n < 1 || nz < 8 || ny < 8 || nx < 8) return 0;
    return carve_acts(nullptr, n, nz, ny, nx, u->base, training != 0).bytes;
}

extern "C" psl_status unet_init(psl_unet *u, uint64_t seed, void *stream) {
    PSL_REQUIRE(u && u->params && u->params_bf16, "NULL network");
    PSL_REQUIRE(u->levels == 4 && u->base == 16, "unsupported architecture");
    Net net = make_net(u->base);
    PSL_REQUIRE(u->n_params == net.n_params, "n_params mismatch");
    if (psl_status s = check_device()) return s;
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_fill_f32, dim3(nblk(net.n_params)), dim3(256), 0, st,
                       u->params, net.n_params, 0.0f);
    for (int i = 0; i < N_CONV; ++i) {
        const ConvL &l = net.L[i];
        const float stdv = std::sqrt(2.0f / (27.0f * (float)l.cin));
        hipLaunchKernelGGL(k_init_layer, dim3(nblk((int64_t)l.cout * l.kp)),
                           dim3(256), 0, st, u->params + l.w_off, l.cout,
                           l.kp, 27 * l.cin, stdv, seed, (uint32_t)i);
    }
    // the head starts at zero: the initial prediction is the input dose
    hipLaunchKernelGGL(k_to_bf16, dim3(nblk(net.n_params)), dim3(256), 0, st,
                       u->params, net.n_params, u->params_bf16);
    PSL_LAUNCHED();
    return PSL_OK;
}

extern "C" psl_status unet_set_brick_blocks(int32_t max_blocks) {
    PSL_REQUIRE(max_blocks >= 0, "max_blocks = %d < 0", max_blocks);
    g_brick_blocks.store(max_blocks, std::memory_order_relaxed);
    return PSL_OK;
}

extern "C" psl_status unet_set_params(psl_unet *u, void *stream) {
    PSL_REQUIRE(u && u->params && u->params_bf16, "NULL network");
    PSL_REQUIRE(u->levels == 4 && u->base == 16, "unsupported architecture");
    PSL_REQUIRE(u->n_params == make_net(u->base).n_params,
                "n_params mismatch");
    if (psl_status s = check_device()) return s;
    hipLaunchKernelGGL(k_to_bf16, dim3(nblk(u->n_params)), dim3(256), 0,
                       (hipStream_t)stream, u->params, u->n_params,
                       u->params_bf16);
    PSL_LAUNCHED();
    return PSL_OK;
}

extern "C" psl_status unet_forward(const psl_unet *u, const float *d_dose,
                                   const float *d_density, int32_t n,
                                   int32_t nz, int32_t ny, int32_t nx,
                                   float *d_out, void *d_ws, size_t ws_bytes,
                                   void *stream) {
    psl_status s = check_net(u, n, nz, ny, nx);
    if (s) return s;
    PSL_REQUIRE(d_dose && d_density && d_out, "NULL argument");
    Acts need = carve_acts(nullptr, n, nz, ny, nx, u->base, false);
    if (!d_ws || ws_bytes < need.bytes) {
        set_error("workspace %zu bytes < %zu required", ws_bytes, need.bytes);
        return PSL_ENOSPC;
    }
    if ((s = check_device())) return s;
    hipStream_t st = (hipStream_t)stream;
    Acts a = carve_acts(d_ws, n, nz, ny, nx, u->base, false);
    Ctx c{make_net(u->base), u->params, u->params_bf16, st};
    if ((s = forward(c, a, d_dose, d_density, false))) return s;
    const int64_t nv = a.V[0].voxels();
    hipLaunchKernelGGL(k_out_scale, dim3(nblk(nv)), dim3(256), 0, st, a.out,
                       nv, nv / n, a.scale, d_out);
    PSL_LAUNCHED();
    return PSL_OK;
}

extern "C" psl_status unet_backward(const psl_unet *u, const float *d_dose,
                                    const float *d_density,
                                    const float *d_target, int32_t n,
                                    int32_t nz, int32_t ny, int32_t nx,
                                    float *d_grads, double *d_loss,
                                    void *d_ws, size_t ws_bytes,
                                    void *stream) {
    psl_status s = check_net(u, n, nz, ny, nx);
    if (s) return s;
    PSL_REQUIRE(d_dose && d_density && d_target && d_grads && d_loss,
                "NULL argument");
    Acts need = carve_acts(nullptr, n, nz, ny, nx, u->base, true);
    if (!d_ws || ws_bytes < need.bytes) {
        set_error("workspace %zu bytes < %zu required", ws_bytes, need.bytes);
        return PSL_ENOSPC;
    }
    if ((s = check_device())) return s;
    hipStream_t st = (hipStream_t)stream;
    Acts a = carve_acts(d_ws, n, nz, ny, nx, u->base, true);
    Ctx c{make_net(u->base), u->params, u->params_bf16, st};
    if ((s = forward(c, a, d_dose, d_density, true))) return s;
    return backward(c, a, d_target, d_grads, d_loss);
}

extern "C" psl_status unet_adam_step(psl_unet *u, float *d_grads, float *d_m,
                                     float *d_v, float lr, float beta1,
                                     float beta2, float eps, int32_t step,
                                     void *stream) {
    PSL_REQUIRE(u && u->params && u->params_bf16 && d_grads && d_m && d_v,
                "NULL argument");
    PSL_REQUIRE(step >= 1, "step counts from 1");
    PSL_REQUIRE(lr > 0 && beta1 >= 0 && beta1 < 1 && beta2 >= 0 && beta2 < 1 &&
                    eps > 0,
                "bad Adam hyper-parameters");
    if (psl_status s = check_device()) return s;
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = u->n_params;
    const float c1 = 1.0f / (1.0f - std::pow(beta1, (float)step));
    const float c2 = 1.0f / (1.0f - std::pow(beta2, (float)step));
    hipLaunchKernelGGL(k_adam, dim3(nblk(n)), dim3(256), 0, st, u->params,
                       d_grads, d_m, d_v, n, lr, beta1, beta2, eps, c1, c2);
    hipLaunchKernelGGL(k_to_bf16, dim3(nblk(n)), dim3(256), 0, st, u->params,
                       n, u->params_bf16);
    hipLaunchKernelGGL(k_fill_f32, dim3(nblk(n)), dim3(256), 0, st, d_grads, n,
                       0.0f);
    PSL_LAUNCHED();
    return PSL_OK;
}

extern "C" psl_status dose_denoise(const float *d_dose,
                                   const float *d_density, int32_t nx,
                                   int32_t ny, int32_t nz,
                                   const psl_unet *net, float *d_out,
                                   void *d_ws, size_t ws_bytes,
                                   void *stream) {
    return unet_forward(net, d_dose, d_density, 1, nz, ny, nx, d_out, d_ws,
                        ws_bytes, stream);
}
