// Learned preconditioner: a 2D convolutional U-Net trained on the GPU.
//
// Architecture (NHWC activations in BF16, FP32 accumulation, channel counts
// padded to multiples of 16):
//   in(16) -> e0: 3x3 conv 16->16, 16->16  (ReLU after every 3x3 conv)
//   pool2  -> e1: 16->32, 32->32
//   pool2  -> e2: 32->64, 64->64
//   pool2  -> e3: 64->64, 64->64
//   up2 ++ e2 (128) -> d2: 128->64, 64->64
//   up2 ++ e1 (96)  -> d1: 96->32, 32->32
//   up2 ++ e0 (48)  -> d0: 48->16, 16->16
//   1x1 head 16->2 (linear, FP32 out)
// Inputs per cell: residual (re, im) scaled to unit RMS per sample,
// ln(D_i / mean D), and tau m_i / D_i (re, im): the shift's share of the
// diagonal.  The head predicts e D_i / s_r, from which the correction
// e = (K + tau M)^{-1} r is rebuilt.
//
// 3x3 convolutions are implicit GEMMs on v_mfma_f32_16x16x16_bf16: one
// wavefront computes 16 consecutive pixels of one image row times all
// output channels; K runs over the 9 taps x input channels.  The input
// gradient is the same kernel with the weights flipped and transposed; the
// weight gradient is a split-K GEMM over pixels on the same instruction.
#include "unet.h"

#include <cmath>
#include <cstring>
#include <random>

namespace lt {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f2bf(float x) {
    // round to nearest even
    uint32_t u = __float_as_uint(x);
    uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(r >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float(((uint32_t)b) << 16); }

// ---------------------------------------------------------------- 3x3 convolution (MFMA)
// X [P][cin] bf16 (P = B*H*W pixels, NHWC), Wt [9][cout][cin] bf16, bias [cout] fp32 (nullable).
// mode 0: Y bf16 = relu?(conv + bias); mode 1: Yf fp32 = conv (overwrite); mode 2: Yf += conv.
// A wavefront takes NT of the cout / 16 output-channel tiles, from tile NT * blockIdx.y on:
// small images split their channels over more workgroups (the sums of a tile are the same
// either way).
template <int NT>
__global__ __launch_bounds__(256) void k_conv3(const unsigned short* __restrict__ X, const unsigned short* __restrict__ Wt,
                                               const float* __restrict__ bias, int B, int H, int W, int cin,
                                               int cout, int relu, int mode, unsigned short* __restrict__ Y,
                                               float* __restrict__ Yf) {
    const int cofs = 16 * NT * blockIdx.y;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long long P = (long long)B * H * W;
    const long long p0 = ((long long)blockIdx.x * 4 + wave) * 16;  // 16 pixels of one row
    if (p0 >= P) return;
    const int w0 = (int)(p0 % W);
    const long long rowi = p0 / W;  // b * H + h
    const int h = (int)(rowi % H);
    const int pw = w0 + (lane & 15);      // this lane's A row (pixel) in the row
    const int kq = 4 * (lane >> 4);       // this lane's k offset inside a 16-chunk
    v4f acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = (v4f){0, 0, 0, 0};
    // one stencil row (three taps) at a time: all of its input and weight loads are issued
    // before the first product (addresses clamped into the image, out-of-image inputs zeroed)
    for (int dy = -1; dy <= 1; ++dy) {
        const int hh = h + dy;
        const bool rin = hh >= 0 && hh < H;
        const long long rowc = rin ? rowi + dy : rowi;
        for (int c0 = 0; c0 < cin; c0 += 16) {
            v4s a[3], b[3][NT];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int ww = pw + j - 1;
                const bool in = rin && ww >= 0 && ww < W;
                const int wc = min(max(ww, 0), W - 1);
                const v4s v = *reinterpret_cast<const v4s*>(X + (rowc * W + wc) * (long long)cin + c0 + kq);
                a[j] = in ? v : (v4s){0, 0, 0, 0};
                const unsigned short* wp = Wt + (size_t)((dy + 1) * 3 + j) * cout * cin;
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    b[j][t] = *reinterpret_cast<const v4s*>(wp + (size_t)(cofs + 16 * t + (lane & 15)) * cin + c0 + kq);
            }
#pragma unroll
            for (int j = 0; j < 3; ++j)
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[j], b[j][t], acc[t], 0, 0, 0);
        }
    }
    // lane holds column co = 16 t + lane%16, rows (pixels) 4 (lane/16) + i
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int co = cofs + 16 * t + (lane & 15);
        const float bb = bias ? bias[co] : 0.0f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const long long p = p0 + kq + i;
            float v = acc[t][i] + bb;
            if (mode == 0) {
                if (relu) v = fmaxf(v, 0.0f);
                Y[p * cout + co] = f2bf(v);
            } else if (mode == 1) {
                Yf[p * cout + co] = v;
            } else {
                Yf[p * cout + co] += v;
            }
        }
    }
}

// dW[tap][co][ci] += sum_p dZ[p][co] X[p + off(tap)][ci] and db[co] += sum_p dZ[p][co]
// (split-K over pixel chunks along blockIdx.x, FP32 atomics).  Every wave takes one
// (tap, ci-tile) combination (blockIdx.y selects a group of four) and all co-tiles; the
// wave of combination 0 also forms the bias gradient as a product with a ones operand.
template <int NT>
__global__ __launch_bounds__(256) void k_wgrad3(const unsigned short* __restrict__ X, const unsigned short* __restrict__ dZ,
                                                int B, int H, int W, int cin, int chunk, float* __restrict__ dW,
                                                float* __restrict__ db) {
    constexpr int cout = 16 * NT;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long long P = (long long)B * H * W;
    const long long pb = (long long)blockIdx.x * chunk;
    const long long pe = pb + chunk < P ? pb + chunk : P;
    const int nci = cin / 16;
    const int ncombo = 9 * nci;
    const int cb = blockIdx.y * 4 + wave;
    if (cb < ncombo) {
        const int tap = cb / nci, ct = cb % nci;
        const bool bias = db != nullptr && cb == 0;
        const v4s ones = (v4s){(short)0x3f80, (short)0x3f80, (short)0x3f80, (short)0x3f80};  // bf16 1.0
        v4f accb[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) accb[t] = (v4f){0, 0, 0, 0};
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        v4f acc[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = (v4f){0, 0, 0, 0};
        // W is a multiple of 16 and so are pb and pe: a group of 16 pixels lies in one row,
        // whose coordinates are found once per group (32-bit: P < 2^31)
        for (int q0 = (int)pb; q0 < (int)pe; q0 += 16) {
            const int row = q0 / W;  // b * H + h
            const int w0 = q0 - row * W;
            const int hh = row % H + dy;
            const bool rowok = hh >= 0 && hh < H;
            const unsigned short* xrow = X + (long long)(row + dy) * W * cin + 16 * ct + (lane & 15);
            // B operand: X at pixels q0 + 4 (lane/16) + i shifted by the tap, channel ci = 16 ct + lane%16
            v4s bx;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int ww = w0 + 4 * (lane >> 4) + i + dx;
                bx[i] = (short)((rowok && ww >= 0 && ww < W) ? xrow[(long long)ww * cin] : (unsigned short)0);
            }
            const unsigned short* zp = dZ + (long long)(q0 + 4 * (lane >> 4)) * cout + (lane & 15);
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                v4s az;
#pragma unroll
                for (int i = 0; i < 4; ++i) az[i] = (short)zp[i * cout + 16 * t];
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(az, bx, acc[t], 0, 0, 0);
                if (bias) accb[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(az, ones, accb[t], 0, 0, 0);
            }
        }
        // every column of accb holds the row sums: column 0 gives db
        if (bias && (lane & 15) == 0) {
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int i = 0; i < 4; ++i) atomicAdd(&db[16 * t + 4 * (lane >> 4) + i], accb[t][i]);
        }
        // lane: column ci = 16 ct + lane%16, rows co = 16 t + 4 (lane/16) + i
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int co = 16 * t + 4 * (lane >> 4) + i;
                atomicAdd(&dW[((size_t)tap * cout + co) * cin + 16 * ct + (lane & 15)], acc[t][i]);
            }
    }
}

// dZ = bf16(dY * (Y > 0))  (ReLU backward; Y is the post-activation output)
__global__ void k_relu_back(const float* __restrict__ dY, const unsigned short* __restrict__ Y, long long n,
                            unsigned short* __restrict__ dZ) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dZ[i] = f2bf(bf2f(Y[i]) > 0.0f ? dY[i] : 0.0f);
}

// 2x2 average pool, NHWC bf16
__global__ void k_pool(const unsigned short* __restrict__ X, int B, int H, int W, int C, unsigned short* __restrict__ Y) {
    const long long n = (long long)B * (H / 2) * (W / 2) * C;
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = (int)(i % C);
    long long q = i / C;
    const int w = (int)(q % (W / 2));
    q /= (W / 2);
    const int h = (int)(q % (H / 2));
    const long long b = q / (H / 2);
    const long long base = ((b * H + 2 * h) * W + 2 * w) * C + c;
    float s = bf2f(X[base]) + bf2f(X[base + C]) + bf2f(X[base + (long long)W * C]) + bf2f(X[base + (long long)W * C + C]);
    Y[i] = f2bf(0.25f * s);
}

// dX (fp32, +=) from dY of the pool: every child gets a quarter
__global__ void k_pool_back(const float* __restrict__ dY, int B, int H, int W, int C, float* __restrict__ dX) {
    const long long n = (long long)B * H * W * C;
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = (int)(i % C);
    long long q = i / C;
    const int w = (int)(q % W);
    q /= W;
    const int h = (int)(q % H);
    const long long b = q / H;
    dX[i] += 0.25f * dY[((b * (H / 2) + h / 2) * (W / 2) + w / 2) * C + c];
}

// out[p] = [ up2(lo)[p] (c1 channels) , skip[p] (c2 channels) ]
__global__ void k_upcat(const unsigned short* __restrict__ lo, const unsigned short* __restrict__ skip, int B, int H,
                        int W, int c1, int c2, unsigned short* __restrict__ out) {
    const int C = c1 + c2;
    const long long n = (long long)B * H * W * C;
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = (int)(i % C);
    const long long p = i / C;
    if (c < c1) {
        const int w = (int)(p % W);
        const long long q = p / W;
        const int h = (int)(q % H);
        const long long b = q / H;
        out[i] = lo[((b * (H / 2) + h / 2) * (W / 2) + w / 2) * c1 + c];
    } else {
        out[i] = skip[p * c2 + (c - c1)];
    }
}

// split d(upcat) into d(lo) (sum over the 2x2 children, overwrite) and d(skip) (+=)
__global__ void k_upcat_back_lo(const float* __restrict__ dOut, int B, int H, int W, int c1, int c2,
                                float* __restrict__ dLo) {
    const int C = c1 + c2;
    const long long n = (long long)B * (H / 2) * (W / 2) * c1;
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = (int)(i % c1);
    long long q = i / c1;
    const int w = (int)(q % (W / 2));
    q /= (W / 2);
    const int h = (int)(q % (H / 2));
    const long long b = q / (H / 2);
    const long long p = (b * H + 2 * h) * W + 2 * w;
    dLo[i] = dOut[p * C + c] + dOut[(p + 1) * C + c] + dOut[(p + W) * C + c] + dOut[(p + W + 1) * C + c];
}
__global__ void k_upcat_back_skip(const float* __restrict__ dOut, long long P, int c1, int c2, float* __restrict__ dSkip) {
    const long long n = P * c2;
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const long long p = i / c2;
    const int c = (int)(i % c2);
    dSkip[i] += dOut[p * (c1 + c2) + c1 + c];
}

// head: out[p][o] = sum_c X[p][c] Wh[o][c] + bh[o]  (16 -> 2)
__global__ void k_head(const unsigned short* __restrict__ X, const float* __restrict__ Wh, const float* __restrict__ bh,
                       long long P, float* __restrict__ out) {
    long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    float a0 = bh[0], a1 = bh[1];
    for (int c = 0; c < 16; ++c) {
        const float x = bf2f(X[p * 16 + c]);
        a0 += Wh[c] * x;
        a1 += Wh[16 + c] * x;
    }
    out[2 * p] = a0;
    out[2 * p + 1] = a1;
}

// head backward: dX[p][c] = sum_o dOut[p][o] Wh[o][c] (fp32 overwrite); dWh, dbh by block reduction
__global__ void k_head_back(const unsigned short* __restrict__ X, const float* __restrict__ Wh,
                            const float* __restrict__ dOut, long long P, float* __restrict__ dX,
                            float* __restrict__ dWh, float* __restrict__ dbh) {
    __shared__ float red[34][4];
    float g[34];
    for (int k = 0; k < 34; ++k) g[k] = 0;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (long long)gridDim.x * blockDim.x) {
        const float d0 = dOut[2 * p], d1 = dOut[2 * p + 1];
        for (int c = 0; c < 16; ++c) {
            const float x = bf2f(X[p * 16 + c]);
            dX[p * 16 + c] = d0 * Wh[c] + d1 * Wh[16 + c];
            g[c] += d0 * x;
            g[16 + c] += d1 * x;
        }
        g[32] += d0;
        g[33] += d1;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int k = 0; k < 34; ++k) {
        float v = g[k];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) red[k][wv] = v;
    }
    __syncthreads();
    if (threadIdx.x < 34) {
        float v = red[threadIdx.x][0] + red[threadIdx.x][1] + red[threadIdx.x][2] + red[threadIdx.x][3];
        if (threadIdx.x < 32) atomicAdd(&dWh[threadIdx.x], v);
        else atomicAdd(&dbh[threadIdx.x - 32], v);
    }
}

// Adam on the FP32 master parameters; refresh the BF16 copies of conv weights in both layouts.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       long long n, float lr, float b1, float b2, float eps, float c1, float c2) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1 - b1) * gi;
    const float vi = b2 * v[i] + (1 - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Wf[tap][co][ci] = bf16(W[tap][co][ci]);  Wb[tap][ci][co] = bf16(W[8 - tap][co][ci]) (flipped, transposed)
__global__ void k_wcast(const float* __restrict__ Wm, int cin, int cout, unsigned short* __restrict__ Wf,
                        unsigned short* __restrict__ Wb) {
    const int n = 9 * cin * cout;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int ci = i % cin, co = (i / cin) % cout, tap = i / (cin * cout);
    const unsigned short b = f2bf(Wm[i]);
    Wf[i] = b;
    Wb[((size_t)(8 - tap) * cin + ci) * cout + co] = b;
}

// ---------------------------------------------------------------- features, targets, loss
// Features of sample r: re, im of the residual / s_r, ln(D / Dbar), re, im of tau m / D.
// x: complex planes [B][2][N] of type T (one sample per right-hand side), s: per-sample RMS (out).
template <typename T>
__global__ void k_features(const T* __restrict__ x, int N, const double* __restrict__ D, const double* __restrict__ m,
                           double lnDbar, double tr, double ti, const float* __restrict__ rms,
                           unsigned short* __restrict__ F) {
    const int b = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const float s = rms[b] > 0 ? 1.0f / rms[b] : 0.0f;
    const double d = D[i];
    unsigned short* f = F + ((size_t)b * N + i) * 16;
    f[0] = f2bf((float)x[(size_t)b * 2 * N + i] * s);
    f[1] = f2bf((float)x[(size_t)b * 2 * N + N + i] * s);
    f[2] = f2bf((float)(log(d) - lnDbar));
    f[3] = f2bf((float)(tr * m[i] / d));
    f[4] = f2bf((float)(ti * m[i] / d));
    for (int c = 5; c < 16; ++c) f[c] = 0;
}

// rms[b] = sqrt(mean |x_b|^2) over the N cells: kRmsBlocks partial sums per sample
// (blockIdx.y), then one wavefront per sample adds them
constexpr int kRmsBlocks = 64;
template <typename T>
__global__ void k_rms_part(const T* __restrict__ x, int N, double* __restrict__ part) {
    const int b = blockIdx.y;
    double s = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < 2 * N; i += gridDim.x * blockDim.x) {
        const double v = (double)x[(size_t)b * 2 * N + i];
        s += v * v;
    }
    __shared__ double red[16];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0;
        for (int q = 0; q < (int)blockDim.x / 64; ++q) t += red[q];
        part[(size_t)b * gridDim.x + blockIdx.x] = t;
    }
}
__global__ void k_rms_final(const double* __restrict__ part, int N, float* __restrict__ rms) {
    const int b = blockIdx.x;
    double s = threadIdx.x < kRmsBlocks ? part[(size_t)b * kRmsBlocks + threadIdx.x] : 0.0;
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (threadIdx.x == 0) rms[b] = (float)sqrt(s / N);
}

// normalised target: tgt[p][c] = e * D / s_r
template <typename T>
__global__ void k_target(const T* __restrict__ e, int N, const double* __restrict__ D, const float* __restrict__ rms,
                         float* __restrict__ tgt) {
    const int b = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const float s = rms[b] > 0 ? 1.0f / rms[b] : 0.0f;
    tgt[((size_t)b * N + i) * 2] = (float)(e[(size_t)b * 2 * N + i] * D[i]) * s;
    tgt[((size_t)b * N + i) * 2 + 1] = (float)(e[(size_t)b * 2 * N + N + i] * D[i]) * s;
}

// e = out * s_r / D  back to complex planes (overwrite), only for active samples
template <typename T>
__global__ void k_unfeature(const float* __restrict__ out, int N, const double* __restrict__ D,
                            const float* __restrict__ rms, T* __restrict__ e, const int* __restrict__ active) {
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double s = rms[b] / D[i];
    e[(size_t)b * 2 * N + i] = (T)(out[((size_t)b * N + i) * 2] * s);
    e[(size_t)b * 2 * N + N + i] = (T)(out[((size_t)b * N + i) * 2 + 1] * s);
}

// Scale-free loss per sample: with o and t the complex output and target fields
// (re, im channels), the best complex multiple alpha o leaves the relative error
//   L_b = min_alpha ||alpha o - t||^2 / ||t||^2 = 1 - |<o, t>|^2 / (||o||^2 ||t||^2),
// <o, t> = sum conj(o) t = P + i Q.  With a, b the re, im channels of o and x, y of t:
//   dL/da = -2 (P x + Q y) / (oo tt) + 2 (P^2 + Q^2) a / (oo^2 tt),
//   dL/db = -2 (P y - Q x) / (oo tt) + 2 (P^2 + Q^2) b / (oo^2 tt),
// divided by B for the mean over samples.  The solver applies the network's
// direction with the residual-minimising multiple, so only the direction is learnt.
__global__ void k_loss(const float* __restrict__ o, const float* __restrict__ t, int N, int B, float* __restrict__ dO,
                       float* __restrict__ loss) {
    const int b = blockIdx.x;
    double P = 0, Q = 0, oo = 0, tt = 0;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const double a = o[((size_t)b * N + i) * 2], bb = o[((size_t)b * N + i) * 2 + 1];
        const double x = t[((size_t)b * N + i) * 2], y = t[((size_t)b * N + i) * 2 + 1];
        P += a * x + bb * y;
        Q += a * y - bb * x;
        oo += a * a + bb * bb;
        tt += x * x + y * y;
    }
    __shared__ double red[4][16];
    __shared__ double tot[4];
    double v[4] = {P, Q, oo, tt};
    for (int k = 0; k < 4; ++k) {
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
        if ((threadIdx.x & 63) == 0) red[k][threadIdx.x >> 6] = v[k];
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double s = 0;
        for (int q = 0; q < (int)blockDim.x / 64; ++q) s += red[threadIdx.x][q];
        tot[threadIdx.x] = s;
    }
    __syncthreads();
    P = tot[0];
    Q = tot[1];
    oo = tot[2];
    tt = tot[3];
    const bool ok = oo > 0 && tt > 0;
    if (threadIdx.x == 0) loss[b] = ok ? (float)(1.0 - (P * P + Q * Q) / (oo * tt)) : 1.0f;
    if (!dO) return;
    const double c1 = ok ? 2.0 / (oo * tt) / B : 0.0, c2 = ok ? 2.0 * (P * P + Q * Q) / (oo * oo * tt) / B : 0.0;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const size_t q = ((size_t)b * N + i) * 2;
        const double a = o[q], bb = o[q + 1], x = t[q], y = t[q + 1];
        dO[q] = (float)(-c1 * (P * x + Q * y) + c2 * a);
        dO[q + 1] = (float)(-c1 * (P * y - Q * x) + c2 * bb);
    }
}

// ---------------------------------------------------------------- host side
static inline unsigned nb(long long n, int b = 256) { return (unsigned)((n + b - 1) / b); }

static const int kCin[14] = {16, 16, 16, 32, 32, 64, 64, 64, 128, 64, 96, 32, 48, 16};
static const int kCout[14] = {16, 16, 32, 32, 64, 64, 64, 64, 64, 64, 32, 32, 16, 16};

UNet::UNet() {
    size_t off = 0;
    for (int l = 0; l < 14; ++l) {
        layers[l].cin = kCin[l];
        layers[l].cout = kCout[l];
        layers[l].w_off = off;
        off += 9 * (size_t)kCin[l] * kCout[l];
        layers[l].b_off = off;
        off += kCout[l];
    }
    head_w = off;
    off += 32;
    head_b = off;
    off += 2;
    nparams = off;
}

int unet_init_params(UNet* u, unsigned long long seed, std::vector<float>& p) {
    p.assign(u->nparams, 0.0f);
    std::mt19937_64 g(seed);
    for (int l = 0; l < 14; ++l) {
        const int fan_in = 9 * u->layers[l].cin;
        std::normal_distribution<float> nd(0.0f, std::sqrt(2.0f / fan_in));
        for (size_t k = 0; k < 9 * (size_t)u->layers[l].cin * u->layers[l].cout; ++k) p[u->layers[l].w_off + k] = nd(g);
    }
    std::normal_distribution<float> nh(0.0f, std::sqrt(1.0f / 16.0f));
    for (int k = 0; k < 32; ++k) p[u->head_w + k] = nh(g);
    return 0;
}

template <typename T> static T* ubuf(UNet* u, const char* name, size_t count, int* rc) {
    DevBuf& b = u->ws[name];
    int r = b.reserve(count * sizeof(T));
    if (r < 0) { *rc = r; return nullptr; }
    return b.as<T>();
}

int unet_upload(UNet* u, hipStream_t st, const float* host_params) {
    int rc = 0;
    float* p = ubuf<float>(u, "params", u->nparams, &rc);
    if (!p) return rc;
    LT_HIP(hipMemcpyAsync(p, host_params, u->nparams * sizeof(float), hipMemcpyHostToDevice, st));
    return unet_refresh_bf16(u, st);
}

int unet_refresh_bf16(UNet* u, hipStream_t st) {
    int rc = 0;
    float* p = ubuf<float>(u, "params", u->nparams, &rc);
    if (!p) return rc;
    for (int l = 0; l < 14; ++l) {
        const int n = 9 * u->layers[l].cin * u->layers[l].cout;
        std::string a = "wf" + std::to_string(l), b = "wb" + std::to_string(l);
        unsigned short* wf = ubuf<unsigned short>(u, a.c_str(), n, &rc);
        unsigned short* wb = ubuf<unsigned short>(u, b.c_str(), n, &rc);
        if (!wf || !wb) return rc;
        k_wcast<<<nb(n), 256, 0, st>>>(p + u->layers[l].w_off, u->layers[l].cin, u->layers[l].cout, wf, wb);
    }
    LT_HIP(hipGetLastError());
    return 0;
}

static int conv3(hipStream_t st, const unsigned short* X, const unsigned short* Wt, const float* bias, int B, int H,
                 int W, int cin, int cout, int relu, int mode, unsigned short* Y, float* Yf) {
    const long long P = (long long)B * H * W;
    const unsigned grid = (unsigned)((P / 16 + 3) / 4);
    const int nt = cout / 16;
    if (grid < 512 && nt > 1) {
        // too few pixel workgroups to fill the chip: one output-channel tile per wavefront
        k_conv3<1><<<dim3(grid, nt), 256, 0, st>>>(X, Wt, bias, B, H, W, cin, cout, relu, mode, Y, Yf);
    } else {
        switch (nt) {
            case 1: k_conv3<1><<<grid, 256, 0, st>>>(X, Wt, bias, B, H, W, cin, cout, relu, mode, Y, Yf); break;
            case 2: k_conv3<2><<<grid, 256, 0, st>>>(X, Wt, bias, B, H, W, cin, cout, relu, mode, Y, Yf); break;
            case 3: k_conv3<3><<<grid, 256, 0, st>>>(X, Wt, bias, B, H, W, cin, cout, relu, mode, Y, Yf); break;
            case 4: k_conv3<4><<<grid, 256, 0, st>>>(X, Wt, bias, B, H, W, cin, cout, relu, mode, Y, Yf); break;
            case 6: k_conv3<6><<<grid, 256, 0, st>>>(X, Wt, bias, B, H, W, cin, cout, relu, mode, Y, Yf); break;
            case 8: k_conv3<8><<<grid, 256, 0, st>>>(X, Wt, bias, B, H, W, cin, cout, relu, mode, Y, Yf); break;
            default: set_last_error("unet: unsupported channel count"); return LT_EUNSUPPORTED;
        }
    }
    LT_HIP(hipGetLastError());
    return 0;
}

static int wgrad3(hipStream_t st, const unsigned short* X, const unsigned short* dZ, int B, int H, int W, int cin,
                  int cout, float* dW, float* db) {
    const long long P = (long long)B * H * W;
    if (W % 16 || P >= (1LL << 31)) {
        set_last_error("unet: weight gradient needs a width that is a multiple of 16 and < 2^31 pixels");
        return LT_EUNSUPPORTED;
    }
    // pixel chunks (multiples of 16) sized so the grid has a few hundred workgroups
    const int chunk = P >= 65536 ? 512 : 256;
    const dim3 grid((unsigned)((P + chunk - 1) / chunk), (unsigned)((9 * (cin / 16) + 3) / 4));
    switch (cout / 16) {
        case 1: k_wgrad3<1><<<grid, 256, 0, st>>>(X, dZ, B, H, W, cin, chunk, dW, db); break;
        case 2: k_wgrad3<2><<<grid, 256, 0, st>>>(X, dZ, B, H, W, cin, chunk, dW, db); break;
        case 4: k_wgrad3<4><<<grid, 256, 0, st>>>(X, dZ, B, H, W, cin, chunk, dW, db); break;
        default: set_last_error("unet: unsupported channel count"); return LT_EUNSUPPORTED;
    }
    LT_HIP(hipGetLastError());
    return 0;
}

// Activation buffers for a batch: per layer output (bf16), pooled inputs, concatenations.
struct Acts {
    unsigned short* in;
    unsigned short* y[14];
    unsigned short* pool[3];
    unsigned short* cat[3];
    float* out;
};

static int acts(UNet* u, int B, int H, int W, Acts* a) {
    int rc = 0;
    const long long P0 = (long long)B * H * W;
    auto lvl = [&](int l) { return P0 >> (2 * l); };
    // layer -> level: e0a,e0b:0  e1a,e1b:1  e2a,e2b:2  e3a,e3b:3  d2a,d2b:2  d1a,d1b:1  d0a,d0b:0
    static const int L[14] = {0, 0, 1, 1, 2, 2, 3, 3, 2, 2, 1, 1, 0, 0};
    a->in = ubuf<unsigned short>(u, "a_in", P0 * 16, &rc);
    for (int l = 0; l < 14; ++l) {
        std::string n = "a_y" + std::to_string(l);
        a->y[l] = ubuf<unsigned short>(u, n.c_str(), lvl(L[l]) * kCout[l], &rc);
    }
    const int pc[3] = {16, 32, 64};
    for (int k = 0; k < 3; ++k) {
        std::string n = "a_pool" + std::to_string(k);
        a->pool[k] = ubuf<unsigned short>(u, n.c_str(), lvl(k + 1) * pc[k], &rc);
    }
    const int cc[3] = {48, 96, 128};  // concatenation at level 0, 1, 2
    for (int k = 0; k < 3; ++k) {
        std::string n = "a_cat" + std::to_string(k);
        a->cat[k] = ubuf<unsigned short>(u, n.c_str(), lvl(k) * cc[k], &rc);
    }
    a->out = ubuf<float>(u, "a_out", P0 * 2, &rc);
    if (rc < 0) return rc;
    for (int l = 0; l < 14; ++l)
        if (!a->y[l]) return LT_ENOMEM;
    return (a->in && a->out) ? 0 : LT_ENOMEM;
}

int unet_forward(UNet* u, hipStream_t st, int B, int H, int W) {
    if (H % 8 || W % 16 || (W >> 3) % 16) {
        set_last_error("unet: H must be a multiple of 8 and W of 128");
        return LT_EUNSUPPORTED;
    }
    Acts a;
    LT_TRY(acts(u, B, H, W, &a));
    int rc = 0;
    float* p = ubuf<float>(u, "params", u->nparams, &rc);
    if (!p) return rc;
    auto wf = [&](int l) { return u->ws["wf" + std::to_string(l)].as<unsigned short>(); };
    auto bias = [&](int l) { return p + u->layers[l].b_off; };
    int h = H, w = W;
    const unsigned short* x = a.in;
    // encoder
    for (int lev = 0; lev < 4; ++lev) {
        const int la = 2 * lev, lb = 2 * lev + 1;
        LT_TRY(conv3(st, x, wf(la), bias(la), B, h, w, kCin[la], kCout[la], 1, 0, a.y[la], nullptr));
        LT_TRY(conv3(st, a.y[la], wf(lb), bias(lb), B, h, w, kCin[lb], kCout[lb], 1, 0, a.y[lb], nullptr));
        if (lev < 3) {
            const long long n = (long long)B * (h / 2) * (w / 2) * kCout[lb];
            k_pool<<<nb(n), 256, 0, st>>>(a.y[lb], B, h, w, kCout[lb], a.pool[lev]);
            x = a.pool[lev];
            h /= 2;
            w /= 2;
        }
    }
    // decoder
    const unsigned short* lo = a.y[7];
    int clo = 64;
    for (int lev = 2; lev >= 0; --lev) {
        h *= 2;
        w *= 2;
        const int skip_layer = 2 * lev + 1;
        const int c2 = kCout[skip_layer];
        const long long n = (long long)B * h * w * (clo + c2);
        k_upcat<<<nb(n), 256, 0, st>>>(lo, a.y[skip_layer], B, h, w, clo, c2, a.cat[lev]);
        const int la = 8 + 2 * (2 - lev), lb = la + 1;
        LT_TRY(conv3(st, a.cat[lev], wf(la), bias(la), B, h, w, kCin[la], kCout[la], 1, 0, a.y[la], nullptr));
        LT_TRY(conv3(st, a.y[la], wf(lb), bias(lb), B, h, w, kCin[lb], kCout[lb], 1, 0, a.y[lb], nullptr));
        lo = a.y[lb];
        clo = kCout[lb];
    }
    const long long P = (long long)B * H * W;
    k_head<<<nb(P), 256, 0, st>>>(a.y[13], p + u->head_w, p + u->head_b, P, a.out);
    LT_HIP(hipGetLastError());
    return 0;
}

// Backward from dOut (fp32 [P][2] in ws "g_out"); accumulates parameter gradients into ws "grad".
int unet_backward(UNet* u, hipStream_t st, int B, int H, int W, float* dIn) {
    Acts a;
    LT_TRY(acts(u, B, H, W, &a));
    int rc = 0;
    float* p = ubuf<float>(u, "params", u->nparams, &rc);
    float* g = ubuf<float>(u, "grad", u->nparams, &rc);
    const long long P0 = (long long)B * H * W;
    float* dOut = ubuf<float>(u, "g_out", P0 * 2, &rc);
    float* gA = ubuf<float>(u, "g_a", P0 * 128, &rc);   // gradient w.r.t. a layer output (fp32)
    float* gB = ubuf<float>(u, "g_b", P0 * 128, &rc);   // gradient w.r.t. a layer input (fp32)
    float* gS[3];
    const int sc[3] = {16, 32, 64};
    for (int k = 0; k < 3; ++k) {
        std::string n = "g_skip" + std::to_string(k);
        gS[k] = ubuf<float>(u, n.c_str(), (P0 >> (2 * k)) * sc[k], &rc);
    }
    unsigned short* dZ = ubuf<unsigned short>(u, "g_dz", P0 * 128, &rc);
    if (rc < 0 || !p || !g || !dOut || !gA || !gB || !dZ) return rc < 0 ? rc : LT_ENOMEM;
    auto wb = [&](int l) { return u->ws["wb" + std::to_string(l)].as<unsigned short>(); };
    // layer inputs (bf16) for the weight gradients
    const unsigned short* lin[14] = {a.in, a.y[0], a.pool[0], a.y[2], a.pool[1], a.y[4], a.pool[2], a.y[6],
                                     a.cat[2], a.y[8], a.cat[1], a.y[10], a.cat[0], a.y[12]};
    static const int L[14] = {0, 0, 1, 1, 2, 2, 3, 3, 2, 2, 1, 1, 0, 0};
    for (int k = 0; k < 3; ++k)
        LT_HIP(hipMemsetAsync(gS[k], 0, (P0 >> (2 * k)) * sc[k] * sizeof(float), st));
    // head
    k_head_back<<<256, 256, 0, st>>>(a.y[13], p + u->head_w, dOut, P0, gA, g + u->head_w, g + u->head_b);
    // gA holds d(y13).  Walk the layers backwards.
    auto conv_back = [&](int l, float* dy, float* dx, int mode_dx) -> int {
        const long long P = P0 >> (2 * L[l]);
        const int h = H >> L[l], w = W >> L[l];
        const int ci = kCin[l], co = kCout[l];
        k_relu_back<<<nb(P * co), 256, 0, st>>>(dy, a.y[l], P * co, dZ);
        LT_TRY(wgrad3(st, lin[l], dZ, B, h, w, ci, co, g + u->layers[l].w_off, g + u->layers[l].b_off));
        if (dx) LT_TRY(conv3(st, dZ, wb(l), nullptr, B, h, w, co, ci, 0, mode_dx, nullptr, dx));
        return 0;
    };
    // decoder, level 0 .. 2
    float* cur = gA;
    float* oth = gB;
    for (int lev = 0; lev <= 2; ++lev) {
        const int la = 8 + 2 * (2 - lev), lb = la + 1;
        LT_TRY(conv_back(lb, cur, oth, 1));  // d(y_la)
        std::swap(cur, oth);
        LT_TRY(conv_back(la, cur, oth, 1));  // d(cat)
        std::swap(cur, oth);
        const int h = H >> lev, w = W >> lev;
        const int skip_layer = 2 * lev + 1;
        const int c2 = kCout[skip_layer];
        static const int kLoC[3] = {32, 64, 64};  // channels of the upsampled decoder input per level
        const int c1 = kLoC[lev];
        const long long P = P0 >> (2 * lev);
        k_upcat_back_skip<<<nb(P * c2), 256, 0, st>>>(cur, P, c1, c2, gS[lev]);
        k_upcat_back_lo<<<nb((P / 4) * c1), 256, 0, st>>>(cur, B, h, w, c1, c2, oth);
        std::swap(cur, oth);  // cur = d(lower decoder output or e3b)
    }
    // encoder, level 3 .. 0 ; cur = d(y7)
    for (int lev = 3; lev >= 0; --lev) {
        const int la = 2 * lev, lb = la + 1;
        if (lev < 3) {
            // d(y_lb) = skip gradient + pool backward of d(pool_lev)
            const long long P = P0 >> (2 * lev);
            const int c = kCout[lb];
            LT_HIP(hipMemcpyAsync(oth, gS[lev], P * c * sizeof(float), hipMemcpyDeviceToDevice, st));
            k_pool_back<<<nb(P * c), 256, 0, st>>>(cur, B, H >> lev, W >> lev, c, oth);
            std::swap(cur, oth);
        }
        LT_TRY(conv_back(lb, cur, oth, 1));
        std::swap(cur, oth);
        LT_TRY(conv_back(la, cur, lev == 0 ? dIn : oth, 1));
        if (lev > 0) std::swap(cur, oth);
    }
    LT_HIP(hipGetLastError());
    return 0;
}

template <typename T>
int unet_features(UNet* u, hipStream_t st, const LevelView<double>& L0, double lnDbar, cdouble tau, int B,
                  const T* x) {
    int rc = 0;
    const long long P0 = (long long)B * L0.N;
    float* rms = ubuf<float>(u, "rms", B, &rc);
    double* rmsp = ubuf<double>(u, "rmsp", (size_t)B * kRmsBlocks, &rc);
    unsigned short* F = ubuf<unsigned short>(u, "a_in", P0 * 16, &rc);
    if (!rms || !rmsp || !F) return rc;
    static_assert(kRmsBlocks <= 64, "one wavefront adds the partial sums");
    k_rms_part<T><<<dim3(kRmsBlocks, B), 256, 0, st>>>(x, L0.N, rmsp);
    k_rms_final<<<B, 64, 0, st>>>(rmsp, L0.N, rms);
    k_features<T><<<dim3(nb(L0.N), B), 256, 0, st>>>(x, L0.N, L0.D, L0.m, lnDbar, tau.real(), tau.imag(), rms, F);
    LT_HIP(hipGetLastError());
    return 0;
}

template <typename T>
int unet_apply(UNet* u, hipStream_t st, const LevelView<double>& L0, double lnDbar, cdouble tau, int B, const T* r,
               T* e, const int* active) {
    LT_TRY(unet_features<T>(u, st, L0, lnDbar, tau, B, r));
    LT_TRY(unet_forward(u, st, B, L0.ny, L0.nx));
    float* rms = u->ws["rms"].as<float>();
    float* out = u->ws["a_out"].as<float>();
    k_unfeature<T><<<dim3(nb(L0.N), B), 256, 0, st>>>(out, L0.N, L0.D, rms, e, active);
    LT_HIP(hipGetLastError());
    return 0;
}
template int unet_features<double>(UNet*, hipStream_t, const LevelView<double>&, double, cdouble, int,
                                   const double*);
template int unet_apply<float>(UNet*, hipStream_t, const LevelView<double>&, double, cdouble, int, const float*,
                               float*, const int*);
template int unet_apply<double>(UNet*, hipStream_t, const LevelView<double>&, double, cdouble, int, const double*,
                                double*, const int*);

int unet_loss_and_grad(UNet* u, hipStream_t st, const LevelView<double>& L0, int B, const double* e,
                       float* loss_dev) {
    int rc = 0;
    const long long P0 = (long long)B * L0.N;
    float* tgt = ubuf<float>(u, "tgt", P0 * 2, &rc);
    float* dOut = ubuf<float>(u, "g_out", P0 * 2, &rc);
    if (!tgt || !dOut) return rc;
    float* rms = u->ws["rms"].as<float>();
    k_target<double><<<dim3(nb(L0.N), B), 256, 0, st>>>(e, L0.N, L0.D, rms, tgt);
    k_loss<<<B, 256, 0, st>>>(u->ws["a_out"].as<float>(), tgt, L0.N, B, dOut, loss_dev);
    LT_HIP(hipGetLastError());
    return 0;
}

int unet_adam(UNet* u, hipStream_t st, float lr) {
    int rc = 0;
    float* p = ubuf<float>(u, "params", u->nparams, &rc);
    float* g = ubuf<float>(u, "grad", u->nparams, &rc);
    float* m = ubuf<float>(u, "adam_m", u->nparams, &rc);
    float* v = ubuf<float>(u, "adam_v", u->nparams, &rc);
    if (!p || !g || !m || !v) return rc;
    if (u->adam_t == 0) {
        LT_HIP(hipMemsetAsync(m, 0, u->nparams * sizeof(float), st));
        LT_HIP(hipMemsetAsync(v, 0, u->nparams * sizeof(float), st));
    }
    u->adam_t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - std::pow(b1, (float)u->adam_t), c2 = 1.0f - std::pow(b2, (float)u->adam_t);
    k_adam<<<nb((long long)u->nparams), 256, 0, st>>>(p, g, m, v, (long long)u->nparams, lr, b1, b2, 1e-8f, c1, c2);
    LT_HIP(hipGetLastError());
    return unet_refresh_bf16(u, st);
}

}  // namespace lt
