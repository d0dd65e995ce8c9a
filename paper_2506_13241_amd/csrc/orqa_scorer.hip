// Learned truncation scorer on gfx950: string features, a 160-128-128-1 GELU
// network with bf16 MFMA forward (fp32 accumulation), fp32 backward and Adam.
//
// The network estimates, from a string's key alone, the log10 of the weight
// |g_I| with which the string will still reach <Z> after the remaining
// circuit; truncation then keeps strings by |c_I| * g_I instead of |c_I|
// (the paper leaves truncation schemes tailored to the problem as future work,
// Conclusion and Appendix D).
#include <algorithm>

#include "orqa_scorer.h"

namespace orqa {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// round to nearest even: the same bits as scorer_bf16 for finite values, in
// one instruction (v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, static_cast<__bf16>(f)); }
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(static_cast<uint32_t>(b) << 16); }

// erf by Hastings' rational approximation (Abramowitz & Stegun, Handbook of
// Mathematical Functions, 7.1.26): for u >= 0, erf(u) = 1 - t (a1 + t (a2 +
// t (a3 + t (a4 + t a5)))) exp(-u^2) with t = 1 / (1 + p u), |error| <= 1.5e-7,
// far below the bf16 rounding the activations get next.  Branch-free: one
// exponential and one reciprocal instead of a piecewise polynomial.
__device__ __forceinline__ float erf_as(float x) {
    // fused multiply-adds written out: the library builds without contraction
    // (the merge's products and sums must round as written), the scorer does not
    const float u = fabsf(x);
    // the hardware reciprocal (about one ulp) is far inside the formula's own
    // error; a correctly rounded one costs the whole division sequence
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, u, 1.0f));
    float p = fmaf(t, 1.061405429f, -1.453152027f);
    p = fmaf(t, p, 1.421413741f);
    p = fmaf(t, p, -0.284496736f);
    p = fmaf(t, p, 0.254829592f);
    p *= t;
    const float e = fmaf(-p, __expf(-u * u), 1.0f);
    return copysignf(e, x);
}
__device__ __forceinline__ float gelu(float x) {
    const float h = 0.5f * x;
    return fmaf(h, erf_as(x * 0.70710678118654752f), h);
}
__device__ __forceinline__ float gelu_grad(float x) {
    const float cdf = 0.5f * (1.0f + erf_as(x * 0.70710678118654752f));
    const float pdf = 0.3989422804014327f * __expf(-0.5f * x * x);
    return cdf + x * pdf;
}

// Feature f of a string: popcount of (letter mask of the string) & qmask[f],
// times scale[f].  Letters: 0 X, 1 Y, 2 Z, 3 any non-identity.
__device__ __forceinline__ float feature(const ulonglong2& mx, const ulonglong2& my, const ulonglong2& mz,
                                         const ulonglong2& ma, const ulonglong2& q, uint32_t letter, float scale) {
    // two-level select on the letter's bits (Y and "any" have bit 0, Z and
    // "any" bit 1): three conditional moves per dword
    const bool b0 = (letter & 1u) != 0u, b1 = (letter & 2u) != 0u;
    const uint64_t lo = b1 ? (b0 ? ma.x : mz.x) : (b0 ? my.x : mx.x);
    const uint64_t hi = b1 ? (b0 ? ma.y : mz.y) : (b0 ? my.y : mx.y);
    return scale * static_cast<float>(__popcll(lo & q.x) + __popcll(hi & q.y));
}

// Shared memory of the forward kernel: the network and the feature table,
// staged once per workgroup and read by all of its waves.
// Weight rows are padded (160 -> 164 and 128 -> 132 bf16, i.e. 82 and 66
// dwords) so that the 16 rows one A fragment reads fall on distinct LDS banks.
constexpr int kW1Ld = kScIn + 4;
constexpr int kW2Ld = kScH + 4;
struct FwdLds {
    alignas(16) uint16_t W1[kScH * kW1Ld];
    alignas(16) uint16_t W2[kScH * kW2Ld];
    float W3[kScH];
    float b1[kScH], b2[kScH], b3;
    ulonglong2 qmask[kScIn];
    float fscale[kScIn];
    uint8_t letter[kScIn];
};

// Forward over strings [0, n) of a (virtual) key array.  Each wave scores 16
// strings at a time and computes every layer transposed, out-features x
// strings: with the mfma_f32_16x16x16 bf16 operand layout (lane l holds
// A[l%16][4(l/16)+i], B[4(l/16)+i][l%16], D[4(l/16)+i][l%16]) the output tile
// of one layer is exactly the B operand of the next, so the hidden
// activations never leave registers.  Lane l works on string l%16; its B
// operand of layer 1 (features 4(l/16)..+3 of a 16-feature block) is computed
// in place from the key.  Weights are the A operands, read from LDS.
// Writes y (log10 of the predicted weight) and, for training, z1, z2 (the
// pre-activations) and the bf16 features.
__global__ __launch_bounds__(kScThreads) void k_scorer_forward(ScorerFwdArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    FwdLds& L = *reinterpret_cast<FwdLds*>(smem);
    const int tid = threadIdx.x;
    const ScorerDev& S = A.net;
    for (int i = tid; i < kScH * kScIn; i += kScThreads) L.W1[(i / kScIn) * kW1Ld + i % kScIn] = S.W1[i];
    for (int i = tid; i < kScH * kScH; i += kScThreads) L.W2[(i / kScH) * kW2Ld + i % kScH] = S.W2[i];
    for (int i = tid; i < kScH; i += kScThreads) {
        L.W3[i] = bf2f(S.W3[i]);
        L.b1[i] = S.b1[i];
        L.b2[i] = S.b2[i];
    }
    for (int i = tid; i < kScIn; i += kScThreads) {
        L.qmask[i] = S.qmask[i];
        L.fscale[i] = S.fscale[i];
        L.letter[i] = S.letter[i];
    }
    if (tid == 0) L.b3 = S.b3[0];
    const uint64_t n = A.nf_ptr ? A.nf_ptr[0] + A.nb_ptr[0] : A.n;
    const uint64_t nf = A.nf_ptr ? A.nf_ptr[0] : n;
    if (A.counters && blockIdx.x == 0 && tid == 0) {
        atomicAdd(reinterpret_cast<unsigned long long*>(&A.counters[0]), static_cast<unsigned long long>(n));
        atomicAdd(reinterpret_cast<unsigned long long*>(&A.counters[1]), 1ull);
    }
    __syncthreads();
    const int lane = tid & 63;
    const int r = lane & 15, kq = (lane >> 4) * 4;
    constexpr int kWaves = kScThreads / 64;
    const uint64_t nwt = (n + 15) / 16;

    for (uint64_t wt = uint64_t(blockIdx.x) * kWaves + (tid >> 6); wt < nwt; wt += uint64_t(gridDim.x) * kWaves) {
        const uint64_t i = wt * 16 + r;
        const bool live = i < n;
        ulonglong2 x = make_ulonglong2(0, 0), z = make_ulonglong2(0, 0);
        if (live) {
            const uint64_t p = i < nf ? i : A.cap - 1 - (i - nf);
            x = A.X[p];
            z = A.Z[p];
            if (A.xrot) x = rotl_n(x, A.xrot, A.nq);
        }
        const ulonglong2 mx = make_ulonglong2(x.x & ~z.x, x.y & ~z.y);
        const ulonglong2 my = make_ulonglong2(x.x & z.x, x.y & z.y);
        const ulonglong2 mz = make_ulonglong2(z.x & ~x.x, z.y & ~x.y);
        const ulonglong2 ma = make_ulonglong2(x.x | z.x, x.y | z.y);

        // ---- layer 1: z1^T = W1 f^T (+ b1)
        floatx4 acc[kScH / 16];
#pragma unroll
        for (int mt = 0; mt < kScH / 16; ++mt) acc[mt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
        for (int kt = 0; kt < kScIn / 16; ++kt) {
            bf16x4 b;
            uint16_t fv[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int f = kt * 16 + kq + q;
                fv[q] = f2bf(feature(mx, my, mz, ma, L.qmask[f], L.letter[f], L.fscale[f]));
                b[q] = static_cast<short>(fv[q]);
            }
            if (A.f_out && live) {
                uint2 pk;
                pk.x = uint32_t(fv[0]) | (uint32_t(fv[1]) << 16);
                pk.y = uint32_t(fv[2]) | (uint32_t(fv[3]) << 16);
                *reinterpret_cast<uint2*>(A.f_out + i * kScIn + kt * 16 + kq) = pk;
            }
#pragma unroll
            for (int mt = 0; mt < kScH / 16; ++mt) {
                const bf16x4 a = *reinterpret_cast<const bf16x4*>(L.W1 + (mt * 16 + r) * kW1Ld + kt * 16 + kq);
                acc[mt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[mt], 0, 0, 0);
            }
        }
        // h1 = gelu(z1) in bf16: already laid out as layer 2's B operand
        bf16x4 h1[kScH / 16];
#pragma unroll
        for (int mt = 0; mt < kScH / 16; ++mt) {
            float zz[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                zz[q] = acc[mt][q] + L.b1[mt * 16 + kq + q];
                h1[mt][q] = static_cast<short>(f2bf(gelu(zz[q])));
            }
            if (A.z1_out && live)
                *reinterpret_cast<float4*>(A.z1_out + i * kScH + mt * 16 + kq) = make_float4(zz[0], zz[1], zz[2], zz[3]);
        }

        // ---- layers 2 and 3: z2^T = W2 h1^T (+ b2), then y = W3 . bf16(gelu(z2))
        // + b3 in fp32.  Two output tiles at a time keep the register count low;
        // the four lanes of a string hold disjoint feature sets and are summed
        // by two shuffles.
        float y = 0.f;
#pragma unroll
        for (int mt = 0; mt < kScH / 16; mt += 2) {
            floatx4 c0 = floatx4{0.f, 0.f, 0.f, 0.f}, c1 = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kt = 0; kt < kScH / 16; ++kt) {  // static: h1[kt] is a register
                const bf16x4 a0 = *reinterpret_cast<const bf16x4*>(L.W2 + (mt * 16 + r) * kW2Ld + kt * 16 + kq);
                const bf16x4 a1 = *reinterpret_cast<const bf16x4*>(L.W2 + (mt * 16 + 16 + r) * kW2Ld + kt * 16 + kq);
                c0 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0, h1[kt], c0, 0, 0, 0);
                c1 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, h1[kt], c1, 0, 0, 0);
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const floatx4& c = h ? c1 : c0;
                const int m = mt + h;
                float zz[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int k = m * 16 + kq + q;
                    zz[q] = c[q] + L.b2[k];
                    y = fmaf(bf2f(f2bf(gelu(zz[q]))), L.W3[k], y);
                }
                if (A.z2_out && live)
                    *reinterpret_cast<float4*>(A.z2_out + i * kScH + m * 16 + kq) =
                        make_float4(zz[0], zz[1], zz[2], zz[3]);
            }
            // keep the scheduler from hoisting the next tiles' weight loads
            // (it would otherwise hold all 64 fragments in registers and spill)
            __builtin_amdgcn_sched_barrier(0);
        }
        y += __shfl_xor(y, 16, 64);
        y += __shfl_xor(y, 32, 64);
        if (lane < 16 && live) A.y_out[i] = y + L.b3;
    }
}

// ---- backward, per sample: dy, dz2 = dy W3 * gelu'(z2), dz1 = (W2^T dz2) * gelu'(z1)
__global__ __launch_bounds__(kThreads) void k_scorer_backward_rows(ScorerBwdArgs A) {
    __shared__ float sW2[kScH * kScH];
    __shared__ float sW3[kScH];
    for (int i = threadIdx.x; i < kScH * kScH; i += kThreads) sW2[i] = bf2f(A.net.W2[i]);
    for (int i = threadIdx.x; i < kScH; i += kThreads) sW3[i] = bf2f(A.net.W3[i]);
    __syncthreads();
    const float inv = 2.0f / static_cast<float>(A.n);
    for (uint64_t s = blockIdx.x * uint64_t(kThreads) + threadIdx.x; s < A.n; s += uint64_t(gridDim.x) * kThreads) {
        const float dy = inv * (A.y[s] - A.target[s]);
        A.dy[s] = dy;
        float dz2[kScH];
#pragma unroll 8
        for (int k = 0; k < kScH; ++k) {
            dz2[k] = dy * sW3[k] * gelu_grad(A.z2[s * kScH + k]);
            A.dz2[s * kScH + k] = dz2[k];
        }
        for (int j = 0; j < kScH; ++j) {
            float h = 0.f;
#pragma unroll 8
            for (int k = 0; k < kScH; ++k) h += sW2[k * kScH + j] * dz2[k];
            A.dz1[s * kScH + j] = h * gelu_grad(A.z1[s * kScH + j]);
        }
    }
}

// ---- weight gradients: out[i][j] = sum_s D[s][i] * B(s, j), j == J gives the
// bias column (B = 1).  B is gelu(z) (mode 0, fp32 [N][J]) or bf16 features
// (mode 1).  One workgroup per 16x16 output tile, samples in a fixed order.
__global__ __launch_bounds__(kThreads) void k_scorer_atb(const float* __restrict__ D, int I, const void* __restrict__ B,
                                                        int J, int mode, uint64_t N, float* __restrict__ outW,
                                                        float* __restrict__ outB) {
    __shared__ float sD[64][16];
    __shared__ float sB[64][17];
    const int ti = blockIdx.y * 16, tj = blockIdx.x * 16;
    const int li = threadIdx.x >> 4, lj = threadIdx.x & 15;
    float acc = 0.f;
    for (uint64_t s0 = 0; s0 < N; s0 += 64) {
        for (int t = threadIdx.x; t < 64 * 16; t += kThreads) {
            const int ss = t >> 4, c = t & 15;
            const uint64_t s = s0 + ss;
            const int i = ti + c, j = tj + c;
            sD[ss][c] = (s < N && i < I) ? D[s * I + i] : 0.f;
            float bv = 0.f;
            if (s < N) {
                if (j == J) bv = 1.f;
                else if (j < J) bv = mode == 0 ? gelu(static_cast<const float*>(B)[s * J + j])
                                               : bf2f(static_cast<const uint16_t*>(B)[s * J + j]);
            }
            sB[ss][c] = bv;
        }
        __syncthreads();
#pragma unroll 8
        for (int ss = 0; ss < 64; ++ss) acc += sD[ss][li] * sB[ss][lj];
        __syncthreads();
    }
    const int i = ti + li, j = tj + lj;
    if (i < I && j < J) outW[i * J + j] = acc;
    if (i < I && j == J) outB[i] = acc;
}

// ---- mean squared error (deterministic: fixed blocks, fixed tree)
__global__ void k_scorer_loss(const float* __restrict__ y, const float* __restrict__ t, uint64_t n,
                              double* __restrict__ out) {
    __shared__ double s[kThreads];
    double acc = 0.0;
    for (uint64_t i = threadIdx.x; i < n; i += kThreads) {
        const double r = double(y[i]) - double(t[i]);
        acc += r * r;
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int o = kThreads / 2; o > 0; o >>= 1) {
        if (int(threadIdx.x) < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = s[0] / double(n);
}

// ---- Adam on the fp32 master parameters; refreshes the bf16 weights.
__global__ void k_scorer_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                              float* __restrict__ v, int n, float lr, float b1, float b2, float eps, float c1,
                              float c2, ScorerDev net) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        p[i] = pi;
        scorer_store_param(net, i, pi);
    }
}

__global__ void k_scorer_set(const float* __restrict__ p, int n, ScorerDev net) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        scorer_store_param(net, i, p[i]);
}

hipError_t launch_scorer_forward(const ScorerFwdArgs& a, hipStream_t s, int grid) {
    static bool attr = false;
    if (!attr) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_scorer_forward),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, int(sizeof(FwdLds)));
        if (e != hipSuccess) return e;
        attr = true;
    }
    k_scorer_forward<<<dim3(grid), dim3(kScThreads), sizeof(FwdLds), s>>>(a);
    return hipGetLastError();
}

hipError_t launch_scorer_backward(const ScorerBwdArgs& a, const uint16_t* f, float* grad, hipStream_t s) {
    const int nb = int(std::min<uint64_t>((a.n + kThreads - 1) / kThreads, 1024));
    k_scorer_backward_rows<<<dim3(nb), dim3(kThreads), 0, s>>>(a);
    // gradients straight into the flat parameter layout
    k_scorer_atb<<<dim3((kScIn + 1 + 15) / 16, kScH / 16), dim3(kThreads), 0, s>>>(
        a.dz1, kScH, f, kScIn, 1, a.n, grad + kScOffW1, grad + kScOffB1);
    k_scorer_atb<<<dim3((kScH + 1 + 15) / 16, kScH / 16), dim3(kThreads), 0, s>>>(
        a.dz2, kScH, a.z1, kScH, 0, a.n, grad + kScOffW2, grad + kScOffB2);
    k_scorer_atb<<<dim3((kScH + 1 + 15) / 16, 1), dim3(kThreads), 0, s>>>(
        a.dy, 1, a.z2, kScH, 0, a.n, grad + kScOffW3, grad + kScOffB3);
    return hipGetLastError();
}

hipError_t launch_scorer_loss(const float* y, const float* t, uint64_t n, double* out, hipStream_t s) {
    k_scorer_loss<<<1, kThreads, 0, s>>>(y, t, n, out);
    return hipGetLastError();
}

hipError_t launch_scorer_adam(float* p, const float* g, float* m, float* v, int n, float lr, int step,
                              const ScorerDev& net, hipStream_t s) {
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, float(step)), c2 = 1.f - powf(b2, float(step));
    k_scorer_adam<<<dim3((n + 255) / 256), dim3(256), 0, s>>>(p, g, m, v, n, lr, b1, b2, 1e-8f, c1, c2, net);
    return hipGetLastError();
}

hipError_t launch_scorer_set(const float* p, int n, const ScorerDev& net, hipStream_t s) {
    k_scorer_set<<<dim3((n + 255) / 256), dim3(256), 0, s>>>(p, n, net);
    return hipGetLastError();
}

}  // namespace orqa
