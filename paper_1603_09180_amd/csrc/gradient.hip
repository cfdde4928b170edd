// gradient.hip -- gfx950 kernels of the gradient front-end: the image the
// paper thins in its illustration (Fig. 1) is a Deriche gradient magnitude.
//
// Deriche's smoothing kernel f(n) = k (a|n| + 1) r^|n| and derivative kernel
// g(n) = -c n r^|n| (r = exp(-a); k gives unit sum, c unit response to a
// unit ramp) are each the sum of a causal and an anticausal second-order
// recursion.  The 2-D gradient is separable: a column pass runs f and g down
// every column (A = f_i F, B = g_i F), a row pass runs g and f along every
// row (gx = g_j A, gy = f_j B) and stores min(top, rint(|(gx, gy)| * gain)).
// Signals are extended by their edge values: each recursion starts from the
// steady state of that constant extension.
//
// One thread runs one column (coalesced across a wave) or one row.  Every
// product and sum is rounded on its own, in the association order written
// below (no contraction into fused multiply-adds), so the float32 result is
// reproducible bit for bit.
#include "thin_internal.h"

#pragma clang fp contract(off)

namespace thin {

namespace {

constexpr int kGradThreads = 64;   // one wave per block: the few lines spread over many CUs
constexpr int CH = 16;             // samples loaded ahead per thread (loads in flight)

// The four recursions, one sample each; s1, s2 hold the last two outputs and
// are advanced.  Association order as in the comments above.
__device__ __forceinline__ float smooth_causal(const GradCoef& co, float x, float xp, float& s1,
                                               float& s2)
{
    const float y = ((co.a0 * x + co.a1 * xp) + co.b1 * s1) + co.b2 * s2;
    s2 = s1;
    s1 = y;
    return y;
}

__device__ __forceinline__ float deriv_causal(const GradCoef& co, float xp, float& s1, float& s2)
{
    const float y = (co.d1 * xp + co.b1 * s1) + co.b2 * s2;
    s2 = s1;
    s1 = y;
    return y;
}

__device__ __forceinline__ float smooth_anti(const GradCoef& co, float x1, float x2, float& s1,
                                             float& s2)
{
    const float y = ((co.a2 * x1 + co.a3 * x2) + co.b1 * s1) + co.b2 * s2;
    s2 = s1;
    s1 = y;
    return y;
}

__device__ __forceinline__ float deriv_anti(const GradCoef& co, float x1, float& s1, float& s2)
{
    const float y = (co.d2 * x1 + co.b1 * s1) + co.b2 * s2;
    s2 = s1;
    s1 = y;
    return y;
}

template <typename T>
__global__ __launch_bounds__(kGradThreads) void k_grad_cols(const T* __restrict__ src,
                                                            int64_t pitch, int h, int w,
                                                            float* __restrict__ A,
                                                            float* __restrict__ B, GradCoef co)
{
    const int j = blockIdx.x * kGradThreads + threadIdx.x;
    if (j >= w || h <= 0) return;
    const T* col = src + j;
    // causal halves: y+(i) from x(i), x(i-1), y+(i-1), y+(i-2); stored
    const float x0 = (float)col[0];
    float xp = x0;
    float sa1 = co.s_plus * x0, sa2 = sa1;
    float sb1 = co.d_plus * x0, sb2 = sb1;
    int i = 0;
    for (; i + CH <= h; i += CH) {
        float xs[CH];
#pragma unroll
        for (int t = 0; t < CH; ++t) xs[t] = (float)col[(int64_t)(i + t) * pitch];
#pragma unroll
        for (int t = 0; t < CH; ++t) {
            const int64_t o = (int64_t)(i + t) * w + j;
            A[o] = smooth_causal(co, xs[t], xp, sa1, sa2);
            B[o] = deriv_causal(co, xp, sb1, sb2);
            xp = xs[t];
        }
    }
    for (; i < h; ++i) {
        const float x = (float)col[(int64_t)i * pitch];
        const int64_t o = (int64_t)i * w + j;
        A[o] = smooth_causal(co, x, xp, sa1, sa2);
        B[o] = deriv_causal(co, xp, sb1, sb2);
        xp = x;
    }
    // anticausal halves: y-(i) from x(i+1), x(i+2), y-(i+1), y-(i+2); added
    const float xl = (float)col[(int64_t)(h - 1) * pitch];
    float x1 = xl, x2 = xl;
    sa1 = co.s_minus * xl;
    sa2 = sa1;
    sb1 = co.d_minus * xl;
    sb2 = sb1;
    i = h - 1;
    for (; i + 1 >= CH; i -= CH) {
        float xs[CH], as[CH], bs[CH];
#pragma unroll
        for (int t = 0; t < CH; ++t) {
            const int64_t o = (int64_t)(i - t) * w + j;
            xs[t] = (float)col[(int64_t)(i - t) * pitch];
            as[t] = A[o];
            bs[t] = B[o];
        }
#pragma unroll
        for (int t = 0; t < CH; ++t) {
            const int64_t o = (int64_t)(i - t) * w + j;
            A[o] = as[t] + smooth_anti(co, x1, x2, sa1, sa2);
            B[o] = bs[t] + deriv_anti(co, x1, sb1, sb2);
            x2 = x1;
            x1 = xs[t];
        }
    }
    for (; i >= 0; --i) {
        const int64_t o = (int64_t)i * w + j;
        A[o] = A[o] + smooth_anti(co, x1, x2, sa1, sa2);
        B[o] = B[o] + deriv_anti(co, x1, sb1, sb2);
        x2 = x1;
        x1 = (float)col[(int64_t)i * pitch];
    }
}

template <typename T>
__device__ __forceinline__ void row_output(const GradCoef& co, float gxc, float gyc, float p,
                                           float q, float gain, float top, T* out, float* mrow,
                                           int j)
{
    const float gx = gxc + p;
    const float gy = gyc + q;
    const float sq = gx * gx + gy * gy;
    const float m = sqrtf(sq);
    if (mrow) mrow[j] = m;
    out[j] = (T)fminf(rintf(m * gain), top);
}

template <typename T>
__global__ __launch_bounds__(kGradThreads) void k_grad_rows(
    const float* __restrict__ A, const float* __restrict__ B, int h, int w,
    float* __restrict__ P, float* __restrict__ Q, T* __restrict__ dst, int64_t dst_pitch,
    float* __restrict__ mag, GradCoef co, float gain, float top)
{
    const int i = blockIdx.x * kGradThreads + threadIdx.x;
    if (i >= h || w <= 0) return;
    const float* a = A + (int64_t)i * w;
    const float* b = B + (int64_t)i * w;
    float* p = P + (int64_t)i * w;
    float* q = Q + (int64_t)i * w;
    // anticausal halves first (gx from A through g, gy from B through f)
    const float al = a[w - 1], bl = b[w - 1];
    float a1 = al, a2 = al, b1 = bl, b2 = bl;
    float gx1 = co.d_minus * al, gx2 = gx1;
    float gy1 = co.s_minus * bl, gy2 = gy1;
    int j = w - 1;
    for (; j + 1 >= CH; j -= CH) {
        float as[CH], bs[CH];
#pragma unroll
        for (int t = 0; t < CH; ++t) {
            as[t] = a[j - t];
            bs[t] = b[j - t];
        }
#pragma unroll
        for (int t = 0; t < CH; ++t) {
            p[j - t] = deriv_anti(co, a1, gx1, gx2);
            q[j - t] = smooth_anti(co, b1, b2, gy1, gy2);
            a2 = a1;
            a1 = as[t];
            b2 = b1;
            b1 = bs[t];
        }
    }
    for (; j >= 0; --j) {
        p[j] = deriv_anti(co, a1, gx1, gx2);
        q[j] = smooth_anti(co, b1, b2, gy1, gy2);
        a2 = a1;
        a1 = a[j];
        b2 = b1;
        b1 = b[j];
    }
    (void)a2;
    // causal halves, the sum, the magnitude and the stored value
    const float a0v = a[0], b0v = b[0];
    float ap = a0v, bp = b0v;
    gx1 = co.d_plus * a0v;
    gx2 = gx1;
    gy1 = co.s_plus * b0v;
    gy2 = gy1;
    T* out = dst + (int64_t)i * dst_pitch;
    float* mrow = mag ? mag + (int64_t)i * w : nullptr;
    j = 0;
    for (; j + CH <= w; j += CH) {
        float as[CH], bs[CH], ps[CH], qs[CH];
#pragma unroll
        for (int t = 0; t < CH; ++t) {
            as[t] = a[j + t];
            bs[t] = b[j + t];
            ps[t] = p[j + t];
            qs[t] = q[j + t];
        }
#pragma unroll
        for (int t = 0; t < CH; ++t) {
            const float gxc = deriv_causal(co, ap, gx1, gx2);
            const float gyc = smooth_causal(co, bs[t], bp, gy1, gy2);
            row_output(co, gxc, gyc, ps[t], qs[t], gain, top, out, mrow, j + t);
            ap = as[t];
            bp = bs[t];
        }
    }
    for (; j < w; ++j) {
        const float av = a[j], bv = b[j];
        const float gxc = deriv_causal(co, ap, gx1, gx2);
        const float gyc = smooth_causal(co, bv, bp, gy1, gy2);
        row_output(co, gxc, gyc, p[j], q[j], gain, top, out, mrow, j);
        ap = av;
        bp = bv;
    }
}

}  // namespace

hipError_t launch_gradient(hipStream_t stream, const void* src, int64_t src_pitch, int src_dtype,
                           int h, int w, float* A, float* B, float* P, float* Q, void* dst,
                           int64_t dst_pitch, int dst_dtype, float* mag, GradCoef co, float gain)
{
    const dim3 block(kGradThreads);
    const dim3 gc((w + kGradThreads - 1) / kGradThreads);
    const dim3 gr((h + kGradThreads - 1) / kGradThreads);
    if (src_dtype == 1)
        hipLaunchKernelGGL(k_grad_cols<uint8_t>, gc, block, 0, stream,
                           static_cast<const uint8_t*>(src), src_pitch, h, w, A, B, co);
    else
        hipLaunchKernelGGL(k_grad_cols<uint16_t>, gc, block, 0, stream,
                           static_cast<const uint16_t*>(src), src_pitch, h, w, A, B, co);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (dst_dtype == 1)
        hipLaunchKernelGGL(k_grad_rows<uint8_t>, gr, block, 0, stream, A, B, h, w, P, Q,
                           static_cast<uint8_t*>(dst), dst_pitch, mag, co, gain, 255.0f);
    else
        hipLaunchKernelGGL(k_grad_rows<uint16_t>, gr, block, 0, stream, A, B, h, w, P, Q,
                           static_cast<uint16_t*>(dst), dst_pitch, mag, co, gain, 65535.0f);
    return hipGetLastError();
}

}  // namespace thin
