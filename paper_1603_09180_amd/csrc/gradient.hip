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
// Each of the four recursions of a pass (causal and anticausal, smoothing
// and derivative) runs in its own thread, one thread per column (coalesced
// across a wave) or per row, writing its own plane; the row pass adds the
// two halves of its input as it reads them, and a last elementwise pass adds
// the halves of gx and gy and stores the result.  Every product and sum is
// rounded on its own, in the association order written below (no
// contraction into fused multiply-adds), so the float32 result is
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

// Loads sample n of a line: column j of the source image (column pass) or
// row i of the sum of two scratch planes (row pass: A = A+ + A-, B = B+ + B-).
template <typename T>
struct ColLine {
    const T* col;
    int64_t pitch;
    __device__ __forceinline__ float operator()(int n) const { return (float)col[(int64_t)n * pitch]; }
};

struct SumLine {
    const float* u;
    const float* v;
    __device__ __forceinline__ float operator()(int n) const { return u[n] + v[n]; }
};

// One recursion along a line of n samples: kind 0 smoothing causal, 1
// smoothing anticausal, 2 derivative causal, 3 derivative anticausal.
// Output sample m goes to out[m * ostride].
template <int KIND, typename Line>
__device__ __forceinline__ void run_line(const GradCoef& co, const Line& x, int n,
                                         float* __restrict__ out, int64_t ostride)
{
    constexpr bool causal = KIND == 0 || KIND == 2;
    constexpr bool smooth = KIND == 0 || KIND == 1;
    const float edge = causal ? x(0) : x(n - 1);
    float s1 = edge * (causal ? (smooth ? co.s_plus : co.d_plus) : (smooth ? co.s_minus : co.d_minus));
    float s2 = s1;
    float x1 = edge, x2 = edge;   // previous inputs: x(m-1) (causal) or x(m+1), x(m+2)
    auto step = [&](float xm, int m) {
        float y;
        if (causal) {
            y = smooth ? smooth_causal(co, xm, x1, s1, s2) : deriv_causal(co, x1, s1, s2);
            x1 = xm;
        } else {
            y = smooth ? smooth_anti(co, x1, x2, s1, s2) : deriv_anti(co, x1, s1, s2);
            x2 = x1;
            x1 = xm;
        }
        out[(int64_t)m * ostride] = y;
    };
    int done = 0;
    for (; done + CH <= n; done += CH) {
        float xs[CH];
#pragma unroll
        for (int t = 0; t < CH; ++t) xs[t] = x(causal ? done + t : n - 1 - done - t);
#pragma unroll
        for (int t = 0; t < CH; ++t) step(xs[t], causal ? done + t : n - 1 - done - t);
    }
    for (; done < n; ++done) {
        const int m = causal ? done : n - 1 - done;
        step(x(m), m);
    }
}

// Column pass: blockIdx.y picks the recursion, one thread per column.
// Planes: out + kind * plane (A+, A-, B+, B-).
template <typename T>
__global__ __launch_bounds__(kGradThreads) void k_grad_cols(const T* __restrict__ src,
                                                            int64_t pitch, int h, int w,
                                                            float* __restrict__ out,
                                                            int64_t plane, GradCoef co)
{
    const int j = blockIdx.x * kGradThreads + threadIdx.x;
    if (j >= w || h <= 0) return;
    const ColLine<T> line{src + j, pitch};
    float* o = out + (int64_t)blockIdx.y * plane + j;
    switch (blockIdx.y) {
    case 0: run_line<0>(co, line, h, o, w); break;
    case 1: run_line<1>(co, line, h, o, w); break;
    case 2: run_line<2>(co, line, h, o, w); break;
    default: run_line<3>(co, line, h, o, w); break;
    }
}

// Row pass: blockIdx.y picks gx+ (derivative causal of A), gx- (derivative
// anticausal of A), gy+ (smoothing causal of B) or gy- (smoothing
// anticausal of B), one thread per row.  Planes in: A+, A-, B+, B-; out:
// gx+, gx-, gy+, gy-.
__global__ __launch_bounds__(kGradThreads) void k_grad_rows(const float* __restrict__ in,
                                                            int h, int w, int64_t plane,
                                                            float* __restrict__ out, GradCoef co)
{
    const int i = blockIdx.x * kGradThreads + threadIdx.x;
    if (i >= h || w <= 0) return;
    const int k = blockIdx.y;
    const int64_t row = (int64_t)i * w;
    const float* u = in + (k < 2 ? 0 : 2 * plane) + row;
    const SumLine line{u, u + plane};
    float* o = out + (int64_t)k * plane + row;
    switch (k) {
    case 0: run_line<2>(co, line, w, o, 1); break;
    case 1: run_line<3>(co, line, w, o, 1); break;
    case 2: run_line<0>(co, line, w, o, 1); break;
    default: run_line<1>(co, line, w, o, 1); break;
    }
}

// gx = gx+ + gx-, gy = gy+ + gy-, magnitude, stored value; one thread per pixel.
template <typename T>
__global__ __launch_bounds__(256) void k_grad_out(const float* __restrict__ g, int h, int w,
                                                  int64_t plane, T* __restrict__ dst,
                                                  int64_t dst_pitch, float* __restrict__ mag,
                                                  float gain, float top)
{
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (n >= plane) return;
    const float gx = g[n] + g[plane + n];
    const float gy = g[2 * plane + n] + g[3 * plane + n];
    const float sq = gx * gx + gy * gy;
    const float m = sqrtf(sq);
    if (mag) mag[n] = m;
    const int64_t i = n / w, j = n - i * w;
    dst[i * dst_pitch + j] = (T)fminf(rintf(m * gain), top);
}

}  // namespace

hipError_t launch_gradient(hipStream_t stream, const void* src, int64_t src_pitch, int src_dtype,
                           int h, int w, float* scratch, void* dst, int64_t dst_pitch,
                           int dst_dtype, float* mag, GradCoef co, float gain)
{
    const int64_t plane = (int64_t)h * w;
    float* cols = scratch;              // A+, A-, B+, B-
    float* rows = scratch + 4 * plane;  // gx+, gx-, gy+, gy-
    const dim3 block(kGradThreads);
    const dim3 gc((w + kGradThreads - 1) / kGradThreads, 4);
    const dim3 gr((h + kGradThreads - 1) / kGradThreads, 4);
    if (src_dtype == 1)
        hipLaunchKernelGGL(k_grad_cols<uint8_t>, gc, block, 0, stream,
                           static_cast<const uint8_t*>(src), src_pitch, h, w, cols, plane, co);
    else
        hipLaunchKernelGGL(k_grad_cols<uint16_t>, gc, block, 0, stream,
                           static_cast<const uint16_t*>(src), src_pitch, h, w, cols, plane, co);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_grad_rows, gr, block, 0, stream, cols, h, w, plane, rows, co);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const dim3 go((unsigned)((plane + 255) / 256));
    if (dst_dtype == 1)
        hipLaunchKernelGGL(k_grad_out<uint8_t>, go, dim3(256), 0, stream, rows, h, w, plane,
                           static_cast<uint8_t*>(dst), dst_pitch, mag, gain, 255.0f);
    else
        hipLaunchKernelGGL(k_grad_out<uint16_t>, go, dim3(256), 0, stream, rows, h, w, plane,
                           static_cast<uint16_t*>(dst), dst_pitch, mag, gain, 65535.0f);
    return hipGetLastError();
}

}  // namespace thin
