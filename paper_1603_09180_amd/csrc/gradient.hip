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
// across a wave; columns of up to 1024 samples split into segments, below)
// or per row, writing its own plane; the row pass adds the two halves of
// its input as it reads them, and a last elementwise pass adds the halves
// of gx and gy and stores the result.  Every product and sum is rounded on
// its own, in the association order written below (no contraction into
// fused multiply-adds), so the float32 result is reproducible bit for bit
// on a given image size.
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

// Columns of at most kSegLen * kSegMax samples also run split into segments
// of kSegLen samples, one wave per segment and 64 lines per block (one per
// lane), so a short column's recursion is not one thread's chain of n
// dependent steps.  Each recursion is linear in its output state: a
// segment first runs from a zero state (the first segment from the edge's
// steady state, which is its true state), then lane by lane wave 0 carries
// the true state from segment to segment (the true final state of a full
// segment is its zero-state final state plus E times its entering state, E
// the 2 x 2 map of the homogeneous recursion over kSegLen steps), and each
// segment adds z1[t] Y1 + z2[t] Y2 to its samples, z1 and z2 the homogeneous
// responses to the entering state (Y1, Y2) = (y[start - 1], y[start - 2]).
// The sums associate differently from the one-chain form, so the result
// agrees with it to rounding (the tests compare both with float64), not bit
// for bit.
constexpr int kSegLen = 64;
constexpr int kSegMax = 16;

template <int KIND, typename Line>
__device__ __forceinline__ void run_line_seg(const GradCoef& co, const Line& x, int n, bool live,
                                             float* __restrict__ out, int64_t ostride, int seg,
                                             int nseg, float2 (*s_state)[64], int lane)
{
    constexpr bool causal = KIND == 0 || KIND == 2;
    constexpr bool smooth = KIND == 0 || KIND == 1;
    auto at = [&](int p) { return causal ? p : n - 1 - p; };  // sample of processing position p
    const int p0 = seg * kSegLen;
    float y[kSegLen];
    float s1 = 0.f, s2 = 0.f;
    if (live && p0 < n) {
        const float edge = x(at(0));
        if (seg == 0) {
            s1 = edge * (causal ? (smooth ? co.s_plus : co.d_plus) : (smooth ? co.s_minus : co.d_minus));
            s2 = s1;
        }
        float x1 = p0 >= 1 ? x(at(p0 - 1)) : edge;
        float x2 = p0 >= 2 ? x(at(p0 - 2)) : edge;
#pragma unroll
        for (int t = 0; t < kSegLen; ++t) {
            if (p0 + t < n) {
                const float xm = x(at(p0 + t));
                if (causal) {
                    y[t] = smooth ? smooth_causal(co, xm, x1, s1, s2) : deriv_causal(co, x1, s1, s2);
                    x1 = xm;
                } else {
                    y[t] = smooth ? smooth_anti(co, x1, x2, s1, s2) : deriv_anti(co, x1, s1, s2);
                    x2 = x1;
                    x1 = xm;
                }
            }
        }
    }
    s_state[seg][lane] = make_float2(s1, s2);  // zero-state final (y[last], y[last - 1])
    __syncthreads();
    if (seg == 0) {
        // E from the homogeneous recursion z[t] = b1 z[t-1] + b2 z[t-2] over kSegLen steps
        float a1 = 1.f, a2 = 0.f, c1 = 0.f, c2 = 1.f;  // (z[t-1], z[t-2]) of both bases
        for (int t = 0; t < kSegLen; ++t) {
            const float an = co.b1 * a1 + co.b2 * a2, cn = co.b1 * c1 + co.b2 * c2;
            a2 = a1;
            a1 = an;
            c2 = c1;
            c1 = cn;
        }
        float Y1 = s_state[0][lane].x, Y2 = s_state[0][lane].y;
        for (int k = 1; k < nseg; ++k) {
            const float2 loc = s_state[k][lane];
            s_state[k][lane] = make_float2(Y1, Y2);
            const float n1 = loc.x + (a1 * Y1 + c1 * Y2), n2 = loc.y + (a2 * Y1 + c2 * Y2);
            Y1 = n1;
            Y2 = n2;
        }
    }
    __syncthreads();
    if (!live || p0 >= n) return;
    if (seg > 0) {
        const float Y1 = s_state[seg][lane].x, Y2 = s_state[seg][lane].y;
        float a1 = 1.f, a2 = 0.f, c1 = 0.f, c2 = 1.f;
#pragma unroll
        for (int t = 0; t < kSegLen; ++t) {
            const float an = co.b1 * a1 + co.b2 * a2, cn = co.b1 * c1 + co.b2 * c2;
            a2 = a1;
            a1 = an;
            c2 = c1;
            c1 = cn;
            y[t] = y[t] + (an * Y1 + cn * Y2);
        }
    }
#pragma unroll
    for (int t = 0; t < kSegLen; ++t)
        if (p0 + t < n) out[(int64_t)at(p0 + t) * ostride] = y[t];
}

// Column pass on segments: blockIdx.y picks the recursion, lane = column,
// threadIdx.y = segment.
template <typename T>
__global__ __launch_bounds__(64 * kSegMax) void k_grad_cols_seg(const T* __restrict__ src,
                                                                 int64_t pitch, int h, int w,
                                                                 float* __restrict__ out,
                                                                 int64_t plane, GradCoef co)
{
    __shared__ float2 s_state[kSegMax][64];
    const int lane = threadIdx.x, seg = threadIdx.y, nseg = blockDim.y;
    const int j = blockIdx.x * 64 + lane;
    const bool live = j < w;
    const ColLine<T> line{src + (live ? j : 0), pitch};
    float* o = out + (int64_t)blockIdx.y * plane + (live ? j : 0);
    switch (blockIdx.y) {
    case 0: run_line_seg<0>(co, line, h, live, o, w, seg, nseg, s_state, lane); break;
    case 1: run_line_seg<1>(co, line, h, live, o, w, seg, nseg, s_state, lane); break;
    case 2: run_line_seg<2>(co, line, h, live, o, w, seg, nseg, s_state, lane); break;
    default: run_line_seg<3>(co, line, h, live, o, w, seg, nseg, s_state, lane); break;
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
    // Segmented passes for lines of at most kSegLen * kSegMax samples (a
    // pass has only 4 x (lines) chains, too few to fill the device); longer
    // lines run one chain per thread.
    const int seg_c = (h + kSegLen - 1) / kSegLen;
    const dim3 sgc((w + 63) / 64, 4);
    if (seg_c <= kSegMax) {
        if (src_dtype == 1)
            hipLaunchKernelGGL(k_grad_cols_seg<uint8_t>, sgc, dim3(64, seg_c), 0, stream,
                               static_cast<const uint8_t*>(src), src_pitch, h, w, cols, plane, co);
        else
            hipLaunchKernelGGL(k_grad_cols_seg<uint16_t>, sgc, dim3(64, seg_c), 0, stream,
                               static_cast<const uint16_t*>(src), src_pitch, h, w, cols, plane, co);
    } else if (src_dtype == 1) {
        hipLaunchKernelGGL(k_grad_cols<uint8_t>, gc, block, 0, stream,
                           static_cast<const uint8_t*>(src), src_pitch, h, w, cols, plane, co);
    } else {
        hipLaunchKernelGGL(k_grad_cols<uint16_t>, gc, block, 0, stream,
                           static_cast<const uint16_t*>(src), src_pitch, h, w, cols, plane, co);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // (The row pass stays one chain per row: its lanes walk different rows,
    // and with segments eight times as many waves share each CU's cache
    // for those scattered lines; measured 24 -> 50 us at 512 x 512.)
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
