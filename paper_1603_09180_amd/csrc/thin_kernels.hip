// thin_kernels.hip -- gfx950 kernels of the lambda-leveling loop.
//
// A parity step t lowers, all at once, the lambda-destructible pixels of the
// parity class s = t mod 4 (classes (i mod 2, j mod 2) = (0,0), (0,1), (1,0),
// (1,1)).  Pixels of one class are never 8-adjacent, so their decisions read
// only pixels no other candidate of the step writes; the result equals
// lowering the class pixel by pixel.
//
// Characterisation of a candidate x with value v (section 2.1):
//   U = {ring neighbours >= v} (Gamma+), L = ring minus U (Gamma--);
//   destructible <=> T+ = #C_n[x, U] = 1 and T-- = #C_n'[x, L] = 1 (a table
//   lookup on the 8-bit mask U);
//   otherwise, when T-- = k >= 2 and lambda > 0, x is lambda-destructible if at
//   least k-1 counted lower components c have v - max_c F <= lambda, i.e.
//   contain a pixel y with v - F(y) <= lambda;
//   a lambda-destructible x gets F(x) := alpha- = max F over L.
//
// Two engines:
//   k_step   one parity step per launch, straight from global memory;
//   k_round  LDS tiles with a halo of K pixels: one residency runs K parity
//            steps (the exact region shrinks by one pixel per step), reading
//            one ping-pong buffer and writing the other.  A tile whose 3x3
//            tile neighbourhood lowered nothing during the last 4 steps
//            cannot lower anything in the coming K steps (K <= tile side:
//            every pixel it could read was already examined at the same
//            values), so it is skipped; it only copies itself across the
//            ping-pong pair when it changed during the previous round.
#include "thin_internal.h"

#include <climits>

namespace thin {

namespace {

constexpr int kThreads = 256;

// Decision and new value for one candidate; nb in ring order E, NE, N, NW,
// W, SW, S, SE.  lut points at the 256 entries of the image's adjacency.
__device__ __forceinline__ bool decide(uint32_t v, const uint32_t (&nb)[8], const TopoEntry* lut,
                                       uint32_t lambda, uint32_t& alpha)
{
    uint32_t u = 0;
#pragma unroll
    for (int p = 0; p < 8; ++p) u |= (uint32_t)(nb[p] >= v) << p;
    const TopoEntry e = lut[u];
    bool lower = (e.flags & 1u) != 0u;
    if (!lower && lambda != 0u) {
        const uint32_t k = (e.flags >> 4) & 7u;
        if (k >= 2u) {
            uint32_t q = 0;  // lower neighbours within lambda of v
#pragma unroll
            for (int p = 0; p < 8; ++p) q |= (uint32_t)(nb[p] < v && v - nb[p] <= lambda) << p;
            const uint32_t hit = e.comps & (q * 0x01010101u);
            const uint32_t nonzero = (((hit & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | hit) & 0x80808080u;
            lower = (uint32_t)__popc(nonzero) + 1u >= k;
        }
    }
    if (lower) {
        uint32_t a = 0;
#pragma unroll
        for (int p = 0; p < 8; ++p) a = max(a, nb[p] < v ? nb[p] : 0u);
        alpha = a;
    }
    return lower;
}

__device__ __forceinline__ uint32_t load_px(const void* base, int dtype, int64_t idx)
{
    return dtype == 1 ? (uint32_t)static_cast<const uint8_t*>(base)[idx]
                      : (uint32_t)static_cast<const uint16_t*>(base)[idx];
}

__device__ __forceinline__ void store_px(void* base, int dtype, int64_t idx, uint32_t v)
{
    if (dtype == 1) static_cast<uint8_t*>(base)[idx] = (uint8_t)v;
    else static_cast<uint16_t*>(base)[idx] = (uint16_t)v;
}

// ------------------------------------------------------------------ k_init

__global__ void k_init_state(ImgCnt* cnt, int nimg, int32_t* tile_last, int ntiles)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nimg) {
        cnt[i].lowerings = 0ull;
        cnt[i].tile_rounds = 0ull;
        cnt[i].last_step = -1;
        cnt[i].pad = 0;
    }
    if (i < ntiles) tile_last[i] = -1;
}

// ------------------------------------------------------------------ k_step

template <typename T>
__global__ __launch_bounds__(kThreads) void k_step(const ImgDev* __restrict__ img, ImgCnt* cnt,
                                                   int step, const TopoEntry* __restrict__ lut_g)
{
    __shared__ TopoEntry s_lut[256];
    const ImgDev d = *img;
    for (int i = threadIdx.x; i < 256; i += kThreads) s_lut[i] = lut_g[d.adj * 256 + i];
    __syncthreads();
    const int s = step & 3, si = s >> 1, sj = s & 1;
    const int i = 2 * (int)blockIdx.y + si;
    const int j = 2 * (int)(blockIdx.x * kThreads + threadIdx.x) + sj;
    bool lowered = false;
    if (i >= 1 && i <= d.h - 2 && j >= 1 && j <= d.w - 2) {
        T* px = static_cast<T*>(d.buf[0]) + (int64_t)i * d.pitch + j;
        const int64_t P = d.pitch;
        const uint32_t v = px[0];
        const uint32_t nb[8] = {px[1], px[-P + 1], px[-P], px[-P - 1],
                                px[-1], px[P - 1], px[P], px[P + 1]};
        uint32_t alpha;
        if (decide(v, nb, s_lut, d.lambda, alpha)) {
            px[0] = (T)alpha;
            lowered = true;
        }
    }
    const unsigned long long ballot = __ballot(lowered);
    if ((threadIdx.x & 63) == 0 && ballot != 0ull) {
        atomicAdd(&cnt->lowerings, (unsigned long long)__popcll(ballot));
        atomicMax(&cnt->last_step, step);
    }
}

// ----------------------------------------------------------------- k_round

template <int TH, int TW, int K>
struct RoundGeom {
    static constexpr int RH = TH + 2 * K;
    static constexpr int RW = TW + 2 * K;
    static constexpr int RWP = RW;  // LDS row pitch in elements
    // lanes across a candidate row: next power of two >= RW/2, at most 64
    static constexpr int LW = (RW / 2 <= 8) ? 8 : (RW / 2 <= 16) ? 16 : (RW / 2 <= 32) ? 32 : 64;
    static_assert(K <= TH && K <= TW, "halo must not exceed the tile side");
};

template <int TH, int TW, int K>
__global__ __launch_bounds__(kThreads) void k_round(const ImgDev* __restrict__ imgs,
                                                    ImgCnt* cnt,
                                                    const int32_t* __restrict__ tile_img,
                                                    int32_t* tile_last, int ntiles, int round,
                                                    const TopoEntry* __restrict__ lut_g)
{
    using G = RoundGeom<TH, TW, K>;
    constexpr int RH = G::RH, RW = G::RW, RWP = G::RWP, LW = G::LW;
    __shared__ uint16_t s_img[RH * RWP];
    __shared__ TopoEntry s_lut[512];
    __shared__ int s_count;

    const int tid = threadIdx.x;
    for (int i = tid; i < 512; i += kThreads) s_lut[i] = lut_g[i];

    for (int g = blockIdx.x; g < ntiles; g += gridDim.x) {
        const int ii = tile_img[g];
        const ImgDev d = imgs[ii];
        const int r = round - d.round0;
        if (r < 0) continue;
        const int t0 = r * K;
        const int nsteps = min(K, d.max_steps - t0);
        if (nsteps <= 0) continue;
        const int lt = g - d.tile0;
        const int ty = lt / d.tiles_x, tx = lt - ty * d.tiles_x;

        // Neighbouring tiles of this round may update their tile_last while
        // it is read here (values only grow, which can only add work), so one
        // thread decides and the barrier broadcasts a block-uniform answer.
        // The barrier also orders this tile's LDS writes after the previous
        // tile's readers.
        int vote = 0;
        if (tid == 0) {
            int32_t m = INT_MIN;
            for (int dy = -1; dy <= 1; ++dy) {
                const int y = ty + dy;
                if (y < 0 || y >= d.tiles_y) continue;
                for (int dx = -1; dx <= 1; ++dx) {
                    const int x = tx + dx;
                    if (x < 0 || x >= d.tiles_x) continue;
                    m = max(m, tile_last[d.tile0 + y * d.tiles_x + x]);
                }
            }
            vote = (r == 0 || m >= t0 - 4) ? 1 : 0;
        }
        const bool active = __syncthreads_or(vote) != 0;
        const int32_t own_last = tile_last[g];  // written only by this block

        const void* src = d.buf[r & 1];
        void* dst = d.buf[(r + 1) & 1];
        const int gy0 = ty * TH, gx0 = tx * TW;  // tile interior origin
        const int ih = min(TH, d.h - gy0), iw = min(TW, d.w - gx0);

        if (!active) {
            // Stable for this round.  The output buffer already equals the
            // input unless the tile changed during the previous round.
            if (own_last >= t0 - K) {
                for (int idx = tid; idx < TH * TW; idx += kThreads) {
                    const int y = idx / TW, x = idx - y * TW;
                    if (y < ih && x < iw) {
                        const int64_t o = (int64_t)(gy0 + y) * d.pitch + (gx0 + x);
                        store_px(dst, d.dtype, o, load_px(src, d.dtype, o));
                    }
                }
            }
            continue;
        }

        // Stage the tile and its K-pixel halo (zeros outside the image; they
        // are never read by a candidate, whose 3x3 lies inside the image).
        const int ry0 = gy0 - K, rx0 = gx0 - K;
        if (tid == 0) s_count = 0;
        for (int idx = tid; idx < RH * RW; idx += kThreads) {
            const int y = idx / RW, x = idx - y * RW;
            const int gi = ry0 + y, gj = rx0 + x;
            uint32_t v = 0;
            if (gi >= 0 && gi < d.h && gj >= 0 && gj < d.w)
                v = load_px(src, d.dtype, (int64_t)gi * d.pitch + gj);
            s_img[y * RWP + x] = (uint16_t)v;
        }
        __syncthreads();

        const TopoEntry* lut = s_lut + d.adj * 256;
        const uint32_t lambda = d.lambda;
        int my_count = 0;
        int last_tau = -1;
        for (int tau = 0; tau < nsteps; ++tau) {
            const int s = (t0 + tau) & 3, si = s >> 1, sj = s & 1;
            // Exact region after tau steps, clipped to the image interior.
            const int r_lo = max(tau + 1, 1 - ry0), r_hi = min(RH - 2 - tau, d.h - 2 - ry0);
            const int c_lo = max(tau + 1, 1 - rx0), c_hi = min(RW - 2 - tau, d.w - 2 - rx0);
            const int r_first = r_lo + ((si - ry0 - r_lo) & 1);
            const int c_first = c_lo + ((sj - rx0 - c_lo) & 1);
            const int na = r_hi >= r_first ? (r_hi - r_first) / 2 + 1 : 0;
            const int nb = c_hi >= c_first ? (c_hi - c_first) / 2 + 1 : 0;
            bool inner = false;
            for (int a = tid / LW; a < na; a += kThreads / LW) {
                const int lr = r_first + 2 * a;
                for (int b = tid % LW; b < nb; b += LW) {
                    const int lc = c_first + 2 * b;
                    uint16_t* p = s_img + lr * RWP + lc;
                    const uint32_t v = p[0];
                    const uint32_t nbv[8] = {p[1], p[-RWP + 1], p[-RWP], p[-RWP - 1],
                                             p[-1], p[RWP - 1], p[RWP], p[RWP + 1]};
                    uint32_t alpha;
                    if (decide(v, nbv, lut, lambda, alpha)) {
                        p[0] = (uint16_t)alpha;
                        if (lr >= K && lr < K + TH && lc >= K && lc < K + TW) {
                            ++my_count;
                            inner = true;
                        }
                    }
                }
            }
            if (__syncthreads_or(inner)) last_tau = tau;
        }

        for (int idx = tid; idx < TH * TW; idx += kThreads) {
            const int y = idx / TW, x = idx - y * TW;
            if (y < ih && x < iw)
                store_px(dst, d.dtype, (int64_t)(gy0 + y) * d.pitch + (gx0 + x),
                         s_img[(K + y) * RWP + (K + x)]);
        }
        if (my_count) atomicAdd(&s_count, my_count);
        __syncthreads();
        if (tid == 0) {
            atomicAdd(&cnt[ii].tile_rounds, 1ull);
            if (last_tau >= 0) {
                tile_last[g] = t0 + last_tau;
                atomicAdd(&cnt[ii].lowerings, (unsigned long long)s_count);
                atomicMax(&cnt[ii].last_step, t0 + last_tau);
            }
        }
    }
}

template <int TH, int TW, int K>
hipError_t launch_round_t(hipStream_t stream, const ImgDev* imgs, ImgCnt* cnt,
                          const int32_t* tile_img, int32_t* tile_last, int ntiles, int round,
                          const TopoEntry* lut, int grid_blocks)
{
    const int grid = max(1, min(ntiles, grid_blocks));
    hipLaunchKernelGGL((k_round<TH, TW, K>), dim3(grid), dim3(kThreads), 0, stream, imgs, cnt,
                       tile_img, tile_last, ntiles, round, lut);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_init_state(hipStream_t stream, ImgCnt* cnt, int nimg, int32_t* tile_last,
                             int ntiles)
{
    const int n = max(nimg, ntiles);
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_init_state, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0,
                       stream, cnt, nimg, tile_last, ntiles);
    return hipGetLastError();
}

hipError_t launch_step(hipStream_t stream, const ImgDev* img_host, const ImgDev* img_dev,
                       ImgCnt* cnt, int step, const TopoEntry* lut)
{
    const int lat_w = (img_host->w + 1) / 2;
    const int lat_h = (img_host->h + 1) / 2;
    if (lat_h > 65535) return hipErrorInvalidValue;
    dim3 grid((lat_w + kThreads - 1) / kThreads, lat_h);
    if (img_host->dtype == 1)
        hipLaunchKernelGGL(k_step<uint8_t>, grid, dim3(kThreads), 0, stream, img_dev, cnt, step, lut);
    else
        hipLaunchKernelGGL(k_step<uint16_t>, grid, dim3(kThreads), 0, stream, img_dev, cnt, step, lut);
    return hipGetLastError();
}

#define THIN_ROUND_SHAPES(X) \
    X(32, 32, 8)             \
    X(32, 32, 16)            \
    X(64, 64, 16)            \
    X(64, 64, 32)

bool tile_shape_supported(TileShape s)
{
#define X(a, b, c) if (s.th == a && s.tw == b && s.k == c) return true;
    THIN_ROUND_SHAPES(X)
#undef X
    return false;
}

int round_blocks_per_cu(TileShape s)
{
    // LDS per block: region of u16 plus the 4 KiB table; 160 KiB per CU.
    const int lds = (s.th + 2 * s.k) * (s.tw + 2 * s.k) * 2 + 4096 + 64;
    int by_lds = (160 * 1024) / lds;
    return max(1, min(8, by_lds));
}

hipError_t launch_round(hipStream_t stream, TileShape shape, const ImgDev* imgs, ImgCnt* cnt,
                        const int32_t* tile_img, int32_t* tile_last, int ntiles, int round,
                        const TopoEntry* lut, int grid_blocks)
{
#define X(a, b, c)                                                                       \
    if (shape.th == a && shape.tw == b && shape.k == c)                                  \
        return launch_round_t<a, b, c>(stream, imgs, cnt, tile_img, tile_last, ntiles,   \
                                       round, lut, grid_blocks);
    THIN_ROUND_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

}  // namespace thin
