// thin_kernels.hip -- gfx950 kernels of the lambda-leveling loop and the
// lambda-skeleton.
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
// The lambda-skeleton (section 2.2's algorithm box) lowers instead the
// lambda-deletable points that are not lambda-end points: a peak (T+ = 0) is
// lowered too when v - alpha- <= lambda, and an end point (one upper
// n-neighbour) is kept when v - alpha- > lambda.  Its tables carry the peak
// and end bits; the images' table index selects the operator.
//
// Kernels:
//   k_step   one parity step per launch, straight from global memory;
//   k_round  one round: LDS tiles with a halo of K pixels, one residency
//            running K parity steps (the exact region shrinks by one pixel
//            per step), reading one ping-pong buffer and writing the other.
//            A tile whose 3x3 tile neighbourhood lowered nothing during the
//            last 4 steps cannot lower anything in the coming K steps
//            (K <= tile side: every pixel it could read was already examined
//            at the same values), so it is skipped; it only copies itself
//            across the ping-pong pair when it changed during the previous
//            round.  Residency variants (Tile, RTile, BTile) differ only in
//            how a step finds and examines its candidates;
//   k_coop   the rounds of k_round in one cooperative launch.
#include "thin_internal.h"

#include <climits>
#include <type_traits>

#include <hip/hip_cooperative_groups.h>

namespace thin {

namespace {

constexpr int kThreads = 256;
constexpr int STAGE_CHUNK = 8;  // global loads in flight per thread while staging a tile

// Upper-neighbour mask of a candidate of value v: bit p set when ring
// neighbour p (order E, NE, N, NW, W, SW, S, SE) has a value >= v.
__device__ __forceinline__ uint32_t upper_mask(uint32_t v, const uint32_t (&nb)[8])
{
    uint32_t u = 0;
#pragma unroll
    for (int p = 0; p < 8; ++p) u |= (uint32_t)(nb[p] >= v) << p;
    return u;
}

// Decision and new value for one candidate with upper mask u and its table
// entry e = lut[u] (the entries of the image's adjacency and operator).
__device__ __forceinline__ bool decide_entry_branchy(uint32_t v, const uint32_t (&nb)[8],
                                                     uint32_t u, TopoEntry e, uint32_t lambda,
                                                     uint32_t& alpha)
{
    bool lower = (e.flags & 1u) != 0u;
    const uint32_t k = (e.flags >> 4) & 7u;  // T--
    if (!lower && lambda != 0u && k >= 2u) {
        // lower neighbours y with v - F(y) <= lambda, i.e. F(y) >= v - lambda
        const uint32_t floor_v = v > lambda ? v - lambda : 0u;
        uint32_t q = 0;
#pragma unroll
        for (int p = 0; p < 8; ++p) q |= (uint32_t)(nb[p] >= floor_v) << p;
        q &= ~u;
        const uint32_t hit = e.comps & (q * 0x01010101u);
        const uint32_t nonzero = (((hit & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | hit) & 0x80808080u;
        lower = (uint32_t)__popc(nonzero) + 1u >= k;
    }
    // Skeleton tables mark peaks (bit 1) and end points (bit 2); leveling
    // tables mark neither.  A peak is lowered when its contrast v - alpha- is
    // at most lambda; an end point that passed the test above is kept when
    // its contrast exceeds lambda (a lambda-end point).
    const uint32_t pe = e.flags & 6u;
    if (lower || pe != 0u) {
        // max over L: the eight masked values are independent, the maxima
        // form a tree of depth three
        uint32_t m[8];
#pragma unroll
        for (int p = 0; p < 8; ++p) m[p] = ((u >> p) & 1u) ? 0u : nb[p];
        const uint32_t a = max(max(max(m[0], m[1]), max(m[2], m[3])),
                               max(max(m[4], m[5]), max(m[6], m[7])));
        alpha = a;
        if (pe != 0u) lower = (lower || pe == 2u) && v - a <= lambda;
    }
    return lower;
}

// The same decision in straight-line form.
__device__ __forceinline__ bool decide_entry_straight(uint32_t v, const uint32_t (&nb)[8],
                                                      uint32_t u, TopoEntry e, uint32_t lambda,
                                                      uint32_t& alpha)
{
    // Straight-line form: every term is computed and selected (inside a
    // wave both sides of a data-dependent branch usually run anyway).
    const uint32_t k = (e.flags >> 4) & 7u;  // T--
    // lower neighbours y with v - F(y) <= lambda, i.e. F(y) >= v - lambda
    const uint32_t floor_v = v > lambda ? v - lambda : 0u;
    uint32_t q = 0;
#pragma unroll
    for (int p = 0; p < 8; ++p) q |= (uint32_t)(nb[p] >= floor_v) << p;
    q &= ~u;
    const uint32_t hit = e.comps & (q * 0x01010101u);
    const uint32_t nonzero = (((hit & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | hit) & 0x80808080u;
    const bool divergent_ok = lambda != 0u && k >= 2u && (uint32_t)__popc(nonzero) + 1u >= k;
    bool lower = (e.flags & 1u) != 0u || divergent_ok;
    // max over L: the eight masked values are independent, the maxima form
    // a tree of depth three
    uint32_t m[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) m[p] = ((u >> p) & 1u) ? 0u : nb[p];
    const uint32_t a = max(max(max(m[0], m[1]), max(m[2], m[3])),
                           max(max(m[4], m[5]), max(m[6], m[7])));
    // Skeleton tables mark peaks (bit 1) and end points (bit 2); leveling
    // tables mark neither.  A peak is lowered when its contrast v - alpha- is
    // at most lambda; an end point that passed the test above is kept when
    // its contrast exceeds lambda (a lambda-end point).
    const uint32_t pe = e.flags & 6u;
    const bool small = v - a <= lambda;
    lower = pe == 0u ? lower : ((lower || pe == 2u) && small);
    alpha = a;
    return lower;
}

// Decision and new value for one candidate; nb in ring order E, NE, N, NW,
// W, SW, S, SE.  lut points at the 256 entries of the image's adjacency and
// operator.  STRAIGHT selects the straight-line form (measured faster where
// whole waves examine candidates together: the register-window and bit-flag
// residencies) over the branching one (faster for the flag residencies).
template <bool STRAIGHT>
__device__ __forceinline__ bool decide(uint32_t v, const uint32_t (&nb)[8], const TopoEntry* lut,
                                       uint32_t lambda, uint32_t& alpha)
{
    const uint32_t u = upper_mask(v, nb);
    // both words in one 64-bit load, so the lambda test waits for no second read
    const uint64_t raw = reinterpret_cast<const uint64_t*>(lut)[u];
    TopoEntry e;
    e.flags = (uint32_t)raw;
    e.comps = (uint32_t)(raw >> 32);
    return STRAIGHT ? decide_entry_straight(v, nb, u, e, lambda, alpha)
                    : decide_entry_branchy(v, nb, u, e, lambda, alpha);
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

__global__ void k_init_state(ImgCnt* cnt, int nimg, int32_t* tile_last, int ntiles,
                             int32_t* hist_round, WorkList wl)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (wl.list != nullptr) {
        if (i < ntiles) wl.listed[i] = -1;
        if (i < 3) wl.count[i] = 0;
        if (i < 6) wl.grab[i] = 0;
    }
    if (hist_round && i < 2 * ntiles) hist_round[i] = -1;
    if (i < nimg) {
        cnt[i].lowerings = 0ull;
        cnt[i].tile_rounds = 0ull;
        cnt[i].last_step = -1;
        cnt[i].pad = -1;
        cnt[i].examinations = 0ull;
    }
    if (tile_last && i < 2 * ntiles) tile_last[i] = -1;
}

__global__ void k_set_desc(ImgDev* dst, ImgDev d)
{
    if (threadIdx.x == 0) *dst = d;
}

__global__ void k_advance(int32_t* round_base, int n)
{
    if (threadIdx.x == 0) *round_base += n;
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
    const bool inside = i >= 1 && i <= d.h - 2 && j >= 1 && j <= d.w - 2;
    if (inside) {
        T* px = static_cast<T*>(d.buf[0]) + (int64_t)i * d.pitch + j;
        const int64_t P = d.pitch;
        const uint32_t v = px[0];
        const uint32_t nb[8] = {px[1], px[-P + 1], px[-P], px[-P - 1],
                                px[-1], px[P - 1], px[P], px[P + 1]};
        uint32_t alpha;
        if (decide<false>(v, nb, s_lut, d.lambda, alpha)) {
            px[0] = (T)alpha;
            lowered = true;
        }
    }
    const unsigned long long ballot = __ballot(lowered);
    const unsigned long long seen = __ballot(inside);
    if ((threadIdx.x & 63) == 0 && seen != 0ull)
        atomicAdd(&cnt->examinations, (unsigned long long)__popcll(seen));
    if ((threadIdx.x & 63) == 0 && ballot != 0ull) {
        atomicAdd(&cnt->lowerings, (unsigned long long)__popcll(ballot));
        atomicMax(&cnt->last_step, step);
    }
}

// ------------------------------------------------------------ tile residency

// Scalar fields of an image used inside a residency (no arrays, so the
// compiler keeps them in registers).
struct View {
    int64_t pitch;
    int32_t h, w;
    int32_t dtype;
    uint32_t lambda;
};

__device__ __forceinline__ View view_of(const ImgDev* d)
{
    View v;
    v.pitch = d->pitch;
    v.h = d->h;
    v.w = d->w;
    v.dtype = d->dtype;
    v.lambda = d->lambda;
    return v;
}

// Ping-pong buffer read by round r (src) and written by it (dst).  The
// descriptor stays in global memory: copying it into a local and indexing its
// array by r & 1 would push the copy into scratch.
__device__ __forceinline__ const void* round_src(const ImgDev* d, int r)
{
    return d->buf[r & 1];
}

__device__ __forceinline__ void* round_dst(const ImgDev* d, int r)
{
    return d->buf[(r + 1) & 1];
}

// ------------------------------------------------------- wide tile transfers
//
// Groups of 4 pixels move as one dword (u8) or two (u16) when both
// ping-pong buffers and the pitch are aligned to a group (the twin is
// 256-byte aligned, so the caller's buffer and pitch decide).  Region and
// interior columns start at multiples of 4, so a group lies wholly left of
// the image or starts inside it; only the last group of a row can be cut by
// the right border, and it moves pixel by pixel.

__device__ __forceinline__ bool wide_ok(const View& d, const void* a, const void* b)
{
    const uintptr_t al = d.dtype == 1 ? 4u : 8u;
    return (d.pitch & 3) == 0 && ((uintptr_t)a % al) == 0 && ((uintptr_t)b % al) == 0;
}

// 4 pixels as two u16 pairs (pixel 0 in the low half of .x).
__device__ __forceinline__ uint2 load4(const uint8_t* p)
{
    const uint32_t w = *reinterpret_cast<const uint32_t*>(p);
    return make_uint2((w & 0xFFu) | ((w << 8) & 0xFF0000u), ((w >> 16) & 0xFFu) | ((w >> 8) & 0xFF0000u));
}
__device__ __forceinline__ uint2 load4(const uint16_t* p) { return *reinterpret_cast<const uint2*>(p); }

__device__ __forceinline__ void store4(uint8_t* p, uint2 v)
{
    *reinterpret_cast<uint32_t*>(p) = (v.x & 0xFFu) | ((v.x >> 8) & 0xFF00u) | ((v.y & 0xFFu) << 16) |
                                      ((v.y << 8) & 0xFF000000u);
}
__device__ __forceinline__ void store4(uint16_t* p, uint2 v) { *reinterpret_cast<uint2*>(p) = v; }

template <typename P>
__device__ __forceinline__ uint2 load_partial(const P* p, int n)
{
    uint32_t q[4] = {0u, 0u, 0u, 0u};
    for (int i = 0; i < n; ++i) q[i] = p[i];
    return make_uint2(q[0] | (q[1] << 16), q[2] | (q[3] << 16));
}

template <typename P>
__device__ __forceinline__ void store_partial(P* p, uint2 v, int n)
{
    const uint32_t q[4] = {v.x & 0xFFFFu, v.x >> 16, v.y & 0xFFFFu, v.y >> 16};
    for (int i = 0; i < n; ++i) p[i] = (P)q[i];
}

// Region rows [0, RH) x columns [0, RW) of src, origin (ry0, rx0), into
// s_img (u16, row pitch RWP); zeros outside the image.
template <typename P, int RH, int RW, int RWP, int NT>
__device__ __forceinline__ void stage_wide(const View& d, const P* src, int ry0, int rx0,
                                           uint16_t* s_img, int tid)
{
    static_assert(RW % 4 == 0 && RWP % 4 == 0, "groups of 4 pixels");
    constexpr int GW = RW / 4, NG = RH * GW;
    constexpr int ITER = (NG + NT - 1) / NT;
    constexpr int CH = ITER < STAGE_CHUNK ? ITER : STAGE_CHUNK;
#pragma unroll 1
    for (int k0 = 0; k0 < ITER; k0 += CH) {
        uint2 v[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int g = tid + (k0 + c) * NT;
            const int y = g / GW, x = 4 * (g - (g / GW) * GW);
            const int gi = ry0 + y, gj = rx0 + x;
            v[c] = make_uint2(0u, 0u);
            if (g < NG && gi >= 0 && gi < d.h && gj >= 0 && gj < d.w) {
                const P* row = src + (int64_t)gi * d.pitch + gj;
                v[c] = gj + 4 <= d.w ? load4(row) : load_partial(row, d.w - gj);
            }
        }
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int g = tid + (k0 + c) * NT;
            if (g < NG) {
                const int y = g / GW, x = 4 * (g - (g / GW) * GW);
                *reinterpret_cast<uint2*>(s_img + y * RWP + x) = v[c];
            }
        }
    }
}

// Interior rows [0, TH) x columns [0, TW) of s_img (origin (OY, OX) in it)
// to dst at (gy0, gx0), clipped to the image.
template <typename P, int TH, int TW, int RWP, int OY, int OX, int NT>
__device__ __forceinline__ void store_wide(const View& d, P* dst, int gy0, int gx0,
                                           const uint16_t* s_img, int tid)
{
    static_assert(TW % 4 == 0 && OX % 4 == 0 && RWP % 4 == 0, "groups of 4 pixels");
    constexpr int GW = TW / 4;
    const int ih = min(TH, d.h - gy0), iw = min(TW, d.w - gx0);
    for (int g = tid; g < TH * GW; g += NT) {
        const int y = g / GW, x = 4 * (g - (g / GW) * GW);
        if (y < ih && x < iw) {
            const uint2 v = *reinterpret_cast<const uint2*>(s_img + (OY + y) * RWP + OX + x);
            P* q = dst + (int64_t)(gy0 + y) * d.pitch + gx0 + x;
            if (x + 4 <= iw) store4(q, v);
            else store_partial(q, v, iw - x);
        }
    }
}

// Region rows [0, RH) x columns [0, RW) of src, origin (ry0, rx0), into
// s_img at (y + OY, x + OX) with row pitch RWP, one pixel per load, up to
// STAGE_CHUNK loads in flight per thread (more would cost registers that
// the steps need); zeros outside the image.
template <int RH, int RW, int RWP, int OY, int OX, int NT>
__device__ __forceinline__ void stage_scalar(const View& d, const void* src, int ry0, int rx0,
                                             uint16_t* s_img, int tid)
{
    constexpr int ITER = (RH * RW + NT - 1) / NT;
    constexpr int CH = ITER < STAGE_CHUNK ? ITER : STAGE_CHUNK;
#pragma unroll 1
    for (int k0 = 0; k0 < ITER; k0 += CH) {
        uint32_t vals[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int idx = tid + (k0 + c) * NT;
            const int y = idx / RW, x = idx - y * RW;
            const int gi = ry0 + y, gj = rx0 + x;
            vals[c] = 0;
            if (idx < RH * RW && gi >= 0 && gi < d.h && gj >= 0 && gj < d.w)
                vals[c] = load_px(src, d.dtype, (int64_t)gi * d.pitch + gj);
        }
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int idx = tid + (k0 + c) * NT;
            const int y = idx / RW, x = idx - y * RW;
            if (idx < RH * RW) s_img[(y + OY) * RWP + x + OX] = (uint16_t)vals[c];
        }
    }
}

// Staging with groups of 4 pixels where the buffers allow it.
template <int RH, int RW, int RWP, int NT>
__device__ __forceinline__ void stage_region(const View& d, const void* src, const void* dst,
                                             int ry0, int rx0, uint16_t* s_img, int tid)
{
    if (wide_ok(d, src, dst)) {
        if (d.dtype == 1)
            stage_wide<uint8_t, RH, RW, RWP, NT>(d, static_cast<const uint8_t*>(src), ry0, rx0,
                                                 s_img, tid);
        else
            stage_wide<uint16_t, RH, RW, RWP, NT>(d, static_cast<const uint16_t*>(src), ry0, rx0,
                                                  s_img, tid);
    } else {
        stage_scalar<RH, RW, RWP, 0, 0, NT>(d, src, ry0, rx0, s_img, tid);
    }
}

// Interior of the staged region (origin (OY, OX) in s_img) to dst.
template <int TH, int TW, int RWP, int OY, int OX, int NT>
__device__ __forceinline__ void store_region(const View& d, const void* src, void* dst, int gy0,
                                             int gx0, const uint16_t* s_img, int tid)
{
    if constexpr (OX % 4 == 0 && RWP % 4 == 0 && TW % 4 == 0) {
        if (wide_ok(d, src, dst)) {
            if (d.dtype == 1)
                store_wide<uint8_t, TH, TW, RWP, OY, OX, NT>(d, static_cast<uint8_t*>(dst), gy0,
                                                             gx0, s_img, tid);
            else
                store_wide<uint16_t, TH, TW, RWP, OY, OX, NT>(d, static_cast<uint16_t*>(dst), gy0,
                                                              gx0, s_img, tid);
            return;
        }
    }
    const int ih = min(TH, d.h - gy0), iw = min(TW, d.w - gx0);
    for (int idx = tid; idx < TH * TW; idx += NT) {
        const int y = idx / TW, x = idx - y * TW;
        if (y < ih && x < iw)
            store_px(dst, d.dtype, (int64_t)(gy0 + y) * d.pitch + (gx0 + x),
                     s_img[(OY + y) * RWP + (OX + x)]);
    }
}

// Staging and store with the LDS tile in the image's own pixel type E (u8
// tiles take half the LDS of u16 ones).  Groups of 4 pixels move unchanged
// between global memory and LDS where the buffers allow it.
template <typename E>
__device__ __forceinline__ void copy4(E* dst, const E* src)
{
    if constexpr (sizeof(E) == 1) *reinterpret_cast<uint32_t*>(dst) = *reinterpret_cast<const uint32_t*>(src);
    else *reinterpret_cast<uint2*>(dst) = *reinterpret_cast<const uint2*>(src);
}

template <typename E, int RH, int RW, int RWP, int NT>
__device__ __forceinline__ void stage_native(const View& d, const void* srcv, const void* dstv,
                                             int ry0, int rx0, E* s_img, int tid)
{
    static_assert(RW % 4 == 0 && RWP % 4 == 0, "groups of 4 pixels");
    const E* src = static_cast<const E*>(srcv);
    if (!wide_ok(d, srcv, dstv)) {
        constexpr int ITER = (RH * RW + NT - 1) / NT;
        constexpr int CH = ITER < STAGE_CHUNK ? ITER : STAGE_CHUNK;
#pragma unroll 1
        for (int k0 = 0; k0 < ITER; k0 += CH) {
            E vals[CH];
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const int idx = tid + (k0 + c) * NT;
                const int y = idx / RW, x = idx - y * RW;
                const int gi = ry0 + y, gj = rx0 + x;
                vals[c] = 0;
                if (idx < RH * RW && gi >= 0 && gi < d.h && gj >= 0 && gj < d.w)
                    vals[c] = src[(int64_t)gi * d.pitch + gj];
            }
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const int idx = tid + (k0 + c) * NT;
                const int y = idx / RW, x = idx - y * RW;
                if (idx < RH * RW) s_img[y * RWP + x] = vals[c];
            }
        }
        return;
    }
    using V = typename std::conditional<sizeof(E) == 1, uint32_t, uint2>::type;
    constexpr int GW = RW / 4, NG = RH * GW;
    constexpr int ITER = (NG + NT - 1) / NT;
    constexpr int CH = ITER < STAGE_CHUNK ? ITER : STAGE_CHUNK;
#pragma unroll 1
    for (int k0 = 0; k0 < ITER; k0 += CH) {
        V v[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int g = tid + (k0 + c) * NT;
            const int y = g / GW, x = 4 * (g - (g / GW) * GW);
            const int gi = ry0 + y, gj = rx0 + x;
            v[c] = V{};
            if (g < NG && gi >= 0 && gi < d.h && gj >= 0 && gj < d.w) {
                const E* row = src + (int64_t)gi * d.pitch + gj;
                if (gj + 4 <= d.w) {
                    v[c] = *reinterpret_cast<const V*>(row);
                } else {
                    E q[4] = {0, 0, 0, 0};
                    for (int i = 0; i < d.w - gj; ++i) q[i] = row[i];
                    v[c] = *reinterpret_cast<const V*>(q);
                }
            }
        }
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int g = tid + (k0 + c) * NT;
            if (g < NG) {
                const int y = g / GW, x = 4 * (g - (g / GW) * GW);
                *reinterpret_cast<V*>(s_img + y * RWP + x) = v[c];
            }
        }
    }
}

template <typename E, int TH, int TW, int RWP, int OY, int OX, int NT>
__device__ __forceinline__ void store_native(const View& d, const void* srcv, void* dstv, int gy0,
                                             int gx0, const E* s_img, int tid)
{
    static_assert(TW % 4 == 0 && OX % 4 == 0 && RWP % 4 == 0, "groups of 4 pixels");
    E* dst = static_cast<E*>(dstv);
    const int ih = min(TH, d.h - gy0), iw = min(TW, d.w - gx0);
    if (!wide_ok(d, srcv, dstv)) {
        for (int idx = tid; idx < TH * TW; idx += NT) {
            const int y = idx / TW, x = idx - y * TW;
            if (y < ih && x < iw)
                dst[(int64_t)(gy0 + y) * d.pitch + (gx0 + x)] = s_img[(OY + y) * RWP + (OX + x)];
        }
        return;
    }
    constexpr int GW = TW / 4;
    for (int g = tid; g < TH * GW; g += NT) {
        const int y = g / GW, x = 4 * (g - (g / GW) * GW);
        if (y < ih && x < iw) {
            const E* s = s_img + (OY + y) * RWP + OX + x;
            E* q = dst + (int64_t)(gy0 + y) * d.pitch + gx0 + x;
            if (x + 4 <= iw) copy4(q, s);
            else
                for (int i = 0; i < iw - x; ++i) q[i] = s[i];
        }
    }
}

// History handed from one round to the next: for every tile processed in a
// round, a bitmap (TH rows of TW/32 words) of the interior pixels that were
// lowered during the last 4 steps of its residency, and the round it was
// written in.  Two copies alternate by round parity, so a tile of round r
// reads its neighbours' round r-1 bitmaps while they may be writing their
// round r ones.
struct Seed {
    const uint32_t* prev_bits;   // copy written in round r - 1 (unused when r == 0)
    const int32_t* prev_round;
    uint32_t* cur_bits;          // copy this round writes
    int32_t* cur_round;
    int r;                       // image-local round of the residency
    int tile0, tiles_x, tiles_y; // tile grid of the image
    int ty, tx, g;               // this tile
};

// Word `a` (global columns 32a..32a+31) of row gi of the previous round's
// change bitmaps; 0 outside the tile grid or where a tile has no bitmap for
// round r - 1 (it was skipped then, so nothing in it changed).
template <int TH, int TW>
__device__ __forceinline__ uint32_t history_word_t(const Seed* sd, int gi, int a)
{
    constexpr int WPR = TW / 32;
    if (a < 0) return 0u;
    const int tcol = a / WPR, trow = gi / TH;
    if (tcol >= sd->tiles_x || trow >= sd->tiles_y) return 0u;
    const int n = sd->tile0 + trow * sd->tiles_x + tcol;
    // both reads go out together: the bitmap of any tile of the grid may be
    // read, and is discarded unless the tile wrote it in round r - 1
    const uint32_t bits = sd->prev_bits[((int64_t)n * TH + (gi - trow * TH)) * WPR + (a - tcol * WPR)];
    return sd->prev_round[n] == sd->r - 1 ? bits : 0u;
}

// Geometry of a tile residency: a TH x TW interior plus a K-pixel halo,
// staged in LDS as u16, processed by NT threads.
template <int TH, int TW, int K, int NT, bool SEED>
struct Tile {
    using Elem = uint16_t;
    static constexpr int RH = TH + 2 * K;
    static constexpr int RW = TW + 2 * K;
    static constexpr int RWP = RW;  // LDS row pitch in elements
    static constexpr int IMG_ELEMS = RH * RWP;    // LDS elements of the image tile
    static constexpr int DIRTY_ELEMS = RH * RWP;  // LDS re-examination flags
    // lanes across a candidate row: next power of two >= RW/2, at most 64
    static constexpr int LAT_H = RH / 2, LAT_W = RW / 2;  // candidate lattice of one class
    static constexpr int PPT = (LAT_H * LAT_W + NT - 1) / NT;  // lattice cells per thread
    static constexpr int WPR = TW >= 32 ? TW / 32 : 1;  // bitmap words per interior row
    static constexpr int RWW = (RW + 31) / 32;           // change-map words per region row
    // LDS words of the history arrays (one when the residency keeps no history)
    static constexpr int BITS_WORDS = SEED ? TH * WPR : 1;
    static constexpr int CW_WORDS = SEED ? RH * RWW : 1;
    static_assert(K <= TH && K <= TW, "halo must not exceed the tile side");
    static_assert(!SEED || TW % 32 == 0, "history bitmaps need a tile width multiple of 32");
    static_assert(!SEED || 2 * K <= TH, "history seeding needs the region inside the 3x3 tile block");
    static_assert(TH % 2 == 0 && TW % 2 == 0 && K % 2 == 0, "tile sides and halo must be even");


    // Tile and halo from src into s_img (no barrier).
    // Work a residency can start before the block knows whether the tile
    // runs (none for this type).
    static __device__ __forceinline__ void prefetch(const View&, int, int, const Seed*, uint8_t*,
                                                    uint32_t*, int)
    {
    }

    static __device__ __forceinline__ void stage(const View& d, int gy0, int gx0, const void* src,
                                                 const void* dst, uint16_t* s_img, int tid)
    {
        stage_region<RH, RW, RWP, NT>(d, src, dst, gy0 - K, gx0 - K, s_img, tid);
    }

    // Interior of the staged tile to dst.
    static __device__ __forceinline__ void store(const View& d, int gy0, int gx0, const void* src,
                                                 void* dst, const uint16_t* s_img, int tid)
    {
        store_region<TH, TW, RWP, K, K, NT>(d, src, dst, gy0, gx0, s_img, tid);
    }

    // Runs nsteps parity steps on the tile staged by stage() (followed by a
    // barrier), starting at image step t0, and writes the interior to dst.  Returns the number of
    // interior lowerings (same value in every thread) and, in last_tau
    // (block-uniform), the last step index within the residency that lowered
    // an interior pixel (-1 if none).  Must be entered by all NT threads after
    // a barrier that ends the previous use of the shared arrays.
    //
    // A candidate is examined only when its 3x3 neighbourhood may have
    // changed since it was last examined (re-examination rule of section
    // 2.2): s_dirty starts at 1 everywhere (no history at staging), a
    // candidate clears its flag when examined, and a lowered pixel marks its
    // whole 3x3.  The decision is a function of the 3x3 only, so skipping
    // clean candidates changes nothing.  Within a step no candidate reads or
    // writes another candidate's flag: the 8 neighbours of a candidate belong
    // to other parity classes.
    //
    // With a Seed (sd != nullptr, round > 0) the flags start from history
    // instead: a candidate examined at step t0 + tau (tau < 4) was last
    // examined at step t0 + tau - 4, in the previous round, by the tile that
    // owned it (or earlier, by a tile that was then skipped because its
    // neighbourhood was quiet).  Only pixels lowered during the last 4 steps
    // of that round can have changed its 3x3 since, so the 3x3 of each such
    // pixel is marked.  The region lies inside the 3x3 tile block (K <= tile
    // side / 2), so the neighbours' bitmaps hold every pixel that matters.
    static __device__ __forceinline__ int run(const View d, int gy0, int gx0, int t0, int nsteps,
                              const void* src, void* dst, uint16_t* s_img, uint8_t* s_dirty,
                              uint32_t* s_bits, uint32_t* s_cw, const Seed* sd,
                              const TopoEntry* lut, int* s_count, int* s_last, int* s_exam,
                              int tid, int& last_tau)
    {
        const int ry0 = gy0 - K, rx0 = gx0 - K;
        const bool seeded = SEED && sd != nullptr && sd->r > 0;
        if (tid == 0) {
            *s_count = 0;
            *s_last = -1;
            *s_exam = 0;
        }
        if constexpr (SEED)
            for (int i = tid; i < TH * WPR; i += NT) s_bits[i] = 0u;
        if (!seeded) {
            uint32_t* f = reinterpret_cast<uint32_t*>(s_dirty);
            for (int i = tid; i < RH * RWP / 4; i += NT) f[i] = 0x01010101u;
        }
        __syncthreads();
        if constexpr (SEED) if (seeded) {
            // Change map of the region in 32-pixel words (row y, word j covers
            // region columns 32j..32j+31), gathered from the neighbours'
            // tile-aligned bitmaps with a funnel shift, then dilated by the 3x3
            // and expanded into the byte flags.
            for (int it = tid; it < RH * RWW; it += NT) {
                const int y = it / RWW, j = it - y * RWW;
                const int gi = ry0 + y;
                uint32_t word = 0u;
                if (gi >= 0 && gi < d.h) {
                    const int c0 = rx0 + 32 * j;                  // first global column
                    const int a = (c0 >= 0) ? (c0 >> 5) : -((31 - c0) >> 5);
                    const int sh = c0 - 32 * a;                   // 0..31
                    const uint32_t lo = history_word_t<TH, TW>(sd, gi, a);
                    const uint32_t hi = history_word_t<TH, TW>(sd, gi, a + 1);
                    word = sh ? ((lo >> sh) | (hi << (32 - sh))) : lo;
                }
                s_cw[it] = word;
            }
            __syncthreads();
            for (int it = tid; it < RH * RWW; it += NT) {
                const int y = it / RWW, j = it - y * RWW;
                uint32_t m = 0u;
                for (int dy = -1; dy <= 1; ++dy) {
                    const int yy = y + dy;
                    if (yy < 0 || yy >= RH) continue;
                    const uint32_t c = s_cw[yy * RWW + j];
                    const uint32_t l = j > 0 ? s_cw[yy * RWW + j - 1] : 0u;
                    const uint32_t r = j + 1 < RWW ? s_cw[yy * RWW + j + 1] : 0u;
                    m |= c | (c << 1) | (c >> 1) | (l >> 31) | (r << 31);
                }
                uint8_t* row = s_dirty + y * RWP + 32 * j;
                const int n = min(32, RW - 32 * j);
                for (int b = 0; b < n; ++b) row[b] = (uint8_t)((m >> b) & 1u);
            }
            __syncthreads();
        }

        const uint32_t lambda = d.lambda;
        int my_count = 0, my_last = -1;  // interior lowerings, last step with one
        int my_exams = 0;                // candidates characterised
        // Each thread owns fixed positions of the candidate lattice (one in
        // four pixels, rows and columns of the step's parity): the region's
        // origin is even (tile side and halo are even), so the candidate of
        // lattice cell (a, b) in class (si, sj) is region pixel
        // (2a + si, 2b + sj).  The exact region and the image interior only
        // mask cells out step by step.
        for (int tau = 0; tau < nsteps; ++tau) {
            const int s = (t0 + tau) & 3, si = s >> 1, sj = s & 1;
            // Exact region after tau steps, clipped to the image interior.
            const int r_lo = max(tau + 1, 1 - ry0), r_hi = min(RH - 2 - tau, d.h - 2 - ry0);
            const int c_lo = max(tau + 1, 1 - rx0), c_hi = min(RW - 2 - tau, d.w - 2 - rx0);
            bool inner = false;
            // The loop over the thread's cells stays rolled: unrolled, the
            // compiler interleaves cells and runs out of registers.
#pragma unroll 1
            for (int idx = tid; idx < LAT_H * LAT_W; idx += NT) {
                const int a = idx / LAT_W;
                const int lr = 2 * a + si, lc = 2 * (idx - a * LAT_W) + sj;
                if (lr < r_lo || lr > r_hi || lc < c_lo || lc > c_hi) continue;
                const int o = lr * RWP + lc;
                {
                    if (!s_dirty[o]) continue;
                    s_dirty[o] = 0;
                    ++my_exams;
                    uint16_t* p = s_img + o;
                    const uint32_t v = p[0];
                    const uint32_t nbv[8] = {p[1], p[-RWP + 1], p[-RWP], p[-RWP - 1],
                                             p[-1], p[RWP - 1], p[RWP], p[RWP + 1]};
                    uint32_t alpha;
                    if (decide<false>(v, nbv, lut, lambda, alpha)) {
                        p[0] = (uint16_t)alpha;
                        uint8_t* q = s_dirty + o;
                        q[-RWP - 1] = 1; q[-RWP] = 1; q[-RWP + 1] = 1;
                        q[-1] = 1;       q[0] = 1;    q[1] = 1;
                        q[RWP - 1] = 1;  q[RWP] = 1;  q[RWP + 1] = 1;
                        if (lr >= K && lr < K + TH && lc >= K && lc < K + TW) {
                            ++my_count;
                            inner = true;
                            if constexpr (SEED) {
                                if (tau >= nsteps - 4) {
                                    const int y = lr - K, x = lc - K;
                                    atomicOr(&s_bits[y * WPR + (x >> 5)], 1u << (x & 31));
                                }
                            }
                        }
                    }
                }
            }
            if (inner) my_last = tau;
            __syncthreads();
        }

        store(d, gy0, gx0, src, dst, s_img, tid);
        if (my_count) {
            atomicAdd(s_count, my_count);
            atomicMax(s_last, my_last);
        }
        if (my_exams) atomicAdd(s_exam, my_exams);
        __syncthreads();
        if constexpr (SEED) {
            if (sd != nullptr) {
                for (int i = tid; i < TH * WPR; i += NT)
                    sd->cur_bits[(int64_t)sd->g * TH * WPR + i] = s_bits[i];
                if (tid == 0) sd->cur_round[sd->g] = sd->r;
            }
        }
        last_tau = *s_last;
        return *s_count;
    }
};

// Residency with register windows.  Each thread owns fixed cells of the 2x2
// lattice of the region and keeps, per cell, the 4x4 window of pixels covered
// by the 3x3 neighbourhoods of the cell's four candidates (one per parity
// class).  A parity step changes only pixels of its class, which occupy four
// window positions, one of them the cell's own candidate; so before each
// step a thread re-reads from LDS the three positions of the previous step's
// class that belong to other cells.  A candidate is examined only when a
// pixel of its 3x3 changed since it was last examined (one bit per class and
// cell, set by re-read values that differ and by the cell's own lowerings):
// the re-examination rule of section 2.2, as in the flag variant.  LDS holds
// the whole region as the exchange medium between cells and as the source of
// the final interior store.
template <int TH, int TW, int K, int NT>
struct RTile {
    using Elem = uint16_t;
    static constexpr int RH = TH + 2 * K;
    static constexpr int RW = TW + 2 * K;
    static constexpr int RWP = RW + 2;                // a spare column on each side
    static constexpr int IMG_ELEMS = (RH + 2) * RWP;  // a spare row above and below
    static constexpr int DIRTY_ELEMS = 1;
    static constexpr int LAT_H = RH / 2, LAT_W = RW / 2;
    static constexpr int PPT = (LAT_H * LAT_W + NT - 1) / NT;  // lattice cells per thread
    static constexpr int WPR = 1, BITS_WORDS = 1, CW_WORDS = 1;
    static_assert(K % 4 == 0, "a residency must start at parity class 0");
    static_assert(K <= TH && K <= TW, "halo must not exceed the tile side");
    static_assert(TH % 2 == 0 && TW % 2 == 0, "tile sides must be even");

    // LDS index of region pixel (y, x), y in [-1, RH], x in [-1, RW].
    static __device__ __forceinline__ int at(int y, int x) { return (y + 1) * RWP + x + 1; }

    // Classes whose candidate's 3x3 contains window position (i, j); the
    // candidate of class (ci, cj) sits at (1 + ci, 1 + cj).
    static constexpr uint32_t affect(int i, int j)
    {
        uint32_t m = 0;
        for (int ci = 0; ci < 2; ++ci)
            for (int cj = 0; cj < 2; ++cj)
                if (ci <= i && i <= ci + 2 && cj <= j && j <= cj + 2) m |= 1u << (2 * ci + cj);
        return m;
    }


    // Tile and halo from src into s_img, spare rows and columns zeroed (they
    // are read into windows but never used by a candidate); no barrier.
    // Work a residency can start before the block knows whether the tile
    // runs (none for this type).
    static __device__ __forceinline__ void prefetch(const View&, int, int, const Seed*, uint8_t*,
                                                    uint32_t*, int)
    {
    }

    static __device__ __forceinline__ void stage(const View& d, int gy0, int gx0, const void* src,
                                                 const void*, uint16_t* s_img, int tid)
    {
        for (int i = tid; i < 2 * RWP + 2 * RH; i += NT) {
            int o;
            if (i < RWP) o = i;
            else if (i < 2 * RWP) o = (RH + 1) * RWP + (i - RWP);
            else if (i < 2 * RWP + RH) o = (i - 2 * RWP + 1) * RWP;
            else o = (i - 2 * RWP - RH + 1) * RWP + RWP - 1;
            s_img[o] = 0;
        }
        stage_scalar<RH, RW, RWP, 1, 1, NT>(d, src, gy0 - K, gx0 - K, s_img, tid);
    }

    static __device__ __forceinline__ void store(const View& d, int gy0, int gx0, const void* src,
                                                 void* dst, const uint16_t* s_img, int tid)
    {
        store_region<TH, TW, RWP, K + 1, K + 1, NT>(d, src, dst, gy0, gx0, s_img, tid);
    }

    struct Cells {
        uint32_t win[PPT][16];  // 4x4 windows, row-major
        int base[PPT];          // LDS index of window position (0, 0)
        int cr[PPT], cc[PPT];   // region position of the cell's (0,0) candidate
        uint32_t pend[PPT];     // bit c: the class-c candidate needs examining
    };

    // One parity step of class C (steps of a residency start at class 0).
    template <int C>
    static __device__ __forceinline__ void step(Cells& q, uint16_t* s_img, int tau, int r_lo,
                                                int r_hi, int c_lo, int c_hi,
                                                const TopoEntry* lut, uint32_t lambda,
                                                int& my_count, int& my_exams, bool& inner)
    {
        constexpr int si = C >> 1, sj = C & 1;
        constexpr int P = (C + 3) & 3, pi = P >> 1, pj = P & 1;
        if (tau > 0) {
            // Window rows of class-P pixels are 1 - pi and 3 - pi, columns
            // 1 - pj and 3 - pj; (1 + pi, 1 + pj) is the cell's own.
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
#pragma unroll
                for (int di = 0; di < 2; ++di) {
#pragma unroll
                    for (int dj = 0; dj < 2; ++dj) {
                        if (di == pi && dj == pj) continue;
                        const int i = 1 - pi + 2 * di, j = 1 - pj + 2 * dj;
                        const uint32_t nv = s_img[q.base[k] + i * RWP + j];
                        if (nv != q.win[k][4 * i + j]) {
                            q.win[k][4 * i + j] = nv;
                            q.pend[k] |= affect(i, j);
                        }
                    }
                }
            }
        }
        constexpr int ci = 1 + si, cj = 1 + sj;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int lr = q.cr[k] + si, lc = q.cc[k] + sj;
            if (lr < r_lo || lr > r_hi || lc < c_lo || lc > c_hi) continue;
            if (((q.pend[k] >> C) & 1u) == 0u) continue;
            q.pend[k] &= ~(1u << C);
            ++my_exams;
            uint32_t(&w)[16] = q.win[k];
            const uint32_t nb[8] = {w[4 * ci + cj + 1],       w[4 * (ci - 1) + cj + 1],
                                    w[4 * (ci - 1) + cj],     w[4 * (ci - 1) + cj - 1],
                                    w[4 * ci + cj - 1],       w[4 * (ci + 1) + cj - 1],
                                    w[4 * (ci + 1) + cj],     w[4 * (ci + 1) + cj + 1]};
            uint32_t alpha;
            if (decide<true>(w[4 * ci + cj], nb, lut, lambda, alpha)) {
                w[4 * ci + cj] = alpha;
                s_img[q.base[k] + ci * RWP + cj] = (uint16_t)alpha;
                q.pend[k] = 0xFu;
                if (lr >= K && lr < K + TH && lc >= K && lc < K + TW) {
                    ++my_count;
                    inner = true;
                }
            }
        }
    }

    template <int C>
    static __device__ __forceinline__ void full_step(Cells& q, const View& d, int ry0, int rx0,
                                                     uint16_t* s_img, int tau,
                                                     const TopoEntry* lut, int& my_last,
                                                     int& my_count, int& my_exams)
    {
        // Exact region after tau steps, clipped to the image interior.
        const int r_lo = max(tau + 1, 1 - ry0), r_hi = min(RH - 2 - tau, d.h - 2 - ry0);
        const int c_lo = max(tau + 1, 1 - rx0), c_hi = min(RW - 2 - tau, d.w - 2 - rx0);
        bool inner = false;
        step<C>(q, s_img, tau, r_lo, r_hi, c_lo, c_hi, lut, d.lambda, my_count, my_exams, inner);
        if (inner) my_last = tau;
        __syncthreads();
    }

    // Same contract as Tile::run (history arguments unused).
    static __device__ __forceinline__ int run(const View d, int gy0, int gx0, int t0, int nsteps,
                              const void* src, void* dst, uint16_t* s_img, uint8_t*, uint32_t*,
                              uint32_t*, const Seed*, const TopoEntry* lut, int* s_count,
                              int* s_last, int* s_exam, int tid, int& last_tau)
    {
        (void)t0;  // a multiple of 4: step tau has class tau mod 4
        const int ry0 = gy0 - K, rx0 = gx0 - K;
        if (tid == 0) {
            *s_count = 0;
            *s_last = -1;
            *s_exam = 0;
        }
        // The barrier after the windows are read also orders the counter
        // reset above before the steps' updates.
        Cells q;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int idx = tid + k * NT;
            const bool valid = idx < LAT_H * LAT_W;
            const int a = valid ? idx / LAT_W : 0, b = valid ? idx % LAT_W : 0;
            q.cr[k] = valid ? 2 * a : RH;  // RH: never in range
            q.cc[k] = 2 * b;
            q.base[k] = 2 * a * RWP + 2 * b;  // at(2a - 1, 2b - 1)
            q.pend[k] = 0xFu;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t* row = reinterpret_cast<const uint32_t*>(s_img + q.base[k] + i * RWP);
                const uint32_t w0 = row[0], w1 = row[1];
                q.win[k][4 * i + 0] = w0 & 0xFFFFu;
                q.win[k][4 * i + 1] = w0 >> 16;
                q.win[k][4 * i + 2] = w1 & 0xFFFFu;
                q.win[k][4 * i + 3] = w1 >> 16;
            }
        }
        __syncthreads();

        int my_count = 0, my_last = -1;  // interior lowerings, last step with one
        int my_exams = 0;                // candidates characterised
        for (int tau = 0; tau < nsteps; tau += 4) {
            full_step<0>(q, d, ry0, rx0, s_img, tau, lut, my_last, my_count, my_exams);
            if (tau + 1 < nsteps)
                full_step<1>(q, d, ry0, rx0, s_img, tau + 1, lut, my_last, my_count, my_exams);
            if (tau + 2 < nsteps)
                full_step<2>(q, d, ry0, rx0, s_img, tau + 2, lut, my_last, my_count, my_exams);
            if (tau + 3 < nsteps)
                full_step<3>(q, d, ry0, rx0, s_img, tau + 3, lut, my_last, my_count, my_exams);
        }

        store(d, gy0, gx0, src, dst, s_img, tid);
        if (my_count) {
            atomicAdd(s_count, my_count);
            atomicMax(s_last, my_last);
        }
        if (my_exams) atomicAdd(s_exam, my_exams);
        __syncthreads();
        last_tau = *s_last;
        return *s_count;
    }
};

// Inclusive prefix sum over the 64 lanes of a wave with DPP moves: shifts by
// 1, 2, 4 and 8 lanes within each row of 16, then the last lane of row 0 and
// of row 2 broadcast into the next row, then lane 31 into rows 2 and 3.
// Lanes a move cannot reach add the 0 kept in `old`.
__device__ __forceinline__ int wave_inclusive_sum(int v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return v;
}

// Residency with bit flags and dense work lists.  Two sets of bitmaps, one
// bit per lattice cell and parity class (4 x LAT_H rows of LWW words each):
// "pending" holds the candidates to examine from the residency's start (all
// ones, or with SEED from the previous round's change bitmaps), "lowered"
// holds, per class, the cells lowered by that class's latest step.  A step
// of class c needs the candidates whose 3x3 changed since their examination
// 4 steps earlier (section 2.2 re-examination rule): the cell itself if it
// was lowered then, and any pixel of its 3x3 lowered by the 3 steps since,
// one class each; the owner of each bitmap word gathers those from the
// lowered bitmaps with word shifts (pull), so a lowering costs one LDS
// atomic.  Every wave takes the candidates of its run of words (one word per
// lane) and writes them into a run of the step's list that it reserves with
// one LDS atomic, at offsets from a wave prefix sum; after one barrier the
// block examines the list densely, so clean candidates cost nothing beyond
// their share of one word.
// The seeded start: a candidate whose 3x3 saw none of the pixels lowered
// during the last 4 steps of round r - 1 (dilated by the 3x3) was examined 4
// steps earlier at the same values.
template <int TH, int TW, int K, int NT, bool SEED, typename E>
struct BTile {
    using Elem = E;  // LDS pixel type: the image's own
    static constexpr int RH = TH + 2 * K;
    static constexpr int RW = TW + 2 * K;
    static constexpr int RWP = RW;
    static constexpr int IMG_ELEMS = RH * RWP;
    static constexpr int LAT_H = RH / 2, LAT_W = RW / 2;
    static constexpr int NCELL = LAT_H * LAT_W;
    static constexpr int LWW = (LAT_W + 31) / 32;     // bitmap words per lattice row
    static constexpr int CLASS_WORDS = LAT_H * LWW;   // bitmap words per class
    static constexpr int NWAVE = NT / 64;
    // Bitmap words of a class are dealt to the waves in runs of WAVE_WORDS
    // (one per lane, whole lattice rows), so each wave's run of the list is
    // in raster order and neighbouring lanes examine neighbouring cells.
    static constexpr int WAVE_ROWS = (LAT_H + NWAVE - 1) / NWAVE;
    static constexpr int WAVE_WORDS = WAVE_ROWS * LWW;
    static constexpr int LIST_ELEMS = (NCELL + 1) & ~1;
    // LDS bytes behind the flag pointer: 4 pending bitmaps, 4 lowered
    // bitmaps, a ring of 8 list lengths and 8 "lowered" flags (by step),
    // 4 "has seeds" flags (by class), the step's list
    static constexpr int DIRTY_ELEMS = 32 * CLASS_WORDS + 32 + 16 + 2 * LIST_ELEMS;
    static constexpr int WPR = TW >= 32 ? TW / 32 : 1;
    static constexpr int RWW = (RW + 31) / 32;
    static constexpr int BITS_WORDS = SEED ? TH * WPR : 1;
    static constexpr int CW_WORDS = SEED ? RH * RWW : 1;
    static_assert(K % 4 == 0, "a residency must start at parity class 0");
    static_assert(K <= TH && K <= TW, "halo must not exceed the tile side");
    static_assert(TH % 4 == 0 && TW % 4 == 0, "tile sides must be multiples of 4");
    static_assert(NT % 64 == 0 && CLASS_WORDS <= NT, "one bitmap word per thread");
    static_assert(WAVE_WORDS <= 64, "one bitmap word per lane");
    static_assert(LWW + 1 <= 8, "reads one row and word past the lowered bitmaps stay in the ring");
    static_assert(LIST_ELEMS >= NT, "every thread may read the first list entry");
    static_assert(LAT_H <= 256 && LAT_W <= 256, "list entries hold a row and a column byte");
    static_assert(!SEED || TW % 32 == 0, "history bitmaps need a tile width multiple of 32");
    static_assert(!SEED || 2 * K <= TH, "history seeding needs the region inside the 3x3 tile block");


    // Everything a residency can start before the block knows whether the
    // tile runs, so that it overlaps the staging loads instead of following
    // them: the ring slots and flags, the cleared lowered bitmaps and, when
    // seeded, the previous round's change map of the region in 32-pixel
    // words (two dependent global reads per word).  None of it is read by the
    // previous tile's tail (which reads only the change bitmap s_bits and the
    // block counters, both set up after the decision).
    static __device__ __forceinline__ void prefetch(const View& d, int gy0, int gx0, const Seed* sd,
                                                    uint8_t* s_flags, uint32_t* s_cw, int tid)
    {
        uint32_t* s_dl = reinterpret_cast<uint32_t*>(s_flags) + 4 * CLASS_WORDS;
        int* s_total = reinterpret_cast<int*>(s_dl + 4 * CLASS_WORDS);
        uint8_t* s_low = reinterpret_cast<uint8_t*>(s_total + 8);
        uint8_t* s_seeds = s_low + 8;
        const bool seeded = SEED && sd != nullptr && sd->r > 0;
        for (int i = tid; i < 4 * CLASS_WORDS; i += NT) s_dl[i] = 0u;
        if (tid < 8) {
            s_total[tid] = 0;
            s_low[tid] = 0;
            s_seeds[tid] = seeded ? 0 : 1;
        }
        if constexpr (SEED) {
            if (seeded) {
                const int ry0 = gy0 - K, rx0 = gx0 - K;
                for (int it = tid; it < RH * RWW; it += NT) {
                    const int y = it / RWW, j = it - y * RWW;
                    const int gi = ry0 + y;
                    uint32_t word = 0u;
                    if (gi >= 0 && gi < d.h) {
                        const int c0 = rx0 + 32 * j;
                        const int a = (c0 >= 0) ? (c0 >> 5) : -((31 - c0) >> 5);
                        const int sh = c0 - 32 * a;
                        const uint32_t lo = history_word_t<TH, TW>(sd, gi, a);
                        const uint32_t hi = history_word_t<TH, TW>(sd, gi, a + 1);
                        word = sh ? ((lo >> sh) | (hi << (32 - sh))) : lo;
                    }
                    s_cw[it] = word;
                }
            }
        }
    }

    static __device__ __forceinline__ void stage(const View& d, int gy0, int gx0, const void* src,
                                                 const void* dst, E* s_img, int tid)
    {
        stage_native<E, RH, RW, RWP, NT>(d, src, dst, gy0 - K, gx0 - K, s_img, tid);
    }

    static __device__ __forceinline__ void store(const View& d, int gy0, int gx0, const void* src,
                                                 void* dst, const E* s_img, int tid)
    {
        store_native<E, TH, TW, RWP, K, K, NT>(d, src, dst, gy0, gx0, s_img, tid);
    }

    // Bits of lattice word j that exist (cells b < LAT_W).
    static __device__ __forceinline__ uint32_t valid_bits(int j)
    {
        constexpr int tail = LAT_W - 32 * (LWW - 1);
        return (j < LWW - 1 || tail == 32) ? ~0u : ((1u << tail) - 1u);
    }

    // Even bits of x packed into the low 16 bits.
    static __device__ __forceinline__ uint32_t even_bits(uint32_t x)
    {
        x &= 0x55555555u;
        x = (x | (x >> 1)) & 0x33333333u;
        x = (x | (x >> 2)) & 0x0F0F0F0Fu;
        x = (x | (x >> 4)) & 0x00FF00FFu;
        x = (x | (x >> 8)) & 0x0000FFFFu;
        return x;
    }

    // Same contract as Tile::run.
    static __device__ __forceinline__ int run(const View d, int gy0, int gx0, int t0, int nsteps,
                                              const void* src, void* dst, E* s_img,
                                              uint8_t* s_flags, uint32_t* s_bits, uint32_t* s_cw,
                                              const Seed* sd, const TopoEntry* lut, int* s_count,
                                              int* s_last, int* s_exam, int tid, int& last_tau)
    {
        (void)t0;  // a multiple of 4: step tau has class tau mod 4
        uint32_t* s_db = reinterpret_cast<uint32_t*>(s_flags);           // [4][LAT_H][LWW]
        uint32_t* s_dl = s_db + 4 * CLASS_WORDS;                         // [4][LAT_H][LWW]
        int* s_total = reinterpret_cast<int*>(s_dl + 4 * CLASS_WORDS);   // [8]: step tau & 7
        uint8_t* s_low = reinterpret_cast<uint8_t*>(s_total + 8);        // [8]: step tau & 7
        uint8_t* s_seeds = s_low + 8;                                    // [4]: class
        uint16_t* s_list = reinterpret_cast<uint16_t*>(s_seeds + 8);
        const int ry0 = gy0 - K, rx0 = gx0 - K;
        const bool seeded = SEED && sd != nullptr && sd->r > 0;
        if (tid == 0) {
            *s_count = 0;
            *s_last = -1;
            *s_exam = 0;
        }
        if constexpr (SEED)
            for (int i = tid; i < TH * WPR; i += NT) s_bits[i] = 0u;
        if (!seeded)
            for (int i = tid; i < 4 * CLASS_WORDS; i += NT) s_db[i] = valid_bits(i % LWW);
        if constexpr (SEED) if (seeded) {
            // Flag word j of class (si, sj) at lattice row a covers region
            // row 2a + si, columns 64j + sj + 2t (t < 32): the 3x3-dilated
            // changed map there, odd or even columns packed.
            for (int i = tid; i < 4 * CLASS_WORDS; i += NT) {
                const int c = i / CLASS_WORDS, rem = i - c * CLASS_WORDS;
                const int a = rem / LWW, j = rem - a * LWW;
                const int y = 2 * a + (c >> 1), sj = c & 1;
                // every read is unconditional (clamped into the map, the
                // value masked), so all of them go out together
                uint32_t half[2];
#pragma unroll
                for (int hw = 0; hw < 2; ++hw) {
                    const int w = 2 * j + hw;
                    const int wc = w < RWW ? w : RWW - 1;
                    const int wl = wc > 0 ? wc - 1 : 0, wr = wc + 1 < RWW ? wc + 1 : wc;
                    uint32_t m = 0u;
#pragma unroll
                    for (int dy = -1; dy <= 1; ++dy) {
                        const int yy = y + dy;
                        const int yc = yy < 0 ? 0 : (yy >= RH ? RH - 1 : yy);
                        const uint32_t cc = s_cw[yc * RWW + wc];
                        const uint32_t l = s_cw[yc * RWW + wl];
                        const uint32_t r = s_cw[yc * RWW + wr];
                        const uint32_t row = cc | (cc << 1) | (cc >> 1) | (wc > 0 ? l >> 31 : 0u) |
                                             (wc + 1 < RWW ? r << 31 : 0u);
                        m |= (yy >= 0 && yy < RH) ? row : 0u;
                    }
                    half[hw] = w < RWW ? even_bits(m >> sj) : 0u;
                }
                const uint32_t word = (half[0] | (half[1] << 16)) & valid_bits(j);
                s_db[i] = word;
                if (word) s_seeds[c] = 1;
            }
        }
        __syncthreads();

        const uint32_t lambda = d.lambda;
        const int wave = tid >> 6, lane = tid & 63;
        // The bitmap word this lane owns; lanes without one read a valid word
        // (the last) and take nothing.  Every read below is unconditional, so
        // a step's reads go out together: a word of a neighbouring row or
        // column outside the lattice reads some other word of the flag area
        // (they all lie inside it) and is masked to zero.
        const bool has_word = lane < WAVE_WORDS && wave * WAVE_WORDS + lane < CLASS_WORDS;
        const int myw = has_word ? wave * WAVE_WORDS + lane : CLASS_WORDS - 1;
        const int wa = myw / LWW, wj = myw - (myw / LWW) * LWW;
        const bool up_ok = wa > 0, dn_ok = wa + 1 < LAT_H, lt_ok = wj > 0, rt_ok = wj + 1 < LWW;
        const uint32_t* own_dl = s_dl + myw;  // word (wa, wj) of class 0's lowered bitmap
        int my_count = 0, my_last = -1;  // interior lowerings, last step with one
        int my_exams = 0;                // candidates characterised (thread 0 counts the lists)
        bool done = false;               // block-uniform: no later step can lower anything

        // One step of class C = tau mod 4.  A step's candidates come from the
        // residency's seeds (first 4 steps) and from pixels lowered during the
        // 4 steps before it.  When neither exists the step cannot lower
        // anything; once 4 steps in a row are quiet and the seeds are used up,
        // no later step of the residency can either.  The flags were written
        // before the last barrier, so every thread takes the same branch.  A
        // skipped step still clears the two ring slots it owns (its "lowered"
        // flag, and the list length of step tau + 4, whose last readers were
        // at step tau - 4).
        auto step = [&](auto cls, int tau) __attribute__((always_inline)) {
            constexpr int c = decltype(cls)::value, si = c >> 1, sj = c & 1;
            const uint64_t lw = *reinterpret_cast<const uint64_t*>(s_low);
            const bool seeds_c = s_seeds[c] != 0;
            // Candidates of this word: still pending from the residency's
            // start, lowered themselves 4 steps ago, or next to a pixel
            // lowered during the last 3 steps (the lowered bitmap of each
            // other class, spread over the cells whose 3x3 holds it: rows a
            // or a+-1 and columns b or b+-1 by parity).  Read before the quiet
            // test; in a quiet step every one of these words is zero.
            uint32_t want = s_db[c * CLASS_WORDS + myw] | own_dl[c * CLASS_WORDS];
#pragma unroll
            for (int k = 1; k < 4; ++k) {
                const int o = (c + k) & 3, oi = o >> 1, oj = o & 1;
                const uint32_t* bm = own_dl + o * CLASS_WORDS;  // word (wa, wj) of class o
                // rows of o next to row wa of c: wa itself when oi == si, else
                // wa - 1 and wa (oi > si) or wa and wa + 1 (oi < si)
                const int dr = oi > si ? -LWW : LWW;
                const bool r_ok = oi > si ? up_ok : dn_ok;
                uint32_t w0 = bm[0], prev = 0u, next = 0u;
                if (oj > sj) prev = bm[-1];
                if (oj < sj) next = bm[1];
                if (oi != si) {
                    const uint32_t x0 = bm[dr];
                    const uint32_t xp = oj > sj ? bm[dr - 1] : 0u;
                    const uint32_t xn = oj < sj ? bm[dr + 1] : 0u;
                    w0 |= r_ok ? x0 : 0u;
                    prev |= r_ok ? xp : 0u;
                    next |= r_ok ? xn : 0u;
                }
                if (oj == sj) {
                    want |= w0;
                } else if (oj > sj) {  // cells b - 1 and b
                    want |= w0 | (w0 << 1) | ((lt_ok ? prev : 0u) >> 31);
                } else {               // cells b and b + 1
                    want |= w0 | (w0 >> 1) | ((rt_ok ? next : 0u) << 31);
                }
            }
            {
                const int sh = 8 * ((tau + 4) & 7);  // slots tau-4 .. tau-1, in ring order
                const uint64_t rot = sh ? ((lw >> sh) | (lw << (64 - sh))) : lw;
                const uint64_t recent = rot & 0xFFFFFFFFull;
                if (recent == 0ull && !(tau < 4 && seeds_c)) {
                    if (tau >= 4) {
                        done = true;
                        return;
                    }
                    if (tid == 0) {
                        s_low[tau & 7] = 0;
                        s_total[(tau + 4) & 7] = 0;
                    }
                    return;
                }
            }
            if (tid == 0) s_low[tau & 7] = 0;
            if (has_word) {
                s_db[c * CLASS_WORDS + myw] = 0u;
                s_dl[c * CLASS_WORDS + myw] = 0u;
            }
            // Exact region after tau steps, clipped to the image interior,
            // as lattice rows a (region row 2a + si) and columns b (2b + sj).
            const int r_lo = max(tau + 1, 1 - ry0), r_hi = min(RH - 2 - tau, d.h - 2 - ry0);
            const int c_lo = max(tau + 1, 1 - rx0), c_hi = min(RW - 2 - tau, d.w - 2 - rx0);
            const int a_lo = (r_lo - si + 1) >> 1, a_hi = (r_hi - si) >> 1;
            const int b_lo = (c_lo - sj + 1) >> 1, b_hi = (c_hi - sj) >> 1;
            uint32_t take = 0u;
            {
                const int lo = max(b_lo - 32 * wj, 0), hi = min(b_hi - 32 * wj, 31);
                if (has_word && wa >= a_lo && wa <= a_hi && lo <= hi) {
                    const uint32_t mask = (hi == 31 ? ~0u : ((2u << hi) - 1u)) & ~((1u << lo) - 1u);
                    take = want & mask;
                }
            }
            // Each wave reserves a run of the step's list with one LDS atomic
            // (the counter of the other parity was read a step ago and is
            // cleared for the next step while this one is examined).
            const int cnt = __popc(take);
            const int incl = wave_inclusive_sum(cnt);
            const int wave_total = __builtin_amdgcn_readlane(incl, 63);
            int base = 0;
            if (lane == 63 && wave_total) base = atomicAdd(&s_total[tau & 7], wave_total);
            base = __builtin_amdgcn_readlane(base, 63);
            if (take) {
                int off = base + incl - cnt;
                uint32_t t = take;
                while (t) {
                    // entry: lattice row in the high byte, column in the low
                    s_list[off++] = (uint16_t)((wa << 8) | (32 * wj + __ffs(t) - 1));
                    t &= t - 1u;
                }
            }
            __syncthreads();
            // the first entry is read with the length (it is in the list
            // whenever tid < total)
            const int total = s_total[tau & 7];
            int next_cell = s_list[tid];
            if (tid == 0) {
                s_total[(tau + 4) & 7] = 0;
                my_exams += total;
            }
            bool inner = false, lowered = false;
            for (int i = tid; i < total; i += NT) {
                const int cell = next_cell;
                if (i + NT < total) next_cell = s_list[i + NT];
                const int a = cell >> 8, b = cell & 0xFF;
                const int lr = 2 * a + si, lc = 2 * b + sj;
                E* p = s_img + lr * RWP + lc;
                const uint32_t v = p[0];
                const uint32_t nbv[8] = {p[1], p[-RWP + 1], p[-RWP], p[-RWP - 1],
                                         p[-1], p[RWP - 1], p[RWP], p[RWP + 1]};
                uint32_t alpha;
                if (decide<true>(v, nbv, lut, lambda, alpha)) {
                    p[0] = (E)alpha;
                    lowered = true;
                    atomicOr(&s_dl[c * CLASS_WORDS + a * LWW + (b >> 5)], 1u << (b & 31));
                    if (lr >= K && lr < K + TH && lc >= K && lc < K + TW) {
                        ++my_count;
                        inner = true;
                        if constexpr (SEED) {
                            if (tau >= nsteps - 4) {
                                const int y = lr - K, x = lc - K;
                                atomicOr(&s_bits[y * WPR + (x >> 5)], 1u << (x & 31));
                            }
                        }
                    }
                }
            }
            // one store per wave (the lanes would all write the same byte)
            if (__ballot(lowered) != 0ull && lane == 0) s_low[tau & 7] = 1;
            if (inner) my_last = tau;
            __syncthreads();
        };
        using C0 = std::integral_constant<int, 0>;
        using C1 = std::integral_constant<int, 1>;
        using C2 = std::integral_constant<int, 2>;
        using C3 = std::integral_constant<int, 3>;
        for (int tau = 0; tau < nsteps && !done; tau += 4) {
            step(C0{}, tau);
            if (tau + 1 < nsteps && !done) step(C1{}, tau + 1);
            if (tau + 2 < nsteps && !done) step(C2{}, tau + 2);
            if (tau + 3 < nsteps && !done) step(C3{}, tau + 3);
        }

        store(d, gy0, gx0, src, dst, s_img, tid);
        if (my_count) {
            atomicAdd(s_count, my_count);
            atomicMax(s_last, my_last);
        }
        if (my_exams) atomicAdd(s_exam, my_exams);
        __syncthreads();
        if constexpr (SEED) {
            if (sd != nullptr) {
                for (int i = tid; i < TH * WPR; i += NT)
                    sd->cur_bits[(int64_t)sd->g * TH * WPR + i] = s_bits[i];
                if (tid == 0) sd->cur_round[sd->g] = sd->r;
            }
        }
        last_tau = *s_last;
        return *s_count;
    }
};

// Residency type of a variant; E is the LDS pixel type of the bit-flag
// variants (the other variants keep u16).
template <int TH, int TW, int K, int NT, int VAR, typename E = uint16_t>
using TileOf = typename std::conditional<
    VAR == kVarRegs, RTile<TH, TW, K, NT>,
    typename std::conditional<VAR == kVarBits || VAR == kVarBitsSeeded,
                              BTile<TH, TW, K, NT, VAR == kVarBitsSeeded, E>,
                              Tile<TH, TW, K, NT, VAR == kVarSeeded>>::type>::type;

// Waves per SIMD that the LDS of one residency of T allows (blocks per CU
// times waves per block over the 4 SIMDs).  The large bit-flag tiles of the
// batched path ask the compiler to fit their registers to it, so that
// register growth never costs them a resident block (their register needs
// sit just under that budget); the other shapes need more registers than
// their LDS occupancy would leave them, and ask for nothing (1).
template <typename T, int NT, int TH, int VAR>
constexpr int lds_waves_per_eu()
{
    if constexpr (!(TH >= 128 && (VAR == kVarBits || VAR == kVarBitsSeeded))) return 1;
    constexpr int lds = (int)sizeof(typename T::Elem) * T::IMG_ELEMS + T::DIRTY_ELEMS +
                        4 * T::BITS_WORDS + 4 * T::CW_WORDS + (int)sizeof(TopoEntry) * 256 + 64;
    constexpr int by_lds = (160 * 1024) / lds;
    constexpr int by_threads = 2048 / NT;
    constexpr int blocks = by_lds < by_threads ? by_lds : by_threads;
    constexpr int w = (blocks < 1 ? 1 : blocks) * (NT / 64) / 4;
    return w < 1 ? 1 : (w > 8 ? 8 : w);
}

// ----------------------------------------------------------------- k_round

// One tile of one round (launch-per-round and cooperative engines).
// Returns 1 when the tile was processed (active), 0 when skipped.  All NT
// threads must call it together.
// Queues tile g for launch round `next` (once per round).
__device__ __forceinline__ void enqueue(const WorkList& wl, int g, int next)
{
    if (atomicMax(&wl.listed[g], next) < next) {
        const int pos = atomicAdd(&wl.count[next % 3], 1);
        wl.list[(next & 1) * wl.cap + pos] = g;
    }
}

template <int TH, int TW, int K, int NT, int VAR, typename E>
__device__ __forceinline__ int round_tile(const ImgDev* __restrict__ imgs, ImgCnt* cnt,
                          const int32_t* __restrict__ tile_img, int32_t* tile_state, int g,
                          int round, int ntiles, uint32_t* hist_bits, int32_t* hist_round,
                          typename TileOf<TH, TW, K, NT, VAR, E>::Elem* s_img, uint8_t* s_dirty,
                          uint32_t* s_bits, uint32_t* s_cw, const TopoEntry* __restrict__ lut_g,
                          TopoEntry* s_lut, int& lut_adj, int* s_count, int* s_last,
                          int* s_exam, const WorkList& wl, int kflags)
{
    using T = TileOf<TH, TW, K, NT, VAR, E>;
    const int tid = threadIdx.x;
    const int ii = (kflags & kOneImage) ? 0 : tile_img[g];
    const ImgDev* d = imgs + ii;
    // A tile that is not this launch's returns at once; the barrier keeps the
    // block's tile hand-out (written by thread 0 before the tile, read by all
    // after it) ordered as a visited tile's barriers do.  Every condition
    // here is the same for the whole block.
    if (((kflags & kOnlyU8) && d->dtype != 1) || ((kflags & kOnlyU16) && d->dtype != 2)) {
        __syncthreads();
        return 0;
    }
    const int r = round - d->round0;
    if (r < 0) {
        __syncthreads();
        return 0;
    }
    const int t0 = r * K;
    const int nsteps = min(K, d->max_steps - t0);
    if (nsteps <= 0) {
        __syncthreads();
        return 0;
    }
    const int lt = g - d->tile0;
    const int ty = lt / d->tiles_x, tx = lt - ty * d->tiles_x;
    const int slot = d->slot;
    // this tile's state pair
    int32_t* st = tile_state + 2 * ((kflags & kStateIsTile) ? (int64_t)g : d->state0 + lt);

    // tile_state[2g] is the latest round for which a tile of g's 3x3 tile
    // neighbourhood asked g to be active (it lowered something during the
    // last 4 steps of the round before); tile_state[2g + 1] is the last round
    // in which g itself lowered something.  Neighbours of this round may raise
    // tile_state[2g] to r + 1 while it is read here (only adding work), so one
    // thread decides and the barrier broadcasts a block-uniform answer.  The
    // tile is staged (and the residency's set-up started) before the answer
    // is known, so its loads overlap the state read; the barrier also
    // completes the staging and orders it after the previous tile's readers
    // of LDS.
    int act = 0, chg = 0;
    if (tid == 0) {
        act = __hip_atomic_load(&st[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        chg = __hip_atomic_load(&st[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const void* src = round_src(d, r);
    void* dst = round_dst(d, r);
    const int gy0 = ty * TH, gx0 = tx * TW;
    const View v = view_of(d);
    if (d->adj != lut_adj) {
        // The block's table follows the image's pairing; the previous tile's
        // readers are past its last barrier, and the decision barrier below
        // orders these writes before this tile's steps.
        lut_adj = d->adj;
        for (int i = tid; i < 256; i += NT) s_lut[i] = lut_g[lut_adj * 256 + i];
    }
    Seed sd{};
    const int64_t words = var_seeded(VAR) ? (int64_t)ntiles * TH * T::WPR : 0;
    sd.prev_bits = hist_bits + ((r + 1) & 1) * words;
    sd.prev_round = hist_round + ((r + 1) & 1) * ntiles;
    sd.cur_bits = hist_bits + (r & 1) * words;
    sd.cur_round = hist_round + (r & 1) * ntiles;
    sd.r = r;
    sd.tile0 = d->tile0;
    sd.tiles_x = d->tiles_x;
    sd.tiles_y = d->tiles_y;
    sd.ty = ty;
    sd.tx = tx;
    sd.g = g;
    T::stage(v, gy0, gx0, src, dst, s_img, tid);
    T::prefetch(v, gy0, gx0, var_seeded(VAR) ? &sd : nullptr, s_dirty, s_cw, tid);
    const int vote = tid == 0 ? ((r == 0 || act >= r) ? 1 : (chg == r - 1 ? 2 : 0)) : 0;
    const int decision = __syncthreads_or(vote == 1) ? 1 : (__syncthreads_or(vote == 2) ? 2 : 0);
    if (decision != 1) {
        // Stable for this round.  The output buffer already equals the input
        // unless the tile changed during the previous round.
        if (decision == 2) {
            T::store(v, gy0, gx0, src, dst, s_img, tid);
            __syncthreads();  // the next tile's staging overwrites s_img
        }
        return 0;
    }
    int last_tau;
    const int count = T::run(v, gy0, gx0, t0, nsteps, src, dst, s_img, s_dirty, s_bits, s_cw,
                             var_seeded(VAR) ? &sd : nullptr, s_lut, s_count, s_last, s_exam,
                             tid, last_tau);
    // Counters and the tiles the next round must visit, from the lanes of
    // wave 0 in parallel (one lane per tile of the 3x3 tile block), so the
    // block's next tile is not held up by a chain of dependent atomics.
    if (tid < 64) {
        if (tid == 0) {
            atomicAdd(&cnt[slot].tile_rounds, 1ull);
            atomicAdd(&cnt[slot].examinations, (unsigned long long)*s_exam);
            if (last_tau >= 0) {
                __hip_atomic_store(&st[1], r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                atomicAdd(&cnt[slot].lowerings, (unsigned long long)count);
                atomicMax(&cnt[slot].last_step, t0 + last_tau);
            }
        }
        // Lowered during the last 4 steps: the tile and those of its 8
        // neighbours within reach must run the next round.  Only pixels next
        // to a pixel lowered during the last 4 steps can be pending, and a
        // change travels at most one pixel per step, so in the next K steps
        // a neighbour's interior can change only if one of those lowerings
        // lies within K of it; a tile none of whose 3x3 tile block is within
        // reach cannot change (K <= tile side).  The seeded variants know
        // where those lowerings are (their change bitmap): wave 0 takes the
        // bounding box and spares the neighbours beyond K + 1 (one pixel of
        // margin); the others ask the whole 3x3 block.  Lowered earlier: the
        // tile itself is visited again (to copy itself across the ping-pong
        // pair).
        if (last_tau >= nsteps - 4) {
            uint32_t ask = 0x1FFu;  // bit 3 (dy + 1) + (dx + 1)
            if constexpr (var_seeded(VAR)) {
                if (nsteps >= 4) {
                    int rmin = TH, rmax = -1, cmin = TW, cmax = -1;
                    for (int i = tid; i < TH * T::WPR; i += 64) {
                        const uint32_t w = s_bits[i];
                        if (!w) continue;
                        const int row = i / T::WPR, c0 = 32 * (i - row * T::WPR);
                        rmin = min(rmin, row);
                        rmax = max(rmax, row);
                        cmin = min(cmin, c0 + __ffs(w) - 1);
                        cmax = max(cmax, c0 + 31 - __clz(w));
                    }
#pragma unroll
                    for (int o = 32; o >= 1; o >>= 1) {
                        rmin = min(rmin, __shfl_xor(rmin, o));
                        rmax = max(rmax, __shfl_xor(rmax, o));
                        cmin = min(cmin, __shfl_xor(cmin, o));
                        cmax = max(cmax, __shfl_xor(cmax, o));
                    }
                    if (rmax >= 0) {
                        constexpr int REACH = K + 1;
                        const bool up = rmin <= REACH, down = rmax >= TH - 1 - REACH;
                        const bool left = cmin <= REACH, right = cmax >= TW - 1 - REACH;
                        const uint32_t rows = (up ? 1u : 0u) | 2u | (down ? 4u : 0u);
                        const uint32_t cols = (left ? 1u : 0u) | 2u | (right ? 4u : 0u);
                        ask = 0u;
#pragma unroll
                        for (int q = 0; q < 9; ++q)
                            if (((rows >> (q / 3)) & 1u) && ((cols >> (q % 3)) & 1u)) ask |= 1u << q;
                    }
                }
            }
            if (tid < 9 && ((ask >> tid) & 1u)) {
                const int y = ty + tid / 3 - 1, x = tx + tid % 3 - 1;
                if (y >= 0 && y < d->tiles_y && x >= 0 && x < d->tiles_x) {
                    __hip_atomic_fetch_max(&tile_state[2 * (d->state0 + y * d->tiles_x + x)],
                                           r + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (wl.list != nullptr) enqueue(wl, d->tile0 + y * d->tiles_x + x, round + 1);
                }
            }
        } else if (last_tau >= 0 && tid == 0 && wl.list != nullptr) {
            enqueue(wl, g, round + 1);
        }
    }
    return 1;
}

template <int TH, int TW, int K, int NT, int VAR, typename E>
__global__ __attribute__((amdgpu_flat_work_group_size(1, NT),
                          amdgpu_waves_per_eu(lds_waves_per_eu<TileOf<TH, TW, K, NT, VAR, E>, NT, TH, VAR>())))
void k_round(const ImgDev* __restrict__ imgs, ImgCnt* cnt,
                                              const int32_t* __restrict__ tile_img,
                                              int32_t* tile_last, int ntiles, int round,
                                              const TopoEntry* __restrict__ lut_g,
                                              uint32_t* hist_bits, int32_t* hist_round,
                                              WorkList wl, const int32_t* round_base,
                                              int kflags)
{
    using T = TileOf<TH, TW, K, NT, VAR, E>;
    if (round_base != nullptr) round += *round_base;
    __shared__ __align__(16) typename T::Elem s_img[T::IMG_ELEMS];
    __shared__ __align__(16) uint8_t s_dirty[T::DIRTY_ELEMS];
    __shared__ uint32_t s_bits[T::BITS_WORDS];
    __shared__ uint32_t s_cw[T::CW_WORDS];
    __shared__ TopoEntry s_lut[256];
    __shared__ int s_count, s_last, s_exam;
    int lut_adj = -1;
    const bool all = wl.list == nullptr || round == wl.full;
    const int n = all ? ntiles : wl.count[round % 3];
    if (wl.list != nullptr && blockIdx.x == 0 && threadIdx.x == 0) {
        wl.count[(round + 2) % 3] = 0;
        wl.grab[2 * ((round + 2) % 3)] = 0;
        wl.grab[2 * ((round + 2) % 3) + 1] = 0;
    }
    const int32_t* mine = all ? nullptr : wl.list + (round & 1) * wl.cap;
    // Each block takes its first tile by its index and every later one from
    // a counter shared by the round's blocks, so blocks that drew cheap
    // tiles take more of them (tiles differ widely in cost: partial tiles
    // at image borders, quiet ones that are skipped).  Thread 0 claims the
    // next position while the current tile runs; two slots, so that a slot
    // is written again only after every thread has passed a barrier of the
    // tile in between.  The u8 and u16 launches of one round draw from
    // counters of their own.
    __shared__ int s_next[2];
    int32_t* grab = wl.list != nullptr ? wl.grab + 2 * (round % 3) + ((kflags & kOnlyU16) ? 1 : 0)
                                       : nullptr;
    int i = blockIdx.x;
    for (int k = 0; i < n; ++k) {
        if (threadIdx.x == 0)
            s_next[k & 1] = grab ? (int)gridDim.x + atomicAdd(grab, 1) : i + (int)gridDim.x;
        round_tile<TH, TW, K, NT, VAR, E>(imgs, cnt, tile_img, tile_last, all ? i : mine[i], round,
                                          ntiles, hist_bits, hist_round, s_img, s_dirty, s_bits,
                                          s_cw, lut_g, s_lut, lut_adj, &s_count, &s_last, &s_exam,
                                          wl, kflags);
        i = s_next[k & 1];
    }
}

// ------------------------------------------------------------------ k_coop
//
// All rounds in one cooperative launch (every block resident): each round
// processes the tile list like k_round, then the whole grid synchronises.
// active[round % 3] counts the tiles processed in a round; a round in which
// no tile was active means every image is stable (a tile is skipped only when
// its neighbourhood was quiet for the last 4 steps), so all blocks leave
// together.  The counter of round r is read by every block right after the
// grid barrier of round r and is cleared during round r + 2, after the next
// barrier has proved those reads complete.

template <int TH, int TW, int K, int NT, int VAR, typename E>
__global__ __attribute__((amdgpu_flat_work_group_size(1, NT),
                          amdgpu_waves_per_eu(lds_waves_per_eu<TileOf<TH, TW, K, NT, VAR, E>, NT, TH, VAR>())))
void k_coop(const ImgDev* __restrict__ imgs, ImgCnt* cnt,
                                             const int32_t* __restrict__ tile_img,
                                             int32_t* tile_last, int ntiles,
                                             const TopoEntry* __restrict__ lut_g, int32_t* active,
                                             int32_t* rounds_out, int max_rounds,
                                             uint32_t* hist_bits, int32_t* hist_round, int kflags)
{
    using T = TileOf<TH, TW, K, NT, VAR, E>;
    __shared__ __align__(16) typename T::Elem s_img[T::IMG_ELEMS];
    __shared__ __align__(16) uint8_t s_dirty[T::DIRTY_ELEMS];
    __shared__ uint32_t s_bits[T::BITS_WORDS];
    __shared__ uint32_t s_cw[T::CW_WORDS];
    __shared__ TopoEntry s_lut[256];
    __shared__ int s_count, s_last, s_exam;
    const int tid = threadIdx.x;
    int lut_adj = -1;
    cooperative_groups::grid_group grid = cooperative_groups::this_grid();
    int round = 0;
    for (;; ++round) {
        if (blockIdx.x == 0 && tid == 0)
            __hip_atomic_store(&active[(round + 1) % 3], 0, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        int mine = 0;
        for (int g = blockIdx.x; g < ntiles; g += gridDim.x)
            mine += round_tile<TH, TW, K, NT, VAR, E>(imgs, cnt, tile_img, tile_last, g, round,
                                                 ntiles, hist_bits, hist_round, s_img, s_dirty,
                                                 s_bits, s_cw, lut_g, s_lut, lut_adj, &s_count,
                                                 &s_last, &s_exam, WorkList{}, kflags);
        if (tid == 0 && mine) atomicAdd(&active[round % 3], mine);
        // Stores of every wave must be acknowledged before the grid barrier
        // publishes them.
        __builtin_amdgcn_s_waitcnt(0);
        grid.sync();
        const int a = __hip_atomic_load(&active[round % 3], __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
        if (a == 0 || round + 1 >= max_rounds) break;
    }
    if (blockIdx.x == 0 && tid == 0) *rounds_out = round + 1;
}

template <int TH, int TW, int K, int NT, int VAR, typename E>
hipError_t launch_coop_t(hipStream_t stream, const ImgDev* imgs, ImgCnt* cnt,
                         const int32_t* tile_img, int32_t* tile_last, int ntiles,
                         const TopoEntry* lut, int32_t* active, int32_t* rounds_out,
                         int max_rounds, int num_cus, uint32_t* hist_bits, int32_t* hist_round,
                         int kflags)
{
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, reinterpret_cast<const void*>(&k_coop<TH, TW, K, NT, VAR, E>), NT, 0);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    const int grid = max(1, min(ntiles, per_cu * num_cus));
    void* args[] = {(void*)&imgs,       (void*)&cnt,       (void*)&tile_img,
                    (void*)&tile_last,  (void*)&ntiles,    (void*)&lut,
                    (void*)&active,     (void*)&rounds_out, (void*)&max_rounds,
                    (void*)&hist_bits,  (void*)&hist_round, (void*)&kflags};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_coop<TH, TW, K, NT, VAR, E>),
                                      dim3(grid), dim3(NT), args, 0, stream);
}

template <int TH, int TW, int K, int NT, int VAR, typename E>
hipError_t launch_round_t(hipStream_t stream, const ImgDev* imgs, ImgCnt* cnt,
                          const int32_t* tile_img, int32_t* tile_last, int ntiles, int round,
                          const TopoEntry* lut, int num_cus, uint32_t* hist_bits,
                          int32_t* hist_round, WorkList wl, const int32_t* round_base, int kflags)
{
    // As many blocks as fit on the device at once (registers, LDS and thread
    // slots of this instantiation), each looping over the tiles.
    static int per_cu = 0;
    if (per_cu == 0) {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &n, reinterpret_cast<const void*>(&k_round<TH, TW, K, NT, VAR, E>), NT, 0) !=
                hipSuccess ||
            n < 1)
            n = 1;
        per_cu = n;
    }
    const int grid = max(1, min(ntiles, per_cu * num_cus));
    hipLaunchKernelGGL((k_round<TH, TW, K, NT, VAR, E>), dim3(grid), dim3(NT), 0, stream, imgs, cnt,
                       tile_img, tile_last, ntiles, round, lut, hist_bits, hist_round, wl,
                       round_base, kflags);
    return hipGetLastError();
}

// -------------------------------------------------------------- k_worklist
//
// The re-examination rule of section 2.2 as explicit per-class candidate
// lists.  A candidate is pending when a pixel of its 3x3 (itself included)
// was lowered since its last examination; the visit of its class examines
// every pending candidate of that class once and clears it; a lowered pixel
// marks its 3x3 pending (one bit per lattice cell and class, set with an
// atomic so each cell enters its class's list once).  The class being
// visited receives no marks from its own step except the lowered pixels
// themselves, which become the next list of that class.  Started with every
// interior candidate pending, the engine examines exactly the candidates
// the sequential dirty-pixel sweep examines.
//
// Lists hold (lattice row << 16) | lattice column and live in LDS; a list
// that overflows is dropped and its class's next visit scans the bitmap
// instead (the bitmap is always exact).  The pending bitmaps stay in LDS when
// they fit, else in global memory.  One block of kWlThreads threads per image;
// two barriers per step.

// Pending-bitmap access of k_worklist.  In global memory the words are read
// and written with device-scope atomics, which go to L2 like the bit-setting
// atomics, so no wave reads a stale copy from its CU's L1.
template <bool GBITS>
__device__ __forceinline__ uint32_t wl_load(uint32_t* w)
{
    if constexpr (GBITS) return __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else return *w;
}
template <bool GBITS>
__device__ __forceinline__ void wl_store(uint32_t* w, uint32_t v)
{
    if constexpr (GBITS) __hip_atomic_store(w, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else *w = v;
}
template <bool GBITS>
__device__ __forceinline__ uint32_t wl_or(uint32_t* w, uint32_t m)
{
    if constexpr (GBITS) return __hip_atomic_fetch_or(w, m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else return atomicOr(w, m);
}
template <bool GBITS>
__device__ __forceinline__ void wl_and(uint32_t* w, uint32_t m)
{
    if constexpr (GBITS) __hip_atomic_fetch_and(w, m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else atomicAnd(w, m);
}

template <typename E, bool GBITS>
__global__ __launch_bounds__(kWlThreads) void k_worklist(const WlImg* __restrict__ imgs,
                                                       ImgCnt* cnt,
                                                       const TopoEntry* __restrict__ lut_g,
                                                       int32_t* steps_out)
{
    __shared__ TopoEntry s_lut[256];
    __shared__ uint32_t s_lbits[GBITS ? 1 : kWlLdsWords];
    __shared__ uint32_t s_list[5][kWlListCap];
    __shared__ int s_n[5], s_ovf[5], s_map[4];
    __shared__ int s_j, s_low, s_quiet, s_step, s_last;
    __shared__ unsigned long long s_exam, s_lowsum;
    const int tid = threadIdx.x;
    const WlImg im = imgs[blockIdx.x];
    E* img = static_cast<E*>(im.image);
    const int64_t P = im.pitch;
    const int H = im.h, W = im.w;
    const int LH = (H + 1) / 2, LW = (W + 1) / 2, LWW = (LW + 31) / 32, CW = LH * LWW;
    uint32_t* bits = GBITS ? im.gbits : s_lbits;
    for (int i = tid; i < 256; i += kWlThreads) s_lut[i] = lut_g[im.adj * 256 + i];
    if (tid < 5) {
        s_n[tid] = 0;
        s_ovf[tid] = 1;   // first visit of each class scans its bitmap
    }
    if (tid < 4) s_map[tid] = tid;
    if (tid == 0) {
        s_j = 4;
        s_low = 0;
        s_quiet = 0;
        s_step = im.step0;
        s_last = -1;
        s_exam = 0ull;
        s_lowsum = 0ull;
    }
    // Initial pending sets.  Cell (a, b) of class (si, sj) is pixel
    // (2a + si, 2b + sj); only interior pixels are ever pending.  With init 1
    // a candidate is pending when a pixel of its 3x3 differs from the state
    // one tiled round earlier: a pixel-change bitmap (1 bit per pixel, rows of
    // DW words) is built first, in the list storage while it is unused when
    // it fits there.
    const int DW = (W + 31) / 32;
    uint32_t* dmap = &s_list[0][0];
    const bool dfast = im.init == 1 && H * DW <= 5 * kWlListCap;
    if (dfast) {
        const E* prev = static_cast<const E*>(im.prev);
        for (int wd = tid; wd < H * DW; wd += kWlThreads) {
            const int y = wd / DW, x0 = 32 * (wd - y * DW);
            const E* ra = img + (int64_t)y * P + x0;
            const E* rb = prev + (int64_t)y * P + x0;
            const int nx = min(32, W - x0);
            uint32_t m = 0u;
            for (int t = 0; t < nx; ++t) m |= (uint32_t)(ra[t] != rb[t]) << t;
            dmap[wd] = m;
        }
        __syncthreads();
    }
    for (int wd = tid; wd < 4 * CW; wd += kWlThreads) {
        const int c = wd / CW, rem = wd - c * CW;
        const int a = rem / LWW, j0 = 32 * (rem - a * LWW);
        const int i = 2 * a + (c >> 1);
        uint32_t word = 0u;
        if (i >= 1 && i <= H - 2) {
            for (int t = 0; t < 32; ++t) {
                const int j = 2 * (j0 + t) + (c & 1);
                if (j < 1 || j > W - 2) continue;
                bool pend = true;
                if (dfast) {
                    pend = false;
                    for (int di = -1; di <= 1; ++di) {
                        const uint32_t* row = dmap + (i + di) * DW;
                        for (int dj = -1; dj <= 1; ++dj) {
                            const int x = j + dj;
                            pend |= ((row[x >> 5] >> (x & 31)) & 1u) != 0u;
                        }
                    }
                } else if (im.init == 1) {
                    const E* prev = static_cast<const E*>(im.prev);
                    pend = false;
                    for (int di = -1; di <= 1 && !pend; ++di)
                        for (int dj = -1; dj <= 1; ++dj) {
                            const int64_t o = (int64_t)(i + di) * P + (j + dj);
                            if (img[o] != prev[o]) {
                                pend = true;
                                break;
                            }
                        }
                }
                if (pend) word |= 1u << t;
            }
        }
        wl_store<GBITS>(&bits[wd], word);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    const uint32_t lambda = im.lambda;
    unsigned long long my_exam = 0ull;
    for (;;) {
        const int t = s_step;
        if (s_quiet >= 4 || t >= im.max_steps) break;
        const int c = t & 3, si = c >> 1, sj = c & 1;
        const int L = s_map[c], J = s_j;
        const bool scan = s_ovf[L] != 0;
        const int n = scan ? CW : min(s_n[L], kWlListCap);
        int my_low = 0;
        // one candidate (or, scanning, one bitmap word) per iteration
        for (int k = tid; k < n; k += kWlThreads) {
            uint32_t cells, wbase;
            int a, b0;
            if (scan) {
                cells = wl_load<GBITS>(&bits[c * CW + k]);
                if (!cells) continue;
                wl_store<GBITS>(&bits[c * CW + k], 0u);   // no other thread touches it this step
                a = k / LWW;
                b0 = 32 * (k - a * LWW);
                wbase = c * CW + k;
            } else {
                const uint32_t e = s_list[L][k];
                a = (int)(e >> 16);
                const int b = (int)(e & 0xFFFFu);
                b0 = b & ~31;
                cells = 1u << (b & 31);
                wbase = c * CW + a * LWW + (b >> 5);
                wl_and<GBITS>(&bits[wbase], ~cells);
            }
            uint32_t relower = 0u;
            while (cells) {
                const int bit = __ffs(cells) - 1;
                cells &= cells - 1u;
                ++my_exam;
                const int i = 2 * a + si, j = 2 * (b0 + bit) + sj;
                E* p = img + (int64_t)i * P + j;
                const uint32_t v = p[0];
                const uint32_t nbv[8] = {p[1], p[-P + 1], p[-P], p[-P - 1],
                                         p[-1], p[P - 1], p[P], p[P + 1]};
                uint32_t alpha;
                if (!decide<false>(v, nbv, s_lut, lambda, alpha)) continue;
                p[0] = (E)alpha;
                ++my_low;
                relower |= 1u << bit;
                // itself: the next list of this class
                const int pos = atomicAdd(&s_n[J], 1);
                if (pos < kWlListCap) s_list[J][pos] = ((uint32_t)a << 16) | (uint32_t)(b0 + bit);
                else s_ovf[J] = 1;
                // its 8 neighbours (other classes), interior only
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int di = q < 3 ? -1 : (q < 5 ? 0 : 1);
                    const int dj = q < 3 ? q - 1 : (q == 3 ? -1 : (q == 4 ? 1 : q - 6));
                    const int y = i + di, x = j + dj;
                    if (y < 1 || y > H - 2 || x < 1 || x > W - 2) continue;
                    const int cy = ((y & 1) << 1) | (x & 1);
                    const int ay = y >> 1, by = x >> 1;
                    const uint32_t m = 1u << (by & 31);
                    const uint32_t old = wl_or<GBITS>(&bits[cy * CW + ay * LWW + (by >> 5)], m);
                    if (old & m) continue;
                    const int lk = s_map[cy];
                    const int pp = atomicAdd(&s_n[lk], 1);
                    if (pp < kWlListCap) s_list[lk][pp] = ((uint32_t)ay << 16) | (uint32_t)by;
                    else s_ovf[lk] = 1;
                }
            }
            if (relower) {
                // lowered cells are pending again for their next visit
                wl_or<GBITS>(&bits[wbase], relower);
            }
        }
        if (my_low) atomicAdd(&s_low, my_low);
        // The image and (in global memory) the bitmaps are shared through
        // memory: every wave's writes must be complete before the barrier.
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (tid == 0) {
            // the lowered pixels of this step are the next list of class c
            s_map[c] = J;
            s_j = L;
            s_n[L] = 0;
            s_ovf[L] = 0;
            if (s_low) {
                s_quiet = 0;
                s_last = t - im.step0;
                s_lowsum += (unsigned long long)s_low;
            } else {
                ++s_quiet;
            }
            s_low = 0;
            s_step = t + 1;
        }
        __syncthreads();
    }
    if (my_exam) atomicAdd(&s_exam, my_exam);
    __syncthreads();
    if (tid == 0) {
        ImgCnt* ct = cnt + im.slot;
        atomicAdd(&ct->lowerings, s_lowsum);
        atomicAdd(&ct->examinations, s_exam);
        if (s_last >= 0) atomicMax(&ct->last_step, im.step0 + s_last);
        steps_out[blockIdx.x] = s_step;
    }
}

}  // namespace

hipError_t launch_init_state(hipStream_t stream, ImgCnt* cnt, int nimg, int32_t* tile_last,
                             int ntiles, int32_t* hist_round, WorkList wl)
{
    const int n = max(max(nimg, 2 * ntiles), 3);
    hipLaunchKernelGGL(k_init_state, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0,
                       stream, cnt, nimg, tile_last, ntiles, hist_round, wl);
    return hipGetLastError();
}

hipError_t launch_worklist(hipStream_t stream, const WlImg* imgs, int nimg, int dtype,
                           bool gbits, ImgCnt* cnt, const TopoEntry* lut, int32_t* steps_out)
{
    if (nimg <= 0) return hipSuccess;
    const dim3 grid(nimg), block(kWlThreads);
    if (dtype == 1) {
        if (gbits) hipLaunchKernelGGL((k_worklist<uint8_t, true>), grid, block, 0, stream, imgs, cnt, lut, steps_out);
        else hipLaunchKernelGGL((k_worklist<uint8_t, false>), grid, block, 0, stream, imgs, cnt, lut, steps_out);
    } else {
        if (gbits) hipLaunchKernelGGL((k_worklist<uint16_t, true>), grid, block, 0, stream, imgs, cnt, lut, steps_out);
        else hipLaunchKernelGGL((k_worklist<uint16_t, false>), grid, block, 0, stream, imgs, cnt, lut, steps_out);
    }
    return hipGetLastError();
}

hipError_t launch_set_desc(hipStream_t stream, ImgDev* dst, const ImgDev& d)
{
    hipLaunchKernelGGL(k_set_desc, dim3(1), dim3(64), 0, stream, dst, d);
    return hipGetLastError();
}

hipError_t launch_advance(hipStream_t stream, int32_t* round_base, int n)
{
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, stream, round_base, n);
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

// Compiled tile shapes: (tile height, tile width, halo = steps per residency,
// threads per tile, residency variant).
#define THIN_SHAPES(X)      \
    X(16, 16, 8, 256, 0)    \
    X(32, 32, 8, 256, 0)    \
    X(32, 32, 8, 512, 0)    \
    X(32, 32, 16, 256, 0)   \
    X(32, 32, 16, 1024, 0)  \
    X(32, 32, 16, 1024, 1)  \
    X(64, 64, 16, 1024, 0)  \
    X(64, 64, 16, 1024, 1)  \
    X(64, 64, 32, 1024, 0)  \
    X(64, 64, 8, 1024, 0)   \
    X(64, 64, 16, 512, 0)   \
    X(64, 64, 16, 256, 0)   \
    X(64, 64, 32, 512, 0)   \
    X(64, 64, 8, 512, 0)    \
    X(48, 48, 16, 512, 0)   \
    X(32, 32, 16, 512, 0)   \
    X(128, 128, 16, 512, 0) \
    X(128, 128, 16, 512, 1) \
    X(64, 64, 16, 512, 1)   \
    X(32, 32, 16, 256, 3)   \
    X(64, 64, 16, 256, 3)   \
    X(64, 64, 16, 256, 4)   \
    X(128, 128, 16, 256, 4) \
    X(32, 32, 16, 512, 3)   \
    X(64, 64, 16, 512, 3)   \
    X(64, 64, 16, 512, 4)   \
    X(64, 64, 32, 512, 3)   \
    X(64, 64, 32, 512, 4)   \
    X(128, 128, 16, 512, 3) \
    X(128, 128, 16, 512, 4) \
    X(128, 128, 32, 512, 4) \
    X(128, 128, 8, 512, 4)  \
    X(128, 128, 24, 512, 4) \
    X(64, 64, 16, 512, 2)   \
    X(32, 32, 16, 512, 2)   \
    X(16, 16, 8, 256, 2)    \
    X(16, 16, 16, 576, 2)   \
    X(16, 16, 16, 256, 2)   \
    X(24, 24, 12, 576, 2)   \
    X(16, 16, 16, 576, 0)   \
    X(32, 32, 8, 256, 2)    \
    X(32, 32, 16, 256, 2)   \
    X(32, 32, 16, 1024, 2)  \
    X(32, 32, 32, 1024, 2)  \
    X(64, 64, 16, 1024, 2)  \
    X(64, 64, 32, 1024, 2)

bool tile_shape_supported(TileShape s)
{
#define X(a, b, c, n, e) \
    if (s.th == a && s.tw == b && s.k == c && s.nt == n && s.var == e) return true;
    THIN_SHAPES(X)
#undef X
    return false;
}

int compiled_shapes(TileShape* out, int cap)
{
    int n = 0;
#define X(a, b, c, t, e)                                  \
    if (n < cap && out) out[n] = TileShape{a, b, c, t, e}; \
    ++n;
    THIN_SHAPES(X)
#undef X
    return n;
}

TileShape complete_shape(int th, int tw, int k)
{
#define X(a, b, c, n, e) \
    if (th == a && tw == b && k == c) return TileShape{a, b, c, n, e};
    THIN_SHAPES(X)
#undef X
    return TileShape{0, 0, 0, 0, 0};
}

static int lds_bytes(TileShape s)
{
    if (s.var == kVarRegs) return (s.th + 2 * s.k + 2) * (s.tw + 2 * s.k + 2) * 2 + 2048 + 64;
    const int region = (s.th + 2 * s.k) * (s.tw + 2 * s.k);
    const int hist = var_seeded(s.var)
                         ? (s.th * (s.tw / 32) + (s.th + 2 * s.k) * ((s.tw + 2 * s.k + 31) / 32)) * 4
                         : 8;
    if (s.var == kVarBits || s.var == kVarBitsSeeded) {
        const int lat_h = (s.th + 2 * s.k) / 2, lat_w = (s.tw + 2 * s.k) / 2;
        const int flags = 16 * lat_h * ((lat_w + 31) / 32) + 2 * lat_h * lat_w + 64;
        return region * 2 + flags + hist + 2048 + 64;
    }
    return region * 3 + hist + 2048 + 64;
}

int history_words(TileShape s) { return var_seeded(s.var) ? s.th * (s.tw / 32) : 1; }

int round_blocks_per_cu(TileShape s)
{
    const int by_lds = (160 * 1024) / lds_bytes(s);
    const int by_threads = 2048 / max(64, s.nt);
    return max(1, min(by_lds, by_threads));
}

hipError_t launch_round(hipStream_t stream, TileShape shape, const ImgDev* imgs, ImgCnt* cnt,
                        const int32_t* tile_img, int32_t* tile_last, int ntiles, int round,
                        const TopoEntry* lut, int num_cus, uint32_t* hist_bits,
                        int32_t* hist_round, WorkList wl, const int32_t* round_base, int kflags)
{
    // The bit-flag variants keep u8 images as u8 in LDS: a launch with
    // kOnlyU8 takes that instantiation.
    const bool u8 = (kflags & kOnlyU8) != 0;
#define X(a, b, c, n, e)                                                                      \
    if (shape.th == a && shape.tw == b && shape.k == c && shape.nt == n && shape.var == e) {  \
        if constexpr (e == kVarBits || e == kVarBitsSeeded)                                   \
            if (u8)                                                                           \
                return launch_round_t<a, b, c, n, e, uint8_t>(stream, imgs, cnt, tile_img,    \
                                                              tile_last, ntiles, round, lut,   \
                                                              num_cus, hist_bits,              \
                                                              hist_round, wl, round_base,      \
                                                              kflags);                         \
        return launch_round_t<a, b, c, n, e, uint16_t>(stream, imgs, cnt, tile_img, tile_last, \
                                                       ntiles, round, lut, num_cus,             \
                                                       hist_bits, hist_round, wl, round_base,   \
                                                       kflags);                                 \
    }
    THIN_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_coop(hipStream_t stream, TileShape shape, const ImgDev* imgs, ImgCnt* cnt,
                       const int32_t* tile_img, int32_t* tile_last, int ntiles,
                       const TopoEntry* lut, int32_t* active, int32_t* rounds_out,
                       int max_rounds, int num_cus, uint32_t* hist_bits, int32_t* hist_round,
                       int kflags)
{
    const bool u8 = (kflags & kOnlyU8) != 0;
#define X(a, b, c, n, e)                                                                      \
    if (shape.th == a && shape.tw == b && shape.k == c && shape.nt == n && shape.var == e) {  \
        if constexpr (e == kVarBits || e == kVarBitsSeeded)                                   \
            if (u8)                                                                           \
                return launch_coop_t<a, b, c, n, e, uint8_t>(stream, imgs, cnt, tile_img,     \
                                                             tile_last, ntiles, lut, active,   \
                                                             rounds_out, max_rounds, num_cus,  \
                                                             hist_bits, hist_round, kflags);   \
        return launch_coop_t<a, b, c, n, e, uint16_t>(stream, imgs, cnt, tile_img, tile_last,  \
                                                      ntiles, lut, active, rounds_out,          \
                                                      max_rounds, num_cus, hist_bits,           \
                                                      hist_round, kflags);                      \
    }
    THIN_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

}  // namespace thin
