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

#include <hip/hip_cooperative_groups.h>

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
    if (lower) {
        uint32_t a = 0;
#pragma unroll
        for (int p = 0; p < 8; ++p) a = max(a, ((u >> p) & 1u) ? 0u : nb[p]);
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

__global__ void k_init_state(ImgCnt* cnt, int nimg, int32_t* tile_last, int ntiles,
                             int32_t* hist_round)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (hist_round && i < 2 * ntiles) hist_round[i] = -1;
    if (i < nimg) {
        cnt[i].lowerings = 0ull;
        cnt[i].tile_rounds = 0ull;
        cnt[i].last_step = -1;
        cnt[i].final_round = -1;
    }
    if (tile_last && i < 2 * ntiles) tile_last[i] = -1;
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
    if (sd->prev_round[n] != sd->r - 1) return 0u;
    return sd->prev_bits[((int64_t)n * TH + (gi - trow * TH)) * WPR + (a - tcol * WPR)];
}

// Geometry of a tile residency: a TH x TW interior plus a K-pixel halo,
// staged in LDS as u16, processed by NT threads.
template <int TH, int TW, int K, int NT, bool SEED>
struct Tile {
    static constexpr int RH = TH + 2 * K;
    static constexpr int RW = TW + 2 * K;
    static constexpr int RWP = RW;  // LDS row pitch in elements
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

    // Interior copy src -> dst (a stable tile keeping the ping-pong pair equal).
    static __device__ void copy_interior(const View d, int gy0, int gx0, const void* src,
                                         void* dst, int tid)
    {
        const int ih = min(TH, d.h - gy0), iw = min(TW, d.w - gx0);
        for (int idx = tid; idx < TH * TW; idx += NT) {
            const int y = idx / TW, x = idx - y * TW;
            if (y < ih && x < iw) {
                const int64_t o = (int64_t)(gy0 + y) * d.pitch + (gx0 + x);
                store_px(dst, d.dtype, o, load_px(src, d.dtype, o));
            }
        }
    }

    // Stages the tile and its halo from src, runs nsteps parity steps starting
    // at image step t0, writes the interior to dst.  Returns the number of
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
    static __device__ int run(const View d, int gy0, int gx0, int t0, int nsteps,
                              const void* src, void* dst, uint16_t* s_img, uint8_t* s_dirty,
                              uint32_t* s_bits, uint32_t* s_cw, const Seed* sd,
                              const TopoEntry* lut, int* s_count, int* s_last, int tid,
                              int& last_tau)
    {
        const int ry0 = gy0 - K, rx0 = gx0 - K;
        const bool seeded = SEED && sd != nullptr && sd->r > 0;
        if (tid == 0) {
            *s_count = 0;
            *s_last = -1;
        }
        if constexpr (SEED)
            for (int i = tid; i < TH * WPR; i += NT) s_bits[i] = 0u;
        // All global loads of the region are issued before the first one is
        // waited for.  Zeros outside the image are never read by a candidate:
        // every candidate is an interior pixel whose 3x3 lies inside the image.
        constexpr int ITER = (RH * RW + NT - 1) / NT;
        uint32_t vals[ITER];
#pragma unroll
        for (int k = 0; k < ITER; ++k) {
            const int idx = tid + k * NT;
            const int y = idx / RW, x = idx - y * RW;
            const int gi = ry0 + y, gj = rx0 + x;
            vals[k] = 0;
            if (idx < RH * RW && gi >= 0 && gi < d.h && gj >= 0 && gj < d.w)
                vals[k] = load_px(src, d.dtype, (int64_t)gi * d.pitch + gj);
        }
#pragma unroll
        for (int k = 0; k < ITER; ++k) {
            const int idx = tid + k * NT;
            const int y = idx / RW, x = idx - y * RW;
            if (idx < RH * RW) {
                s_img[y * RWP + x] = (uint16_t)vals[k];
                s_dirty[y * RWP + x] = seeded ? 0 : 1;
            }
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
        int my_count = 0;
        // Each thread owns fixed positions of the candidate lattice (one in
        // four pixels, rows and columns of the step's parity): the region's
        // origin is even (tile side and halo are even), so the candidate of
        // lattice cell (a, b) in class (si, sj) is region pixel
        // (2a + si, 2b + sj).  The exact region and the image interior only
        // mask cells out step by step.
        int cell_r[PPT], cell_c[PPT];
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int idx = tid + k * NT;
            cell_r[k] = idx < LAT_H * LAT_W ? (idx / LAT_W) * 2 : RH;  // RH: never in range
            cell_c[k] = idx < LAT_H * LAT_W ? (idx % LAT_W) * 2 : 0;
        }
        for (int tau = 0; tau < nsteps; ++tau) {
            const int s = (t0 + tau) & 3, si = s >> 1, sj = s & 1;
            // Exact region after tau steps, clipped to the image interior.
            const int r_lo = max(tau + 1, 1 - ry0), r_hi = min(RH - 2 - tau, d.h - 2 - ry0);
            const int c_lo = max(tau + 1, 1 - rx0), c_hi = min(RW - 2 - tau, d.w - 2 - rx0);
            bool inner = false;
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const int lr = cell_r[k] + si, lc = cell_c[k] + sj;
                if (lr < r_lo || lr > r_hi || lc < c_lo || lc > c_hi) continue;
                const int o = lr * RWP + lc;
                {
                    if (!s_dirty[o]) continue;
                    s_dirty[o] = 0;
                    uint16_t* p = s_img + o;
                    const uint32_t v = p[0];
                    const uint32_t nbv[8] = {p[1], p[-RWP + 1], p[-RWP], p[-RWP - 1],
                                             p[-1], p[RWP - 1], p[RWP], p[RWP + 1]};
                    uint32_t alpha;
                    if (decide(v, nbv, lut, lambda, alpha)) {
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
            // One lane per wave that lowered an interior pixel records the step.
            if (__ballot(inner) != 0ull && (tid & 63) == 0) atomicMax(s_last, tau);
            __syncthreads();
        }

        const int ih = min(TH, d.h - gy0), iw = min(TW, d.w - gx0);
        for (int idx = tid; idx < TH * TW; idx += NT) {
            const int y = idx / TW, x = idx - y * TW;
            if (y < ih && x < iw)
                store_px(dst, d.dtype, (int64_t)(gy0 + y) * d.pitch + (gx0 + x),
                         s_img[(K + y) * RWP + (K + x)]);
        }
        if (my_count) atomicAdd(s_count, my_count);
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

// Largest tile_last over the 3x3 tile neighbourhood of (ty, tx).
__device__ __forceinline__ int32_t neighbourhood_last(const ImgDev* d, const int32_t* tile_last,
                                                      int ty, int tx)
{
    const int tiles_x = d->tiles_x, tiles_y = d->tiles_y, tile0 = d->tile0;
    int32_t m = INT_MIN;
    for (int dy = -1; dy <= 1; ++dy) {
        const int y = ty + dy;
        if (y < 0 || y >= tiles_y) continue;
        for (int dx = -1; dx <= 1; ++dx) {
            const int x = tx + dx;
            if (x < 0 || x >= tiles_x) continue;
            m = max(m, __hip_atomic_load(&tile_last[tile0 + y * tiles_x + x], __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT));
        }
    }
    return m;
}

// ----------------------------------------------------------------- k_round

// One tile of one round (launch-per-round and cooperative engines).
// Returns 1 when the tile was processed (active), 0 when skipped.  All NT
// threads must call it together.
template <int TH, int TW, int K, int NT, bool SEED>
__device__ int round_tile(const ImgDev* __restrict__ imgs, ImgCnt* cnt,
                          const int32_t* __restrict__ tile_img, int32_t* tile_state, int g,
                          int round, int ntiles, uint32_t* hist_bits, int32_t* hist_round,
                          uint16_t* s_img, uint8_t* s_dirty, uint32_t* s_bits, uint32_t* s_cw,
                          const TopoEntry* s_lut, int* s_count, int* s_last)
{
    using T = Tile<TH, TW, K, NT, SEED>;
    const int tid = threadIdx.x;
    const int ii = tile_img[g];
    const ImgDev* d = imgs + ii;
    const int r = round - d->round0;
    if (r < 0) return 0;
    const int t0 = r * K;
    const int nsteps = min(K, d->max_steps - t0);
    if (nsteps <= 0) return 0;
    const int lt = g - d->tile0;
    const int ty = lt / d->tiles_x, tx = lt - ty * d->tiles_x;
    const int slot = d->slot;
    int32_t* st = tile_state + 2 * (d->state0 + lt);  // this tile's state pair

    // tile_state[2g] is the latest round for which a tile of g's 3x3 tile
    // neighbourhood asked g to be active (it lowered something during the
    // last 4 steps of the round before); tile_state[2g + 1] is the last round
    // in which g itself lowered something.  Neighbours of this round may raise
    // tile_state[2g] to r + 1 while it is read here (only adding work), so one
    // thread decides and the barrier broadcasts a block-uniform answer; the
    // barrier also orders this tile's LDS writes after the previous tile's
    // readers.
    int vote = 0;
    if (tid == 0) {
        const int act = __hip_atomic_load(&st[0], __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
        const int chg = __hip_atomic_load(&st[1], __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
        vote = (r == 0 || act >= r) ? 1 : (chg == r - 1 ? 2 : 0);
    }
    const int decision = __syncthreads_or(vote == 1) ? 1 : (__syncthreads_or(vote == 2) ? 2 : 0);
    const bool active = decision == 1;
    const void* src = round_src(d, r);
    void* dst = round_dst(d, r);
    const int gy0 = ty * TH, gx0 = tx * TW;
    const View v = view_of(d);

    if (!active) {
        // Stable for this round.  The output buffer already equals the input
        // unless the tile changed during the previous round.
        if (decision == 2) T::copy_interior(v, gy0, gx0, src, dst, tid);
        return 0;
    }
    Seed sd{};
    const int64_t words = SEED ? (int64_t)ntiles * TH * T::WPR : 0;
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
    int last_tau;
    const int count = T::run(v, gy0, gx0, t0, nsteps, src, dst, s_img, s_dirty, s_bits, s_cw,
                             SEED ? &sd : nullptr, s_lut + d->adj * 256, s_count, s_last, tid,
                             last_tau);
    if (tid == 0) {
        atomicAdd(&cnt[slot].tile_rounds, 1ull);
        if (last_tau >= 0) {
            __hip_atomic_store(&st[1], r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            atomicAdd(&cnt[slot].lowerings, (unsigned long long)count);
            atomicMax(&cnt[slot].last_step, t0 + last_tau);
        }
        // Lowered during the last 4 steps: the 3x3 tile block must run the next
        // round (a tile whose whole block was quiet for 4 steps cannot change
        // within the next K <= tile-side steps).
        if (last_tau >= nsteps - 4) {
            for (int dy = -1; dy <= 1; ++dy) {
                const int y = ty + dy;
                if (y < 0 || y >= d->tiles_y) continue;
                for (int dx = -1; dx <= 1; ++dx) {
                    const int x = tx + dx;
                    if (x < 0 || x >= d->tiles_x) continue;
                    __hip_atomic_fetch_max(&tile_state[2 * (d->state0 + y * d->tiles_x + x)],
                                           r + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
    }
    return 1;
}

template <int TH, int TW, int K, int NT, bool SEED>
__global__ __launch_bounds__(NT) void k_round(const ImgDev* __restrict__ imgs, ImgCnt* cnt,
                                              const int32_t* __restrict__ tile_img,
                                              int32_t* tile_last, int ntiles, int round,
                                              const TopoEntry* __restrict__ lut_g,
                                              uint32_t* hist_bits, int32_t* hist_round)
{
    using T = Tile<TH, TW, K, NT, SEED>;
    __shared__ uint16_t s_img[T::RH * T::RWP];
    __shared__ uint8_t s_dirty[T::RH * T::RWP];
    __shared__ uint32_t s_bits[T::BITS_WORDS];
    __shared__ uint32_t s_cw[T::CW_WORDS];
    __shared__ TopoEntry s_lut[512];
    __shared__ int s_count, s_last;
    for (int i = threadIdx.x; i < 512; i += NT) s_lut[i] = lut_g[i];
    for (int g = blockIdx.x; g < ntiles; g += gridDim.x)
        round_tile<TH, TW, K, NT, SEED>(imgs, cnt, tile_img, tile_last, g, round, ntiles, hist_bits,
                                  hist_round, s_img, s_dirty, s_bits, s_cw, s_lut, &s_count,
                                  &s_last);
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

template <int TH, int TW, int K, int NT, bool SEED>
__global__ __launch_bounds__(NT) void k_coop(const ImgDev* __restrict__ imgs, ImgCnt* cnt,
                                             const int32_t* __restrict__ tile_img,
                                             int32_t* tile_last, int ntiles,
                                             const TopoEntry* __restrict__ lut_g, int32_t* active,
                                             int32_t* rounds_out, int max_rounds,
                                             uint32_t* hist_bits, int32_t* hist_round)
{
    using T = Tile<TH, TW, K, NT, SEED>;
    __shared__ uint16_t s_img[T::RH * T::RWP];
    __shared__ uint8_t s_dirty[T::RH * T::RWP];
    __shared__ uint32_t s_bits[T::BITS_WORDS];
    __shared__ uint32_t s_cw[T::CW_WORDS];
    __shared__ TopoEntry s_lut[512];
    __shared__ int s_count, s_last;
    const int tid = threadIdx.x;
    for (int i = tid; i < 512; i += NT) s_lut[i] = lut_g[i];
    cooperative_groups::grid_group grid = cooperative_groups::this_grid();
    int round = 0;
    for (;; ++round) {
        if (blockIdx.x == 0 && tid == 0)
            __hip_atomic_store(&active[(round + 1) % 3], 0, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        int mine = 0;
        for (int g = blockIdx.x; g < ntiles; g += gridDim.x)
            mine += round_tile<TH, TW, K, NT, SEED>(imgs, cnt, tile_img, tile_last, g, round, ntiles,
                                              hist_bits, hist_round, s_img, s_dirty, s_bits, s_cw,
                                              s_lut, &s_count, &s_last);
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

template <int TH, int TW, int K, int NT, bool SEED>
hipError_t launch_coop_t(hipStream_t stream, const ImgDev* imgs, ImgCnt* cnt,
                         const int32_t* tile_img, int32_t* tile_last, int ntiles,
                         const TopoEntry* lut, int32_t* active, int32_t* rounds_out,
                         int max_rounds, int num_cus, uint32_t* hist_bits, int32_t* hist_round)
{
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, reinterpret_cast<const void*>(&k_coop<TH, TW, K, NT, SEED>), NT, 0);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    const int grid = max(1, min(ntiles, per_cu * num_cus));
    void* args[] = {(void*)&imgs,       (void*)&cnt,       (void*)&tile_img,
                    (void*)&tile_last,  (void*)&ntiles,    (void*)&lut,
                    (void*)&active,     (void*)&rounds_out, (void*)&max_rounds,
                    (void*)&hist_bits,  (void*)&hist_round};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_coop<TH, TW, K, NT, SEED>),
                                      dim3(grid), dim3(NT), args, 0, stream);
}

template <int TH, int TW, int K, int NT, bool SEED>
hipError_t launch_round_t(hipStream_t stream, const ImgDev* imgs, ImgCnt* cnt,
                          const int32_t* tile_img, int32_t* tile_last, int ntiles, int round,
                          const TopoEntry* lut, int grid_blocks, uint32_t* hist_bits,
                          int32_t* hist_round)
{
    const int grid = max(1, min(ntiles, grid_blocks));
    hipLaunchKernelGGL((k_round<TH, TW, K, NT, SEED>), dim3(grid), dim3(NT), 0, stream, imgs, cnt,
                       tile_img, tile_last, ntiles, round, lut, hist_bits, hist_round);
    return hipGetLastError();
}

// --------------------------------------------------------------- k_persist
//
// One launch runs every image of the work list to stability.  Work item q is
// (round r = q / ntiles, tile g = q % ntiles); items are handed out in order
// by one atomic counter.  Item (r, g) may start once tile g and its 8
// neighbouring tiles have completed round r - 1.  Those items were handed out
// earlier, to blocks that are running, and the oldest item still outstanding
// never waits, so the queue always drains; no co-residency is assumed.
// Publishing a round: every thread fences its stores at device scope, then
// one thread raises progress[g] with release semantics; a waiter observes it
// with acquire semantics before the block reads the halo.
// Convergence: per image, a ring of per-round completion counters finds the
// last tile to finish round r; that tile finalises the image when nothing
// was lowered during the last 4 steps of round r (or the step cap is
// reached).  Ring entries are reused after `ring_w` rounds, more than the
// largest round spread between two tiles of one image (a tile is at most one
// round ahead of each neighbour).  Every wait has a time limit, and so has
// the whole launch: on expiry the block raises sched->error and all blocks
// leave, so every wave reaches the end of the kernel.

// Reads a word other blocks update, as a read-modify-write at device scope.
// A plain relaxed load may be served from this XCD's L2, which is not kept
// coherent with the other XCDs' L2s, so a polling loop could keep reading a
// stale copy; an atomic RMW is performed at the device coherence point and
// returns the latest value without invalidating any cache.
__device__ __forceinline__ int ld_sync(int32_t* p)
{
    return __hip_atomic_fetch_add(p, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int TH, int TW, int K, int NT, bool SEED>
__global__ __launch_bounds__(NT) void k_persist(const ImgDev* __restrict__ imgs, ImgCnt* cnt,
                                                const int32_t* __restrict__ tile_img,
                                                int32_t* tile_last, int32_t* progress,
                                                int32_t* ring, Sched* sched, int ntiles,
                                                const TopoEntry* __restrict__ lut_g,
                                                unsigned long long wait_ticks,
                                                unsigned long long kernel_ticks)
{
    using T = Tile<TH, TW, K, NT, SEED>;
    __shared__ uint16_t s_img[T::RH * T::RWP];
    __shared__ uint8_t s_dirty[T::RH * T::RWP];
    __shared__ uint32_t s_bits[T::BITS_WORDS];
    __shared__ uint32_t s_cw[T::CW_WORDS];
    __shared__ TopoEntry s_lut[512];
    __shared__ int s_count, s_last;
    __shared__ int s_item[4];  // tile, round, active, copy

    const int tid = threadIdx.x;
    for (int i = tid; i < 512; i += NT) s_lut[i] = lut_g[i];
    const unsigned long long kernel_start = wall_clock64();

    for (;;) {
        if (tid == 0) {
            int item_g = -1, item_r = 0, item_active = 0, item_copy = 0;
            const unsigned long long since = wall_clock64();
            for (;;) {
                if (ld_sync(&sched->images_left) <= 0 || ld_sync(&sched->error)) break;
                if (wall_clock64() - since > 2 * wait_ticks ||
                    wall_clock64() - kernel_start > kernel_ticks) {
                    // Items keep being skipped while an image stays unfinished:
                    // give up rather than spin.
                    __hip_atomic_store(&sched->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                const unsigned long long q = atomicAdd(&sched->next, 1ull);
                const int r = (int)(q / (unsigned long long)ntiles);
                const int g = (int)(q % (unsigned long long)ntiles);
                const int ii = tile_img[g];
                const ImgDev* d = imgs + ii;
                const int64_t t0 = (int64_t)r * K;
                if (t0 >= d->max_steps) continue;  // beyond the step cap
                int fr = ld_sync(&cnt[ii].final_round);
                if (fr >= 0 && r >= fr) continue;  // image already final
                const int tiles_x = d->tiles_x, tiles_y = d->tiles_y, tile0 = d->tile0;
                const int lt = g - tile0;
                const int ty = lt / tiles_x, tx = lt - ty * tiles_x;
                bool skip = false, failed = false;
                const unsigned long long w0 = wall_clock64();
                for (;;) {
                    // Poll with device-scope RMW reads (no cache
                    // invalidation); one acquire fence follows success.
                    bool ready = ld_sync(&progress[g]) >= r;
                    for (int dy = -1; dy <= 1 && ready; ++dy) {
                        const int y = ty + dy;
                        if (y < 0 || y >= tiles_y) continue;
                        for (int dx = -1; dx <= 1 && ready; ++dx) {
                            const int x = tx + dx;
                            if (x < 0 || x >= tiles_x || (dx == 0 && dy == 0)) continue;
                            ready = ld_sync(&progress[tile0 + y * tiles_x + x]) >= r;
                        }
                    }
                    if (ready) {
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                        break;
                    }
                    fr = ld_sync(&cnt[ii].final_round);
                    if (fr >= 0 && r >= fr) { skip = true; break; }
                    if (ld_sync(&sched->error) || wall_clock64() - w0 > wait_ticks ||
                        wall_clock64() - kernel_start > kernel_ticks) {
                        failed = true;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                if (failed) {
                    __hip_atomic_store(&sched->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                if (skip) continue;
                item_g = g;
                item_r = r;
                item_active = (r == 0 || neighbourhood_last(d, tile_last, ty, tx) >= (int)t0 - 4);
                item_copy = tile_last[g] >= (int)t0 - K;
                break;
            }
            s_item[0] = item_g;
            s_item[1] = item_r;
            s_item[2] = item_active;
            s_item[3] = item_copy;
        }
        __syncthreads();
        const int g = s_item[0];
        if (g < 0) break;
        const int r = s_item[1];
        const int ii = tile_img[g];
        const ImgDev* d = imgs + ii;
        const int t0 = r * K;
        const int nsteps = min(K, d->max_steps - t0);
        const int lt = g - d->tile0;
        const int ty = lt / d->tiles_x, tx = lt - ty * d->tiles_x;
        const void* src = round_src(d, r);
        void* dst = round_dst(d, r);
        const int gy0 = ty * TH, gx0 = tx * TW;
        const View v = view_of(d);
        int last_tau = -1, count = 0;
        if (s_item[2]) {
            count = T::run(v, gy0, gx0, t0, nsteps, src, dst, s_img, s_dirty, s_bits, s_cw,
                           nullptr, s_lut + d->adj * 256, &s_count, &s_last, tid, last_tau);
        } else if (s_item[3]) {
            T::copy_interior(v, gy0, gx0, src, dst, tid);
        }
        // Publishing: each wave waits until its own stores are acknowledged
        // (a workgroup barrier alone does not wait for them), then one
        // thread's release fence writes the L2 back for other XCDs.
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (tid == 0) {
            if (s_item[2]) atomicAdd(&cnt[ii].tile_rounds, 1ull);
            if (last_tau >= 0) {
                __hip_atomic_store(&tile_last[g], t0 + last_tau, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                atomicAdd(&cnt[ii].lowerings, (unsigned long long)count);
                atomicMax(&cnt[ii].last_step, t0 + last_tau);
            }
            __hip_atomic_store(&progress[g], r + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            const int slot = d->ring0 + r % d->ring_w;
            const int done = __hip_atomic_fetch_add(&ring[slot], 1, __ATOMIC_ACQ_REL,
                                                    __HIP_MEMORY_SCOPE_AGENT) + 1;
            if (done == d->tiles_x * d->tiles_y) {
                // Last tile of round r: every tile's counters of rounds <= r
                // are in.  Later rounds cannot lower anything if this one
                // ended quiet, so last_step decides stability exactly.
                __hip_atomic_store(&ring[slot], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const int ls = ld_sync(&cnt[ii].last_step);
                const int64_t steps = min((int64_t)(r + 1) * K, (int64_t)d->max_steps);
                if ((int64_t)ls < steps - 4 || steps >= d->max_steps) {
                    __hip_atomic_store(&cnt[ii].final_round, r + 1, __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_fetch_add(&sched->images_left, -1, __ATOMIC_ACQ_REL,
                                           __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
    }
}

__global__ void k_init_persist(ImgCnt* cnt, int nimg, int32_t* tile_last, int32_t* progress,
                               int ntiles, int32_t* ring, int nring, Sched* sched)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nimg) {
        cnt[i].lowerings = 0ull;
        cnt[i].tile_rounds = 0ull;
        cnt[i].last_step = -1;
        cnt[i].final_round = -1;
    }
    if (i < ntiles) {
        tile_last[i] = -1;
        progress[i] = 0;
    }
    if (i < nring) ring[i] = 0;
    if (i == 0) {
        sched->next = 0ull;
        sched->images_left = nimg;
        sched->error = 0;
    }
}

template <int TH, int TW, int K, int NT, bool SEED>
hipError_t launch_persist_t(hipStream_t stream, const ImgDev* imgs, ImgCnt* cnt,
                            const int32_t* tile_img, int32_t* tile_last, int32_t* progress,
                            int32_t* ring, Sched* sched, int ntiles, const TopoEntry* lut,
                            int grid_blocks, unsigned long long wait_ticks,
                            unsigned long long kernel_ticks)
{
    hipLaunchKernelGGL((k_persist<TH, TW, K, NT, SEED>), dim3(max(1, grid_blocks)), dim3(NT), 0, stream,
                       imgs, cnt, tile_img, tile_last, progress, ring, sched, ntiles, lut,
                       wait_ticks, kernel_ticks);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_init_state(hipStream_t stream, ImgCnt* cnt, int nimg, int32_t* tile_last,
                             int ntiles, int32_t* hist_round)
{
    const int n = max(nimg, 2 * ntiles);
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_init_state, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0,
                       stream, cnt, nimg, tile_last, ntiles, hist_round);
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
// threads per tile, history seeding).
#define THIN_SHAPES(X)           \
    X(16, 16, 8, 256, false)     \
    X(32, 32, 8, 256, false)     \
    X(32, 32, 8, 512, false)     \
    X(32, 32, 16, 256, false)    \
    X(32, 32, 16, 1024, false)   \
    X(32, 32, 16, 1024, true)    \
    X(64, 64, 16, 1024, false)   \
    X(64, 64, 16, 1024, true)    \
    X(64, 64, 32, 1024, false)

bool tile_shape_supported(TileShape s)
{
#define X(a, b, c, n, e) \
    if (s.th == a && s.tw == b && s.k == c && s.nt == n && s.seed == e) return true;
    THIN_SHAPES(X)
#undef X
    return false;
}

TileShape complete_shape(int th, int tw, int k)
{
#define X(a, b, c, n, e) \
    if (th == a && tw == b && k == c) return TileShape{a, b, c, n, e};
    THIN_SHAPES(X)
#undef X
    return TileShape{0, 0, 0, 0, false};
}

int persist_threads(TileShape s) { return s.nt; }

static int lds_bytes(TileShape s)
{
    const int region = (s.th + 2 * s.k) * (s.tw + 2 * s.k);
    const int hist = s.seed ? (s.th * (s.tw / 32) + (s.th + 2 * s.k) * ((s.tw + 2 * s.k + 31) / 32)) * 4
                            : 8;
    return region * 3 + hist + 4096 + 64;
}

int history_words(TileShape s) { return s.seed ? s.th * (s.tw / 32) : 1; }

int round_blocks_per_cu(TileShape s)
{
    const int by_lds = (160 * 1024) / lds_bytes(s);
    const int by_threads = 2048 / max(64, s.nt);
    return max(1, min(by_lds, by_threads));
}

int persist_blocks_per_cu(TileShape s) { return round_blocks_per_cu(s); }

hipError_t launch_round(hipStream_t stream, TileShape shape, const ImgDev* imgs, ImgCnt* cnt,
                        const int32_t* tile_img, int32_t* tile_last, int ntiles, int round,
                        const TopoEntry* lut, int grid_blocks, uint32_t* hist_bits,
                        int32_t* hist_round)
{
#define X(a, b, c, n, e)                                                                    \
    if (shape.th == a && shape.tw == b && shape.k == c && shape.nt == n && shape.seed == e)  \
        return launch_round_t<a, b, c, n, e>(stream, imgs, cnt, tile_img, tile_last, ntiles, \
                                             round, lut, grid_blocks, hist_bits, hist_round);
    THIN_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_persist(hipStream_t stream, TileShape shape, const ImgDev* imgs, ImgCnt* cnt,
                          const int32_t* tile_img, int32_t* tile_last, int32_t* progress,
                          int32_t* ring, Sched* sched, int ntiles, const TopoEntry* lut,
                          int grid_blocks, unsigned long long wait_ticks,
                          unsigned long long kernel_ticks)
{
#define X(a, b, c, n, e)                                                                     \
    if (shape.th == a && shape.tw == b && shape.k == c && shape.nt == n && shape.seed == e)   \
        return launch_persist_t<a, b, c, n, e>(stream, imgs, cnt, tile_img, tile_last,        \
                                               progress, ring, sched, ntiles, lut, grid_blocks, \
                                               wait_ticks, kernel_ticks);
    THIN_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_coop(hipStream_t stream, TileShape shape, const ImgDev* imgs, ImgCnt* cnt,
                       const int32_t* tile_img, int32_t* tile_last, int ntiles,
                       const TopoEntry* lut, int32_t* active, int32_t* rounds_out,
                       int max_rounds, int num_cus, uint32_t* hist_bits, int32_t* hist_round)
{
#define X(a, b, c, n, e)                                                                    \
    if (shape.th == a && shape.tw == b && shape.k == c && shape.nt == n && shape.seed == e)  \
        return launch_coop_t<a, b, c, n, e>(stream, imgs, cnt, tile_img, tile_last, ntiles,  \
                                            lut, active, rounds_out, max_rounds, num_cus,    \
                                            hist_bits, hist_round);
    THIN_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_init_persist(hipStream_t stream, ImgCnt* cnt, int nimg, int32_t* tile_last,
                               int32_t* progress, int ntiles, int32_t* ring, int nring,
                               Sched* sched)
{
    const int n = max(max(nimg, ntiles), max(nring, 1));
    hipLaunchKernelGGL(k_init_persist, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0,
                       stream, cnt, nimg, tile_last, progress, ntiles, ring, nring, sched);
    return hipGetLastError();
}

}  // namespace thin
