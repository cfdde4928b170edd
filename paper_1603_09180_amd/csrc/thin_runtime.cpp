// thin_runtime.cpp -- host runtime and C ABI of the lambda-leveling library.
//
// The runtime validates arguments, owns the device scratch (ping-pong twins,
// per-tile state, per-image counters, the connectivity table), builds the
// tile work list, launches rounds of the tiled kernel on the context's
// stream and decides convergence from per-image counters copied back
// asynchronously: a round chunk is checked while the next one already runs,
// so the host never waits on the GPU between chunks.
//
// Convergence (the "until stability" of section 2.2): an image is stable once
// four consecutive parity steps -- one of each class -- lowered nothing.  The
// step sequence is fixed, so the pass count is recovered exactly from the
// index of the last step that lowered something: P = last_step / 4 + 2, or 1
// when nothing was ever lowered (the final pass without change is counted).
#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <iterator>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "thin.h"
#include "thin_internal.h"

using thin::ImgCnt;
using thin::ImgDev;
using thin::TileShape;
using thin::TopoEntry;

namespace {

struct DevBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
};

// First-fit allocator of offsets inside one device buffer (host bookkeeping).
class Arena {
public:
    void reset(uint64_t cap)
    {
        cap_ = cap;
        free_.clear();
        if (cap) free_[0] = cap;
    }
    uint64_t capacity() const { return cap_; }
    // Returns an offset aligned to `align`, or UINT64_MAX when nothing fits.
    uint64_t alloc(uint64_t len, uint64_t align)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            const uint64_t start = (it->first + align - 1) / align * align;
            const uint64_t end = it->first + it->second;
            if (start + len > end) continue;
            const uint64_t f0 = it->first;
            free_.erase(it);
            if (start > f0) free_[f0] = start - f0;
            if (end > start + len) free_[start + len] = end - (start + len);
            return start;
        }
        return UINT64_MAX;
    }
    void release(uint64_t off, uint64_t len)
    {
        auto it = free_.emplace(off, len).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }

private:
    uint64_t cap_ = 0;
    std::map<uint64_t, uint64_t> free_;
};

struct Resident {          // one image admitted for serving
    thin_image img;
    uint64_t tag;
    int round0;            // launch round of its first parity step
    uint64_t twin_off, twin_len;    // its twin inside the twin arena
    uint64_t state_off, ntiles;     // its per-tile state inside the state arena (tiles)
    int tiles_x, tiles_y;
    int slot;              // its counters
    int max_steps;
    bool fresh;            // state not yet initialised on the device
};

struct Retired {
    uint64_t tag;
    thin_stats stats;
};

constexpr int kServeSlots = 1 << 14;          // resident images at most
constexpr uint64_t kServeDefaultBudget = 1ull << 30;

}  // namespace

struct thin_ctx {
    int device = 0;
    int engine = THIN_ENGINE_TILED;
    hipStream_t stream = nullptr;
    uint64_t max_device_bytes = 0;
    uint64_t max_passes = 0;
    TileShape forced{0, 0, 0, 0, 0};
    int num_cus = 256;

    TopoEntry* d_lut = nullptr;
    uint64_t allocated = 0;        // bytes of scratch currently held
    DevBuf twin, imgs, cnt, tile_img, tile_last, small, hist_bits, hist_round, wl_list, wl_meta;
    DevBuf wl_imgs, wl_bits;       // pixel work-list engine: descriptors, global pending bitmaps
    DevBuf grad;                   // gradient front-end scratch (8 floats per pixel)
    ImgCnt* h_snap[2] = {nullptr, nullptr};   // pinned snapshots of the counters
    size_t h_snap_cap = 0;
    hipEvent_t ev[2] = {nullptr, nullptr};

    // profiling (THIN_FLAG_PROFILE): a pool of timing events, two per launch
    bool profile = false;
    std::vector<hipEvent_t> prof_ev;
    uint64_t prof_launches = 0;
    double prof_ms = 0.0;
    uint64_t prof_tile_rounds = 0;

    // serving (continuous batching)
    std::vector<Resident> resident;
    std::vector<Retired> retired;  // finished, not yet reported
    std::vector<int> free_slots;
    int serve_round = 0;           // next launch round of the serving clock
    bool serve_ready = false;
    bool serve_dirty = true;       // resident set changed since the device list was built
    int serve_ntiles = 0;          // entries of the device tile list
    TileShape serve_shape{0, 0, 0, 0, false};
    Arena twin_arena, state_arena;
    DevBuf serve_twin, serve_state, serve_cnt, serve_imgs, serve_tile_img;
    ImgCnt* serve_snap = nullptr;  // pinned copy of all counter slots

    // graph mode (THIN_FLAG_GRAPH): instantiated chunk graphs by launch parameters
    bool graph = false;
    hipStream_t cap_stream = nullptr;
    std::map<std::vector<uint64_t>, hipGraphExec_t> graphs;

    // autotuned shapes by size class (log2 total pixels, log2 pixels per image)
    std::map<std::pair<int, int>, TileShape> tuned;
    std::string tune_cache;        // file of tuned shapes ("" = none)
    std::string arch;              // device architecture name, e.g. gfx950

    int last_launches = 0;         // round launches of the last tiled run
    int last_tail_steps = 0;       // steps its work-list tail ran (0: none)
    bool tail = false;             // hand single small images' tails to the work-list kernel
    void* noalloc = nullptr;       // this device's copy of the static scratch array

    std::string last_error;
};

namespace {

int fail(thin_ctx* ctx, int code, const char* fmt, ...)
{
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->last_error = buf;
    }
    return code;
}

#define HIP_TRY(ctx, expr)                                                                  \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail((ctx), THIN_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// Grows `b` to at least `need` bytes (contents not kept).
int ensure(thin_ctx* ctx, DevBuf& b, size_t need)
{
    if (b.bytes >= need) return THIN_OK;
    size_t want = std::max(need, b.bytes + b.bytes / 2);
    want = (want + 255) & ~size_t(255);
    const uint64_t after = ctx->allocated - b.bytes + want;
    if (ctx->max_device_bytes && after > ctx->max_device_bytes) {
        want = (need + 255) & ~size_t(255);
        if (ctx->allocated - b.bytes + want > ctx->max_device_bytes)
            return fail(ctx, THIN_ENOMEM, "scratch of %zu bytes exceeds max_device_bytes %llu",
                        want, (unsigned long long)ctx->max_device_bytes);
    }
    if (b.ptr) {
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        HIP_TRY(ctx, hipFree(b.ptr));
        ctx->allocated -= b.bytes;
        b.ptr = nullptr;
        b.bytes = 0;
    }
    if (hipMalloc(&b.ptr, want) != hipSuccess) {
        (void)hipGetLastError();
        b.ptr = nullptr;
        return fail(ctx, THIN_ENOMEM, "hipMalloc(%zu) failed", want);
    }
    b.bytes = want;
    ctx->allocated += want;
    return THIN_OK;
}

int ensure_snap(thin_ctx* ctx, size_t n)
{
    if (ctx->h_snap_cap >= n) return THIN_OK;
    for (int i = 0; i < 2; ++i) {
        if (ctx->h_snap[i]) (void)hipHostFree(ctx->h_snap[i]);
        ctx->h_snap[i] = nullptr;
    }
    size_t want = std::max<size_t>(n, 64);
    for (int i = 0; i < 2; ++i)
        if (hipHostMalloc((void**)&ctx->h_snap[i], want * sizeof(ImgCnt), hipHostMallocDefault) !=
            hipSuccess)
            return fail(ctx, THIN_ENOMEM, "hipHostMalloc of counter snapshots failed");
    ctx->h_snap_cap = want;
    return THIN_OK;
}

bool bits_variant(TileShape s) { return s.var == thin::kVarBits || s.var == thin::kVarBitsSeeded; }

// One round: a single launch, or for the bit-flag variants (whose LDS tile
// has the image's pixel type) one launch per pixel type present.  dtypes:
// bit 0 when u8 images take part, bit 1 when u16 ones do.
hipError_t launch_rounds_split(hipStream_t stream, TileShape shape, const ImgDev* imgs,
                               ImgCnt* cnt, const int32_t* tile_img, int32_t* tile_last,
                               int ntiles, int round, const TopoEntry* lut, int num_cus,
                               uint32_t* hist_bits, int32_t* hist_round, thin::WorkList wl,
                               const int32_t* round_base, int kflags, int dtypes)
{
    if (!bits_variant(shape))
        return thin::launch_round(stream, shape, imgs, cnt, tile_img, tile_last, ntiles, round, lut,
                                  num_cus, hist_bits, hist_round, wl, round_base, kflags);
    hipError_t e = hipSuccess;
    if (dtypes & 1)
        e = thin::launch_round(stream, shape, imgs, cnt, tile_img, tile_last, ntiles, round, lut,
                               num_cus, hist_bits, hist_round, wl, round_base,
                               kflags | thin::kOnlyU8);
    if (e == hipSuccess && (dtypes & 2))
        e = thin::launch_round(stream, shape, imgs, cnt, tile_img, tile_last, ntiles, round, lut,
                               num_cus, hist_bits, hist_round, wl, round_base,
                               kflags | thin::kOnlyU16);
    return e;
}

// Launches one round, bracketed by timing events when profiling.
int timed_round(thin_ctx* ctx, size_t& ev_used, TileShape shape, const ImgDev* imgs, ImgCnt* cnt,
                const int32_t* tile_img, int32_t* tile_last, int ntiles, int round, int grid,
                uint32_t* hist_bits, int32_t* hist_round, thin::WorkList wl, int kflags,
                int dtypes)
{
    if (ctx->profile) {
        while (ctx->prof_ev.size() < ev_used + 2) {
            hipEvent_t e;
            HIP_TRY(ctx, hipEventCreate(&e));
            ctx->prof_ev.push_back(e);
        }
        HIP_TRY(ctx, hipEventRecord(ctx->prof_ev[ev_used], ctx->stream));
    }
    (void)grid;
    HIP_TRY(ctx, launch_rounds_split(ctx->stream, shape, imgs, cnt, tile_img, tile_last, ntiles,
                                     round, ctx->d_lut, ctx->num_cus, hist_bits, hist_round, wl,
                                     nullptr, kflags, dtypes));
    if (ctx->profile) {
        HIP_TRY(ctx, hipEventRecord(ctx->prof_ev[ev_used + 1], ctx->stream));
        ev_used += 2;
    }
    return THIN_OK;
}

// Adds the durations of the timed launches (the stream must be idle).
int collect_profile(thin_ctx* ctx, size_t ev_used)
{
    for (size_t i = 0; i + 1 < ev_used; i += 2) {
        float ms = 0.f;
        HIP_TRY(ctx, hipEventElapsedTime(&ms, ctx->prof_ev[i], ctx->prof_ev[i + 1]));
        ctx->prof_ms += ms;
        ctx->prof_launches += 1;
    }
    return THIN_OK;
}

// Index of the image's connectivity table on the device (adjacency and operator).
int32_t table_index(const thin_image& im)
{
    return im.adjacency + 2 * im.op;
}

int validate(thin_ctx* ctx, const thin_image& im)
{
    if (im.h < 0 || im.w < 0) return fail(ctx, THIN_EINVAL, "negative image size");
    if (im.dtype != THIN_U8 && im.dtype != THIN_U16) return fail(ctx, THIN_EINVAL, "bad dtype %d", im.dtype);
    if (im.adjacency != THIN_ADJ_8_4 && im.adjacency != THIN_ADJ_4_8)
        return fail(ctx, THIN_EINVAL, "bad adjacency %d", im.adjacency);
    if (im.op != THIN_OP_LEVELING && im.op != THIN_OP_SKELETON)
        return fail(ctx, THIN_EINVAL, "bad operator %d", im.op);
    if (im.pitch_elems != 0 && im.pitch_elems < im.w) return fail(ctx, THIN_EINVAL, "pitch < w");
    if (im.h > (1 << 30) || im.w > (1 << 30)) return fail(ctx, THIN_EINVAL, "image side above 2^30");
    if (im.h * im.w > 0 && im.image == nullptr) return fail(ctx, THIN_EINVAL, "NULL image");
    return THIN_OK;
}

int64_t pitch_of(const thin_image& im) { return im.pitch_elems ? im.pitch_elems : im.w; }

int steps_cap(const thin_ctx* ctx)
{
    if (!ctx->max_passes) return INT_MAX;
    const uint64_t s = ctx->max_passes * 4ull;
    return s > (uint64_t)INT_MAX ? INT_MAX : (int)s;
}

int floor_log2(int64_t v)
{
    int l = 0;
    while (v > 1) {
        v >>= 1;
        ++l;
    }
    return l;
}

std::pair<int, int> size_class(int64_t total_pixels, int64_t images)
{
    return {floor_log2(total_pixels), floor_log2(total_pixels / std::max<int64_t>(images, 1))};
}

// Tune cache file: one line per entry,
//   <arch> <log2 total pixels> <log2 pixels per image> <th> <tw> <k> <threads> <variant> <ms>
// Lines of other architectures, or naming shapes this build does not have,
// are ignored when reading and kept when writing.
void load_tune_cache(thin_ctx* ctx)
{
    if (ctx->tune_cache.empty()) return;
    FILE* f = fopen(ctx->tune_cache.c_str(), "r");
    if (!f) return;
    char arch[64];
    int a, b;
    TileShape sh{};
    double ms;
    while (fscanf(f, "%63s %d %d %d %d %d %d %d %lf", arch, &a, &b, &sh.th, &sh.tw, &sh.k, &sh.nt,
                  &sh.var, &ms) == 9)
        if (ctx->arch == arch && thin::tile_shape_supported(sh)) ctx->tuned[{a, b}] = sh;
    fclose(f);
}

void save_tune_cache(const thin_ctx* ctx, std::pair<int, int> cls, TileShape sh, double ms)
{
    if (ctx->tune_cache.empty()) return;
    std::vector<std::string> keep;
    if (FILE* f = fopen(ctx->tune_cache.c_str(), "r")) {
        char line[256];
        while (fgets(line, sizeof line, f)) {
            char arch[64];
            int a, b;
            if (sscanf(line, "%63s %d %d", arch, &a, &b) == 3 && ctx->arch == arch &&
                a == cls.first && b == cls.second)
                continue;  // replaced below
            keep.push_back(line);
        }
        fclose(f);
    }
    const std::string tmp = ctx->tune_cache + ".tmp";
    FILE* f = fopen(tmp.c_str(), "w");
    if (!f) return;
    for (const std::string& l : keep) fputs(l.c_str(), f);
    fprintf(f, "%s %d %d %d %d %d %d %d %.4f\n", ctx->arch.c_str(), cls.first, cls.second, sh.th,
            sh.tw, sh.k, sh.nt, sh.var, ms);
    fclose(f);
    std::rename(tmp.c_str(), ctx->tune_cache.c_str());
}

TileShape choose_shape(const thin_ctx* ctx, int64_t total_pixels, int64_t images)
{
    if (ctx->forced.th) return ctx->forced;
    auto it = ctx->tuned.find(size_class(total_pixels, images));
    if (it != ctx->tuned.end()) return it->second;
    // Small work lists are bound by the latency of each round: small tiles
    // with one cell per thread and register windows.  Large ones are bound by
    // throughput: dense per-step work lists with seeded flags in 128x128
    // tiles (less halo work per pixel).
    (void)images;
    if (total_pixels <= (int64_t)1 << 20) return TileShape{32, 32, 16, 1024, thin::kVarRegs};
    return TileShape{128, 128, 16, 512, thin::kVarBitsSeeded};
}

void fill_stats(thin_stats* st, const ImgCnt& c, int steps_done, int max_steps, bool trivial)
{
    if (!st) return;
    std::memset(st, 0, sizeof *st);
    if (trivial) {
        st->converged = 1;
        return;
    }
    st->lowerings = c.lowerings;
    st->tile_rounds = c.tile_rounds;
    st->examinations = c.examinations;
    const bool stable = c.last_step < steps_done - 4;
    if (stable) {
        st->converged = 1;
        st->passes = c.last_step < 0 ? 1 : (uint64_t)(c.last_step / 4) + 2;
    } else {
        st->converged = 0;
        st->passes = (uint64_t)std::min(steps_done, max_steps) / 4;
    }
}

// ---------------------------------------------------------------- tiled engine

struct Plan {
    std::vector<ImgDev> imgs;
    std::vector<int32_t> tile_img;
    std::vector<int> src_index;     // position in the caller's array
};

// The instantiated graph for `key`, capturing `record` on the context's
// capture stream the first time.
template <typename F>
int chunk_graph(thin_ctx* ctx, const std::vector<uint64_t>& key, F record, hipGraphExec_t* out)
{
    auto it = ctx->graphs.find(key);
    if (it != ctx->graphs.end()) {
        *out = it->second;
        return THIN_OK;
    }
    if (ctx->graphs.size() >= 64) {
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        for (auto& kv : ctx->graphs) (void)hipGraphExecDestroy(kv.second);
        ctx->graphs.clear();
    }
    if (!ctx->cap_stream)
        HIP_TRY(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    HIP_TRY(ctx, hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
    const hipError_t e = record(ctx->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(ctx->cap_stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(ctx, THIN_EDEVICE, "graph capture failed: %s",
                    hipGetErrorString(e != hipSuccess ? e : e2));
    }
    hipGraphExec_t ge = nullptr;
    const hipError_t e3 = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e3 != hipSuccess) return fail(ctx, THIN_EDEVICE, "graph instantiation failed: %s",
                                      hipGetErrorString(e3));
    ctx->graphs[key] = ge;
    *out = ge;
    return THIN_OK;
}

int launch_worklists(thin_ctx* ctx, std::vector<thin::WlImg>& wl, std::vector<int32_t>& steps,
                     ImgCnt* d_cnt);

// Longest chunk of rounds launched between two counter reads.  A run stops
// at most one chunk past stability, so long chunks cost extra rounds; short
// ones cost a counter copy per chunk in the stream.  Runs whose rounds fit
// in one wave of blocks (small images: a round is a few microseconds of
// latency, an extra one is cheap) take chunks of up to 8 rounds (measured
// 2.5 % faster than 4 on the 512 x 512 workloads); runs with many tiles
// per round (batches, large images) take 4.  THIN_MAX_CHUNK overrides both.
int max_chunk(bool small_rounds)
{
    static int c = -1;
    if (c < 0) {
        const char* e = getenv("THIN_MAX_CHUNK");
        c = e ? std::max(1, atoi(e)) : 0;
    }
    return c ? c : (small_rounds ? 8 : 4);
}

// A single image lowering fewer than this many pixels per round (counted
// over the last chunk of rounds) has its remaining steps run by the pixel
// work-list kernel; THIN_TAIL_RATE overrides it (tuning).
double tail_rate()
{
    static double r = -1.0;
    if (r < 0.0) {
        const char* e = getenv("THIN_TAIL_RATE");
        r = e ? atof(e) : 2048.0;
    }
    return r;
}

// Device memory one tiled run works in (context-owned buffers, or carved out
// of the library's static scratch array by the no-allocation entry point).
struct TiledBufs {
    ImgDev* imgs;
    ImgCnt* cnt;
    int32_t* tile_img;    // tile -> image (unused with one image)
    int32_t* tile_last;   // 2 per tile
    uint32_t* hist_bits;  // 2 * ntiles * history_words(shape)
    int32_t* hist_round;  // 2 per tile
    int32_t* wl_list;     // 2 per tile
    int32_t* wl_meta;     // 12 + 1 per tile
    int32_t* small;       // 16 words
};

// Launches the rounds of a tiled run whose descriptors (host copy h_imgs,
// device copy b.imgs) and tile map are in place, until every image is stable
// or at its step cap, brings every image's state home into its own buffer
// and fills the statistics (stats[src_index[i]] for image i; src_index may
// be null for the identity).  allocate: graphs and profiling events may be
// created (the no-allocation entry point passes false).
int drive_tiled(thin_ctx* ctx, TileShape shape, const ImgDev* h_imgs, int nimg, int ntiles,
                const TiledBufs& b, const int* src_index, thin_stats* stats, bool allocate)
{
    const int K = shape.k;
    int max_steps_all = 0;
    for (int i = 0; i < nimg; ++i) max_steps_all = std::max(max_steps_all, h_imgs[i].max_steps);
    // (Only worth a longer dependency chain per visit when blocks visit
    // several tiles each.)
    const int grid = ctx->num_cus * thin::round_blocks_per_cu(shape);
    thin::WorkList wl{};
    wl.full = 0;
    if (ntiles > 2 * grid) wl.list = b.wl_list;
    wl.count = b.wl_meta;
    wl.grab = wl.count + 4;
    wl.listed = wl.count + 12;
    wl.cap = ntiles;
    HIP_TRY(ctx, thin::launch_init_state(ctx->stream, b.cnt, nimg, b.tile_last, ntiles,
                                         b.hist_round, wl));

    const int rounds_cap =
        (max_steps_all == INT_MAX) ? INT_MAX : (max_steps_all + K - 1) / K;
    size_t ev_used = 0;        // profiling events recorded by this call
    int launched = 0;          // rounds enqueued so far
    int chunk = 2;
    int pending = -1;          // snapshot slot in flight (-1 none)
    int pending_rounds = 0;
    bool done = false;
    auto all_done = [&](const ImgCnt* snap, int rounds) {
        for (int i = 0; i < nimg; ++i) {
            const int steps = (int)std::min<int64_t>((int64_t)rounds * K, h_imgs[i].max_steps);
            const bool stable = snap[i].last_step < steps - 4;
            if (!stable && steps < h_imgs[i].max_steps) return false;
        }
        return true;
    };
    const int kflags = thin::kStateIsTile | (nimg == 1 ? thin::kOneImage : 0);
    int dtypes = 0;
    for (int i = 0; i < nimg; ++i) dtypes |= h_imgs[i].dtype == THIN_U8 ? 1 : 2;
    const bool profile = ctx->profile && allocate;
    // Graph mode: a chunk of rounds is one graph replay; the launches read
    // their round from a device counter that the graph's last node advances.
    const bool use_graph = ctx->graph && !profile && allocate;
    int32_t* d_round = b.small + 8;
    if (use_graph) HIP_TRY(ctx, hipMemsetAsync(d_round, 0, sizeof(int32_t), ctx->stream));
    auto record_rounds = [&](hipStream_t st, int count) -> hipError_t {
        for (int k = 0; k < count; ++k) {
            const hipError_t e = launch_rounds_split(st, shape, b.imgs, b.cnt, b.tile_img,
                                                     b.tile_last, ntiles, k, ctx->d_lut,
                                                     ctx->num_cus, b.hist_bits, b.hist_round, wl,
                                                     d_round, kflags, dtypes);
            if (e != hipSuccess) return e;
        }
        return thin::launch_advance(st, d_round, count);
    };
    int rc;
    // Tail hand-over: one image whose pending bitmaps fit the work-list
    // kernel's LDS, on the default tiled path.
    const bool tail_ok = allocate && ctx->tail && nimg == 1 && !use_graph &&
                         ctx->engine == THIN_ENGINE_TILED && h_imgs[0].h <= 131070 &&
                         h_imgs[0].w <= 131070 &&
                         thin::wl_bitmap_words(h_imgs[0].h, h_imgs[0].w) <= thin::kWlLdsWords;
    bool handover = false;
    unsigned long long prev_low = 0;
    int prev_rounds = -1;
    while (!done) {
        const int n = std::min(chunk, rounds_cap - launched);
        if (use_graph) {
            hipGraphExec_t ge = nullptr;
            if (n == chunk) {
                const std::vector<uint64_t> key = {
                    (uint64_t)shape.th, (uint64_t)shape.tw, (uint64_t)shape.k, (uint64_t)shape.nt,
                    (uint64_t)shape.var, (uint64_t)ntiles, (uint64_t)grid, (uint64_t)n,
                    (uint64_t)(uintptr_t)b.imgs, (uint64_t)(uintptr_t)b.cnt,
                    (uint64_t)(uintptr_t)b.tile_img, (uint64_t)(uintptr_t)b.tile_last,
                    (uint64_t)(uintptr_t)b.hist_bits, (uint64_t)(uintptr_t)b.hist_round,
                    (uint64_t)(uintptr_t)wl.list, (uint64_t)(uintptr_t)wl.count,
                    (uint64_t)(uintptr_t)ctx->d_lut, (uint64_t)(uintptr_t)d_round,
                    // what the recorded launches bake in besides pointers and sizes:
                    // the one-image shortcut and which pixel-type launches exist
                    (uint64_t)kflags, (uint64_t)dtypes};
                if ((rc = chunk_graph(ctx, key, [&](hipStream_t st) { return record_rounds(st, n); },
                                      &ge)))
                    return rc;
                HIP_TRY(ctx, hipGraphLaunch(ge, ctx->stream));
            } else {
                HIP_TRY(ctx, record_rounds(ctx->stream, n));
            }
            launched += n;
        } else {
            for (int k = 0; k < n; ++k) {
                if (profile) {
                    if ((rc = timed_round(ctx, ev_used, shape, b.imgs, b.cnt, b.tile_img,
                                          b.tile_last, ntiles, launched, grid, b.hist_bits,
                                          b.hist_round, wl, kflags, dtypes)))
                        return rc;
                } else {
                    HIP_TRY(ctx, launch_rounds_split(ctx->stream, shape, b.imgs, b.cnt,
                                                     b.tile_img, b.tile_last, ntiles, launched,
                                                     ctx->d_lut, ctx->num_cus, b.hist_bits,
                                                     b.hist_round, wl, nullptr, kflags, dtypes));
                }
                ++launched;
            }
        }
        // Counters are read back one chunk behind (the host never waits for
        // the chunk it just launched), so a run stops at most one chunk past
        // stability; chunks stay short for that reason.
        const int slot = (pending < 0) ? 0 : 1 - pending;
        HIP_TRY(ctx, hipMemcpyAsync(ctx->h_snap[slot], b.cnt, sizeof(ImgCnt) * nimg,
                                    hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(ctx, hipEventRecord(ctx->ev[slot], ctx->stream));
        if (launched >= rounds_cap) break;
        if (pending >= 0) {
            HIP_TRY(ctx, hipEventSynchronize(ctx->ev[pending]));
            if (all_done(ctx->h_snap[pending], pending_rounds)) {
                done = true;
            } else if (tail_ok) {
                const unsigned long long low = ctx->h_snap[pending][0].lowerings;
                if (prev_rounds >= 0 && pending_rounds > prev_rounds &&
                    (double)(low - prev_low) < tail_rate() * (pending_rounds - prev_rounds)) {
                    handover = true;
                    done = true;
                }
                prev_low = low;
                prev_rounds = pending_rounds;
            }
        }
        pending = slot;
        pending_rounds = launched;
        chunk = std::min(chunk * 2, max_chunk(ntiles <= grid));
    }
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    // steps each image has run
    std::vector<int> steps_done(nimg);
    for (int i = 0; i < nimg; ++i)
        steps_done[i] = (int)std::min<int64_t>((int64_t)launched * K, h_imgs[i].max_steps);
    if (handover && steps_done[0] < h_imgs[0].max_steps) {
        // The remaining steps on the pixel work lists, in place on the
        // current state buf[launched & 1]; a candidate starts pending when a
        // pixel of its 3x3 changed during the last round (a superset of the
        // candidates the next steps need, so the result is unchanged).
        const ImgDev& d = h_imgs[0];
        thin::WlImg w{};
        w.image = d.buf[launched & 1];
        w.prev = d.buf[(launched + 1) & 1];
        w.pitch = d.pitch;
        w.h = d.h;
        w.w = d.w;
        w.dtype = d.dtype;
        w.lambda = d.lambda;
        w.adj = d.adj;
        w.step0 = steps_done[0];
        w.max_steps = d.max_steps;
        w.init = 1;
        w.slot = d.slot;
        std::vector<thin::WlImg> wl{w};
        std::vector<int32_t> st;
        if (profile) {
            while (ctx->prof_ev.size() < ev_used + 2) {
                hipEvent_t e;
                HIP_TRY(ctx, hipEventCreate(&e));
                ctx->prof_ev.push_back(e);
            }
            HIP_TRY(ctx, hipEventRecord(ctx->prof_ev[ev_used], ctx->stream));
        }
        if ((rc = launch_worklists(ctx, wl, st, b.cnt))) return rc;
        if (profile) {
            HIP_TRY(ctx, hipEventRecord(ctx->prof_ev[ev_used + 1], ctx->stream));
            HIP_TRY(ctx, hipEventSynchronize(ctx->prof_ev[ev_used + 1]));
            ev_used += 2;
        }
        steps_done[0] = st[0];
        ctx->last_tail_steps = st[0] - w.step0;
    } else {
        ctx->last_tail_steps = 0;
    }
    HIP_TRY(ctx, hipMemcpyAsync(ctx->h_snap[0], b.cnt, sizeof(ImgCnt) * nimg,
                                hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    const ImgCnt* fin = ctx->h_snap[0];
    if (profile) {
        if ((rc = collect_profile(ctx, ev_used))) return rc;
        for (int i = 0; i < nimg; ++i) ctx->prof_tile_rounds += fin[i].tile_rounds;
    }

    // Bring results home: after r rounds an image's state is in buf[r & 1],
    // where r stops growing once its step cap is reached.
    for (int i = 0; i < nimg; ++i) {
        const ImgDev& d = h_imgs[i];
        const int r_img = std::min(launched, (d.max_steps == INT_MAX) ? INT_MAX
                                                                       : (d.max_steps + K - 1) / K);
        if (r_img & 1) {
            const size_t bpp = d.dtype == THIN_U8 ? 1 : 2;
            HIP_TRY(ctx, hipMemcpy2DAsync(d.buf[0], d.pitch * bpp, d.buf[1], d.pitch * bpp,
                                          (size_t)d.w * bpp, (size_t)d.h,
                                          hipMemcpyDeviceToDevice, ctx->stream));
        }
    }
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    ctx->last_launches = launched;

    bool limited = false;
    for (int i = 0; i < nimg; ++i) {
        const ImgDev& d = h_imgs[i];
        thin_stats st;
        fill_stats(&st, fin[i], steps_done[i], d.max_steps, false);
        if (!st.converged) limited = true;
        if (stats) stats[src_index ? src_index[i] : i] = st;
    }
    return limited ? fail(ctx, THIN_ELIMIT, "max_passes reached before stability") : THIN_OK;
}

// Descriptor of image `im` for a tiled run with `shape`, its twin at `twin`,
// its tiles from tile0 on, counter slot `slot`.
ImgDev describe_tiled(const thin_image& im, TileShape shape, void* twin, int32_t tile0,
                      int32_t slot, int max_steps)
{
    ImgDev d{};
    d.buf[0] = im.image;
    d.buf[1] = twin;
    d.pitch = pitch_of(im);
    d.h = (int32_t)im.h;
    d.w = (int32_t)im.w;
    d.dtype = im.dtype;
    d.lambda = im.lambda;
    d.adj = table_index(im);
    d.tiles_y = (int32_t)((im.h + shape.th - 1) / shape.th);
    d.tiles_x = (int32_t)((im.w + shape.tw - 1) / shape.tw);
    d.tile0 = tile0;
    d.round0 = 0;
    d.max_steps = max_steps;
    d.slot = slot;
    d.state0 = d.tile0;
    return d;
}

int run_tiled(thin_ctx* ctx, const thin_image* ims, const std::vector<int>& work, thin_stats* stats)
{
    int64_t total_px = 0;
    for (int i : work) total_px += ims[i].h * ims[i].w;
    const TileShape shape = choose_shape(ctx, total_px, (int64_t)work.size());
    if (!thin::tile_shape_supported(shape))
        return fail(ctx, THIN_EINVAL, "unsupported tile shape %dx%d k=%d", shape.th, shape.tw, shape.k);
    const int max_steps = steps_cap(ctx);

    Plan plan;
    size_t twin_bytes = 0;
    std::vector<size_t> twin_off;
    for (int i : work) {
        const thin_image& im = ims[i];
        const size_t bpp = im.dtype == THIN_U8 ? 1 : 2;
        twin_off.push_back(twin_bytes);
        twin_bytes += ((size_t)im.h * (size_t)pitch_of(im) * bpp + 255) & ~size_t(255);
    }
    int rc = ensure(ctx, ctx->twin, std::max<size_t>(twin_bytes, 256));
    if (rc) return rc;
    for (size_t n = 0; n < work.size(); ++n) {
        const thin_image& im = ims[work[n]];
        const ImgDev d = describe_tiled(im, shape, static_cast<char*>(ctx->twin.ptr) + twin_off[n],
                                        (int32_t)plan.tile_img.size(),
                                        (int32_t)plan.imgs.size(), max_steps);
        const int64_t nt = (int64_t)d.tiles_x * d.tiles_y;
        if ((int64_t)plan.tile_img.size() + nt > INT_MAX / 2)
            return fail(ctx, THIN_EINVAL, "too many tiles in one call");
        for (int64_t t = 0; t < nt; ++t) plan.tile_img.push_back((int32_t)plan.imgs.size());
        plan.imgs.push_back(d);
        plan.src_index.push_back(work[n]);
    }
    const int nimg = (int)plan.imgs.size();
    const int ntiles = (int)plan.tile_img.size();
    if ((rc = ensure(ctx, ctx->imgs, sizeof(ImgDev) * nimg))) return rc;
    if ((rc = ensure(ctx, ctx->cnt, sizeof(ImgCnt) * nimg))) return rc;
    if ((rc = ensure(ctx, ctx->tile_img, sizeof(int32_t) * ntiles))) return rc;
    if ((rc = ensure(ctx, ctx->tile_last, sizeof(int32_t) * 2 * (size_t)ntiles))) return rc;
    if ((rc = ensure(ctx, ctx->hist_bits,
                     sizeof(uint32_t) * 2 * (size_t)ntiles * thin::history_words(shape))))
        return rc;
    if ((rc = ensure(ctx, ctx->hist_round, sizeof(int32_t) * 2 * (size_t)ntiles))) return rc;
    if ((rc = ensure_snap(ctx, nimg))) return rc;
    if ((rc = ensure(ctx, ctx->small, 64))) return rc;
    // Work lists: round 0 visits every tile, later rounds the tiles queued
    // by the round before.
    if ((rc = ensure(ctx, ctx->wl_list, sizeof(int32_t) * 2 * (size_t)ntiles))) return rc;
    if ((rc = ensure(ctx, ctx->wl_meta, sizeof(int32_t) * (12 + (size_t)ntiles)))) return rc;

    TiledBufs b{};
    b.imgs = static_cast<ImgDev*>(ctx->imgs.ptr);
    b.cnt = static_cast<ImgCnt*>(ctx->cnt.ptr);
    b.tile_img = static_cast<int32_t*>(ctx->tile_img.ptr);
    b.tile_last = static_cast<int32_t*>(ctx->tile_last.ptr);
    b.hist_bits = static_cast<uint32_t*>(ctx->hist_bits.ptr);
    b.hist_round = static_cast<int32_t*>(ctx->hist_round.ptr);
    b.wl_list = static_cast<int32_t*>(ctx->wl_list.ptr);
    b.wl_meta = static_cast<int32_t*>(ctx->wl_meta.ptr);
    b.small = static_cast<int32_t*>(ctx->small.ptr);
    HIP_TRY(ctx, hipMemcpyAsync(b.imgs, plan.imgs.data(), sizeof(ImgDev) * nimg,
                                hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(b.tile_img, plan.tile_img.data(), sizeof(int32_t) * ntiles,
                                hipMemcpyHostToDevice, ctx->stream));
    return drive_tiled(ctx, shape, plan.imgs.data(), nimg, ntiles, b, plan.src_index.data(), stats,
                       true);
}

// ---------------------------------------------------------- cooperative engine

int run_coop(thin_ctx* ctx, const thin_image* ims, const std::vector<int>& work, thin_stats* stats)
{
    int64_t total_px = 0;
    int dtypes = 0;
    for (int i : work) {
        total_px += ims[i].h * ims[i].w;
        dtypes |= ims[i].dtype == THIN_U8 ? 1 : 2;
    }
    TileShape shape = choose_shape(ctx, total_px, (int64_t)work.size());
    // One cooperative launch runs every image, so a bit-flag shape (LDS tile
    // in the pixel type) needs a single pixel type; mixed calls take the flag
    // variant.
    if (bits_variant(shape) && dtypes == 3) shape = TileShape{64, 64, 16, 512, thin::kVarFlags};
    const int coop_flags = bits_variant(shape) ? (dtypes == 1 ? thin::kOnlyU8 : thin::kOnlyU16) : 0;
    if (!thin::tile_shape_supported(shape))
        return fail(ctx, THIN_EINVAL, "unsupported tile shape %dx%d k=%d", shape.th, shape.tw, shape.k);
    const int K = shape.k;
    const int max_steps = steps_cap(ctx);

    Plan plan;
    size_t twin_bytes = 0;
    std::vector<size_t> twin_off;
    for (int i : work) {
        const thin_image& im = ims[i];
        const size_t bpp = im.dtype == THIN_U8 ? 1 : 2;
        twin_off.push_back(twin_bytes);
        twin_bytes += ((size_t)im.h * (size_t)pitch_of(im) * bpp + 255) & ~size_t(255);
    }
    int rc = ensure(ctx, ctx->twin, std::max<size_t>(twin_bytes, 256));
    if (rc) return rc;
    for (size_t n = 0; n < work.size(); ++n) {
        const thin_image& im = ims[work[n]];
        ImgDev d{};
        d.buf[0] = im.image;
        d.buf[1] = static_cast<char*>(ctx->twin.ptr) + twin_off[n];
        d.pitch = pitch_of(im);
        d.h = (int32_t)im.h;
        d.w = (int32_t)im.w;
        d.dtype = im.dtype;
        d.lambda = im.lambda;
        d.adj = table_index(im);
        d.tiles_y = (int32_t)((im.h + shape.th - 1) / shape.th);
        d.tiles_x = (int32_t)((im.w + shape.tw - 1) / shape.tw);
        d.tile0 = (int32_t)plan.tile_img.size();
        d.round0 = 0;
        d.max_steps = max_steps;
        d.slot = (int32_t)plan.imgs.size();
        d.state0 = d.tile0;
        const int64_t nt = (int64_t)d.tiles_x * d.tiles_y;
        if ((int64_t)plan.tile_img.size() + nt > INT_MAX / 2)
            return fail(ctx, THIN_EINVAL, "too many tiles in one call");
        for (int64_t t = 0; t < nt; ++t) plan.tile_img.push_back((int32_t)plan.imgs.size());
        plan.imgs.push_back(d);
        plan.src_index.push_back(work[n]);
    }
    const int nimg = (int)plan.imgs.size();
    const int ntiles = (int)plan.tile_img.size();
    if ((rc = ensure(ctx, ctx->imgs, sizeof(ImgDev) * nimg))) return rc;
    if ((rc = ensure(ctx, ctx->cnt, sizeof(ImgCnt) * nimg))) return rc;
    if ((rc = ensure(ctx, ctx->tile_img, sizeof(int32_t) * ntiles))) return rc;
    if ((rc = ensure(ctx, ctx->tile_last, sizeof(int32_t) * 2 * (size_t)ntiles))) return rc;
    if ((rc = ensure(ctx, ctx->small, 64))) return rc;
    if ((rc = ensure(ctx, ctx->hist_bits,
                     sizeof(uint32_t) * 2 * (size_t)ntiles * thin::history_words(shape))))
        return rc;
    if ((rc = ensure(ctx, ctx->hist_round, sizeof(int32_t) * 2 * (size_t)ntiles))) return rc;
    if ((rc = ensure_snap(ctx, nimg))) return rc;

    ImgDev* d_imgs = static_cast<ImgDev*>(ctx->imgs.ptr);
    ImgCnt* d_cnt = static_cast<ImgCnt*>(ctx->cnt.ptr);
    int32_t* d_tile_img = static_cast<int32_t*>(ctx->tile_img.ptr);
    int32_t* d_tile_last = static_cast<int32_t*>(ctx->tile_last.ptr);
    int32_t* d_small = static_cast<int32_t*>(ctx->small.ptr);  // [0..2] active, [3] rounds
    HIP_TRY(ctx, hipMemcpyAsync(d_imgs, plan.imgs.data(), sizeof(ImgDev) * nimg,
                                hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(d_tile_img, plan.tile_img.data(), sizeof(int32_t) * ntiles,
                                hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, hipMemsetAsync(d_small, 0, 4 * sizeof(int32_t), ctx->stream));
    HIP_TRY(ctx, thin::launch_init_state(ctx->stream, d_cnt, nimg, d_tile_last, ntiles,
                                         static_cast<int32_t*>(ctx->hist_round.ptr),
                                         thin::WorkList{}));
    const int rounds_cap = (max_steps == INT_MAX) ? INT_MAX : (max_steps + K - 1) / K;
    size_t ev_used = 0;
    if (ctx->profile) {
        while (ctx->prof_ev.size() < 2) {
            hipEvent_t e;
            HIP_TRY(ctx, hipEventCreate(&e));
            ctx->prof_ev.push_back(e);
        }
        HIP_TRY(ctx, hipEventRecord(ctx->prof_ev[0], ctx->stream));
    }
    HIP_TRY(ctx, thin::launch_coop(ctx->stream, shape, d_imgs, d_cnt, d_tile_img, d_tile_last,
                                   ntiles, ctx->d_lut, d_small, d_small + 3, rounds_cap,
                                   ctx->num_cus, static_cast<uint32_t*>(ctx->hist_bits.ptr),
                                   static_cast<int32_t*>(ctx->hist_round.ptr),
                                   thin::kStateIsTile | (nimg == 1 ? thin::kOneImage : 0) |
                                       coop_flags));
    if (ctx->profile) {
        HIP_TRY(ctx, hipEventRecord(ctx->prof_ev[1], ctx->stream));
        ev_used = 2;
    }
    int32_t rounds = 0;
    HIP_TRY(ctx, hipMemcpyAsync(ctx->h_snap[0], d_cnt, sizeof(ImgCnt) * nimg,
                                hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    HIP_TRY(ctx, hipMemcpy(&rounds, d_small + 3, sizeof rounds, hipMemcpyDeviceToHost));
    const ImgCnt* fin = ctx->h_snap[0];
    if (ctx->profile) {
        if ((rc = collect_profile(ctx, ev_used))) return rc;
        for (int i = 0; i < nimg; ++i) ctx->prof_tile_rounds += fin[i].tile_rounds;
    }
    bool limited = false;
    for (int i = 0; i < nimg; ++i) {
        const ImgDev& d = plan.imgs[i];
        const int r_img = std::min(rounds, (d.max_steps == INT_MAX) ? INT_MAX
                                                                   : (d.max_steps + K - 1) / K);
        if (r_img & 1) {
            const size_t bpp = d.dtype == THIN_U8 ? 1 : 2;
            HIP_TRY(ctx, hipMemcpy2DAsync(d.buf[0], d.pitch * bpp, d.buf[1], d.pitch * bpp,
                                          (size_t)d.w * bpp, (size_t)d.h,
                                          hipMemcpyDeviceToDevice, ctx->stream));
        }
        const int steps = (int)std::min<int64_t>((int64_t)rounds * K, d.max_steps);
        thin_stats st;
        fill_stats(&st, fin[i], steps, d.max_steps, false);
        if (!st.converged) limited = true;
        if (stats) stats[plan.src_index[i]] = st;
    }
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return limited ? fail(ctx, THIN_ELIMIT, "max_passes reached before stability") : THIN_OK;
}

// ----------------------------------------------------------------- step engine

int run_step_engine(thin_ctx* ctx, const thin_image* ims, const std::vector<int>& work,
                    thin_stats* stats)
{
    int rc;
    if ((rc = ensure(ctx, ctx->imgs, sizeof(ImgDev)))) return rc;
    if ((rc = ensure(ctx, ctx->cnt, sizeof(ImgCnt)))) return rc;
    if ((rc = ensure_snap(ctx, 1))) return rc;
    const int max_steps = steps_cap(ctx);
    bool limited = false;
    for (int i : work) {
        const thin_image& im = ims[i];
        if (im.h > 131070) return fail(ctx, THIN_EINVAL, "step engine supports h <= 131070");
        ImgDev d{};
        d.buf[0] = d.buf[1] = im.image;
        d.pitch = pitch_of(im);
        d.h = (int32_t)im.h;
        d.w = (int32_t)im.w;
        d.dtype = im.dtype;
        d.lambda = im.lambda;
        d.adj = table_index(im);
        d.max_steps = max_steps;
        ImgDev* d_img = static_cast<ImgDev*>(ctx->imgs.ptr);
        ImgCnt* d_cnt = static_cast<ImgCnt*>(ctx->cnt.ptr);
        HIP_TRY(ctx, hipMemcpyAsync(d_img, &d, sizeof d, hipMemcpyHostToDevice, ctx->stream));
        HIP_TRY(ctx, thin::launch_init_state(ctx->stream, d_cnt, 1, nullptr, 0, nullptr,
                                             thin::WorkList{}));
        int step = 0;
        for (;;) {
            for (int s = 0; s < 4 && step < max_steps; ++s, ++step)
                HIP_TRY(ctx, thin::launch_step(ctx->stream, &d, d_img, d_cnt, step, ctx->d_lut));
            HIP_TRY(ctx, hipMemcpyAsync(ctx->h_snap[0], d_cnt, sizeof(ImgCnt),
                                        hipMemcpyDeviceToHost, ctx->stream));
            HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
            if (ctx->h_snap[0]->last_step < step - 4 || step >= max_steps) break;
        }
        thin_stats st;
        fill_stats(&st, *ctx->h_snap[0], step, max_steps, false);
        if (!st.converged) limited = true;
        if (stats) stats[i] = st;
    }
    return limited ? fail(ctx, THIN_ELIMIT, "max_passes reached before stability") : THIN_OK;
}

// ------------------------------------------------------- pixel work-list engine

// Runs k_worklist on the images `wl` (descriptors on the host, counters in
// slots 0..n-1 already cleared), one launch per pixel type and bitmap home;
// steps[i] receives one past the last global step image i ran.
int launch_worklists(thin_ctx* ctx, std::vector<thin::WlImg>& wl, std::vector<int32_t>& steps,
                     ImgCnt* d_cnt)
{
    const int n = (int)wl.size();
    int rc;
    uint64_t gwords = 0;
    for (const thin::WlImg& w : wl)
        if (thin::wl_bitmap_words(w.h, w.w) > thin::kWlLdsWords) gwords += thin::wl_bitmap_words(w.h, w.w);
    if ((rc = ensure(ctx, ctx->wl_imgs, sizeof(thin::WlImg) * n + sizeof(int32_t) * n + 256))) return rc;
    if (gwords && (rc = ensure(ctx, ctx->wl_bits, sizeof(uint32_t) * gwords))) return rc;
    uint64_t goff = 0;
    for (thin::WlImg& w : wl) {
        const int64_t words = thin::wl_bitmap_words(w.h, w.w);
        w.gbits = nullptr;
        if (words > thin::kWlLdsWords) {
            w.gbits = static_cast<uint32_t*>(ctx->wl_bits.ptr) + goff;
            goff += (uint64_t)words;
        }
    }
    // group by (pixel type, bitmap home): each group is one launch
    std::vector<thin::WlImg> order;
    std::vector<int> index;
    std::vector<std::pair<int, int>> groups;  // (first, count)
    for (int dt = 1; dt <= 2; ++dt)
        for (int g = 0; g < 2; ++g) {
            const int first = (int)order.size();
            for (int i = 0; i < n; ++i)
                if (wl[i].dtype == dt && (wl[i].gbits != nullptr) == (g == 1)) {
                    order.push_back(wl[i]);
                    index.push_back(i);
                }
            groups.push_back({first, (int)order.size() - first});
        }
    thin::WlImg* d_wl = static_cast<thin::WlImg*>(ctx->wl_imgs.ptr);
    int32_t* d_steps = reinterpret_cast<int32_t*>(d_wl + n);
    HIP_TRY(ctx, hipMemcpyAsync(d_wl, order.data(), sizeof(thin::WlImg) * n, hipMemcpyHostToDevice,
                                ctx->stream));
    for (int k = 0; k < 4; ++k) {
        const int first = groups[k].first, cnt = groups[k].second;
        if (!cnt) continue;
        HIP_TRY(ctx, thin::launch_worklist(ctx->stream, d_wl + first, cnt, 1 + k / 2, (k & 1) != 0,
                                           d_cnt, ctx->d_lut, d_steps + first));
    }
    std::vector<int32_t> st(n);
    HIP_TRY(ctx, hipMemcpyAsync(st.data(), d_steps, sizeof(int32_t) * n, hipMemcpyDeviceToHost,
                                ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    steps.assign(n, 0);
    for (int i = 0; i < n; ++i) steps[index[i]] = st[i];
    return THIN_OK;
}

thin::WlImg describe_worklist(const thin_image& im, int slot, int max_steps)
{
    thin::WlImg w{};
    w.image = im.image;
    w.pitch = pitch_of(im);
    w.h = (int32_t)im.h;
    w.w = (int32_t)im.w;
    w.dtype = im.dtype;
    w.lambda = im.lambda;
    w.adj = table_index(im);
    w.step0 = 0;
    w.max_steps = max_steps;
    w.init = 0;
    w.slot = slot;
    return w;
}

int run_worklist(thin_ctx* ctx, const thin_image* ims, const std::vector<int>& work,
                 thin_stats* stats)
{
    const int n = (int)work.size();
    for (int i : work)
        if (ims[i].h > 131070 || ims[i].w > 131070)
            return fail(ctx, THIN_EINVAL, "the work-list engine takes sides up to 131070");
    int rc;
    if ((rc = ensure(ctx, ctx->cnt, sizeof(ImgCnt) * n))) return rc;
    if ((rc = ensure_snap(ctx, n))) return rc;
    ImgCnt* d_cnt = static_cast<ImgCnt*>(ctx->cnt.ptr);
    HIP_TRY(ctx, thin::launch_init_state(ctx->stream, d_cnt, n, nullptr, 0, nullptr,
                                         thin::WorkList{}));
    const int max_steps = steps_cap(ctx);
    std::vector<thin::WlImg> wl;
    for (int k = 0; k < n; ++k) wl.push_back(describe_worklist(ims[work[k]], k, max_steps));
    std::vector<int32_t> steps;
    if ((rc = launch_worklists(ctx, wl, steps, d_cnt))) return rc;
    HIP_TRY(ctx, hipMemcpyAsync(ctx->h_snap[0], d_cnt, sizeof(ImgCnt) * n, hipMemcpyDeviceToHost,
                                ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    bool limited = false;
    for (int k = 0; k < n; ++k) {
        thin_stats st;
        fill_stats(&st, ctx->h_snap[0][k], steps[k], max_steps, false);
        if (!st.converged) limited = true;
        if (stats) stats[work[k]] = st;
    }
    return limited ? fail(ctx, THIN_ELIMIT, "max_passes reached before stability") : THIN_OK;
}

int run_images(thin_ctx* ctx, const thin_image* ims, int n, thin_stats* stats)
{
    if (!ctx) return THIN_EINVAL;
    if (n < 0 || (n > 0 && !ims)) return fail(ctx, THIN_EINVAL, "bad image list");
    for (int i = 0; i < n; ++i) {
        const int rc = validate(ctx, ims[i]);
        if (rc) return rc;
    }
    std::vector<int> work;
    for (int i = 0; i < n; ++i) {
        if (ims[i].h < 3 || ims[i].w < 3) {
            if (stats) fill_stats(&stats[i], ImgCnt{}, 0, 0, true);
        } else {
            work.push_back(i);
        }
    }
    if (work.empty()) return THIN_OK;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    if (ctx->engine == THIN_ENGINE_STEP) return run_step_engine(ctx, ims, work, stats);
    if (ctx->engine == THIN_ENGINE_WORKLIST) return run_worklist(ctx, ims, work, stats);
    if (ctx->engine == THIN_ENGINE_COOP) return run_coop(ctx, ims, work, stats);
    return run_tiled(ctx, ims, work, stats);
}

// One tiled run over `work` of ims with `shape` forced; wall time in ms
// (the run synchronises the stream before returning).
int timed_run(thin_ctx* ctx, const thin_image* ims, const std::vector<int>& work, TileShape shape,
              double& ms)
{
    const TileShape saved = ctx->forced;
    ctx->forced = shape;
    const auto t0 = std::chrono::steady_clock::now();
    int rc = run_tiled(ctx, ims, work, nullptr);
    const auto t1 = std::chrono::steady_clock::now();
    ctx->forced = saved;
    if (rc == THIN_ELIMIT) rc = THIN_OK;
    ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    return rc;
}

int autotune(thin_ctx* ctx, const thin_image* imgs, int n, int reps, thin_tune_result* out)
{
    if (n <= 0 || !imgs || reps < 1) return fail(ctx, THIN_EINVAL, "bad autotune arguments");
    for (int i = 0; i < n; ++i) {
        const int rc = validate(ctx, imgs[i]);
        if (rc) return rc;
    }
    // Contiguous copies of the images that matter: pristine and working.
    std::vector<thin_image> work_img;
    std::vector<size_t> off;
    size_t bytes = 0;
    int64_t total_px = 0;
    for (int i = 0; i < n; ++i) {
        if (imgs[i].h < 3 || imgs[i].w < 3) continue;
        thin_image c = imgs[i];
        c.pitch_elems = c.w;
        off.push_back(bytes);
        bytes += ((size_t)c.h * (size_t)c.w * (c.dtype == THIN_U8 ? 1 : 2) + 255) & ~size_t(255);
        total_px += c.h * c.w;
        work_img.push_back(c);
    }
    if (work_img.empty()) return fail(ctx, THIN_EINVAL, "no image of at least 3x3 to tune on");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    void *pristine = nullptr, *scratch = nullptr;
    if (hipMalloc(&pristine, bytes) != hipSuccess || hipMalloc(&scratch, bytes) != hipSuccess) {
        (void)hipGetLastError();
        if (pristine) (void)hipFree(pristine);
        return fail(ctx, THIN_ENOMEM, "autotune copies of %zu bytes", 2 * bytes);
    }
    int rc = THIN_OK;
    std::vector<int> work;
    for (size_t k = 0, j = 0; k < (size_t)n; ++k) {
        const thin_image& im = imgs[k];
        if (im.h < 3 || im.w < 3) continue;
        const size_t bpp = im.dtype == THIN_U8 ? 1 : 2;
        const size_t pitch = (size_t)(im.pitch_elems ? im.pitch_elems : im.w) * bpp;
        if (hipMemcpy2DAsync(static_cast<char*>(pristine) + off[j], (size_t)im.w * bpp, im.image,
                             pitch, (size_t)im.w * bpp, (size_t)im.h, hipMemcpyDeviceToDevice,
                             ctx->stream) != hipSuccess) {
            rc = fail(ctx, THIN_EDEVICE, "autotune copy failed");
            break;
        }
        work_img[j].image = static_cast<char*>(scratch) + off[j];
        work.push_back((int)j);
        ++j;
    }
    auto run_one = [&](TileShape shape, double& ms) -> int {
        if (hipMemcpyAsync(scratch, pristine, bytes, hipMemcpyDeviceToDevice, ctx->stream) !=
                hipSuccess ||
            hipStreamSynchronize(ctx->stream) != hipSuccess)
            return fail(ctx, THIN_EDEVICE, "autotune copy failed");
        return timed_run(ctx, work_img.data(), work, shape, ms);
    };
    thin_tune_result res{};
    TileShape best{0, 0, 0, 0, 0};
    if (rc == THIN_OK) {
        // Untuned choice first (also warms the context's buffers).
        const auto cls = size_class(total_px, (int64_t)work_img.size());
        const auto prev = ctx->tuned.find(cls);
        TileShape prev_shape{0, 0, 0, 0, 0};
        if (prev != ctx->tuned.end()) {
            prev_shape = prev->second;
            ctx->tuned.erase(prev);
        }
        const TileShape dflt = choose_shape(ctx, total_px, (int64_t)work_img.size());
        double ms = 0.0;
        if ((rc = run_one(dflt, ms)) == THIN_OK) rc = run_one(dflt, ms);
        res.default_ms = ms;
        std::vector<TileShape> shapes(thin::compiled_shapes(nullptr, 0));
        thin::compiled_shapes(shapes.data(), (int)shapes.size());
        std::vector<std::pair<double, TileShape>> timed;
        for (const TileShape& sh : shapes) {
            if (rc) break;
            double t = 0.0;
            const int r = run_one(sh, t);
            if (r == THIN_EDEVICE) {
                rc = r;
                break;
            }
            if (r == THIN_OK) timed.push_back({t, sh});
        }
        std::sort(timed.begin(), timed.end(),
                  [](const std::pair<double, TileShape>& a, const std::pair<double, TileShape>& b) {
                      return a.first < b.first;
                  });
        const size_t finalists = std::min<size_t>(timed.size(), 3);
        for (size_t f = 0; f < finalists && rc == THIN_OK; ++f)
            for (int k = 1; k < reps && rc == THIN_OK; ++k) {
                double t = 0.0;
                rc = run_one(timed[f].second, t);
                timed[f].first = std::min(timed[f].first, t);
            }
        if (rc == THIN_OK && !timed.empty()) {
            size_t b = 0;
            for (size_t f = 1; f < finalists; ++f)
                if (timed[f].first < timed[b].first) b = f;
            best = timed[b].second;
            res.ms = timed[b].first;
            res.candidates = (int32_t)timed.size();
            ctx->tuned[cls] = best;
            save_tune_cache(ctx, cls, best, res.ms);
        } else if (prev_shape.th) {
            ctx->tuned[cls] = prev_shape;
        }
    }
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(pristine);
    (void)hipFree(scratch);
    if (rc) return rc;
    if (!best.th) return fail(ctx, THIN_EDEVICE, "no tile shape ran");
    res.tile_h = best.th;
    res.tile_w = best.tw;
    res.steps_per_round = best.k;
    res.threads = best.nt;
    res.variant = best.var;
    if (out) *out = res;
    return THIN_OK;
}

// thin_run_noalloc: one image on the tiled engine with every scratch buffer
// carved out of this device's copy of the static scratch array (no device or
// pinned allocation; the counter snapshots were allocated by thin_create).
int run_noalloc(thin_ctx* ctx, const thin_image& im, thin_stats* stats)
{
    int rc = validate(ctx, im);
    if (rc) return rc;
    if (im.h < 3 || im.w < 3) {
        if (stats) fill_stats(stats, ImgCnt{}, 0, 0, true);
        return THIN_OK;
    }
    if (ctx->engine != THIN_ENGINE_TILED)
        return fail(ctx, THIN_EINVAL, "thin_run_noalloc runs on the tiled engine only");
    if (!ctx->noalloc || ctx->h_snap_cap < 1)
        return fail(ctx, THIN_EDEVICE, "the static scratch array was not set up by thin_create");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    const TileShape shape = choose_shape(ctx, im.h * im.w, 1);
    if (!thin::tile_shape_supported(shape))
        return fail(ctx, THIN_EINVAL, "unsupported tile shape %dx%d k=%d", shape.th, shape.tw, shape.k);
    const uint64_t ty = (uint64_t)((im.h + shape.th - 1) / shape.th);
    const uint64_t tx = (uint64_t)((im.w + shape.tw - 1) / shape.tw);
    const uint64_t ntiles = ty * tx;
    const uint64_t bpp = im.dtype == THIN_U8 ? 1 : 2;
    // Layout, each part 256-byte aligned: descriptor, counters, 16 words,
    // per-tile state, change bitmaps and rounds, tile queues, then the twin.
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        const uint64_t at = off;
        off += (bytes + 255) & ~uint64_t(255);
        return at;
    };
    const uint64_t o_imgs = take(sizeof(ImgDev));
    const uint64_t o_cnt = take(sizeof(ImgCnt));
    const uint64_t o_small = take(16 * sizeof(int32_t));
    const uint64_t o_last = take(2 * ntiles * sizeof(int32_t));
    const uint64_t o_bits = take(2 * ntiles * (uint64_t)thin::history_words(shape) * sizeof(uint32_t));
    const uint64_t o_hround = take(2 * ntiles * sizeof(int32_t));
    const uint64_t o_list = take(2 * ntiles * sizeof(int32_t));
    const uint64_t o_meta = take((12 + ntiles) * sizeof(int32_t));
    const uint64_t o_twin = take((uint64_t)im.h * (uint64_t)pitch_of(im) * bpp);
    if (off > thin::kNoAllocScratchBytes || ntiles > (uint64_t)INT_MAX / 2)
        return fail(ctx, THIN_ENOMEM,
                    "a %lldx%lld image needs %llu bytes of scratch; thin_run_noalloc has %llu",
                    (long long)im.h, (long long)im.w, (unsigned long long)off,
                    (unsigned long long)thin::kNoAllocScratchBytes);
    char* base = static_cast<char*>(ctx->noalloc);
    TiledBufs b{};
    b.imgs = reinterpret_cast<ImgDev*>(base + o_imgs);
    b.cnt = reinterpret_cast<ImgCnt*>(base + o_cnt);
    b.tile_img = nullptr;  // one image: the kernels never read the tile map
    b.tile_last = reinterpret_cast<int32_t*>(base + o_last);
    b.hist_bits = reinterpret_cast<uint32_t*>(base + o_bits);
    b.hist_round = reinterpret_cast<int32_t*>(base + o_hround);
    b.wl_list = reinterpret_cast<int32_t*>(base + o_list);
    b.wl_meta = reinterpret_cast<int32_t*>(base + o_meta);
    b.small = reinterpret_cast<int32_t*>(base + o_small);
    const ImgDev d = describe_tiled(im, shape, base + o_twin, 0, 0, steps_cap(ctx));
    HIP_TRY(ctx, thin::launch_set_desc(ctx->stream, b.imgs, d));
    return drive_tiled(ctx, shape, &d, 1, (int)ntiles, b, nullptr, stats, false);
}

}  // namespace

// ------------------------------------------------------------------------- ABI

extern "C" {

int thin_create(thin_ctx** out, const thin_config* cfg)
{
    if (!out) return THIN_EINVAL;
    *out = nullptr;
    thin_config c{};
    if (cfg) c = *cfg;
    if (c.engine < 0 || c.engine > THIN_ENGINE_WORKLIST || c.engine == 3) return THIN_EINVAL;
    if ((c.tile != 0) != (c.steps_per_round != 0)) return THIN_EINVAL;
    TileShape forced{0, 0, 0, 0, 0};
    if (c.tile && c.threads) {
        forced = TileShape{c.tile, c.tile, c.steps_per_round, c.threads, c.variant};
        if (!thin::tile_shape_supported(forced)) return THIN_EINVAL;
    } else if (c.tile) {
        forced = thin::complete_shape(c.tile, c.tile, c.steps_per_round);
        if (!forced.nt) return THIN_EINVAL;
    }
    // THIN_TILE_SHAPE="th,tw,k,threads,variant" selects any compiled shape (tuning).
    if (const char* env = getenv("THIN_TILE_SHAPE")) {
        TileShape e{0, 0, 0, 0, 0};
        if (sscanf(env, "%d,%d,%d,%d,%d", &e.th, &e.tw, &e.k, &e.nt, &e.var) == 5 &&
            thin::tile_shape_supported(e))
            forced = e;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        (void)hipGetLastError();
        return THIN_EDEVICE;
    }
    if (c.device < 0 || c.device >= ndev) return THIN_EINVAL;
    thin_ctx* ctx = new (std::nothrow) thin_ctx();
    if (!ctx) return THIN_ENOMEM;
    ctx->device = c.device;
    ctx->engine = c.engine == THIN_ENGINE_AUTO ? THIN_ENGINE_TILED : c.engine;
    ctx->stream = static_cast<hipStream_t>(c.hip_stream);
    ctx->max_device_bytes = c.max_device_bytes;
    ctx->max_passes = c.max_passes;
    ctx->forced = forced;
    ctx->profile = (c.flags & THIN_FLAG_PROFILE) != 0;
    ctx->tail = (c.flags & THIN_FLAG_TAIL) != 0;
    ctx->graph = (c.flags & THIN_FLAG_GRAPH) != 0;
    int rc = THIN_OK;
    do {
        if (hipSetDevice(c.device) != hipSuccess) { rc = THIN_EDEVICE; break; }
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c.device) == hipSuccess &&
            cus > 0)
            ctx->num_cus = cus;
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, c.device) == hipSuccess) {
            // "gfx950:sramecc+:xnack-" -> "gfx950"
            std::string name = prop.gcnArchName;
            ctx->arch = name.substr(0, name.find(':'));
        }
        if (c.tune_cache) {
            ctx->tune_cache = c.tune_cache;
            load_tune_cache(ctx);
        }
        TopoEntry table[thin::kTables * 256];
        for (int t = 0; t < thin::kTables; ++t)
            thin::build_topology_table(t & 1, t >> 1, table + 256 * t);
        if (hipMalloc((void**)&ctx->d_lut, sizeof table) != hipSuccess) { rc = THIN_ENOMEM; break; }
        if (hipMemcpy(ctx->d_lut, table, sizeof table, hipMemcpyHostToDevice) != hipSuccess) {
            rc = THIN_EDEVICE;
            break;
        }
        for (int i = 0; i < 2; ++i)
            if (hipEventCreateWithFlags(&ctx->ev[i], hipEventDisableTiming) != hipSuccess) {
                rc = THIN_EDEVICE;
                break;
            }
        if (rc != THIN_OK) break;
        // Counter snapshots for up to 64 images now, so that the no-allocation
        // entry point finds them; and this device's copy of its scratch array.
        if (ensure_snap(ctx, 64) != THIN_OK) { rc = THIN_ENOMEM; break; }
        if (thin::noalloc_scratch(c.device, &ctx->noalloc) != hipSuccess) { rc = THIN_EDEVICE; break; }
    } while (0);
    if (rc != THIN_OK) {
        (void)hipGetLastError();
        thin_destroy(ctx);
        return rc;
    }
    *out = ctx;
    return THIN_OK;
}

int thin_run(thin_ctx* ctx, void* image, int64_t h, int64_t w, int32_t dtype, uint32_t lambda,
             int32_t adjacency, thin_stats* stats)
{
    thin_image im{};
    im.image = image;
    im.h = h;
    im.w = w;
    im.pitch_elems = w;
    im.dtype = dtype;
    im.lambda = lambda;
    im.adjacency = adjacency;
    return run_images(ctx, &im, 1, stats);
}

int thin_run_noalloc(thin_ctx* ctx, void* image, int64_t h, int64_t w, int32_t dtype,
                     uint32_t lambda, int32_t adjacency, thin_stats* stats)
{
    if (!ctx) return THIN_EINVAL;
    thin_image im{};
    im.image = image;
    im.h = h;
    im.w = w;
    im.pitch_elems = w;
    im.dtype = dtype;
    im.lambda = lambda;
    im.adjacency = adjacency;
    return run_noalloc(ctx, im, stats);
}

int thin_skeleton(thin_ctx* ctx, void* image, int64_t h, int64_t w, int32_t dtype,
                  uint32_t lambda, int32_t adjacency, thin_stats* stats)
{
    thin_image im{};
    im.image = image;
    im.h = h;
    im.w = w;
    im.pitch_elems = w;
    im.dtype = dtype;
    im.lambda = lambda;
    im.adjacency = adjacency;
    im.op = THIN_OP_SKELETON;
    return run_images(ctx, &im, 1, stats);
}

int thin_run_batch(thin_ctx* ctx, const thin_image* imgs, int32_t n, thin_stats* stats)
{
    return run_images(ctx, imgs, n, stats);
}

int thin_autotune(thin_ctx* ctx, const thin_image* imgs, int32_t n, int32_t reps,
                  thin_tune_result* out)
{
    if (!ctx) return THIN_EINVAL;
    return autotune(ctx, imgs, n, reps, out);
}

int thin_destroy(thin_ctx* ctx)
{
    if (!ctx) return THIN_OK;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    else (void)hipDeviceSynchronize();
    DevBuf* bufs[] = {&ctx->twin,       &ctx->imgs,        &ctx->cnt,        &ctx->tile_img,
                      &ctx->tile_last,  &ctx->small,      &ctx->wl_list,    &ctx->wl_meta,
                      &ctx->hist_bits,  &ctx->hist_round,  &ctx->serve_twin, &ctx->serve_state,
                      &ctx->serve_cnt,  &ctx->serve_imgs,  &ctx->serve_tile_img, &ctx->grad,
                      &ctx->wl_imgs,    &ctx->wl_bits};
    for (DevBuf* b : bufs)
        if (b->ptr) (void)hipFree(b->ptr);
    if (ctx->d_lut) (void)hipFree(ctx->d_lut);
    for (int i = 0; i < 2; ++i) {
        if (ctx->h_snap[i]) (void)hipHostFree(ctx->h_snap[i]);
        if (ctx->ev[i]) (void)hipEventDestroy(ctx->ev[i]);
    }
    for (hipEvent_t e : ctx->prof_ev) (void)hipEventDestroy(e);
    if (ctx->serve_snap) (void)hipHostFree(ctx->serve_snap);
    for (auto& kv : ctx->graphs) (void)hipGraphExecDestroy(kv.second);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    delete ctx;
    return THIN_OK;
}

const char* thin_strerror(int code)
{
    switch (code) {
    case THIN_OK: return "ok";
    case THIN_EINVAL: return "invalid argument";
    case THIN_ENOMEM: return "out of device memory or above max_device_bytes";
    case THIN_EDEVICE: return "HIP device error";
    case THIN_ELIMIT: return "max_passes reached before stability";
    case THIN_EBUSY: return "device-memory budget exhausted; try again later";
    default: return "unknown error";
    }
}

const char* thin_last_error(const thin_ctx* ctx)
{
    return ctx ? ctx->last_error.c_str() : "";
}

int thin_profile(thin_ctx* ctx, thin_profile_info* out, int32_t reset)
{
    if (!ctx || !out) return THIN_EINVAL;
    out->launches = ctx->prof_launches;
    out->kernel_ms = ctx->prof_ms;
    out->tile_rounds = ctx->prof_tile_rounds;
    if (reset) {
        ctx->prof_launches = 0;
        ctx->prof_ms = 0.0;
        ctx->prof_tile_rounds = 0;
    }
    return THIN_OK;
}

namespace {

// Coefficients of the gradient front-end, computed in double from the
// float32 alpha and rounded once to float32.
thin::GradCoef gradient_coef(float alpha)
{
    const double a = alpha;
    const double r = std::exp(-a);
    const double k = (1.0 - r) * (1.0 - r) / (1.0 + 2.0 * a * r - r * r);
    const double c = (1.0 - r) * (1.0 - r) * (1.0 - r) / (2.0 * r * (1.0 + r));
    const double a0 = k, a1 = k * (a - 1.0) * r, a2 = k * (a + 1.0) * r, a3 = -k * r * r;
    const double d1 = -c * r, d2 = c * r, b1 = 2.0 * r, b2 = -r * r;
    const double den = 1.0 - b1 - b2;
    thin::GradCoef co;
    co.a0 = (float)a0;
    co.a1 = (float)a1;
    co.a2 = (float)a2;
    co.a3 = (float)a3;
    co.d1 = (float)d1;
    co.d2 = (float)d2;
    co.b1 = (float)b1;
    co.b2 = (float)b2;
    co.s_plus = (float)((a0 + a1) / den);
    co.s_minus = (float)((a2 + a3) / den);
    co.d_plus = (float)(d1 / den);
    co.d_minus = (float)(d2 / den);
    return co;
}

}  // namespace

int thin_gradient_coefficients(float alpha, float* out, int32_t n)
{
    if (!out || n < 12 || !(alpha > 0.0f) || !std::isfinite(alpha)) return THIN_EINVAL;
    const thin::GradCoef co = gradient_coef(alpha);
    const float v[12] = {co.a0, co.a1, co.a2, co.a3, co.d1, co.d2,
                         co.b1, co.b2, co.s_plus, co.s_minus, co.d_plus, co.d_minus};
    for (int i = 0; i < 12; ++i) out[i] = v[i];
    return THIN_OK;
}

int thin_gradient(thin_ctx* ctx, const void* src, int64_t h, int64_t w, int64_t src_pitch,
                  int32_t src_dtype, float alpha, float gain, void* dst, int64_t dst_pitch,
                  int32_t dst_dtype, float* magnitude)
{
    if (!ctx) return THIN_EINVAL;
    if (h < 0 || w < 0) return fail(ctx, THIN_EINVAL, "negative image size");
    if ((src_dtype != THIN_U8 && src_dtype != THIN_U16) ||
        (dst_dtype != THIN_U8 && dst_dtype != THIN_U16))
        return fail(ctx, THIN_EINVAL, "bad dtype");
    if (!(alpha > 0.0f) || !std::isfinite(alpha))
        return fail(ctx, THIN_EINVAL, "alpha must be positive and finite");
    if (!(gain >= 0.0f) || !std::isfinite(gain))
        return fail(ctx, THIN_EINVAL, "gain must be finite and >= 0");
    if (h > (1 << 30) || w > (1 << 30)) return fail(ctx, THIN_EINVAL, "image side above 2^30");
    if (src_pitch == 0) src_pitch = w;
    if (dst_pitch == 0) dst_pitch = w;
    if (src_pitch < w || dst_pitch < w) return fail(ctx, THIN_EINVAL, "pitch < w");
    if (h * w == 0) return THIN_OK;
    if (!src || !dst) return fail(ctx, THIN_EINVAL, "NULL image");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    const size_t plane = (size_t)h * (size_t)w;
    int rc = ensure(ctx, ctx->grad, thin::kGradPlanes * plane * sizeof(float));
    if (rc) return rc;
    HIP_TRY(ctx, thin::launch_gradient(ctx->stream, src, src_pitch, src_dtype, (int)h, (int)w,
                                       static_cast<float*>(ctx->grad.ptr), dst, dst_pitch,
                                       dst_dtype, magnitude, gradient_coef(alpha), gain));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return THIN_OK;
}

int thin_topology_table(int32_t adjacency, int32_t op, uint32_t* out, int32_t n)
{
    if ((adjacency != THIN_ADJ_8_4 && adjacency != THIN_ADJ_4_8) || !out || n < 512 ||
        (op != THIN_OP_LEVELING && op != THIN_OP_SKELETON))
        return THIN_EINVAL;
    TopoEntry t[256];
    thin::build_topology_table(adjacency, op, t);
    for (int m = 0; m < 256; ++m) {
        out[2 * m] = t[m].flags;
        out[2 * m + 1] = t[m].comps;
    }
    return THIN_OK;
}

int thin_serve_admit(thin_ctx* ctx, const thin_image* img, uint64_t tag)
{
    if (!ctx) return THIN_EINVAL;
    if (!img) return fail(ctx, THIN_EINVAL, "NULL image descriptor");
    int rc = validate(ctx, *img);
    if (rc) return rc;
    if (ctx->engine == THIN_ENGINE_STEP || ctx->engine == THIN_ENGINE_WORKLIST)
        return fail(ctx, THIN_EINVAL, "serving runs on the tiled engine");
    if (img->h < 3 || img->w < 3) {
        Retired d{tag, {}};
        fill_stats(&d.stats, ImgCnt{}, 0, 0, true);
        ctx->retired.push_back(d);
        return THIN_OK;
    }
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    if (!ctx->serve_ready) {
        // Latency first: per-pixel flags in 64x64 tiles (the dense-list
        // variants spend more time per step when little is flagged).
        TileShape shape = ctx->forced.th ? ctx->forced : TileShape{64, 64, 16, 512, thin::kVarFlags};
        shape.var = thin::var_unseeded(shape.var);
        if (!thin::tile_shape_supported(shape))
            return fail(ctx, THIN_EINVAL, "no compiled serving shape %dx%d k=%d", shape.th,
                        shape.tw, shape.k);
        // The serving budget (max_device_bytes, else kServeDefaultBudget) is
        // split once: counters and descriptors for kServeSlots images, 1/32
        // for tile state (8 bytes a tile), 1/64 for the tile list (4 bytes a
        // tile), the rest for twins.
        const uint64_t budget = ctx->max_device_bytes ? ctx->max_device_bytes : kServeDefaultBudget;
        const uint64_t fixed = (sizeof(ImgCnt) + sizeof(ImgDev)) * (uint64_t)kServeSlots;
        const uint64_t state_cap = budget / 32, list_cap = budget / 64;
        if (budget < 2 * (fixed + (1u << 20)))
            return fail(ctx, THIN_ENOMEM, "serving needs max_device_bytes of at least %llu",
                        (unsigned long long)(2 * (fixed + (1u << 20))));
        const uint64_t twin_cap = budget - fixed - state_cap - list_cap;
        if ((rc = ensure(ctx, ctx->serve_twin, twin_cap))) return rc;
        if ((rc = ensure(ctx, ctx->serve_state, state_cap))) return rc;
        if ((rc = ensure(ctx, ctx->serve_tile_img, list_cap))) return rc;
        if ((rc = ensure(ctx, ctx->serve_cnt, sizeof(ImgCnt) * kServeSlots))) return rc;
        if ((rc = ensure(ctx, ctx->serve_imgs, sizeof(ImgDev) * kServeSlots))) return rc;
        if (hipHostMalloc((void**)&ctx->serve_snap, sizeof(ImgCnt) * kServeSlots,
                          hipHostMallocDefault) != hipSuccess)
            return fail(ctx, THIN_ENOMEM, "hipHostMalloc of serving counters failed");
        ctx->twin_arena.reset(twin_cap);
        ctx->state_arena.reset(std::min(state_cap / (2 * sizeof(int32_t)),
                                        list_cap / sizeof(int32_t)));
        ctx->free_slots.clear();
        for (int i = kServeSlots - 1; i >= 0; --i) ctx->free_slots.push_back(i);
        ctx->serve_shape = shape;
        ctx->serve_ready = true;
    }
    const TileShape shape = ctx->serve_shape;
    Resident r{};
    r.img = *img;
    if (!r.img.pitch_elems) r.img.pitch_elems = r.img.w;
    r.tag = tag;
    r.round0 = ctx->serve_round;
    const uint64_t bpp = img->dtype == THIN_U8 ? 1 : 2;
    r.twin_len = (uint64_t)img->h * (uint64_t)r.img.pitch_elems * bpp;
    r.tiles_y = (int)((img->h + shape.th - 1) / shape.th);
    r.tiles_x = (int)((img->w + shape.tw - 1) / shape.tw);
    r.ntiles = (uint64_t)r.tiles_x * r.tiles_y;
    r.max_steps = steps_cap(ctx);
    r.fresh = true;
    if (ctx->free_slots.empty())
        return fail(ctx, THIN_EBUSY, "all %d serving slots are in use", kServeSlots);
    r.twin_off = ctx->twin_arena.alloc(r.twin_len, 256);
    if (r.twin_off == UINT64_MAX)
        return fail(ctx, THIN_EBUSY, "image of %llu bytes does not fit the serving budget",
                    (unsigned long long)r.twin_len);
    r.state_off = ctx->state_arena.alloc(r.ntiles, 1);
    if (r.state_off == UINT64_MAX) {
        ctx->twin_arena.release(r.twin_off, r.twin_len);
        return fail(ctx, THIN_EBUSY, "tile state of the image does not fit the serving budget");
    }
    r.slot = ctx->free_slots.back();
    ctx->free_slots.pop_back();
    ctx->resident.push_back(r);
    ctx->serve_dirty = true;
    return THIN_OK;
}

int thin_serve_step(thin_ctx* ctx, int32_t rounds, uint64_t* done_tags, thin_stats* done_stats,
                    int32_t cap, int32_t* n_done, int32_t* n_resident)
{
    if (n_done) *n_done = 0;
    if (!ctx) return THIN_EINVAL;
    if (rounds < 0 || cap < 0 || (cap > 0 && !done_tags))
        return fail(ctx, THIN_EINVAL, "bad serve_step arguments");
    int rc;
    if (!ctx->resident.empty() && rounds > 0) {
        HIP_TRY(ctx, hipSetDevice(ctx->device));
        const TileShape shape = ctx->serve_shape;
        const int K = shape.k;
        ImgCnt* d_cnt = static_cast<ImgCnt*>(ctx->serve_cnt.ptr);
        int32_t* d_state = static_cast<int32_t*>(ctx->serve_state.ptr);
        // New residents: counters and tile state start empty (-1 everywhere).
        for (Resident& r : ctx->resident) {
            if (!r.fresh) continue;
            ImgCnt c{0ull, 0ull, -1, -1, 0ull};
            ctx->serve_snap[r.slot] = c;
            HIP_TRY(ctx, hipMemcpyAsync(d_cnt + r.slot, &ctx->serve_snap[r.slot], sizeof c,
                                        hipMemcpyHostToDevice, ctx->stream));
            HIP_TRY(ctx, hipMemsetAsync(d_state + 2 * r.state_off, 0xFF,
                                        2 * sizeof(int32_t) * r.ntiles, ctx->stream));
            r.fresh = false;
        }
        if (ctx->serve_dirty) {
            // Descriptors and the tile list of the current residents; an
            // image keeps its round clock, counters and tile state across
            // rebuilds, so only its position in the lists changes.
            std::vector<ImgDev> imgs;
            std::vector<int32_t> tile_img;
            for (const Resident& r : ctx->resident) {
                ImgDev d{};
                d.buf[0] = r.img.image;
                d.buf[1] = static_cast<char*>(ctx->serve_twin.ptr) + r.twin_off;
                d.pitch = r.img.pitch_elems;
                d.h = (int32_t)r.img.h;
                d.w = (int32_t)r.img.w;
                d.dtype = r.img.dtype;
                d.lambda = r.img.lambda;
                d.adj = table_index(r.img);
                d.tiles_x = r.tiles_x;
                d.tiles_y = r.tiles_y;
                d.tile0 = (int32_t)tile_img.size();
                d.round0 = r.round0;
                d.max_steps = r.max_steps;
                d.slot = r.slot;
                d.state0 = (int64_t)r.state_off;
                for (uint64_t t = 0; t < r.ntiles; ++t) tile_img.push_back((int32_t)imgs.size());
                imgs.push_back(d);
            }
            HIP_TRY(ctx, hipMemcpyAsync(ctx->serve_imgs.ptr, imgs.data(), sizeof(ImgDev) * imgs.size(),
                                        hipMemcpyHostToDevice, ctx->stream));
            HIP_TRY(ctx, hipMemcpyAsync(ctx->serve_tile_img.ptr, tile_img.data(),
                                        sizeof(int32_t) * tile_img.size(), hipMemcpyHostToDevice,
                                        ctx->stream));
            // The host vectors are released at scope end: wait for the copies.
            HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
            ctx->serve_ntiles = (int)tile_img.size();
            ctx->serve_dirty = false;
        }
        const int ntiles = ctx->serve_ntiles;
        int dtypes = 0;
        for (const Resident& r : ctx->resident) dtypes |= r.img.dtype == THIN_U8 ? 1 : 2;
        const int grid = ctx->num_cus * thin::round_blocks_per_cu(shape);
        size_t ev_used = 0;
        for (int k = 0; k < rounds; ++k) {
            if ((rc = timed_round(ctx, ev_used, shape, static_cast<ImgDev*>(ctx->serve_imgs.ptr),
                                  d_cnt, static_cast<int32_t*>(ctx->serve_tile_img.ptr), d_state,
                                  ntiles, ctx->serve_round + k, grid,
                                  static_cast<uint32_t*>(ctx->hist_bits.ptr),
                                  static_cast<int32_t*>(ctx->hist_round.ptr), thin::WorkList{},
                                  0, dtypes)))
                return rc;
        }
        ctx->serve_round += rounds;
        int max_slot = 0;
        for (const Resident& r : ctx->resident) max_slot = std::max(max_slot, r.slot + 1);
        HIP_TRY(ctx, hipMemcpyAsync(ctx->serve_snap, d_cnt, sizeof(ImgCnt) * max_slot,
                                    hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        if (ctx->profile && (rc = collect_profile(ctx, ev_used))) return rc;
        // Retire stable images (or images at their pass cap).
        std::vector<Resident> keep;
        for (const Resident& r : ctx->resident) {
            const ImgCnt& c = ctx->serve_snap[r.slot];
            const int cap_rounds = r.max_steps == INT_MAX ? INT_MAX : (r.max_steps + K - 1) / K;
            const int r_img = std::min(ctx->serve_round - r.round0, cap_rounds);
            const int steps = (int)std::min<int64_t>((int64_t)r_img * K, r.max_steps);
            const bool stable = c.last_step < steps - 4;
            if (!stable && steps < r.max_steps) {
                keep.push_back(r);
                continue;
            }
            if (r_img & 1) {
                const size_t bpp = r.img.dtype == THIN_U8 ? 1 : 2;
                const size_t pitch = (size_t)r.img.pitch_elems * bpp;
                HIP_TRY(ctx, hipMemcpy2DAsync(r.img.image, pitch,
                                              static_cast<char*>(ctx->serve_twin.ptr) + r.twin_off,
                                              pitch, (size_t)r.img.w * bpp, (size_t)r.img.h,
                                              hipMemcpyDeviceToDevice, ctx->stream));
            }
            if (ctx->profile) ctx->prof_tile_rounds += c.tile_rounds;
            Retired d{r.tag, {}};
            fill_stats(&d.stats, c, steps, r.max_steps, false);
            ctx->retired.push_back(d);
            ctx->twin_arena.release(r.twin_off, r.twin_len);
            ctx->state_arena.release(r.state_off, r.ntiles);
            ctx->free_slots.push_back(r.slot);
            ctx->serve_dirty = true;
        }
        ctx->resident.swap(keep);
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    }
    // Report retired images, oldest first.
    const int n = std::min<int>(cap, (int)ctx->retired.size());
    for (int i = 0; i < n; ++i) {
        done_tags[i] = ctx->retired[i].tag;
        if (done_stats) done_stats[i] = ctx->retired[i].stats;
    }
    ctx->retired.erase(ctx->retired.begin(), ctx->retired.begin() + n);
    if (n_done) *n_done = n;
    if (n_resident) *n_resident = (int32_t)ctx->resident.size();
    return THIN_OK;
}

}  // extern "C"
