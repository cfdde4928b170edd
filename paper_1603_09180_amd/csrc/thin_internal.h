// thin_internal.h -- structures shared by the HIP kernels and the host runtime
// of the lambda-leveling library.  Not part of the public ABI (include/thin.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace thin {

// One image as the kernels see it.  buf[0] is the caller's image, buf[1] the
// context-owned twin of the same pitch; round r reads buf[r & 1] and writes
// buf[(r + 1) & 1], so after r rounds the current state is in buf[r & 1].
struct ImgDev {
    void* buf[2];
    int64_t pitch;       // row pitch in elements (both buffers)
    int32_t h, w;
    int32_t dtype;       // 1 = u8, 2 = u16
    uint32_t lambda;
    int32_t adj;         // table: adjacency (0 = (8,4), 1 = (4,8)) + 2 * operator
                         // (0 = lambda-leveling, 1 = lambda-skeleton)
    int32_t tiles_x;     // tile grid of this image
    int32_t tiles_y;
    int32_t tile0;       // index of its first tile in the launch's tile arrays
    int32_t round0;      // launch round at which the image's step 0 starts
    int32_t max_steps;   // parity-step cap (4 * max_passes), INT32_MAX if none
    int32_t slot;        // index of its counters (stable while the image is resident)
    int64_t state0;      // index of its first tile in the per-tile state array
};

// Per-image counters, written by the kernels with device-scope atomics.
struct ImgCnt {
    unsigned long long lowerings;
    unsigned long long tile_rounds;
    int32_t last_step;   // image-local index of the last step that lowered, -1 if none
    int32_t pad;
    unsigned long long examinations;  // candidates characterised (section 2.1 tests run)
};

// Tiles a round launch visits.  With list == nullptr every tile is visited.
// Otherwise launch round R visits list[(R & 1) * cap + i] for i < count[R % 3]
// (every tile when R == full), and a tile appends the tiles that must be
// visited in round R + 1 (its 3x3 tile block when it lowered something during
// its last 4 steps, itself when it lowered anything) to the other half,
// deduplicated by listed[g] = last round g was queued for.  count[(R + 2) % 3]
// is cleared during round R, before round R + 1 appends to it.
struct WorkList {
    int32_t* list;
    int32_t* count;
    int32_t* grab;     // [6]: next list position to hand out in round R, one counter per
                       // pixel-type launch of the round (grab[2 * (R % 3) + u16]),
                       // cleared like count
    int32_t* listed;
    int32_t cap;
    int32_t full;    // the launch round that visits every tile (-1: none)
};

// Connectivity table entry for an upper-neighbour mask (see thin_topology_table).
//   flags: bit 0 destructible, bit 1 peak and bit 2 end point (skeleton
//          tables only), bits 4..6 T--, bits 8..10 T+
//   comps: byte c = ring mask of the c-th counted lower component
struct alignas(8) TopoEntry {  // 8-byte aligned: one 64-bit load per lookup
    uint32_t flags;
    uint32_t comps;
};

// Host-side generation of the 256 entries of one (adjacency, operator) table;
// the device holds 4 x 256 entries, table index adjacency + 2 * operator.
constexpr int kTables = 4;
void build_topology_table(int adjacency, int op, TopoEntry out[256]);

// Residency variants.  kVarFlags keeps the tile in LDS with a re-examination
// flag byte per pixel, every thread checking fixed cells each step;
// kVarSeeded also starts those flags from the previous round's change
// bitmaps; kVarRegs keeps each thread's 4x4 windows in registers;
// kVarBits keeps the flags as one bit per candidate and class and gathers
// each step's flagged candidates into a dense list; kVarBitsSeeded adds the
// previous round's change bitmaps to kVarBits.
constexpr int kVarFlags = 0, kVarSeeded = 1, kVarRegs = 2, kVarBits = 3, kVarBitsSeeded = 4;

// Variants that read and write per-tile change bitmaps between rounds.
constexpr bool var_seeded(int v) { return v == kVarSeeded || v == kVarBitsSeeded; }
// The same variant without history (for callers that keep none).
constexpr int var_unseeded(int v)
{
    return v == kVarSeeded ? kVarFlags : (v == kVarBitsSeeded ? kVarBits : v);
}

// Tiled engine geometry chosen at run time among the compiled variants.
struct TileShape {
    int th, tw, k;   // tile height, width, halo = parity steps per residency
    int nt;          // threads per tile
    int var;         // residency variant (kVar*)
};

// The compiled shape with this tile and halo (nt = 0 when there is none).
TileShape complete_shape(int th, int tw, int k);

// Kernel launchers (thin_kernels.hip).  All enqueue on `stream`.
// Clears counters and tile state; with wl.list, listed[] = -1 and counts 0.
hipError_t launch_init_state(hipStream_t stream, ImgCnt* cnt, int nimg, int32_t* tile_last,
                             int ntiles, int32_t* hist_round, WorkList wl);
// The launch's round is `round`, plus *round_base when round_base is not
// null (graph replays: the same launches serve every chunk of rounds).
// Launch flags of the round kernels.
constexpr int kOneImage = 1;     // every tile belongs to image 0 (no tile_img lookup)
constexpr int kStateIsTile = 2;  // a tile's state index is its tile index
constexpr int kOnlyU8 = 4;       // visit only u8 images (bit-flag variants: u8 LDS tiles)
constexpr int kOnlyU16 = 8;      // visit only u16 images
// A grid of as many blocks as fit on num_cus CUs loops over the tiles.
hipError_t launch_round(hipStream_t stream, TileShape shape, const ImgDev* imgs, ImgCnt* cnt,
                        const int32_t* tile_img, int32_t* tile_last, int ntiles, int round,
                        const TopoEntry* lut, int num_cus, uint32_t* hist_bits,
                        int32_t* hist_round, WorkList wl, const int32_t* round_base, int kflags);
// *round_base += n (the last node of a chunk graph).
hipError_t launch_advance(hipStream_t stream, int32_t* round_base, int n);
// Words of one tile's change bitmap (two copies of ntiles bitmaps are needed).
int history_words(TileShape s);
hipError_t launch_step(hipStream_t stream, const ImgDev* img_host, const ImgDev* img_dev,
                       ImgCnt* cnt, int step, const TopoEntry* lut);
// Cooperative engine: every round in one launch, grid-wide barriers between
// rounds.  active: 3 zeroed counters; rounds_out receives the rounds run.
hipError_t launch_coop(hipStream_t stream, TileShape shape, const ImgDev* imgs, ImgCnt* cnt,
                       const int32_t* tile_img, int32_t* tile_last, int ntiles,
                       const TopoEntry* lut, int32_t* active, int32_t* rounds_out,
                       int max_rounds, int num_cus, uint32_t* hist_bits, int32_t* hist_round,
                       int kflags);
bool tile_shape_supported(TileShape s);

// Gradient front-end (gradient.hip): float32 coefficients of Deriche's
// recursive smoothing (a0..a3) and derivative (d1, d2) filters, shared
// feedback (b1, b2) and the steady states of the four recursions for a
// constant input of 1 (the edge rule).
struct GradCoef {
    float a0, a1, a2, a3, d1, d2, b1, b2, s_plus, s_minus, d_plus, d_minus;
};
// Column pass, row pass and output pass on `stream`; scratch holds 8 h*w
// float planes; mag (nullable) receives the float magnitude, h*w contiguous.
constexpr int kGradPlanes = 8;
hipError_t launch_gradient(hipStream_t stream, const void* src, int64_t src_pitch, int src_dtype,
                           int h, int w, float* scratch, void* dst, int64_t dst_pitch,
                           int dst_dtype, float* mag, GradCoef co, float gain);
// Pixel work-list engine (k_worklist): one block per image runs parity
// steps one after the other, examining only the candidates whose 3x3
// changed since their last examination.
struct WlImg {
    void* image;          // the image state, updated in place
    const void* prev;     // init 1: the state one tiled round earlier (same pitch)
    uint32_t* gbits;      // pending bitmaps in global memory (4 * lh * lww words), or null
    int64_t pitch;        // row pitch in elements
    int32_t h, w;
    int32_t dtype;        // 1 = u8, 2 = u16
    uint32_t lambda;
    int32_t adj;          // table index (adjacency + 2 * operator)
    int32_t step0;        // global index of the first step to run
    int32_t max_steps;    // step cap (global index), INT32_MAX if none
    int32_t init;         // 0: every interior candidate pending; 1: those whose 3x3 differs
                          // between image and prev
    int32_t slot;         // counter slot
    int32_t pad;
};
constexpr int kWlThreads = 1024;
constexpr int kWlListCap = 2048;      // entries per candidate list
constexpr int kWlLdsWords = 8192;     // pending-bitmap words kept in LDS (32 KiB)
// Pending-bitmap words of an image (4 classes of ceil(h/2) rows of
// ceil(ceil(w/2)/32) words).
inline int64_t wl_bitmap_words(int64_t h, int64_t w)
{
    return 4 * ((h + 1) / 2) * ((((w + 1) / 2) + 31) / 32);
}
// One block per image; steps_out[i] receives the global index one past the
// last step image i ran.  gbits selects the variant with the pending bitmaps
// in global memory (every image of the launch must have gbits set then).
hipError_t launch_worklist(hipStream_t stream, const WlImg* imgs, int nimg, int dtype,
                           bool gbits, ImgCnt* cnt, const TopoEntry* lut, int32_t* steps_out);

// Writes descriptor d to *dst on `stream` (a kernel argument, so no host
// buffer has to outlive the call).
hipError_t launch_set_desc(hipStream_t stream, ImgDev* dst, const ImgDev& d);

// The static scratch array of the no-allocation entry point (noalloc.hip):
// its size, and the device address of the copy on `device`, looked up once
// per device (the caller makes `device` current).
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
hipError_t noalloc_scratch(int device, void** out);

// Every compiled shape: writes up to cap of them to out, returns the count.
int compiled_shapes(TileShape* out, int cap);
int round_blocks_per_cu(TileShape s);

}  // namespace thin
