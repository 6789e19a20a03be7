// Internal declarations shared by the single-lattice and batched host code of the aqlbm
// library.  Not part of the public interface (include/aqlbm.h).
#pragma once
#include "aq_device.h"

#include "aqlbm.h"

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

namespace aq {

extern thread_local std::string g_err;
int fail(int code, const std::string& msg);

#define HIPCHK(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(AQ_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

inline size_t storage_size(int mode) { return mode == AQ_F64 ? 8 : (mode == AQ_F16S ? 2 : 4); }

struct Layout {
    int pitch;
    long long qs;
    size_t off_a, off_b, off_type, off_uprev, off_tiles, off_tiles2, off_partials, off_counters, off_obs,
        off_walls, off_widx, off_scratch, total;
    int max_tiles, max_tiles2;
};

inline Layout make_layout(const aq_params& P, int n_walls)
{
    Layout L;
    L.pitch = (int)align_up((size_t)P.nx, 64);
    // population arrays sit 64*11 elements past a multiple of 64, so the 13 streams of a
    // node do not start on the same DRAM channel
    L.qs = (long long)align_up((size_t)P.ny * L.pitch, 64) + 64 * 11;
    const size_t es = storage_size(P.storage);
    const size_t pop_bytes = align_up((size_t)NPOP * L.qs * es, 256);
    L.max_tiles = (int)(((P.nx + 63) / 64) * (size_t)P.ny);   // smallest tile is 64x1
    size_t o = 0;
    L.off_a = o; o += pop_bytes;
    L.off_b = o; o += pop_bytes;
    L.off_type = o; o += align_up((size_t)L.qs, 256);
    L.off_uprev = o; o += align_up(3 * (size_t)L.qs * 8, 256);
    L.off_tiles = o; o += align_up((size_t)L.max_tiles * 4, 256);
    L.max_tiles2 = (int)(((P.nx + 63) / 64) * (size_t)((P.ny + 3) / 4));   // fused tiles are 64 x >= 4
    L.off_tiles2 = o; o += align_up((size_t)L.max_tiles2 * 4, 256);
    L.off_partials = o; o += align_up((size_t)L.max_tiles * NRED * 8, 256);
    L.off_counters = o; o += 256;
    L.off_obs = o; o += align_up((size_t)OBS_RING * NRED * 8, 256);
    // wall list: node, id, normal (2 doubles), link fractions (8 doubles)
    L.off_walls = o; o += align_up((size_t)std::max(n_walls, 1) * (4 + 4 + 16 + 64), 256);
    L.off_widx = o; o += align_up((size_t)L.qs * 4, 256);   // node -> wall-list index, -1 off it
    L.off_scratch = o; o += align_up((size_t)P.nx * P.ny * 8, 256);
    L.total = o;
    return L;
}

inline double bytes_per_update(int mode) { return 2.0 * NPOP * storage_size(mode) + 1.0; }

// Lumped-outlet seepage speeds: two doubles in the counters block.
constexpr size_t kUseepOffset = 128;

// Working sets (bytes moved per step) above this use non-temporal population stores; the
// MI355X last-level cache (MALL) holds 256 MB.
constexpr double kMallBytes = 192.0 * 1024 * 1024;

// FP32 lattices with at least this many active nodes run two steps per launch by default.
constexpr long long kFuseMinActive = 1LL << 17;
// F32 and F16S lattices below this many active nodes take 64 x 4 two-step tiles by default
// (twice the blocks of 64 x 8).
constexpr long long kFuse4MaxActive = 1LL << 20;

}  // namespace aq

struct PlainPlan {
    int graph_launches, graph_steps, tail;
};

struct aq_solver {
    aq_params P;
    aq::Layout L;
    int mode;
    char* base = nullptr;
    bool own_mem = false;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = -1;              // HIP device current at creation (-1: not yet known)

    std::vector<uint8_t> htype;   // [ny][pitch]
    int64_t n_active = 0, n_fluid = 0, n_cornea = 0, n_iris = 0;
    std::vector<int> hwall_node, hwall_id;
    std::vector<double> hwall_n, hwall_q;
    int n_walls = 0;

    int tile_x = 64, tile_y = 4, tiles_x = 0, n_tiles = 0, xcd_remap = 1;
    int nt_store = 0;
    int fuse = 1;                 // two steps per launch on the plain steps of an interval
    std::vector<int> htiles2;     // active 64 x fuse_rows tiles
    int fuse_rows = 0;            // rows of a two-step tile: 8, or 4 (F32 and F16S)
    int tiles_x2 = 0, n_tiles2 = 0;
    std::vector<int> htiles;      // active tile indices (host copy of the device list)
    int cur = 0;                  // 0: buffer A holds the state
    int ro_slot = 0;              // lumped outlet: seepage-speed slot the last pull used
    int64_t step = 0;
    unsigned int checks = 0;      // reducing launches enqueued
    int64_t last_check_step = 0;
    bool diverged = false;
    double sf = 1, st = 1;        // F16S scales
    int exp_f = 0, exp_t = 0;

    hipGraphExec_t plain_graph[2] = {nullptr, nullptr};   // by the buffer holding the state
    hipGraph_t plain_graph_src[2] = {nullptr, nullptr};
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    double* obs_pinned = nullptr; // host pinned, 2 * NRED
    double useep_host[2] = {0.0, 0.0};   // lumped outlet: last seepage speeds set from the host

    void* popA() const { return base + L.off_a; }
    void* popB() const { return base + L.off_b; }
};


namespace aq {

StepArgs make_args(const aq_solver* s, bool a_is_src);
StepArgs make_args2(const aq_solver* s, bool a_is_src);
int set_state(aq_solver* s, const double* pops);
int set_useep(aq_solver* s, double now, double before);
StepArgs make_readout_args(const aq_solver* s);
double seepage_speed(const aq_params& P, double p_iop);
int lumped_guard(const aq_params& P, const uint8_t* mask, int stride);
void raw_to_obs(const aq_solver* s, const double* raw, int64_t step, aq_observables* o);
int create_common(const aq_params* P, const uint8_t* mask, const aq_wall_node* walls, int32_t n_walls,
                  void* arena, size_t arena_bytes, void* stream, bool own, aq_solver** out,
                  int fuse_rows = 0);
int validate(const aq_params* P, const uint8_t* mask, const aq_wall_node* walls, int32_t n_walls);
// The reduced storages' 32-bit population offsets cover the lattice (always true in FP64).
bool offsets_fit(const aq_params& P);
int upload_tiles(aq_solver* s);
// Set the two-step tile rows of a solver and rebuild its tile lists (synchronises its stream).
int set_fuse_rows(aq_solver* s, int rows);

}  // namespace aq
