// Shared declarations between the HIP kernels and the host side of the aqlbm library.
// Internal to the library; the public interface is include/aqlbm.h.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace aq {

// Device-side node-type byte.  Bits 0-4 are the input mask byte (class, wall id); the
// library adds the two flags below.
enum : uint8_t {
    CLS_MASK = 7,
    SOLID = 0, FLUID = 1, POROUS = 2, INLET = 3, OUTLET = 4,
    WALL_SHIFT = 3, WALL_BOX = 0, WALL_CORNEA = 1, WALL_IRIS = 2,
    F_WSS = 1 << 5,       // active node listed in the wall-shear-stress set
    F_BOUNDARY = 1 << 6,  // active node with at least one non-active neighbour
};

// Raw per-check-step sums written by the reducing kernel (double).
enum {
    R_DP_FLUID = 0, R_QOUT, R_QIN, R_WSS_C_SUM, R_WSS_C_MAX, R_WSS_I_SUM, R_WSS_I_MAX,
    R_DU2, R_U2, R_DT2, R_T2, R_MASS_F, R_MASS_T, R_UMAX, R_NONFINITE, NRED
};

constexpr int NPOP = 13;    // 8 flow (q = 1..8) + 5 thermal (q = 0..4)
constexpr int OBS_RING = 64;

// Kernel arguments, passed by value.  Physical constants are double, with single-precision
// copies for the storages that compute in FP32.
struct StepArgs {
    const void* src;          // 13 population arrays, qs elements apart
    void* dst;
    long long qs;             // elements between population arrays
    const uint8_t* type;      // [ny][pitch]
    const int* tiles;         // active tile indices (ty * tiles_x + tx)
    int n_tiles, tiles_x, tile_x, tile_y;
    int pitch, nx, ny, xcd_remap;
    int nt_store;             // non-temporal population stores (working set beyond the MALL)

    double omega_f, omega_t;  // 1/tau_f, 1/tau_t
    double w0T, wT, inv_cs2T; // thermal weights (rest, axis) and 1/c_sT^2
    double nuK, drag_den;     // nu/K and 1/(1 + nu/(2K))
    double bx, by;            // g*beta*(sin phi, cos phi)
    double dT0;               // T_ref - T0
    double T_ref;
    double uin_x, uin_y;      // inlet wall velocity
    double dp_out;            // p_out - p_ref
    double tw_cornea, tw_iris, tw_inlet;   // T_w - T_ref
    double sf, inv_sf, st, inv_st;         // F16S scales (flow, thermal)
    // The constants the step uses, rounded to single precision once on the host (the same
    // rounding a conversion in the kernel would give): the FP32-compute storages read
    // these, so no thread converts a double constant.
    float omega_f32, omega_t32, w0T32, wT32, inv_cs2T32, nuK32, drag_den32, bx32, by32, dT032, T_ref32;
    float sf32, inv_sf32, st32, inv_st32;
    float uin_x32, uin_y32, dp_out32, tw_cornea32, tw_iris32, tw_inlet32;   // boundary rules

    // lumped meshwork outlet: OUTLET links are walls moving at the seepage speed *useep
    // along the node's outward direction; the finish kernel re-evaluates it at check steps
    int lumped;
    const double* useep;      // seepage speed the pull uses
    double* useep_state;      // [0] in effect for the next steps, [1] the one before it
    double k_mu, h_tm;        // K_tm / mu (mu = nu at unit density) and the thickness
    double p_ref, p_sc;
    double n_fluid;           // FLUID nodes (IOP mean)

    // reductions (check steps only)
    double* partials;         // [gridDim][NRED]
    double* obs;              // [OBS_RING][NRED]
    unsigned int* obs_count;  // check steps reduced so far
    double* uprev;            // 3 arrays (u_x, u_y, T) of qs doubles
    const int* wall_node;     // sorted node indices (y * pitch + x)
    const int* wall_id;
    const double* wall_n;     // interleaved (n_x, n_y)
    const double* wall_q;     // [n_walls][8] link fractions (-1: no wall on the link)
    const int* widx;          // [qs] wall-list index of a node, -1 off the list
    int n_walls;
    int bc_paper;             // interpolated bounce-back on wall-list links (Bouzidi et al.)
};

// One instance of a batch (device table entry).  `a` has buffer A as src (even parity).
struct InstDesc {
    StepArgs a;
    StepArgs a2;                  // the same instance with its fused (two-step) tile list
    int work_start, work_count;   // this instance's run in its storage mode's work list
    int running, mode;            // mode: the instance's kernel class (storage + 4 * paper scheme)
};

// Arguments of the batched kernels (one storage mode per launch).
struct BatchArgs {
    const InstDesc* inst;
    const int2* work;          // (slot, tile) items, grouped by slot
    const int* n_work;         // number of items (device memory, read at run time)
    const int2* work2;         // (slot, fused tile) items for two-step launches
    const int* n_work2;
    double* partials;          // [work capacity][NRED]
    double* latest;            // [max_slots][NRED]: latest raw sums of every instance
    int parity;                // 0: buffer A is src
    int max_slots;
    int mode;                  // storage mode of this launch
    int kind;                  // kernel class of this launch (instances with InstDesc.mode == kind)
    int nt_store;              // non-temporal population stores
    int bc;                    // 1: the instances of this launch use the paper's boundary schemes
    int tile_y;                // rows of the two-step tiles of this launch (8, or 4 in F32 and F16S)
};

// Host-side launchers (defined in aq_kernels.hip).
hipError_t launch_step(int mode, bool reduce, const StepArgs& a, hipStream_t s);
hipError_t launch_batch_step(int mode, bool reduce, const BatchArgs& b, int grid, hipStream_t s);
// Two plain time steps in one launch (tiles 64 x fused_tile_rows(mode) from a.tiles).
hipError_t launch_step2(int mode, const StepArgs& a, hipStream_t s);
hipError_t launch_batch_step2(int mode, const BatchArgs& b, int grid, hipStream_t s);
int fused_tile_rows(int mode);   // the default two-step tile rows (64 x 8)
bool fused_rows_supported(int mode, int rows);
hipError_t launch_batch_finish(const BatchArgs& b, hipStream_t s);
// Write into a.dst the buffer whose pull gives the pre-collision populations `pops`
// (dense [13][ny][nx] doubles), or, if pops is null, the rest equilibrium with
// p - p_ref = dp0 and T - T_ref = th0.
hipError_t launch_scatter(int mode, const StepArgs& a, const double* pops, double dp0, double th0,
                          hipStream_t s);
// Pull a.src and write one field (0 p, 1 u_x, 2 u_y, 3 T, 4 flow population q, 5 thermal
// population q) to out[ny][nx]; field 6 stores the moments as the residual reference;
// field 7 writes all 13 populations to out[13][ny][nx]; field 8 writes u_x and u_y to
// out[2][ny][nx].
hipError_t launch_unpack(int mode, const StepArgs& a, int field, int q, double p_ref, double* out,
                         hipStream_t s);
// Vortex diagnostics of the state `a` pulls to (field 8 read-out, vorticity, stream
// function); ws holds diagnostics_words(nx, ny) doubles, results in its last 8.
size_t diagnostics_words(int nx, int ny);
hipError_t launch_diagnostics(int mode, const StepArgs& a, double* ws, hipStream_t s);

}  // namespace aq
