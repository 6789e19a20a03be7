// Host side of the aqlbm C-ABI (include/aqlbm.h): solver creation, device layout,
// tile lists, HIP-graph chunks, observables and checkpoints.  No kernels live here; the
// only device object is the fixed diagnostics workspace of aq_diagnose_noalloc.
#include "aq_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace aq;

namespace aq {

thread_local std::string g_err;

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

StepArgs make_args(const aq_solver* s, bool a_is_src)
{
    const aq_params& P = s->P;
    StepArgs a;
    std::memset(&a, 0, sizeof(a));
    a.src = a_is_src ? s->popA() : s->popB();
    a.dst = a_is_src ? s->popB() : s->popA();
    a.qs = s->L.qs;
    a.type = (const uint8_t*)(s->base + s->L.off_type);
    a.tiles = (const int*)(s->base + s->L.off_tiles);
    a.n_tiles = s->n_tiles;
    a.tiles_x = s->tiles_x;
    a.tile_x = s->tile_x;
    a.tile_y = s->tile_y;
    a.pitch = s->L.pitch;
    a.nx = P.nx;
    a.ny = P.ny;
    a.xcd_remap = s->xcd_remap;
    a.nt_store = s->nt_store;
    a.omega_f = 1.0 / P.tau_f;
    a.omega_t = 1.0 / P.tau_t;
    a.w0T = P.w0;
    a.wT = (1.0 - P.w0) / 4.0;
    a.inv_cs2T = 2.0 / (1.0 - P.w0);
    const double nu = (2.0 * P.tau_f - 1.0) / 6.0;   // eq. 10
    a.nuK = nu / P.K;
    a.drag_den = 1.0 / (1.0 + 0.5 * a.nuK);
    a.bx = P.gbeta * std::sin(P.gravity_angle);
    a.by = P.gbeta * std::cos(P.gravity_angle);
    a.dT0 = P.T_ref - P.T0;
    a.T_ref = P.T_ref;
    a.uin_x = P.u_in_x;
    a.uin_y = P.u_in_y;
    a.dp_out = P.p_out - P.p_ref;
    a.tw_cornea = P.T_cornea - P.T_ref;
    a.tw_iris = P.T_iris - P.T_ref;
    a.tw_inlet = P.T_inlet - P.T_ref;
    a.sf = s->sf;
    a.inv_sf = 1.0 / s->sf;
    a.st = s->st;
    a.inv_st = 1.0 / s->st;
    a.omega_f32 = (float)a.omega_f;
    a.uin_x32 = (float)a.uin_x;
    a.uin_y32 = (float)a.uin_y;
    a.dp_out32 = (float)a.dp_out;
    a.tw_cornea32 = (float)a.tw_cornea;
    a.tw_iris32 = (float)a.tw_iris;
    a.tw_inlet32 = (float)a.tw_inlet;
    a.omega_t32 = (float)a.omega_t;
    // thermal weights whose single-precision values sum to one exactly (w0T + 4 wT = 1 in
    // real arithmetic), so the float collision conserves the thermal populations' sum:
    // round the larger of the two groups and take the other as the exact remainder
    if (P.w0 <= 0.5) {
        a.wT32 = (float)a.wT;
        a.w0T32 = 1.0f - 4.0f * a.wT32;           // 4 wT in [1/2, 1]: exact
    } else {
        a.w0T32 = (float)a.w0T;
        a.wT32 = (1.0f - a.w0T32) * 0.25f;        // w0T in (1/2, 1): exact
    }
    a.inv_cs2T32 = (float)a.inv_cs2T;
    a.nuK32 = (float)a.nuK;
    a.drag_den32 = (float)a.drag_den;
    a.bx32 = (float)a.bx;
    a.by32 = (float)a.by;
    a.dT032 = (float)a.dT0;
    a.T_ref32 = (float)a.T_ref;
    a.sf32 = (float)a.sf;
    a.inv_sf32 = (float)a.inv_sf;
    a.st32 = (float)a.st;
    a.inv_st32 = (float)a.inv_st;
    char* b = s->base;
    a.partials = (double*)(b + s->L.off_partials);
    a.obs_count = (unsigned int*)(b + s->L.off_counters + 64);
    a.obs = (double*)(b + s->L.off_obs);
    a.uprev = (double*)(b + s->L.off_uprev);
    a.wall_node = (const int*)(b + s->L.off_walls);
    a.wall_id = (const int*)(b + s->L.off_walls + 4 * (size_t)std::max(s->n_walls, 1));
    a.wall_n = (const double*)(b + s->L.off_walls + 8 * (size_t)std::max(s->n_walls, 1));
    a.wall_q = (const double*)(b + s->L.off_walls + 24 * (size_t)std::max(s->n_walls, 1));
    a.widx = (const int*)(b + s->L.off_widx);
    a.n_walls = s->n_walls;
    a.bc_paper = P.bc_scheme == AQ_BC_PAPER ? 1 : 0;
    a.lumped = P.outlet_mode == AQ_OUTLET_LUMPED ? 1 : 0;
    a.useep_state = (double*)(b + s->L.off_counters + kUseepOffset);
    a.useep = a.useep_state;          // a step pulls with the speed in effect
    a.k_mu = a.lumped ? P.K_tm / nu : 0.0;
    a.h_tm = a.lumped ? P.h_tm : 1.0;
    a.p_ref = P.p_ref;
    a.p_sc = P.p_sc;
    a.n_fluid = (double)s->n_fluid;
    return a;
}

// Arguments of a read-out pull of the current state: the lumped outlet's links must use
// the seepage speed the last step's pull used (a check step replaces the speed in effect).
StepArgs make_readout_args(const aq_solver* s)
{
    StepArgs a = make_args(s, s->cur != 0);
    a.useep = a.useep_state + s->ro_slot;
    return a;
}

// Seepage speed of the lumped meshwork at pressure p_iop (eq. 4 across the thickness).
double seepage_speed(const aq_params& P, double p_iop)
{
    const double nu = (2.0 * P.tau_f - 1.0) / 6.0;
    return P.K_tm / nu * ((p_iop - P.p_sc) / P.h_tm);
}

// Arguments of the two-steps-per-launch kernel: the same lattice with the fused tile list.
StepArgs make_args2(const aq_solver* s, bool a_is_src)
{
    StepArgs a = make_args(s, a_is_src);
    a.tiles = (const int*)(s->base + s->L.off_tiles2);
    a.n_tiles = s->n_tiles2;
    a.tiles_x = s->tiles_x2;
    a.tile_x = 64;
    a.tile_y = s->fuse_rows;
    return a;
}

// The seepage speed of the lumped outlet is explicit over a check interval.  The flow mass
// of the chamber, (5/3) N dp, then relaxes toward its steady level by the factor 1 - D r per
// interval, r = 3 A K_tm / (5 N nu h_tm), where A = sum over links into OUTLET nodes of
// 6 w_i e_i.n is the outflow area.  Accept D r <= 1 (monotone approach; the coupling
// oscillates beyond and diverges past 2).  `mask` holds the mask bytes with row stride
// `stride` (bits above 4 ignored).
int lumped_guard(const aq_params& P, const uint8_t* mask, int stride)
{
    static const int lx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1}, ly[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    if (!(P.K_tm > 0.0 && P.h_tm > 0.0 && std::isfinite(P.K_tm) && std::isfinite(P.h_tm) && std::isfinite(P.p_sc)))
        return fail(AQ_EINVAL, "lumped outlet needs finite K_tm > 0, h_tm > 0 and p_sc");
    double area = 0.0, n_act = 0.0;
    for (int y = 1; y < P.ny - 1; y++)
        for (int x = 1; x < P.nx - 1; x++) {
            const int c = mask[(size_t)y * stride + x] & 7;
            if (c != AQ_FLUID && c != AQ_POROUS) continue;
            n_act += 1.0;
            for (int i = 1; i <= 8; i++) {
                const uint8_t m = mask[(size_t)(y + ly[i]) * stride + x + lx[i]];
                if ((m & 7) != AQ_OUTLET) continue;
                const int d = ((m >> 3) & 3) + 1;
                area += 6.0 * (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0) * (lx[i] * lx[d] + ly[i] * ly[d]);
            }
        }
    if (!(area > 0.0)) return fail(AQ_EINVAL, "lumped outlet: no outflow area (no link into an OUTLET node along its direction)");
    const double nu = (2.0 * P.tau_f - 1.0) / 6.0;
    const double dr = P.check_interval * 3.0 * area * P.K_tm / (5.0 * n_act * nu * P.h_tm);
    if (dr > 1.0)
        return fail(AQ_EINVAL, "lumped outlet: check_interval * 3 A K_tm / (5 N nu h_tm) = " + std::to_string(dr) +
                                   " > 1 (the explicit coupling would overshoot); lower check_interval or K_tm");
    return AQ_OK;
}

bool offsets_fit(const aq_params& P)
{
    if (P.storage != AQ_F32 && P.storage != AQ_F32X && P.storage != AQ_F16S) return true;
    // the kernels of the reduced storages address populations with 32-bit byte offsets from
    // a plane base; a boundary pull's offset reaches two planes beyond the node's own slot
    const Layout L0 = make_layout(P, 0);
    const long long elem = P.storage == AQ_F16S ? 2 : 4;
    return (3 * L0.qs + L0.pitch + 1) * elem <= (1LL << 32);
}

int validate(const aq_params* P, const uint8_t* mask, const aq_wall_node* walls, int32_t n_walls)
{
    if (!P || !mask) return fail(AQ_EINVAL, "null params or mask");
    if (P->struct_size != sizeof(aq_params)) return fail(AQ_EINVAL, "aq_params.struct_size mismatch");
    if (P->nx < 4 || P->ny < 4) return fail(AQ_EINVAL, "nx and ny must be >= 4");
    if ((long long)P->nx * P->ny > (1LL << 30)) return fail(AQ_EINVAL, "lattice too large");
    if (!(P->tau_f > 0.5) || !(P->tau_t > 0.5)) return fail(AQ_EINVAL, "tau_f and tau_t must exceed 1/2");
    if (!offsets_fit(*P))
        return fail(AQ_EINVAL, "lattice too large for the storage: three population planes must stay within 4 GiB");
    if (!(P->w0 >= 0.0 && P->w0 < 1.0)) return fail(AQ_EINVAL, "w0 must be in [0, 1)");
    if (!(P->K > 0.0)) return fail(AQ_EINVAL, "K must be positive");
    if (P->storage < AQ_F64 || P->storage > AQ_F32X) return fail(AQ_EINVAL, "unknown storage");
    if (P->check_interval < 2 || (P->check_interval & 1)) return fail(AQ_EINVAL, "check_interval must be even and >= 2");
    if (P->fp16_exp_flow < -1 || P->fp16_exp_flow > 40 || P->fp16_exp_thermal < -1 || P->fp16_exp_thermal > 40)
        return fail(AQ_EINVAL, "fp16 exponents must be in [-1, 40]");
    if (P->outlet_mode != AQ_OUTLET_PRESSURE && P->outlet_mode != AQ_OUTLET_LUMPED)
        return fail(AQ_EINVAL, "unknown outlet_mode");
    if (P->bc_scheme != AQ_BC_LINKWISE && P->bc_scheme != AQ_BC_PAPER) return fail(AQ_EINVAL, "unknown bc_scheme");
    const int nx = P->nx, ny = P->ny;
    for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++) {
            const uint8_t m = mask[(size_t)y * nx + x];
            const int c = m & 7;
            if (c > AQ_OUTLET || (m >> 5)) return fail(AQ_EINVAL, "invalid mask byte");
            const bool act = c == AQ_FLUID || c == AQ_POROUS;
            if (act && (x == 0 || y == 0 || x == nx - 1 || y == ny - 1))
                return fail(AQ_EINVAL, "active node on the outer frame");
        }
    if (P->outlet_mode == AQ_OUTLET_LUMPED) {
        int rc = lumped_guard(*P, mask, nx);
        if (rc) return rc;
    }
    if (n_walls < 0 || (n_walls > 0 && !walls)) return fail(AQ_EINVAL, "invalid wall list");
    for (int w = 0; w < n_walls; w++) {
        const int k = walls[w].node;
        if (k < 0 || (long long)k >= (long long)nx * ny) return fail(AQ_EINVAL, "wall node out of range");
        if ((mask[k] & 7) != AQ_FLUID) return fail(AQ_EINVAL, "wall node is not FLUID");
        if (walls[w].wall != AQ_WALL_CORNEA && walls[w].wall != AQ_WALL_IRIS) return fail(AQ_EINVAL, "wall id must be CORNEA or IRIS");
        if (w > 0 && walls[w - 1].node >= k) return fail(AQ_EINVAL, "wall list must be sorted by node, without repeats");
        if (!std::isfinite(walls[w].n_x) || !std::isfinite(walls[w].n_y)) return fail(AQ_EINVAL, "non-finite wall normal");
        for (int i = 0; i < 8; i++) {
            const double q = walls[w].q[i];
            if (!(q == -1.0 || (q > 0.0 && q <= 1.0))) return fail(AQ_EINVAL, "wall link fraction must be -1 or in (0, 1]");
        }
    }
    return AQ_OK;
}

// Power-of-two scales for F16S storage: largest s with the expected deviation magnitude
// times 2^s at most 1/4 (see the design notes); clamp to [0, 24].
int auto_exp(double dmax)
{
    if (!(dmax > 0)) return 0;
    int s = (int)std::floor(std::log2(0.25 / dmax));
    return std::max(0, std::min(24, s));
}

void choose_scales(aq_solver* s)
{
    const aq_params& P = s->P;
    const double dT = std::max({std::fabs(P.T_cornea - P.T0), std::fabs(P.T_iris - P.T0),
                                std::fabs(P.T_inlet - P.T0), std::fabs(P.T_init - P.T0), 1e-30});
    const double L = std::max(P.nx, P.ny);
    const double ub = std::sqrt(std::fabs(P.gbeta) * dT * L);
    const double us = std::max({std::fabs(P.u_in_x), std::fabs(P.u_in_y), ub, 1e-12});
    const double dps = std::fabs(P.gbeta) * dT * L + std::fabs(P.p_out - P.p_ref) + std::fabs(P.p_init - P.p_ref);
    const double dflow = (3.0 * us + dps) / 3.0;
    const double dTr = std::max({std::fabs(P.T_cornea - P.T_ref), std::fabs(P.T_iris - P.T_ref),
                                 std::fabs(P.T_inlet - P.T_ref), std::fabs(P.T_init - P.T_ref), 1e-30});
    const double dtherm = 0.5 * dTr * (1.0 + 2.0 * us / (1.0 - P.w0)) + 1e-30;
    s->exp_f = P.fp16_exp_flow >= 0 ? P.fp16_exp_flow : auto_exp(dflow);
    s->exp_t = P.fp16_exp_thermal >= 0 ? P.fp16_exp_thermal : auto_exp(dtherm);
    if (P.storage == AQ_F16S) {
        s->sf = std::ldexp(1.0, s->exp_f);
        s->st = std::ldexp(1.0, s->exp_t);
    } else {
        s->sf = s->st = 1.0;
        s->exp_f = s->exp_t = 0;
    }
}

// Active tiles of shape tw x th in row-major order; returns the tiles per row.
int list_tiles(const aq_solver* s, int tw, int th, std::vector<int>& tiles)
{
    const int nx = s->P.nx, ny = s->P.ny, pitch = s->L.pitch;
    const int tiles_x = (nx + tw - 1) / tw;
    const int tiles_y = (ny + th - 1) / th;
    tiles.clear();
    for (int ty = 0; ty < tiles_y; ty++)
        for (int tx = 0; tx < tiles_x; tx++) {
            bool any = false;
            for (int y = ty * th; y < std::min(ny, (ty + 1) * th) && !any; y++)
                for (int x = tx * tw; x < std::min(nx, (tx + 1) * tw); x++) {
                    const int c = s->htype[(size_t)y * pitch + x] & CLS_MASK;
                    if (c == FLUID || c == POROUS) { any = true; break; }
                }
            if (any) tiles.push_back(ty * tiles_x + tx);
        }
    return tiles_x;
}

void build_tiles(aq_solver* s, std::vector<int>& tiles)
{
    s->tiles_x = list_tiles(s, s->tile_x, s->tile_y, tiles);
    s->n_tiles = (int)tiles.size();
}

int upload_tiles(aq_solver* s)
{
    std::vector<int>& tiles = s->htiles;
    build_tiles(s, tiles);
    if (s->n_tiles > s->L.max_tiles) return fail(AQ_EINVAL, "tile list overflow");
    if (s->n_tiles)
        HIPCHK(hipMemcpyAsync(s->base + s->L.off_tiles, tiles.data(), tiles.size() * 4, hipMemcpyHostToDevice, s->stream));
    s->tiles_x2 = list_tiles(s, 64, s->fuse_rows, s->htiles2);
    s->n_tiles2 = (int)s->htiles2.size();
    if (s->n_tiles2 > s->L.max_tiles2) return fail(AQ_EINVAL, "fused tile list overflow");
    if (s->n_tiles2)
        HIPCHK(hipMemcpyAsync(s->base + s->L.off_tiles2, s->htiles2.data(), s->htiles2.size() * 4, hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return AQ_OK;
}

void drop_graph(aq_solver* s)
{
    for (int p = 0; p < 2; p++) {
        if (s->plain_graph[p]) (void)hipGraphExecDestroy(s->plain_graph[p]);
        if (s->plain_graph_src[p]) (void)hipGraphDestroy(s->plain_graph_src[p]);
        s->plain_graph[p] = nullptr;
        s->plain_graph_src[p] = nullptr;
    }
}

// Switch the two-step tile rows (the tile lists are rebuilt and the graphs captured anew).
int set_fuse_rows(aq_solver* s, int rows)
{
    if (!fused_rows_supported(s->mode, rows)) return fail(AQ_EINVAL, "two-step tile rows not supported");
    if (rows == s->fuse_rows) return AQ_OK;
    HIPCHK(hipStreamSynchronize(s->stream));
    drop_graph(s);
    s->fuse_rows = rows;
    return upload_tiles(s);
}

// The check_interval - 1 plain steps of an interval: `graph_launches` launches replayed
// from a graph (two-step launches when fusion is on, else single steps) covering
// `graph_steps` steps, then `tail` single steps launched directly.  The reducing step that
// closes the interval is always a single step, so the previous buffer pulls back to the
// state at every check step.
static PlainPlan plain_plan(const aq_solver* s)
{
    const int n = s->P.check_interval - 1;
    // F16S rounds where it stores, so its launch schedule is part of its arithmetic: it
    // takes the batch's plan, an even number of two-step launches (the batch keeps every
    // instance's buffer parity), so a solve rounds at the same steps alone and batched
    if (s->fuse && s->mode == AQ_F16S) {
        const int F = (n / 2) & ~1;
        return {F, 2 * F, n - 2 * F};
    }
    if (s->fuse) return {n / 2, 2 * (n / 2), n % 2};
    return {n, n, 0};
}

static void enqueue_graph_part(aq_solver* s, int cur, hipError_t* err)
{
    const PlainPlan pp = plain_plan(s);
    bool a_src = cur == 0;
    *err = hipSuccess;
    for (int i = 0; i < pp.graph_launches && *err == hipSuccess; i++) {
        *err = s->fuse ? launch_step2(s->mode, make_args2(s, a_src), s->stream)
                       : launch_step(s->mode, false, make_args(s, a_src), s->stream);
        a_src = !a_src;
    }
}

// Capture the graph part of an interval starting from buffer `cur` as one graph.
int ensure_graph(aq_solver* s, int cur)
{
    if (s->plain_graph[cur] || plain_plan(s).graph_launches == 0) return AQ_OK;
    HIPCHK(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
    hipError_t err = hipSuccess;
    enqueue_graph_part(s, cur, &err);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(s->stream, &g);
    if (err != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(AQ_EDEVICE, std::string("capture launch: ") + hipGetErrorString(err));
    }
    if (e2 != hipSuccess) return fail(AQ_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e2));
    hipGraphExec_t ge = nullptr;
    hipError_t e3 = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (e3 != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(AQ_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e3));
    }
    s->plain_graph_src[cur] = g;
    s->plain_graph[cur] = ge;
    return AQ_OK;
}

int launch_one(aq_solver* s)
{
    const bool reduce = ((s->step + 1) % s->P.check_interval) == 0;
    StepArgs a = make_args(s, s->cur == 0);
    HIPCHK(launch_step(s->mode, reduce, a, s->stream));
    s->cur ^= 1;
    s->step++;
    s->ro_slot = reduce ? 1 : 0;   // a reducing step's finish kernel moves the speed on
    if (reduce) {
        s->checks++;
        s->last_check_step = s->step;
    }
    return AQ_OK;
}

// Replay the graph part of an interval (the state is at a check step).
static int launch_graph_part(aq_solver* s)
{
    const PlainPlan pp = plain_plan(s);
    if (pp.graph_launches == 0) return AQ_OK;
    int rc = ensure_graph(s, s->cur);
    if (rc) return rc;
    HIPCHK(hipGraphLaunch(s->plain_graph[s->cur], s->stream));
    s->cur ^= pp.graph_launches & 1;
    s->step += pp.graph_steps;
    s->ro_slot = 0;
    return AQ_OK;
}

// The tail single steps and the reducing step that close an interval.
static int launch_interval_end(aq_solver* s)
{
    for (int i = 0; i < plain_plan(s).tail; i++) {
        int rc = launch_one(s);
        if (rc) return rc;
    }
    return launch_one(s);
}

void raw_to_obs(const aq_solver* s, const double* r, int64_t step, aq_observables* o)
{
    const aq_params& P = s->P;
    std::memset(o, 0, sizeof(*o));
    o->step = step;
    o->p_mean_fluid = P.p_ref + (s->n_fluid > 0 ? r[R_DP_FLUID] / (double)s->n_fluid : 0.0);
    o->iop_gauge = o->p_mean_fluid - P.p_out;
    o->q_in = r[R_QIN];
    o->q_out = r[R_QOUT];
    o->wss_cornea_mean = s->n_cornea ? r[R_WSS_C_SUM] / (double)s->n_cornea : 0.0;
    o->wss_cornea_max = r[R_WSS_C_MAX];
    o->wss_iris_mean = s->n_iris ? r[R_WSS_I_SUM] / (double)s->n_iris : 0.0;
    o->wss_iris_max = r[R_WSS_I_MAX];
    const double D = (double)P.check_interval;
    o->resid_u = r[R_U2] > 0 ? std::sqrt(r[R_DU2]) / (D * std::sqrt(r[R_U2])) : std::sqrt(r[R_DU2]) / D;
    o->resid_T = r[R_T2] > 0 ? std::sqrt(r[R_DT2]) / (D * std::sqrt(r[R_T2])) : std::sqrt(r[R_DT2]) / D;
    o->u_max = r[R_UMAX];
    o->mass_flow = r[R_MASS_F];
    o->mass_thermal = r[R_MASS_T];
    o->n_nonfinite = (int64_t)r[R_NONFINITE];
    // the speed the finish kernel derived from this check step (same expression)
    o->u_seep = P.outlet_mode == AQ_OUTLET_LUMPED ? (P.K_tm / ((2.0 * P.tau_f - 1.0) / 6.0)) *
                                                        ((o->p_mean_fluid - P.p_sc) / P.h_tm)
                                                  : 0.0;
}

// Read the raw sums of reduction number `idx` (0-based) after the stream has passed it.
int read_raw(aq_solver* s, unsigned int idx, double* raw)
{
    const double* src = (const double*)(s->base + s->L.off_obs) + (size_t)(idx % OBS_RING) * NRED;
    HIPCHK(hipMemcpyAsync(s->obs_pinned, src, NRED * 8, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    std::memcpy(raw, s->obs_pinned, NRED * 8);
    return AQ_OK;
}

// Set the current pre-collision state to `pops` (device, dense [13][ny][nx]) or, if
// null, to the rest equilibrium of (p_init, T_init): scatter its pre-image into the
// `prev` buffer, collide it into `cur` with one regular step launch, and reset the
// residual reference to its moments.  The step counter and buffer parity are unchanged.
int set_state(aq_solver* s, const double* pops)
{
    const bool prev_is_b = s->cur == 0;
    StepArgs sc = make_args(s, prev_is_b);         // dst = prev
    HIPCHK(launch_scatter(s->mode, sc, pops, s->P.p_init - s->P.p_ref, s->P.T_init - s->P.T_ref, s->stream));
    StepArgs st = make_args(s, !prev_is_b);        // src = prev, dst = cur
    HIPCHK(launch_step(s->mode, false, st, s->stream));
    s->ro_slot = 0;
    HIPCHK(launch_unpack(s->mode, st, 6, 0, s->P.p_ref, nullptr, s->stream));
    return AQ_OK;
}

// Both seepage-speed slots of the lumped outlet (host values, async copy).
int set_useep(aq_solver* s, double now, double before)
{
    s->useep_host[0] = now;
    s->useep_host[1] = before;
    HIPCHK(hipMemcpyAsync(s->base + s->L.off_counters + kUseepOffset, s->useep_host, 16, hipMemcpyHostToDevice,
                          s->stream));
    return AQ_OK;
}

int init_state(aq_solver* s)
{
    s->cur = 0;
    s->step = 0;
    s->checks = 0;
    s->last_check_step = 0;
    s->diverged = false;
    HIPCHK(hipMemsetAsync(s->base + s->L.off_counters, 0, 256, s->stream));
    HIPCHK(hipMemsetAsync(s->base + s->L.off_obs, 0, OBS_RING * NRED * 8, s->stream));
    if (s->P.outlet_mode == AQ_OUTLET_LUMPED) {
        // the first interval drains at the speed the initial pressure drives
        const double u0 = seepage_speed(s->P, s->P.p_init);
        int rc = set_useep(s, u0, u0);
        if (rc) return rc;
    }
    int rc = set_state(s, nullptr);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(s->stream));
    return AQ_OK;
}

int setup(aq_solver* s, const uint8_t* mask, const aq_wall_node* walls, int32_t n_walls)
{
    const aq_params& P = s->P;
    const int nx = P.nx, ny = P.ny, pitch = s->L.pitch;
    s->htype.assign((size_t)s->L.qs, 0);
    for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++) s->htype[(size_t)y * pitch + x] = mask[(size_t)y * nx + x] & 31;
    static const int ex[8] = {1, 0, -1, 0, 1, -1, -1, 1}, ey[8] = {0, 1, 0, -1, 1, 1, -1, -1};
    for (int y = 1; y < ny - 1; y++)
        for (int x = 1; x < nx - 1; x++) {
            uint8_t& t = s->htype[(size_t)y * pitch + x];
            const int c = t & CLS_MASK;
            if (c != FLUID && c != POROUS) continue;
            s->n_active++;
            if (c == FLUID) s->n_fluid++;
            for (int i = 0; i < 8; i++) {
                const int cc = mask[(size_t)(y + ey[i]) * nx + x + ex[i]] & 7;
                if (cc != AQ_FLUID && cc != AQ_POROUS) t |= F_BOUNDARY;
            }
        }
    // the read and written populations of a step exceed the last-level cache: stream the writes
    s->nt_store = (double)s->n_active * bytes_per_update(s->mode) > kMallBytes ? 1 : 0;
    // two steps per launch where it measured faster: the FP64-arithmetic storages always;
    // FP32 from kFuseMinActive active nodes or past the cache (below, even 64 x 4 tiles are
    // too few blocks to fill the chip); F16S always, since its two-step launch rounds to
    // binary16 only where it stores, so the schedule is part of its arithmetic and a batched
    // instance (always two-step) must match
    s->fuse = (s->mode == AQ_F64 || s->mode == AQ_F32X || s->mode == AQ_F16S || s->nt_store ||
               (s->mode == AQ_F32 && s->n_active >= kFuseMinActive)) ? 1 : 0;
    // two-step tile rows: given (the batch: 8), else 4 for mid-size F32 / F16S lattices,
    // whose 64 x 8 tiles leave part of the chip idle (eye check intervals, 64 x 8 against
    // 64 x 4: 1024x512 F32 17.7k / 22.6k MLUPS, F16S 18.6k / 24.6k; 2048x1024 F32 48.1k /
    // 50.3k, F16S 55.1k / 58.6k; 4096x2048 F32 66.7k / 63.1k, F16S 101.0k / 96.7k)
    if (s->fuse_rows == 0)
        s->fuse_rows = ((s->mode == AQ_F32 || s->mode == AQ_F16S) && s->n_active < kFuse4MaxActive) ? 4 : 8;
    if (!fused_rows_supported(s->mode, s->fuse_rows))
        return fail(AQ_EINVAL, "two-step tile rows not supported for the storage");
    s->n_walls = n_walls;
    s->hwall_node.resize(std::max(n_walls, 1));
    s->hwall_id.resize(std::max(n_walls, 1));
    s->hwall_n.resize(2 * (size_t)std::max(n_walls, 1));
    s->hwall_q.assign(8 * (size_t)std::max(n_walls, 1), -1.0);
    std::vector<int> widx((size_t)s->L.qs, -1);
    for (int w = 0; w < n_walls; w++) {
        const int k = walls[w].node, x = k % nx, y = k / nx;
        s->hwall_node[w] = y * pitch + x;
        s->hwall_id[w] = walls[w].wall;
        s->hwall_n[2 * w] = walls[w].n_x;
        s->hwall_n[2 * w + 1] = walls[w].n_y;
        for (int i = 0; i < 8; i++) s->hwall_q[8 * (size_t)w + i] = walls[w].q[i];
        widx[(size_t)y * pitch + x] = w;
        s->htype[(size_t)y * pitch + x] |= F_WSS;
        if (walls[w].wall == AQ_WALL_CORNEA) s->n_cornea++; else s->n_iris++;
    }
    choose_scales(s);

    // device images: populations poisoned with NaN (never read at non-active nodes)
    HIPCHK(hipMemsetAsync(s->base + s->L.off_a, 0xFF, s->L.off_type - s->L.off_a, s->stream));
    HIPCHK(hipMemcpyAsync(s->base + s->L.off_type, s->htype.data(), s->htype.size(), hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipMemsetAsync(s->base + s->L.off_uprev, 0, 3 * (size_t)s->L.qs * 8, s->stream));
    const size_t W = (size_t)std::max(n_walls, 1);
    char* wb = s->base + s->L.off_walls;
    HIPCHK(hipMemcpyAsync(wb, s->hwall_node.data(), 4 * W, hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipMemcpyAsync(wb + 4 * W, s->hwall_id.data(), 4 * W, hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipMemcpyAsync(wb + 8 * W, s->hwall_n.data(), 16 * W, hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipMemcpyAsync(wb + 24 * W, s->hwall_q.data(), 64 * W, hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipMemcpyAsync(s->base + s->L.off_widx, widx.data(), widx.size() * 4, hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));   // the host vector goes out of scope
    int rc = upload_tiles(s);
    if (rc) return rc;
    for (auto& e : s->ev) HIPCHK(hipEventCreate(&e));
    HIPCHK(hipHostMalloc((void**)&s->obs_pinned, 2 * NRED * 8, hipHostMallocDefault));
    return init_state(s);
}

int create_common(const aq_params* P, const uint8_t* mask, const aq_wall_node* walls, int32_t n_walls,
                  void* arena, size_t arena_bytes, void* stream, bool own, aq_solver** out, int fuse_rows)
{
    if (!out) return fail(AQ_EINVAL, "null out");
    int rc = validate(P, mask, walls, n_walls);
    if (rc) return rc;
    aq_solver* s = new aq_solver();
    s->P = *P;
    s->fuse_rows = fuse_rows;   // 0: chosen in setup from the lattice
    s->mode = P->storage;
    s->L = make_layout(*P, n_walls);
    if (hipGetDevice(&s->device) != hipSuccess) s->device = -1;   // resolved where it is needed
    if (own) {
        hipError_t e = hipMalloc((void**)&s->base, s->L.total);
        if (e != hipSuccess) {
            delete s;
            return fail(AQ_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        }
        s->own_mem = true;
    } else {
        if (!arena || ((uintptr_t)arena & 255)) {
            delete s;
            return fail(AQ_EINVAL, "arena must be non-null and 256-byte aligned");
        }
        if (arena_bytes < s->L.total) {
            delete s;
            return fail(AQ_ENOMEM, "arena smaller than aq_required_bytes");
        }
        s->base = (char*)arena;
    }
    if (stream) {
        s->stream = (hipStream_t)stream;
    } else {
        hipError_t e = hipStreamCreate(&s->stream);   // default priority
        if (e != hipSuccess) {
            aq_destroy(s);
            return fail(AQ_EDEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
        }
        s->own_stream = true;
    }
    rc = setup(s, mask, walls, n_walls);
    if (rc) {
        std::string keep = g_err;
        aq_destroy(s);
        g_err = keep;
        return rc;
    }
    *out = s;
    return AQ_OK;
}

// The diagnostics of the state into workspace w (diagnostics_words doubles): the kernels
// write every word they later read, so w needs no clearing.  Synchronises the stream.
int diagnose_into(aq_solver* s, double* w, aq_diagnostics* out)
{
    const size_t words = diagnostics_words(s->P.nx, s->P.ny);
    HIPCHK(launch_diagnostics(s->mode, make_readout_args(s), w, s->stream));
    HIPCHK(hipMemcpyAsync(s->obs_pinned, w + words - 8, 8 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    const double* r = s->obs_pinned;
    out->step = s->step;
    out->vortex_intensity = r[0];
    out->u_max_fluid = r[1];
    out->psi_max = r[2];
    out->psi_max_x = (int32_t)r[3];
    out->psi_max_y = (int32_t)r[4];
    out->psi_min = r[5];
    out->psi_min_x = (int32_t)r[6];
    out->psi_min_y = (int32_t)r[7];
    return AQ_OK;
}

// Fixed workspace of aq_diagnose_noalloc, for callers that cannot allocate device memory.
// Every GPU the library runs on holds its own copy until the process ends.  In host code
// `scratch` names a host-side stand-in, not device memory: its device address on each GPU
// comes from hipGetSymbolAddress (with that GPU current), taken once per device and kept.
constexpr size_t kDiagScratchBytes = size_t(64) << 20;
static __device__ __align__(256) double scratch[kDiagScratchBytes / sizeof(double)];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

int diag_scratch(int device, double** out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (device < 0 || device >= kMaxDevices) return fail(AQ_EDEVICE, "device index out of range");
    if (!g_scratch_ptr[device]) {
        int prev = 0;
        HIPCHK(hipGetDevice(&prev));
        if (prev != device) HIPCHK(hipSetDevice(device));
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (prev != device) HIPCHK(hipSetDevice(prev));
        if (e != hipSuccess) return fail(AQ_EDEVICE, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
        if (!p) return fail(AQ_EDEVICE, "hipGetSymbolAddress returned a null address");
        g_scratch_ptr[device] = (double*)p;
    }
    *out = g_scratch_ptr[device];
    return AQ_OK;
}

}  // namespace

extern "C" {

const char* aq_version(void) { return "aqlbm 0.1 (gfx950)"; }

const char* aq_last_error(void) { return g_err.c_str(); }

int aq_required_bytes(const aq_params* P, const uint8_t* mask, size_t* bytes)
{
    if (!P || !bytes) return fail(AQ_EINVAL, "null argument");
    if (P->struct_size != sizeof(aq_params)) return fail(AQ_EINVAL, "aq_params.struct_size mismatch");
    if (P->nx < 4 || P->ny < 4 || P->storage < AQ_F64 || P->storage > AQ_F32X) return fail(AQ_EINVAL, "invalid size or storage");
    int n_walls = 0;
    if (mask) {
        // an upper bound on the wall list: every FLUID node
        size_t n = (size_t)P->nx * P->ny;
        for (size_t k = 0; k < n; k++) n_walls += (mask[k] & 7) == AQ_FLUID;
    }
    *bytes = make_layout(*P, n_walls).total;
    return AQ_OK;
}

int aq_create(const aq_params* P, const uint8_t* mask, const aq_wall_node* walls, int32_t n_walls, aq_solver** out)
{
    return create_common(P, mask, walls, n_walls, nullptr, 0, nullptr, true, out);
}

int aq_create_ext(const aq_params* P, const uint8_t* mask, const aq_wall_node* walls, int32_t n_walls,
                  void* arena, size_t arena_bytes, void* stream, aq_solver** out)
{
    return create_common(P, mask, walls, n_walls, arena, arena_bytes, stream, false, out);
}

int aq_destroy(aq_solver* s)
{
    if (!s) return AQ_OK;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    drop_graph(s);
    for (auto& e : s->ev)
        if (e) (void)hipEventDestroy(e);
    if (s->obs_pinned) (void)hipHostFree(s->obs_pinned);
    if (s->own_mem && s->base) (void)hipFree(s->base);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
    return AQ_OK;
}

int aq_step(aq_solver* s, int64_t nsteps)
{
    if (!s || nsteps < 0) return fail(AQ_EINVAL, "invalid arguments");
    const int D = s->P.check_interval;
    while (nsteps > 0) {
        if (s->step % D == 0 && nsteps >= D && s->n_tiles > 0) {
            int rc = launch_graph_part(s);
            if (rc == AQ_OK) rc = launch_interval_end(s);
            if (rc) return rc;
            nsteps -= D;
        } else {
            int rc = launch_one(s);
            if (rc) return rc;
            nsteps--;
        }
    }
    return s->diverged ? fail(AQ_EDIVERGED, "non-finite state seen at a check step") : AQ_OK;
}

int aq_observe(aq_solver* s, aq_observables* out)
{
    if (!s || !out) return fail(AQ_EINVAL, "null argument");
    if (s->checks == 0) {
        HIPCHK(hipStreamSynchronize(s->stream));
        std::memset(out, 0, sizeof(*out));
        return AQ_OK;
    }
    double raw[NRED];
    int rc = read_raw(s, s->checks - 1, raw);
    if (rc) return rc;
    raw_to_obs(s, raw, s->last_check_step, out);
    if (out->n_nonfinite) s->diverged = true;
    return AQ_OK;
}

int aq_run_to_steady(aq_solver* s, double tol, int64_t max_steps, aq_observables* out)
{
    if (!s || !out || !(tol > 0)) return fail(AQ_EINVAL, "invalid arguments");
    const int D = s->P.check_interval;
    // align to the check schedule
    const int64_t lead = (D - s->step % D) % D;
    int rc = aq_step(s, std::min<int64_t>(lead, max_steps));
    if (rc) return rc;
    int64_t done = std::min<int64_t>(lead, max_steps);
    // keep one interval in flight while the previous one's residual is checked
    bool have_prev = false;
    unsigned int prev_idx = 0;
    int64_t prev_step = 0;
    while (true) {
        bool launched = false;
        if (done + D <= max_steps) {
            rc = aq_step(s, D);
            if (rc) return rc;
            done += D;
            launched = true;
        }
        if (have_prev) {
            double raw[NRED];
            const double* src = (const double*)(s->base + s->L.off_obs) + (size_t)(prev_idx % OBS_RING) * NRED;
            // the stream may be ahead; the copy below is ordered after the in-flight interval
            HIPCHK(hipMemcpyAsync(s->obs_pinned, src, NRED * 8, hipMemcpyDeviceToHost, s->stream));
            HIPCHK(hipStreamSynchronize(s->stream));
            std::memcpy(raw, s->obs_pinned, NRED * 8);
            aq_observables o;
            raw_to_obs(s, raw, prev_step, &o);
            if (o.n_nonfinite) {
                s->diverged = true;
                *out = o;
                return fail(AQ_EDIVERGED, "non-finite state");
            }
            if (std::max(o.resid_u, o.resid_T) < tol) {
                return aq_observe(s, out);   // the latest interval (one past convergence)
            }
        }
        if (!launched) break;
        have_prev = true;
        prev_idx = s->checks - 1;
        prev_step = s->last_check_step;
    }
    rc = aq_observe(s, out);
    if (rc) return rc;
    if (std::max(out->resid_u, out->resid_T) < tol) return AQ_OK;
    return fail(AQ_ENOTCONVERGED, "max_steps reached before the residual fell below tol");
}

int aq_read_field(aq_solver* s, int32_t field, int32_t q, double* host, size_t count)
{
    if (!s || !host) return fail(AQ_EINVAL, "null argument");
    if (count != (size_t)s->P.nx * s->P.ny) return fail(AQ_EINVAL, "count must be nx*ny");
    if (field < AQ_FIELD_P || field > AQ_FIELD_POP_HEAT) return fail(AQ_EINVAL, "unknown field");
    if (field == AQ_FIELD_POP_FLOW && (q < 1 || q > 8)) return fail(AQ_EINVAL, "flow population q must be 1..8");
    if (field == AQ_FIELD_POP_HEAT && (q < 0 || q > 4)) return fail(AQ_EINVAL, "thermal population q must be 0..4");
    StepArgs a = make_readout_args(s);   // src = prev: pulls to the current state
    double* scratch = (double*)(s->base + s->L.off_scratch);
    HIPCHK(launch_unpack(s->mode, a, field, q, s->P.p_ref, scratch, s->stream));
    HIPCHK(hipMemcpyAsync(host, scratch, count * 8, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return AQ_OK;
}

int aq_write_populations(aq_solver* s, const double* flow, const double* heat, size_t count)
{
    if (!s || !flow || !heat) return fail(AQ_EINVAL, "null argument");
    const size_t n = (size_t)s->P.nx * s->P.ny;
    if (count != n) return fail(AQ_EINVAL, "count must be nx*ny");
    double* tmp = nullptr;
    HIPCHK(hipMalloc((void**)&tmp, NPOP * n * 8));
    hipError_t e = hipMemcpyAsync(tmp, flow, 8 * n * 8, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(tmp + 8 * n, heat, 5 * n * 8, hipMemcpyHostToDevice, s->stream);
    int rc = AQ_OK;
    if (e == hipSuccess) rc = set_state(s, tmp);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    (void)hipFree(tmp);
    if (e != hipSuccess) return fail(AQ_EDEVICE, std::string("write populations: ") + hipGetErrorString(e));
    if (rc) return rc;
    s->diverged = false;
    return AQ_OK;
}

int aq_get_info(aq_solver* s, aq_info* o)
{
    if (!s || !o) return fail(AQ_EINVAL, "null argument");
    std::memset(o, 0, sizeof(*o));
    o->active_nodes = s->n_active;
    o->fluid_nodes = s->n_fluid;
    o->lattice_nodes = (int64_t)s->P.nx * s->P.ny;
    o->nx = s->P.nx;
    o->ny = s->P.ny;
    o->pitch = s->L.pitch;
    o->storage = s->P.storage;
    o->tile_x = s->tile_x;
    o->tile_y = s->tile_y;
    o->n_tiles = s->n_tiles;
    o->check_interval = s->P.check_interval;
    o->fp16_exp_flow = s->exp_f;
    o->fp16_exp_thermal = s->exp_t;
    o->fusion = s->fuse ? 1 : 0;
    o->fused_tile_rows = s->fuse_rows;
    o->graph_launches = plain_plan(s).graph_launches;
    o->nt_store = s->nt_store ? 1 : 0;
    o->step = s->step;
    o->device_bytes = s->L.total;
    o->bytes_per_node_update = bytes_per_update(s->mode);
    return AQ_OK;
}

int aq_set_tile(aq_solver* s, int32_t tx, int32_t ty)
{
    if (!s) return fail(AQ_EINVAL, "null solver");
    if (!(tx == 64 || tx == 128 || tx == 256) || ty < 1 || tx * ty < 64 || tx * ty > 256 || (ty & (ty - 1)))
        return fail(AQ_EINVAL, "tile_x in {64,128,256}, tile_y a power of two, 64 <= tile_x*tile_y <= 256");
    HIPCHK(hipStreamSynchronize(s->stream));
    drop_graph(s);
    s->tile_x = tx;
    s->tile_y = ty;
    return upload_tiles(s);
}

int aq_time_step_kernel(aq_solver* s, int32_t n_launch, double* ms)
{
    if (!s || !ms || n_launch < 2 || (n_launch & 1)) return fail(AQ_EINVAL, "n_launch must be even and >= 2");
    // n_launch steps, all without reductions (a check step that falls inside is not
    // reduced); the step counter advances so the check schedule stays aligned
    HIPCHK(hipEventRecord(s->ev[0], s->stream));
    for (int i = 0; i < n_launch; i++) {
        StepArgs a = make_args(s, s->cur == 0);
        HIPCHK(launch_step(s->mode, false, a, s->stream));
        s->cur ^= 1;
        s->step++;
    }
    s->ro_slot = 0;
    HIPCHK(hipEventRecord(s->ev[1], s->stream));
    HIPCHK(hipEventSynchronize(s->ev[1]));
    float t = 0;
    HIPCHK(hipEventElapsedTime(&t, s->ev[0], s->ev[1]));
    *ms = t / n_launch;
    return AQ_OK;
}

int aq_set_outlet(aq_solver* s, double K_tm, double h_tm, double p_sc)
{
    if (!s) return fail(AQ_EINVAL, "null solver");
    if (s->P.outlet_mode != AQ_OUTLET_LUMPED) return fail(AQ_EINVAL, "the solver's outlet is not the lumped meshwork");
    aq_params P = s->P;
    P.K_tm = K_tm;
    P.h_tm = h_tm;
    P.p_sc = p_sc;
    int rc = lumped_guard(P, s->htype.data(), s->L.pitch);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(s->stream));
    drop_graph(s);          // the captured launches carry the old constants
    // the speed in effect becomes that of the new constants at the last check step's IOP
    // (p_init before the first check); the read-out keeps the speed the last pull used
    double p_iop = P.p_init;
    if (s->checks > 0) {
        double raw[NRED];
        rc = read_raw(s, s->checks - 1, raw);
        if (rc) return rc;
        aq_observables o;
        raw_to_obs(s, raw, s->last_check_step, &o);
        p_iop = o.p_mean_fluid;
    }
    double cur[2];
    HIPCHK(hipMemcpyAsync(cur, s->base + s->L.off_counters + kUseepOffset, 16, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    const double before = s->ro_slot == 0 ? cur[0] : cur[1];
    s->ro_slot = 1;
    s->P = P;
    rc = set_useep(s, seepage_speed(P, p_iop), before);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(s->stream));
    return AQ_OK;
}

int aq_diagnostics_bytes(const aq_params* P, size_t* bytes)
{
    if (!P || !bytes || P->nx < 1 || P->ny < 1) return fail(AQ_EINVAL, "invalid arguments");
    *bytes = diagnostics_words(P->nx, P->ny) * sizeof(double);
    return AQ_OK;
}

int aq_diagnose(aq_solver* s, void* ws, size_t ws_bytes, aq_diagnostics* out)
{
    if (!s || !ws || !out) return fail(AQ_EINVAL, "null argument");
    const size_t words = diagnostics_words(s->P.nx, s->P.ny);
    if (ws_bytes < words * sizeof(double) || ((uintptr_t)ws & 7)) return fail(AQ_EINVAL, "workspace too small or misaligned");
    return diagnose_into(s, (double*)ws, out);
}

int aq_diagnose_noalloc(aq_solver* s, aq_diagnostics* out)
{
    if (!s || !out) return fail(AQ_EINVAL, "null argument");
    const size_t need = diagnostics_words(s->P.nx, s->P.ny) * sizeof(double);
    if (need > kDiagScratchBytes)
        return fail(AQ_EINVAL, "lattice too large for the fixed diagnostics workspace: needs " + std::to_string(need) +
                                   " bytes, " + std::to_string(kDiagScratchBytes) + " available (use aq_diagnose)");
    if (s->device < 0 && hipGetDevice(&s->device) != hipSuccess) {
        s->device = -1;
        return fail(AQ_EDEVICE, "hipGetDevice failed");
    }
    double* w = nullptr;
    const int rc = diag_scratch(s->device, &w);
    if (rc) return rc;
    return diagnose_into(s, w, out);
}

int aq_set_fusion(aq_solver* s, int32_t enable)
{
    if (!s) return fail(AQ_EINVAL, "null solver");
    HIPCHK(hipStreamSynchronize(s->stream));
    drop_graph(s);
    s->fuse = enable ? 1 : 0;
    return AQ_OK;
}

int aq_time_fused_kernel(aq_solver* s, int32_t n_launch, double* ms)
{
    if (!s || !ms || n_launch < 1) return fail(AQ_EINVAL, "n_launch must be >= 1");
    // n_launch two-step launches followed by one single step, so the previous buffer
    // pulls back to the current state again; only the two-step launches are timed
    HIPCHK(hipEventRecord(s->ev[0], s->stream));
    for (int i = 0; i < n_launch; i++) {
        HIPCHK(launch_step2(s->mode, make_args2(s, s->cur == 0), s->stream));
        s->cur ^= 1;
        s->step += 2;
    }
    HIPCHK(hipEventRecord(s->ev[1], s->stream));
    HIPCHK(launch_step(s->mode, false, make_args(s, s->cur == 0), s->stream));
    s->cur ^= 1;
    s->step++;
    s->ro_slot = 0;
    HIPCHK(hipEventSynchronize(s->ev[1]));
    float t = 0;
    HIPCHK(hipEventElapsedTime(&t, s->ev[0], s->ev[1]));
    *ms = t / n_launch;
    return AQ_OK;
}

int aq_set_fused_tile_rows(aq_solver* s, int32_t rows)
{
    if (!s) return fail(AQ_EINVAL, "null solver");
    return set_fuse_rows(s, rows);
}

int aq_autotune_tile(aq_solver* s, int32_t n_launch, int32_t only_256, int32_t* tile_x, int32_t* tile_y,
                     double* ms_per_launch)
{
    if (!s || !tile_x || !tile_y || !ms_per_launch || n_launch < 2 || (n_launch & 1))
        return fail(AQ_EINVAL, "invalid arguments");
    static const int cand[6][2] = {{64, 4}, {128, 2}, {256, 1}, {64, 1}, {64, 2}, {128, 1}};
    const int nc = only_256 ? 3 : 6;
    int best = -1;
    double best_ms = 0;
    for (int c = 0; c < nc; c++) {
        int rc = aq_set_tile(s, cand[c][0], cand[c][1]);
        if (rc) return rc;
        double ms = 0;
        rc = aq_time_step_kernel(s, 2, &ms);          // warm up
        if (rc == AQ_OK) rc = aq_time_step_kernel(s, n_launch, &ms);
        if (rc) return rc;
        if (best < 0 || ms < best_ms) {
            best = c;
            best_ms = ms;
        }
    }
    int rc = aq_set_tile(s, cand[best][0], cand[best][1]);
    if (rc) return rc;
    // the two-step tile, where a storage has two: timed per pair of steps
    if (s->fuse && fused_rows_supported(s->mode, 4)) {
        const int keep = s->fuse_rows;
        int best_rows = keep;
        double best2 = -1;
        for (int rows : {8, 4}) {
            rc = set_fuse_rows(s, rows);
            double ms = 0;
            if (rc == AQ_OK) rc = aq_time_fused_kernel(s, 1, &ms);          // warm up
            if (rc == AQ_OK) rc = aq_time_fused_kernel(s, std::max(1, n_launch / 2), &ms);
            if (rc) {
                (void)set_fuse_rows(s, keep);
                return rc;
            }
            if (best2 < 0 || ms < best2) {
                best2 = ms;
                best_rows = rows;
            }
        }
        rc = set_fuse_rows(s, best_rows);
        if (rc) return rc;
    }
    *tile_x = cand[best][0];
    *tile_y = cand[best][1];
    *ms_per_launch = best_ms;
    return AQ_OK;
}

int aq_run_intervals_timed(aq_solver* s, int32_t n, double* total_ms, double* plain_ms)
{
    if (!s || !total_ms || !plain_ms || n < 1) return fail(AQ_EINVAL, "invalid arguments");
    const int D = s->P.check_interval;
    if (s->step % D) return fail(AQ_ESTATE, "the step count must be a multiple of check_interval");
    if (s->n_tiles == 0) return fail(AQ_ESTATE, "the lattice has no active node");
    int rc = ensure_graph(s, 0);
    if (rc == AQ_OK) rc = ensure_graph(s, 1);
    if (rc) return rc;
    std::vector<hipEvent_t> evs(2 * (size_t)n + 1);
    for (auto& e : evs) HIPCHK(hipEventCreate(&e));
    HIPCHK(hipEventRecord(evs[0], s->stream));
    for (int i = 0; i < n; i++) {
        rc = launch_graph_part(s);
        if (rc) return rc;
        HIPCHK(hipEventRecord(evs[2 * i + 1], s->stream));
        rc = launch_interval_end(s);
        if (rc) return rc;
        HIPCHK(hipEventRecord(evs[2 * i + 2], s->stream));
    }
    HIPCHK(hipEventSynchronize(evs[2 * n]));
    float t = 0;
    double plain = 0;
    for (int i = 0; i < n; i++) {
        HIPCHK(hipEventElapsedTime(&t, evs[2 * i], evs[2 * i + 1]));
        plain += t;
    }
    HIPCHK(hipEventElapsedTime(&t, evs[0], evs[2 * n]));
    *total_ms = t;
    *plain_ms = plain;
    for (auto& e : evs) (void)hipEventDestroy(e);
    return AQ_OK;
}

// A plain device copy in 16-byte words, grid-stride, with non-temporal stores (the step
// kernels' store form past the last-level cache): the bandwidth a streaming kernel reaches
// on this GPU, the context for the step kernels' moved bytes.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void copy_kernel(const u32x4* __restrict__ src, u32x4* __restrict__ dst, size_t n)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        __builtin_nontemporal_store(src[i], &dst[i]);
}

static hipError_t launch_copy(const void* src, void* dst, size_t words16, int blocks, hipStream_t s)
{
    hipLaunchKernelGGL(copy_kernel, dim3(blocks), dim3(256), 0, s, (const u32x4*)src, (u32x4*)dst, words16);
    return hipGetLastError();
}

int aq_copy_bandwidth(size_t bytes, int32_t reps, double* gbs)
{
    if (!gbs || reps < 1 || bytes < ((size_t)1 << 20) || (bytes & 15))
        return fail(AQ_EINVAL, "bytes must be a multiple of 16 and at least 1 MiB, reps at least 1");
    void* src = nullptr;
    void* dst = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    auto release = [&]() {
        if (ev[0]) (void)hipEventDestroy(ev[0]);
        if (ev[1]) (void)hipEventDestroy(ev[1]);
        if (st) (void)hipStreamDestroy(st);
        if (src) (void)hipFree(src);
        if (dst) (void)hipFree(dst);
    };
    hipError_t e = hipMalloc(&src, bytes);
    if (e == hipSuccess) e = hipMalloc(&dst, bytes);
    if (e == hipErrorOutOfMemory) {
        release();
        return fail(AQ_ENOMEM, "the copy buffers do not fit");
    }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    if (e == hipSuccess) e = hipMemsetAsync(src, 0, bytes, st);
    double best = 0;
    for (int r = 0; r <= reps && e == hipSuccess; r++) {   // the first pass warms up
        e = hipEventRecord(ev[0], st);
        if (e == hipSuccess) e = launch_copy(src, dst, bytes / 16, 256 * 8, st);
        if (e == hipSuccess) e = hipEventRecord(ev[1], st);
        if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
        if (e == hipSuccess && r > 0 && ms > 0) best = std::max(best, 2.0 * (double)bytes / ((double)ms * 1e6));
    }
    release();
    if (e != hipSuccess) return fail(AQ_EDEVICE, std::string("copy bandwidth: ") + hipGetErrorString(e));
    *gbs = best;
    return AQ_OK;
}

// Checkpoint file: magic, version, aq_params, step, last check step, exponents, then the
// current and previous population buffers (storage precision) and the residual reference.
int aq_save(aq_solver* s, const char* path)
{
    if (!s || !path) return fail(AQ_EINVAL, "null argument");
    const size_t pop_bytes = (size_t)NPOP * s->L.qs * storage_size(s->mode);
    const size_t up_bytes = 3 * (size_t)s->L.qs * 8;
    std::vector<char> buf(2 * pop_bytes + up_bytes);
    const char* cur = (const char*)(s->cur == 0 ? s->popA() : s->popB());
    const char* prev = (const char*)(s->cur == 0 ? s->popB() : s->popA());
    HIPCHK(hipMemcpyAsync(buf.data(), cur, pop_bytes, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipMemcpyAsync(buf.data() + pop_bytes, prev, pop_bytes, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipMemcpyAsync(buf.data() + 2 * pop_bytes, s->base + s->L.off_uprev, up_bytes, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    FILE* f = std::fopen(path, "wb");
    if (!f) return fail(AQ_EINVAL, std::string("cannot open ") + path);
    const uint32_t magic = 0x4D424C41u, version = 2;   // "ALBM"
    int32_t hdr[4] = {s->exp_f, s->exp_t, (int32_t)s->checks, s->cur};
    int32_t hdr2[2] = {s->ro_slot, 0};
    double useep[2] = {0.0, 0.0};   // lumped outlet: seepage speeds (in effect, previous)
    HIPCHK(hipMemcpyAsync(useep, s->base + s->L.off_counters + kUseepOffset, 16, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    bool ok = std::fwrite(&magic, 4, 1, f) == 1 && std::fwrite(&version, 4, 1, f) == 1 &&
              std::fwrite(&s->P, sizeof(aq_params), 1, f) == 1 && std::fwrite(&s->step, 8, 1, f) == 1 &&
              std::fwrite(&s->last_check_step, 8, 1, f) == 1 && std::fwrite(hdr, 16, 1, f) == 1 &&
              std::fwrite(hdr2, 8, 1, f) == 1 && std::fwrite(useep, 16, 1, f) == 1 &&
              std::fwrite(buf.data(), 1, buf.size(), f) == buf.size();
    std::fclose(f);
    return ok ? AQ_OK : fail(AQ_EINVAL, "short write");
}

int aq_load(aq_solver* s, const char* path)
{
    if (!s || !path) return fail(AQ_EINVAL, "null argument");
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(AQ_EINVAL, std::string("cannot open ") + path);
    uint32_t magic = 0, version = 0;
    aq_params P;
    int64_t step = 0, last = 0;
    int32_t hdr[4], hdr2[2];
    double useep[2];
    bool ok = std::fread(&magic, 4, 1, f) == 1 && std::fread(&version, 4, 1, f) == 1 &&
              std::fread(&P, sizeof(aq_params), 1, f) == 1 && std::fread(&step, 8, 1, f) == 1 &&
              std::fread(&last, 8, 1, f) == 1 && std::fread(hdr, 16, 1, f) == 1 &&
              std::fread(hdr2, 8, 1, f) == 1 && std::fread(useep, 16, 1, f) == 1;
    if (!ok || magic != 0x4D424C41u || version != 2 || std::memcmp(&P, &s->P, sizeof(aq_params)) != 0) {
        std::fclose(f);
        return fail(AQ_EINVAL, "checkpoint does not match this solver");
    }
    const size_t pop_bytes = (size_t)NPOP * s->L.qs * storage_size(s->mode);
    const size_t up_bytes = 3 * (size_t)s->L.qs * 8;
    std::vector<char> buf(2 * pop_bytes + up_bytes);
    ok = std::fread(buf.data(), 1, buf.size(), f) == buf.size();
    std::fclose(f);
    if (!ok) return fail(AQ_EINVAL, "truncated checkpoint");
    HIPCHK(hipStreamSynchronize(s->stream));
    s->cur = hdr[3] & 1;        // which buffer held the state
    void* cur = s->cur == 0 ? s->popA() : s->popB();
    void* prev = s->cur == 0 ? s->popB() : s->popA();
    HIPCHK(hipMemcpyAsync(cur, buf.data(), pop_bytes, hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipMemcpyAsync(prev, buf.data() + pop_bytes, pop_bytes, hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipMemcpyAsync(s->base + s->L.off_uprev, buf.data() + 2 * pop_bytes, up_bytes, hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    s->step = step;
    s->last_check_step = last;
    s->exp_f = hdr[0];
    s->exp_t = hdr[1];
    s->ro_slot = hdr2[0] & 1;
    int rc = set_useep(s, useep[0], useep[1]);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(s->stream));
    s->diverged = false;
    // the observables ring is not part of the checkpoint; the counters keep their
    // device values so the next check step lands in the expected slot
    return AQ_OK;
}

}  // extern "C"
