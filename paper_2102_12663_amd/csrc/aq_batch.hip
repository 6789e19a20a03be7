// Batched serving form of the aqlbm library: many independent lattices (parameter-sweep
// solves of uneven sizes) resident in one HBM arena and stepped together by one
// multi-instance kernel per kernel class (storage x boundary scheme), with a captured HIP
// graph per check interval.
//
// - Admission checks the free arena (first-fit pool), free slots, the work-list capacity
//   and an active-node cap; each admitted instance is an ordinary single-lattice solver
//   carved out of the arena, so its state, fields and checkpoints behave exactly as alone.
// - The kernels read the instance table and the (slot, tile) work lists from device
//   memory; each launch has one block per work item, so the graph is captured again when
//   admissions or retirements change a list's length (not when only instance arguments
//   change, e.g. a new meshwork thickness).
// - After each call to aq_batch_run the latest reductions of every running instance are
//   read back in one copy; converged, diverged and capped instances are retired.
// - An F16S instance whose residual falls below max(tol, 2e-5), or stops falling for 50
//   check intervals, has reached binary16's rounding floor.  If its residual is below tol
//   it is done (AQ_OK).  Otherwise the IOP drift check compares its IOP with the IOP at
//   least kDriftSteps steps earlier: within drift_tol (relative) the state is accepted at
//   the floor (AQ_RESULT_FLOOR); else its state is converted to F32 storage and the solve
//   continues there until the residual falls below tol.  An F16S instance's arena block
//   holds, besides its own layout, the F32 layout and the conversion scratch, so the
//   hand-off never needs memory beyond what admission granted.
#include "aq_internal.h"

#include <map>

using namespace aq;

namespace {

// binary16 rounding keeps the per-step residual of an F16S solve above ~1e-6; its phase
// ends at max(tol, this floor)
constexpr double kF16ResidFloor = 2e-5;
constexpr int kF16Stall = 50;
// the IOP drift check compares the IOP with one taken at least this many steps earlier
constexpr int64_t kDriftSteps = 1000;
constexpr int kIopRing = 32;

// First-fit allocator over [0, size) with coalescing free blocks (offsets in bytes).
class Pool {
public:
    void init(size_t size)
    {
        free_.clear();
        if (size) free_[0] = size;
        size_ = size;
        used_ = 0;
    }
    bool alloc(size_t bytes, size_t* off)
    {
        bytes = align_up(bytes, 256);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t noff = it->first + bytes;
                free_.erase(it);
                if (rest) free_[noff] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = align_up(bytes, 256);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t largest() const
    {
        size_t m = 0;
        for (auto& kv : free_) m = std::max(m, kv.second);
        return m;
    }

private:
    std::map<size_t, size_t> free_;
    size_t size_ = 0, used_ = 0;
};

struct Slot {
    bool used = false, running = false, done = false, reported = false, keep = false;
    double best_resid = 1e300;   // F16S phase: smallest residual so far
    int since_best = 0;          // check intervals since it last fell by 10%
    aq_solver* s = nullptr;
    size_t off = 0, bytes = 0;   // arena block; for F16S: [F16S layout | F32 layout | scratch]
    size_t bytes16 = 0, bytes32 = 0;   // F16S: the first two parts (256-aligned)
    double tol = 0, drift_tol = 0;
    int64_t max_steps = 0, request_id = 0, steps = 0;
    int status = AQ_OK, fallback = 0;
    aq_observables obs;
    int64_t iop_step[kIopRing];  // F16S phase: (step, IOP) at the last check of each run call
    double iop_val[kIopRing];
    int n_iop = 0;
};

// Bytes of the F32 continuation an F16S instance reserves: the F32 layout and the dense
// FP64 image of the state the conversion passes through (13 populations per node).
inline size_t f32_layout_bytes(const aq_params& P, int n_walls)
{
    aq_params Q = P;
    Q.storage = AQ_F32;
    return align_up(make_layout(Q, n_walls).total, 256);
}
inline size_t conversion_scratch_bytes(const aq_params& P)
{
    return align_up((size_t)NPOP * P.nx * P.ny * 8, 256);
}

// IOP drift of an F16S phase: relative change of the IOP against the newest recorded IOP
// taken at least kDriftSteps steps before the current one; false if there is none yet.
bool iop_drift(const Slot& sl, double* drift)
{
    const int64_t now = sl.obs.step;
    for (int j = sl.n_iop - 2; j >= 0 && j >= sl.n_iop - kIopRing; j--) {
        const int r = j % kIopRing;
        if (now - sl.iop_step[r] >= kDriftSteps) {
            const double a = sl.obs.iop_gauge, b0 = sl.iop_val[r];
            *drift = a != 0 ? std::fabs(a - b0) / std::fabs(a) : std::fabs(a - b0);
            return true;
        }
    }
    return false;
}

// Has the current phase reached its residual?  F32/F64: max(resid_u, resid_T) < tol.
// F16S: below max(tol, kF16ResidFloor), or stagnating (no 10% improvement over the last
// kF16Stall check intervals: binary16 rounding noise sets a problem-dependent floor).
bool resid_done(Slot& sl, int mode, int n_intervals)
{
    const double r = std::max(sl.obs.resid_u, sl.obs.resid_T);
    if (mode != AQ_F16S) return r < sl.tol;
    if (r < std::max(sl.tol, kF16ResidFloor)) return true;
    if (r < 0.9 * sl.best_resid) {
        sl.best_resid = r;
        sl.since_best = 0;
    } else {
        sl.since_best += n_intervals;
    }
    return sl.since_best >= kF16Stall;
}

}  // namespace

constexpr int NMODE = 4;            // AQ_F64, AQ_F32, AQ_F16S, AQ_F32X
constexpr int NKIND = 2 * NMODE;    // x boundary scheme

inline int kind_of(const aq_solver* s) { return s->mode + (s->P.bc_scheme == AQ_BC_PAPER ? NMODE : 0); }

struct aq_batch {
    size_t budget = 0;
    char* arena = nullptr;
    Pool pool;
    int max_slots = 0, max_tiles = 0, interval = 0;
    int64_t max_active = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<Slot> slots;
    int64_t step = 0;

    // Instances are grouped into kernel classes ("kinds"): storage mode + NMODE * boundary
    // scheme (the paper's schemes are a compile-time variant of the step kernels).
    InstDesc* d_inst = nullptr;
    int2* d_work[NKIND] = {};
    int2* d_work2[NKIND] = {};
    int* d_nwork = nullptr;         // [0, NKIND) single-step items, [NKIND, 2 NKIND) two-step items
    double* d_partials[NKIND] = {};
    double* d_latest = nullptr;
    double* h_latest = nullptr;     // pinned
    std::vector<InstDesc> h_inst;
    int n_work[NKIND] = {};
    int n_work2[NKIND] = {};

    int nt_store = 0;               // non-temporal stores for the current working set
    int graph_mask = -1;
    int graph_items[2 * NKIND] = {};   // work-list lengths the captured launches were sized for
    // one check interval = graph[0] (the two-step launches of every kernel class) then
    // graph[1] (the remaining single steps, the reducing step and the finishing sums)
    hipGraph_t graph_src[2] = {nullptr, nullptr};
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    int fused_launches = 0;         // two-step launches per kernel class and interval
    // two-step tile rows per kernel class, and the caller's choice (0: by the class's size)
    int rows2[NKIND] = {8, 8, 8, 8, 8, 8, 8, 8};
    int rows_choice = 0;
};

namespace {

BatchArgs batch_args(const aq_batch* b, int kind, int parity)
{
    BatchArgs a;
    a.inst = b->d_inst;
    a.work = b->d_work[kind];
    a.n_work = b->d_nwork + kind;
    a.work2 = b->d_work2[kind];
    a.n_work2 = b->d_nwork + NKIND + kind;
    a.partials = b->d_partials[kind];
    a.latest = b->d_latest;
    a.parity = parity;
    a.max_slots = b->max_slots;
    a.mode = kind % NMODE;
    a.kind = kind;
    a.nt_store = b->nt_store;
    a.bc = kind / NMODE;
    a.tile_y = b->rows2[kind];
    return a;
}

int active_mask(const aq_batch* b)
{
    int m = 0;
    for (int i = 0; i < NKIND; i++)
        if (b->n_work[i] > 0) m |= 1 << i;
    return m;
}

// Work lists and partials of a kernel class, allocated when its first instance arrives.
int ensure_kind(aq_batch* b, int k)
{
    if (b->d_work[k]) return AQ_OK;
    const size_t mt = (size_t)b->max_tiles;
    if (hipMalloc((void**)&b->d_work[k], mt * sizeof(int2)) != hipSuccess ||
        hipMalloc((void**)&b->d_work2[k], mt * sizeof(int2)) != hipSuccess ||
        hipMalloc((void**)&b->d_partials[k], mt * NRED * 8) != hipSuccess) {
        (void)hipFree(b->d_work[k]);
        (void)hipFree(b->d_work2[k]);
        (void)hipFree(b->d_partials[k]);
        b->d_work[k] = b->d_work2[k] = nullptr;
        b->d_partials[k] = nullptr;
        return fail(AQ_ENOMEM, "cannot allocate the batch work lists");
    }
    return AQ_OK;
}

void drop_graph(aq_batch* b)
{
    for (int g = 0; g < 2; g++) {
        if (b->graph[g]) (void)hipGraphExecDestroy(b->graph[g]);
        if (b->graph_src[g]) (void)hipGraphDestroy(b->graph_src[g]);
        b->graph[g] = nullptr;
        b->graph_src[g] = nullptr;
    }
    b->graph_mask = -1;
    std::fill(b->graph_items, b->graph_items + 2 * NKIND, 0);
}

// End a capture on the batch stream and instantiate it into graph slot g.
int finish_capture(aq_batch* b, int g, hipError_t err)
{
    hipGraph_t gr = nullptr;
    const hipError_t e2 = hipStreamEndCapture(b->stream, &gr);
    if (err != hipSuccess || e2 != hipSuccess) {
        if (gr) (void)hipGraphDestroy(gr);
        return fail(AQ_EDEVICE, std::string("batch graph capture: ") + hipGetErrorString(err != hipSuccess ? err : e2));
    }
    hipGraphExec_t ge = nullptr;
    const hipError_t e3 = hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0);
    if (e3 != hipSuccess) {
        (void)hipGraphDestroy(gr);
        return fail(AQ_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e3));
    }
    b->graph_src[g] = gr;
    b->graph[g] = ge;
    return AQ_OK;
}

// One check interval for every kernel class present: interval-1 plain steps, the
// reducing step, and the per-instance finishing sums.  Every launch has one block per work
// item (the hardware dispatcher then balances uneven tiles across the chip), so the graphs
// are captured again whenever admissions or retirements change a work list's length.  The
// interval is two graphs replayed back to back: the two-step launches of every class, then
// the rest (classes are independent, so their order across the two graphs is immaterial).
int ensure_graph(aq_batch* b)
{
    const int mask = active_mask(b);
    bool same = b->graph[0] && b->graph[1] && b->graph_mask == mask;
    for (int m = 0; m < NKIND && same; m++)
        same = b->graph_items[m] == b->n_work[m] && b->graph_items[NKIND + m] == b->n_work2[m];
    if (same) return AQ_OK;
    drop_graph(b);
    // interval - 1 plain steps then the reducing one: an even number F of two-step launches
    // (every storage; F16S: 69.3 against 67.3 GLUPS with single steps on the 512-instance
    // sweep), so every interval swaps the buffers an even number of times and the batch is
    // back at parity 0 (instances are admitted at parity 0)
    const int plain = b->interval - 1;
    const int F = (plain / 2) & ~1;
    b->fused_launches = F;
    HIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    hipError_t err = hipSuccess;
    for (int m = 0; m < NKIND && err == hipSuccess; m++) {
        if (!(mask & (1 << m))) continue;
        int parity = 0;
        for (int j = 0; j < F && err == hipSuccess; j++, parity ^= 1)
            err = launch_batch_step2(m % NMODE, batch_args(b, m, parity), b->n_work2[m], b->stream);
    }
    int rc = finish_capture(b, 0, err);
    if (rc) return rc;
    HIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    for (int m = 0; m < NKIND && err == hipSuccess; m++) {
        if (!(mask & (1 << m))) continue;
        int parity = 0;     // F is even
        for (int j = 2 * F; j < plain && err == hipSuccess; j++, parity ^= 1)
            err = launch_batch_step(m % NMODE, false, batch_args(b, m, parity), b->n_work[m], b->stream);
        if (err == hipSuccess) err = launch_batch_step(m % NMODE, true, batch_args(b, m, parity), b->n_work[m], b->stream);
    }
    for (int m = 0; m < NKIND && err == hipSuccess; m++)
        if (mask & (1 << m)) err = launch_batch_finish(batch_args(b, m, 0), b->stream);
    rc = finish_capture(b, 1, err);
    if (rc) {
        drop_graph(b);
        return rc;
    }
    b->graph_mask = mask;
    std::copy(b->n_work, b->n_work + NKIND, b->graph_items);
    std::copy(b->n_work2, b->n_work2 + NKIND, b->graph_items + NKIND);
    return AQ_OK;
}

// Two-step tile rows of a kernel class: 64 x 4 tiles (six blocks per CU) in F32 and F16S
// while the class's running instances hold fewer than kFuse4MaxActive active nodes, so a
// small batch still spreads over the chip; 64 x 8 otherwise, or as the caller chose.
// Instances whose fused tile list has another height are listed again.
int choose_rows(aq_batch* b, const bool* force8)
{
    int64_t act[NKIND] = {};
    for (const Slot& sl : b->slots)
        if (sl.used && sl.running) act[kind_of(sl.s)] += sl.s->n_active;
    for (int m = 0; m < NKIND; m++) {
        int rows = 8;
        if (fused_rows_supported(m % NMODE, 4) && !force8[m])
            rows = b->rows_choice ? b->rows_choice : (act[m] < kFuse4MaxActive ? 4 : 8);
        if (rows != b->rows2[m]) {
            b->rows2[m] = rows;
            drop_graph(b);                 // the captured launches bake the tile height in
        }
    }
    for (const Slot& sl : b->slots) {
        if (!sl.used || !sl.running || sl.s->fuse_rows == b->rows2[kind_of(sl.s)]) continue;
        const int rc = set_fuse_rows(sl.s, b->rows2[kind_of(sl.s)]);
        if (rc) return rc;
    }
    return AQ_OK;
}

// Rebuild the instance table and the per-mode work lists from the running slots and
// copy them to the device (ordered on the batch stream, then synchronised).  A class whose
// 64 x 4 list would not fit the work-list capacity takes 64 x 8 tiles.
int upload_tables(aq_batch* b)
{
    bool force8[NKIND] = {};
    int rc = choose_rows(b, force8);
    if (rc) return rc;
    for (;;) {
        int64_t n2[NKIND] = {};
        for (const Slot& sl : b->slots)
            if (sl.used && sl.running) n2[kind_of(sl.s)] += (int64_t)sl.s->htiles2.size();
        bool again = false;
        for (int m = 0; m < NKIND; m++)
            if (b->rows2[m] == 4 && n2[m] > b->max_tiles) force8[m] = again = true;
        if (!again) break;
        rc = choose_rows(b, force8);
        if (rc) return rc;
    }
    std::vector<int2> work[NKIND], work2[NKIND];
    double bytes = 0;
    for (const Slot& sl : b->slots)
        if (sl.used && sl.running) bytes += (double)sl.s->n_active * bytes_per_update(sl.s->mode);
    const int nt = bytes > kMallBytes ? 1 : 0;
    if (nt != b->nt_store) {
        b->nt_store = nt;
        drop_graph(b);                 // the captured launches bake the store policy in
    }
    for (int i = 0; i < b->max_slots; i++) {
        InstDesc& d = b->h_inst[i];
        std::memset(&d, 0, sizeof(d));
        const Slot& sl = b->slots[i];
        if (!sl.used || !sl.running) continue;
        const int m = kind_of(sl.s);
        d.a = make_args(sl.s, true);
        d.a.nt_store = nt;
        d.a2 = make_args2(sl.s, true);
        d.a2.nt_store = nt;
        d.work_start = (int)work[m].size();
        d.work_count = sl.s->n_tiles;
        d.running = 1;
        d.mode = m;                    // the instance's kernel class
        for (int t : sl.s->htiles) work[m].push_back(make_int2(i, t));
        for (int t : sl.s->htiles2) work2[m].push_back(make_int2(i, t));
    }
    for (int m = 0; m < NKIND; m++) {
        if ((int)work[m].size() > b->max_tiles || (int)work2[m].size() > b->max_tiles)
            return fail(AQ_EBUSY, "work list capacity exceeded");
        if (!work[m].empty()) {
            rc = ensure_kind(b, m);
            if (rc) return rc;
        }
        b->n_work[m] = (int)work[m].size();
        b->n_work2[m] = (int)work2[m].size();
        if (!work[m].empty())
            HIPCHK(hipMemcpyAsync(b->d_work[m], work[m].data(), work[m].size() * sizeof(int2), hipMemcpyHostToDevice, b->stream));
        if (!work2[m].empty())
            HIPCHK(hipMemcpyAsync(b->d_work2[m], work2[m].data(), work2[m].size() * sizeof(int2), hipMemcpyHostToDevice, b->stream));
    }
    int counts[2 * NKIND];
    for (int m = 0; m < NKIND; m++) {
        counts[m] = b->n_work[m];
        counts[NKIND + m] = b->n_work2[m];
    }
    HIPCHK(hipMemcpyAsync(b->d_nwork, counts, sizeof(counts), hipMemcpyHostToDevice, b->stream));
    HIPCHK(hipMemcpyAsync(b->d_inst, b->h_inst.data(), b->h_inst.size() * sizeof(InstDesc), hipMemcpyHostToDevice, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    return AQ_OK;
}

int64_t running_active(const aq_batch* b)
{
    int64_t n = 0;
    for (const Slot& sl : b->slots)
        if (sl.used && sl.running) n += sl.s->n_active;
    return n;
}

void free_slot(aq_batch* b, int i)
{
    Slot& sl = b->slots[i];
    if (sl.s) aq_destroy(sl.s);
    if (sl.bytes) b->pool.release(sl.off, sl.bytes);
    sl = Slot();
}

// Continue an F16S solve in F32 storage from its current state, inside the instance's
// arena block: the F32 solver goes to the block's second part, the state passes through
// the scratch in its third part, then the first part (the F16S layout) and the scratch
// return to the pool.
int convert_to_f32(aq_batch* b, int i)
{
    Slot& sl = b->slots[i];
    aq_solver* s16 = sl.s;
    const size_t n = (size_t)s16->P.nx * s16->P.ny;
    aq_params P = s16->P;
    P.storage = AQ_F32;
    if (!sl.bytes16 || !sl.bytes32) return fail(AQ_ESTATE, "instance has no F32 reservation");
    // the new solver needs the mask and the wall list again: rebuild them from the old one
    std::vector<uint8_t> mask(n);
    for (int y = 0; y < P.ny; y++)
        for (int x = 0; x < P.nx; x++) mask[(size_t)y * P.nx + x] = s16->htype[(size_t)y * s16->L.pitch + x] & 31;
    std::vector<aq_wall_node> walls(std::max(s16->n_walls, 1));
    for (int w = 0; w < s16->n_walls; w++) {
        const int k = s16->hwall_node[w];
        walls[w].node = (k / s16->L.pitch) * P.nx + k % s16->L.pitch;
        walls[w].wall = s16->hwall_id[w];
        walls[w].n_x = s16->hwall_n[2 * w];
        walls[w].n_y = s16->hwall_n[2 * w + 1];
        for (int i = 0; i < 8; i++) walls[w].q[i] = s16->hwall_q[8 * (size_t)w + i];
    }
    const size_t off32 = sl.off + sl.bytes16, off_scr = off32 + sl.bytes32;
    const size_t scr_bytes = sl.bytes - sl.bytes16 - sl.bytes32;
    double* dense = (double*)(b->arena + off_scr);
    StepArgs a = make_readout_args(s16);   // src = prev: pulls to the current state
    hipError_t e = launch_unpack(s16->mode, a, 7, 0, P.p_ref, dense, b->stream);
    aq_solver* s32 = nullptr;
    int rc = AQ_OK;
    if (e == hipSuccess) {
        rc = create_common(&P, mask.data(), walls.data(), s16->n_walls, b->arena + off32, sl.bytes32, b->stream, false, &s32,
                           fused_tile_rows(AQ_F32));
        if (rc == AQ_OK) rc = aq_set_tile(s32, s16->tile_x, s16->tile_y);
        if (rc == AQ_OK) {
            // lumped outlet: the seepage speeds carry over with the state
            const size_t uo = s32->L.off_counters + kUseepOffset;
            e = hipMemcpyAsync(s32->base + uo, s16->base + s16->L.off_counters + kUseepOffset, 16,
                               hipMemcpyDeviceToDevice, b->stream);
            if (e != hipSuccess) rc = fail(AQ_EDEVICE, std::string("seepage speed copy: ") + hipGetErrorString(e));
        }
        if (rc == AQ_OK) rc = set_state(s32, dense);
        if (rc == AQ_OK) {
            s32->step = s16->step;
            s32->checks = 0;
            s32->last_check_step = s16->last_check_step;
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess || rc != AQ_OK) {
        if (s32) aq_destroy(s32);
        return rc != AQ_OK ? rc : fail(AQ_EDEVICE, std::string("state conversion: ") + hipGetErrorString(e));
    }
    aq_destroy(s16);
    b->pool.release(sl.off, sl.bytes16);
    if (scr_bytes) b->pool.release(off_scr, scr_bytes);
    sl.s = s32;
    sl.off = off32;
    sl.bytes = sl.bytes32;
    sl.bytes16 = sl.bytes32 = 0;
    sl.fallback = 1;
    return AQ_OK;
}

// Enqueue n_intervals check intervals (both graphs of each); with events, ev[2i] and
// ev[2i+1] bracket the two-step part of interval i and ev[2n] follows the last interval.
int enqueue_intervals(aq_batch* b, int n_intervals, hipEvent_t* ev)
{
    int rc = ensure_graph(b);
    if (rc) return rc;
    for (int i = 0; i < n_intervals; i++) {
        if (ev) HIPCHK(hipEventRecord(ev[2 * i], b->stream));
        HIPCHK(hipGraphLaunch(b->graph[0], b->stream));
        if (ev) HIPCHK(hipEventRecord(ev[2 * i + 1], b->stream));
        HIPCHK(hipGraphLaunch(b->graph[1], b->stream));
    }
    if (ev) HIPCHK(hipEventRecord(ev[2 * n_intervals], b->stream));
    return AQ_OK;
}

// After n_intervals have been enqueued: read back the latest reductions of every running
// instance (synchronising the stream) and retire the finished ones.
int after_intervals(aq_batch* b, int n_intervals)
{
    const int64_t dn = (int64_t)n_intervals * b->interval;
    b->step += dn;
    HIPCHK(hipMemcpyAsync(b->h_latest, b->d_latest, (size_t)b->max_slots * NRED * 8, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    bool changed = false;
    int rc = AQ_OK;
    for (int i = 0; i < b->max_slots; i++) {
        Slot& sl = b->slots[i];
        if (!sl.used || !sl.running) continue;
        aq_solver* s = sl.s;
        s->step += dn;
        s->ro_slot = 1;   // every interval ends with a reducing step and its finish kernel
        s->checks += n_intervals;
        s->last_check_step = s->step;
        sl.steps += dn;
        raw_to_obs(s, b->h_latest + (size_t)i * NRED, s->step, &sl.obs);
        if (s->mode == AQ_F16S) {
            const int r = sl.n_iop % kIopRing;
            sl.iop_step[r] = sl.obs.step;
            sl.iop_val[r] = sl.obs.iop_gauge;
            sl.n_iop++;
        }
        bool finish = false;
        if (sl.obs.n_nonfinite > 0) {
            sl.status = AQ_EDIVERGED;
            s->diverged = true;
            finish = true;
        } else if (resid_done(sl, s->mode, n_intervals)) {
            double drift = 0;
            if (s->mode != AQ_F16S || std::max(sl.obs.resid_u, sl.obs.resid_T) < sl.tol) {
                sl.status = AQ_OK;
                finish = true;
            } else if (iop_drift(sl, &drift) && drift <= sl.drift_tol) {
                sl.status = AQ_RESULT_FLOOR;          // accepted at binary16's floor
                finish = true;
            } else if (sl.n_iop >= 2 && iop_drift(sl, &drift)) {
                const int rc2 = convert_to_f32(b, i);  // the IOP still drifts: continue in F32
                if (rc2 != AQ_OK) {
                    sl.status = rc2;
                    finish = true;
                    rc = rc2;
                }
                changed = true;
            }                                          // else: no IOP history yet, keep going
        }
        if (!finish && sl.running && sl.steps >= sl.max_steps) {
            sl.status = AQ_ENOTCONVERGED;
            finish = true;
        }
        if (finish) {
            sl.running = false;
            sl.done = true;
            changed = true;
        }
    }
    (void)rc;   // a failed hand-off is reported through that request's status
    if (changed) return upload_tables(b);
    return AQ_OK;
}

}  // namespace

extern "C" {

int aq_batch_create(size_t budget_bytes, int32_t max_slots, int64_t max_active_nodes, int32_t max_tiles,
                    int32_t check_interval, void* hip_stream, aq_batch** out)
{
    if (!out || max_slots < 1 || max_slots > 65536 || max_tiles < 1 || budget_bytes < (1u << 20) ||
        check_interval < 2 || (check_interval & 1) || max_active_nodes < 0)
        return fail(AQ_EINVAL, "invalid batch parameters");
    aq_batch* b = new aq_batch();
    b->budget = align_up(budget_bytes, 256);
    b->max_slots = max_slots;
    b->max_tiles = max_tiles;
    b->max_active = max_active_nodes;
    b->interval = check_interval;
    b->slots.resize(max_slots);
    b->h_inst.resize(max_slots);
    auto cleanup = [&](int rc) {
        std::string keep = aq_last_error();
        aq_batch_destroy(b);
        g_err = keep;
        return rc;
    };
    if (hipMalloc((void**)&b->arena, b->budget) != hipSuccess) return cleanup(fail(AQ_ENOMEM, "cannot allocate the batch arena"));
    b->pool.init(b->budget);
    if (hip_stream) {
        b->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreate(&b->stream) != hipSuccess) return cleanup(fail(AQ_EDEVICE, "hipStreamCreate failed"));
        b->own_stream = true;
    }
    bool ok = hipMalloc((void**)&b->d_inst, (size_t)max_slots * sizeof(InstDesc)) == hipSuccess &&
              hipMalloc((void**)&b->d_nwork, 2 * NKIND * sizeof(int)) == hipSuccess &&
              hipMalloc((void**)&b->d_latest, (size_t)max_slots * NRED * 8) == hipSuccess &&
              hipHostMalloc((void**)&b->h_latest, (size_t)max_slots * NRED * 8, hipHostMallocDefault) == hipSuccess;
    if (!ok) return cleanup(fail(AQ_ENOMEM, "cannot allocate the batch tables"));
    int rc = upload_tables(b);
    if (rc) return cleanup(rc);
    *out = b;
    return AQ_OK;
}

int aq_batch_destroy(aq_batch* b)
{
    if (!b) return AQ_OK;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    for (int i = 0; i < (int)b->slots.size(); i++)
        if (b->slots[i].used) free_slot(b, i);
    (void)hipFree(b->d_inst);
    (void)hipFree(b->d_nwork);
    (void)hipFree(b->d_latest);
    if (b->h_latest) (void)hipHostFree(b->h_latest);
    for (int m = 0; m < NKIND; m++) {
        (void)hipFree(b->d_work[m]);
        (void)hipFree(b->d_work2[m]);
        (void)hipFree(b->d_partials[m]);
    }
    (void)hipFree(b->arena);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return AQ_OK;
}

int aq_batch_admit(aq_batch* b, const aq_params* P, const uint8_t* mask, const aq_wall_node* walls,
                   int32_t n_walls, int32_t tile_x, int32_t tile_y, double tol, double drift_tol,
                   int64_t max_steps, int64_t request_id, int32_t keep, int32_t* slot)
{
    if (!b || !slot) return fail(AQ_EINVAL, "null argument");
    if (!(tol > 0) || !(drift_tol > 0) || max_steps < 1) return fail(AQ_EINVAL, "tol, drift_tol and max_steps must be positive");
    if (tile_x * tile_y != 256) return fail(AQ_EINVAL, "batched instances use 256-thread tiles");
    int rc = validate(P, mask, walls, n_walls);
    if (rc) return rc;
    if (P->storage == AQ_F16S) {
        aq_params Q = *P;
        Q.storage = AQ_F32;
        if (!offsets_fit(Q))
            return fail(AQ_EINVAL, "lattice too large for the FP32 continuation of an F16S solve: three population "
                                   "planes must stay within 4 GiB");
    }
    if (P->check_interval != b->interval) return fail(AQ_EINVAL, "check_interval differs from the batch's");
    int free_i = -1;
    for (int i = 0; i < b->max_slots; i++)
        if (!b->slots[i].used) { free_i = i; break; }
    if (free_i < 0) return fail(AQ_EBUSY, "no free slot");
    const Layout L = make_layout(*P, n_walls);
    // an F16S instance also reserves its F32 continuation (layout and conversion scratch)
    const size_t b16 = align_up(L.total, 256);
    const size_t b32 = P->storage == AQ_F16S ? f32_layout_bytes(*P, n_walls) : 0;
    const size_t total = b16 + (P->storage == AQ_F16S ? b32 + conversion_scratch_bytes(*P) : 0);
    size_t off = 0;
    if (!b->pool.alloc(total, &off)) return fail(AQ_EBUSY, "not enough free HBM in the batch arena");
    aq_solver* s = nullptr;
    rc = create_common(P, mask, walls, n_walls, b->arena + off, L.total, b->stream, false, &s,
                       fused_tile_rows(P->storage));
    if (rc == AQ_OK) rc = aq_set_tile(s, tile_x, tile_y);
    if (rc == AQ_OK && b->max_active && running_active(b) + s->n_active > b->max_active)
        rc = fail(AQ_EBUSY, "active-node cap reached");
    if (rc == AQ_OK && b->n_work[kind_of(s)] + s->n_tiles > b->max_tiles)
        rc = fail(AQ_EBUSY, "work list capacity reached");
    if (rc != AQ_OK) {
        std::string keep_err = aq_last_error();
        if (s) aq_destroy(s);
        b->pool.release(off, total);
        g_err = keep_err;
        return rc;
    }
    Slot& sl = b->slots[free_i];
    sl = Slot();
    sl.used = sl.running = true;
    sl.keep = keep != 0;
    sl.s = s;
    sl.off = off;
    sl.bytes = total;
    if (P->storage == AQ_F16S) {
        sl.bytes16 = b16;
        sl.bytes32 = b32;
    }
    sl.tol = tol;
    sl.drift_tol = drift_tol;
    sl.max_steps = max_steps;
    sl.request_id = request_id;
    std::memset(&sl.obs, 0, sizeof(sl.obs));
    rc = upload_tables(b);
    if (rc) {
        std::string keep_err = aq_last_error();
        free_slot(b, free_i);
        (void)upload_tables(b);
        g_err = keep_err;
        return rc;
    }
    *slot = free_i;
    return AQ_OK;
}

int aq_batch_run(aq_batch* b, int32_t n_intervals)
{
    if (!b || n_intervals < 1) return fail(AQ_EINVAL, "invalid arguments");
    if (active_mask(b) == 0) return AQ_OK;
    int rc = enqueue_intervals(b, n_intervals, nullptr);
    if (rc) return rc;
    return after_intervals(b, n_intervals);
}

int aq_batch_run_timed(aq_batch* b, int32_t n_intervals, double* total_ms, double* fused_ms, int32_t* fused_launches)
{
    if (!b || n_intervals < 1 || !total_ms || !fused_ms || !fused_launches) return fail(AQ_EINVAL, "invalid arguments");
    if (active_mask(b) == 0) return fail(AQ_ESTATE, "no running instance");
    std::vector<hipEvent_t> ev(2 * (size_t)n_intervals + 1, nullptr);
    for (auto& e : ev) HIPCHK(hipEventCreate(&e));
    int rc = enqueue_intervals(b, n_intervals, ev.data());
    if (rc == AQ_OK) {
        HIPCHK(hipEventSynchronize(ev[2 * n_intervals]));
        float t = 0;
        double fused = 0;
        for (int i = 0; i < n_intervals; i++) {
            HIPCHK(hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]));
            fused += t;
        }
        HIPCHK(hipEventElapsedTime(&t, ev[0], ev[2 * n_intervals]));
        *total_ms = t;
        *fused_ms = fused;
        int classes = 0;
        for (int m = 0; m < NKIND; m++)
            if (active_mask(b) & (1 << m)) classes++;
        *fused_launches = b->fused_launches * classes * n_intervals;
        rc = after_intervals(b, n_intervals);
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    return rc;
}

int aq_batch_poll(aq_batch* b, aq_result* done, int32_t cap, int32_t* n_done)
{
    if (!b || !n_done || (cap > 0 && !done)) return fail(AQ_EINVAL, "invalid arguments");
    int n = 0;
    for (int i = 0; i < b->max_slots && n < cap; i++) {
        Slot& sl = b->slots[i];
        if (!sl.used || !sl.done || sl.reported) continue;
        aq_result& r = done[n++];
        std::memset(&r, 0, sizeof(r));
        r.request_id = sl.request_id;
        r.slot = i;
        r.status = sl.status;
        r.storage = sl.s->mode;
        r.fallback = sl.fallback;
        r.steps = sl.steps;
        r.obs = sl.obs;
        sl.reported = true;
        if (!sl.keep) free_slot(b, i);
    }
    *n_done = n;
    return AQ_OK;
}

int aq_batch_read_field(aq_batch* b, int32_t slot, int32_t field, int32_t q, double* host, size_t count)
{
    if (!b || slot < 0 || slot >= b->max_slots || !b->slots[slot].used) return fail(AQ_EINVAL, "no such slot");
    return aq_read_field(b->slots[slot].s, field, q, host, count);
}

int aq_batch_observe(aq_batch* b, int32_t slot, aq_observables* out)
{
    if (!b || slot < 0 || slot >= b->max_slots || !b->slots[slot].used) return fail(AQ_EINVAL, "no such slot");
    return aq_observe(b->slots[slot].s, out);
}

int aq_batch_set_outlet(aq_batch* b, int32_t slot, double K_tm, double h_tm, double p_sc)
{
    if (!b || slot < 0 || slot >= b->max_slots || !b->slots[slot].used) return fail(AQ_EINVAL, "no such slot");
    HIPCHK(hipStreamSynchronize(b->stream));
    int rc = aq_set_outlet(b->slots[slot].s, K_tm, h_tm, p_sc);
    if (rc) return rc;
    return upload_tables(b);    // the instance table carries the constants
}

int aq_batch_resume(aq_batch* b, int32_t slot, double tol, int64_t max_steps)
{
    if (!b || slot < 0 || slot >= b->max_slots || !b->slots[slot].used) return fail(AQ_EINVAL, "no such slot");
    Slot& sl = b->slots[slot];
    if (!sl.keep || !sl.done || sl.running) return fail(AQ_ESTATE, "only a finished instance admitted with keep can resume");
    if (!(tol > 0) || max_steps < 1) return fail(AQ_EINVAL, "tol and max_steps must be positive");
    if (sl.status != AQ_OK && sl.status != AQ_ENOTCONVERGED && sl.status != AQ_RESULT_FLOOR)
        return fail(AQ_ESTATE, "the instance failed");
    if (b->max_active && running_active(b) + sl.s->n_active > b->max_active) return fail(AQ_EBUSY, "active-node cap reached");
    if (b->n_work[kind_of(sl.s)] + sl.s->n_tiles > b->max_tiles) return fail(AQ_EBUSY, "work list capacity reached");
    sl.running = true;
    sl.done = sl.reported = false;
    sl.tol = tol;
    sl.max_steps = sl.steps + max_steps;
    sl.best_resid = 1e300;
    sl.since_best = 0;
    sl.n_iop = 0;
    sl.status = AQ_OK;
    return upload_tables(b);
}

int aq_batch_diagnose(aq_batch* b, int32_t slot, void* ws, size_t ws_bytes, aq_diagnostics* out)
{
    if (!b || slot < 0 || slot >= b->max_slots || !b->slots[slot].used) return fail(AQ_EINVAL, "no such slot");
    return aq_diagnose(b->slots[slot].s, ws, ws_bytes, out);
}

int aq_batch_release(aq_batch* b, int32_t slot)
{
    if (!b || slot < 0 || slot >= b->max_slots || !b->slots[slot].used) return fail(AQ_EINVAL, "no such slot");
    Slot& sl = b->slots[slot];
    const bool was_running = sl.running;
    free_slot(b, slot);
    if (was_running) return upload_tables(b);
    return AQ_OK;
}

int aq_batch_get_info(aq_batch* b, aq_batch_info* o)
{
    if (!b || !o) return fail(AQ_EINVAL, "null argument");
    std::memset(o, 0, sizeof(*o));
    o->max_slots = b->max_slots;
    for (const Slot& sl : b->slots) {
        if (!sl.used) continue;
        if (sl.running) o->running++;
        else o->finished++;
    }
    for (int m = 0; m < NKIND; m++) o->n_work[m % NMODE] += b->n_work[m];
    o->active_nodes = running_active(b);
    o->budget_bytes = b->budget;
    o->used_bytes = b->pool.used();
    o->largest_free_bytes = b->pool.largest();
    o->step = b->step;
    for (int m = 0; m < NMODE; m++) o->fused_tile_rows[m] = b->rows2[m];
    return AQ_OK;
}

int aq_batch_set_fused_tile_rows(aq_batch* b, int32_t rows)
{
    if (!b) return fail(AQ_EINVAL, "null batch");
    if (rows != 0 && rows != 4 && rows != 8) return fail(AQ_EINVAL, "two-step tile rows must be 0 (by size), 4 or 8");
    b->rows_choice = rows;
    return upload_tables(b);
}

}  // extern "C"
