// HIP kernels (gfx950) for one time step of the coupled lattice Boltzmann model of
// arXiv:2102.12663, section 2.3.
//
// One launch = one time step over the active tiles.  Each thread owns one node and
//   1. pulls its 8 flow and 5 thermal post-collision populations from the upstream
//      neighbours (buffer src), or from its own opposite slot through the link's boundary
//      rule when the upstream node is not active (half-way bounce-back, moving-wall inlet,
//      anti-bounce-back pressure outlet, anti-bounce-back / adiabatic thermal walls);
//   2. takes the moments u = sum e_i h_i, p - p_ref = 3/5 (sum h_i + S_0(u))      (eq. 9)
//      and T = T_ref + sum g_i                                                  (eq. 13);
//   3. forms the buoyant force g beta (T - T0)(sin phi, cos phi) (eq. 15-16) and, in
//      porous nodes, the Darcy drag -(nu/K) u_D on the mid-step velocity          (eq. 4);
//   4. relaxes both distributions toward their equilibria (eq. 6-8, eq. 11-12) and adds
//      the force term (eq. 17 for buoyancy on the axis links; weights 3 w_i for the drag);
//   5. stores the 13 post-collision values to dst at its own index (SoA, coalesced).
// Every stored value is read exactly once in the next step, so HBM traffic per active
// node is one read and one write of each live population plus the type byte.
//
// On check steps the same kernel also reduces the IOP, outlet/inlet fluxes, wall shear
// stress, residuals, masses and max |u| in double: wavefront shuffles and one partial per
// block, then a one-block kernel sums the partials in a fixed order (deterministic, with
// no fences or atomics inside the step kernel).
#include "aq_device.h"

#include <math.h>

namespace aq {

// D2Q9 link directions (e_2, e_4 are the gravity axis of eq. 17) and opposites.
__device__ constexpr int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

// Storage precision: how a population is stored and in which type it is computed.
template <int MODE> struct Traits;
// L is the element type of the two-step kernels' LDS image: it holds values decoded from the
// storage (exact in single precision for every storage but FP64), or in F16S the single-
// precision intermediate step itself.
template <> struct Traits<0> {   // AQ_F64
    using S = double;
    using R = double;
    using L = double;
    using Acc = double;      // exact-enough sums of a node's stored values
    __device__ static R ld(const S* p, R) { return *p; }
    __device__ static R ldv(S v, R) { return v; }
    __device__ static void st(S* p, R v, R) { *p = v; }
    __device__ static S enc(Acc v, R) { return v; }
    __device__ static Acc dec(S s, R) { return s; }
};
template <> struct Traits<1> {   // AQ_F32
    using S = float;
    using R = float;
    using L = float;
    using Acc = double;
    __device__ static R ld(const S* p, R) { return *p; }
    __device__ static R ldv(S v, R) { return v; }
    __device__ static void st(S* p, R v, R) { *p = v; }
    __device__ static S enc(Acc v, R) { return (S)v; }
    __device__ static Acc dec(S s, R) { return s; }
};
template <> struct Traits<2> {   // AQ_F16S: binary16 of (deviation * 2^s)
    // The step computes in units of the stored values (deviation * 2^s, the flow and the
    // thermal lattice each with its own power-of-two scale): loads and stores are bare
    // conversions, and the few constants that carry physical units are scaled instead
    // (see fscale / tscale).  Scaling by a power of two is exact, so every rounding is the
    // physical-unit arithmetic's, scaled.  st() writes a physical value (state installation).
    using S = _Float16;
    using R = float;
    using L = float;
    using Acc = float;       // float sums of binary16 values are far finer than their ulp
    __device__ static R ld(const S* p, R) { return (R)(*p); }
    __device__ static R ldv(S v, R) { return (R)v; }
    __device__ static void st(S* p, R v, R sc) { *p = (S)(v * sc); }
    __device__ static S enc(Acc v, R) { return (S)v; }
    __device__ static Acc dec(S s, R) { return (R)s; }
};
template <> struct Traits<3> {   // AQ_F32X: FP32 storage, FP64 arithmetic
    using S = float;
    using R = double;
    using L = float;
    using Acc = double;
    __device__ static R ld(const S* p, R) { return *p; }
    __device__ static R ldv(S v, R) { return v; }
    __device__ static void st(S* p, R v, R) { *p = (S)v; }
    __device__ static S enc(Acc v, R) { return (S)v; }
    __device__ static Acc dec(S s, R) { return s; }
};

// A step constant in the compute type: the double itself, or its single-precision copy
// (rounded on the host), so that FP32 compute converts no constant per node.
template <typename R> __device__ __forceinline__ R cst(double d, float f);
template <> __device__ __forceinline__ double cst<double>(double d, float) { return d; }
template <> __device__ __forceinline__ float cst<float>(double, float f) { return f; }

// Compute units of a storage: F16S computes in stored units, so a physical flow quantity
// enters multiplied by fscale and a physical thermal quantity by tscale (the per-solver
// powers of two 2^s); the other storages compute in physical units (factor one, folded).
template <int MODE, typename R> __device__ __forceinline__ R fscale(const StepArgs& a)
{
    if constexpr (MODE == 2) return R(a.sf32);
    else return R(1);
}
template <int MODE, typename R> __device__ __forceinline__ R tscale(const StepArgs& a)
{
    if constexpr (MODE == 2) return R(a.st32);
    else return R(1);
}

template <typename R> struct Node {
    R h[9];   // h[1..8] flow (h[0] unused)
    R g[5];   // g[0..4] thermal
    R qin, qout;
};

// Weight of link i in eq. 8 and lambda_i of eq. 7 (lambda_i = 3 w_i).
template <typename R> __device__ __forceinline__ R wflow(int i) { return i <= 4 ? R(1.0 / 9.0) : R(1.0 / 36.0); }
template <typename R> __device__ __forceinline__ R lam(int i) { return i <= 4 ? R(1.0 / 3.0) : R(1.0 / 12.0); }

__device__ __forceinline__ bool is_active(uint8_t t)
{
    uint8_t c = t & CLS_MASK;
    return c == FLUID || c == POROUS;
}

// ------------------------------------------------------------------------------ moments
template <typename R> struct Moments {
    R sum, ux, uy, uu, dp, th;   // th = T - T_ref
};

template <typename R>
__device__ __forceinline__ Moments<R> moments(const Node<R>& n)
{
    Moments<R> m;
    const R* h = n.h;
    if constexpr (sizeof(R) == 4) {
        // single precision: the velocity from differences of opposite links, which near
        // equilibrium hold nearly equal values (lambda_i (p - p_ref) dominates both), so
        // each difference is exact and u carries no rounding of the pressure part
        const R d13 = h[1] - h[3], d24 = h[2] - h[4], d57 = h[5] - h[7], d68 = h[6] - h[8];
        m.ux = d13 + (d57 - d68);
        m.uy = d24 + (d57 + d68);
        m.sum = ((h[1] + h[3]) + (h[2] + h[4])) + ((h[5] + h[7]) + (h[6] + h[8]));
    } else {
        m.sum = ((h[1] + h[2]) + (h[3] + h[4])) + ((h[5] + h[6]) + (h[7] + h[8]));
        m.ux = (h[1] - h[3]) + (h[5] - h[6]) + (h[8] - h[7]);
        m.uy = (h[2] - h[4]) + (h[5] + h[6]) - (h[7] + h[8]);
    }
    m.uu = fma(m.ux, m.ux, m.uy * m.uy);
    // p - p_ref = c^2/(4 sigma) [sum h_i + S_0(u)], S_0 = -(2/3)|u|^2, sigma = 5/12
    m.dp = R(0.6) * (m.sum - R(2.0 / 3.0) * m.uu);
    m.th = (n.g[0] + n.g[1]) + (n.g[2] + n.g[3]) + n.g[4];
    return m;
}

// The moments in double of a node held in the compute type R: the check-step reductions
// and the field read-out of the single-precision forms widen the node's values (exactly)
// and take the moments from them, so the reduced IOP, residuals and read-out fields carry
// no single-precision rounding of their own.  In double this is `moments` itself.
template <int MODE, typename R>
__device__ __forceinline__ Moments<double> wide_moments(const StepArgs& a, const Node<R>& n, Node<double>& w)
{
    // back to physical units (F16S: exact division by the powers of two)
    const double uf = MODE == 2 ? a.inv_sf : 1.0, ut = MODE == 2 ? a.inv_st : 1.0;
#pragma unroll
    for (int i = 1; i <= 8; i++) w.h[i] = (double)n.h[i] * uf;
#pragma unroll
    for (int i = 0; i <= 4; i++) w.g[i] = (double)n.g[i] * ut;
    w.qin = (double)n.qin * uf;
    w.qout = (double)n.qout * uf;
    return moments(w);
}

// ------------------------------------------------------------------------------ addressing
// Element at byte offset `kb` from `p + off` elements, where p + off is the same for every
// thread of the block (a plane base shifted by a link): the base goes through a scalar
// register, so a load or store takes it with the 32-bit per-node offset as its offset
// operand and no thread does 64-bit address arithmetic.  The offsets stay below 4 GiB: the
// node-type bytes (at most 2^30 nodes) and, in the F32, F32X and F16S storages, three
// population planes (the reach of a boundary pull; checked at creation).
__device__ __forceinline__ const char* uniform_base(const void* p)
{
#if defined(__HIP_DEVICE_COMPILE__)
    const unsigned long long b = (unsigned long long)p;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
    typedef const __attribute__((address_space(1))) char GlobalChar;
    return (const char*)(GlobalChar*)(((unsigned long long)hi << 32) | lo);
#else
    return (const char*)p;
#endif
}

template <typename S>
__device__ __forceinline__ const S* at(const S* p, long long off, unsigned kb)
{
    return (const S*)(uniform_base(p + off) + kb);
}

template <typename S>
__device__ __forceinline__ S* at(S* p, long long off, unsigned kb)
{
    return (S*)(const_cast<char*>(uniform_base(p + off)) + kb);
}

// ------------------------------------------------------------------------------ pull
// All 13 loads are issued without intervening branches: a boundary node first reads its
// 8 neighbours' type bytes, each load address is then selected (upstream slot, or the
// node's own opposite slot for a link into a non-active node), and the link rules are
// applied to the loaded values afterwards.  Interior nodes skip the type reads.
// The three phases of the pull, separable so that a thread owning several nodes can issue
// the loads of all of them before waiting on any.
// (1) Types of the 8 neighbours (boundary nodes only; interior nodes see all FLUID).
__device__ __forceinline__ void pull_types(const StepArgs& a, int k, bool boundary, uint8_t* nt)
{
    if (boundary) {
#pragma unroll
        for (int i = 1; i <= 8; i++) nt[i] = *at(a.type, -(EY[i] * a.pitch + EX[i]), (unsigned)k);
    } else {
#pragma unroll
        for (int i = 1; i <= 8; i++) nt[i] = FLUID;
    }
}

// (2) The 13 loads: upstream slot, or the own opposite slot for a link into a non-active
// node.  In the FP32-compute storages an interior node (all neighbours active) pulls every
// link from upstream with one addressing form: a plane base shifted by the link (uniform,
// scalar arithmetic) plus the node's own byte offset, the same for all 13 loads; that
// saves the integer work of the compute-bound formats.  FP64 keeps one 64-bit address per
// load and the per-link selects: with this interior path, or one with 64-bit addresses, its
// single step took 2-4% longer and its two-step launch 1-4%.
template <int MODE>
__device__ __forceinline__ void pull_loads(const StepArgs& a, const typename Traits<MODE>::S* src, int k,
                                           bool boundary, const uint8_t* nt, Node<typename Traits<MODE>::R>& n)
{
    using T = Traits<MODE>;
    using R = typename T::R;
    using S = typename T::S;
    const R inv_f = cst<R>(a.inv_sf, a.inv_sf32), inv_t = cst<R>(a.inv_st, a.inv_st32);
    const unsigned kb = (unsigned)k * (unsigned)sizeof(S);
    if (MODE != 0 && !boundary) {
#pragma unroll
        for (int i = 1; i <= 8; i++) n.h[i] = T::ld(at(src, (i - 1) * a.qs - (EY[i] * a.pitch + EX[i]), kb), inv_f);
        n.g[0] = T::ld(at(src, 8 * a.qs, kb), inv_t);
#pragma unroll
        for (int i = 1; i <= 4; i++) n.g[i] = T::ld(at(src, (8 + i) * a.qs - (EY[i] * a.pitch + EX[i]), kb), inv_t);
        // keeps the compiler from merging these loads with the boundary path's into one set
        // with per-lane 64-bit addresses (it waits for nothing: no loaded value is used)
        __asm__ volatile("" ::: "memory");
        return;
    }
    if constexpr (MODE != 0) {
        // a boundary node: the upstream slot, or the node's own opposite slot for a link from
        // a non-active node, both as one plane base (uniform) plus a 32-bit per-node offset.
        // The base is the lower of the two slots' planes (opposite links are two planes
        // apart, and a plane is longer than a row plus one), so both offsets are k's own
        // byte offset plus a non-negative uniform distance.
#pragma unroll
        for (int i = 1; i <= 8; i++) {
            const long long up_k0 = (long long)(i - 1) * a.qs - (EY[i] * a.pitch + EX[i]);   // slot of node 0
            const long long own_k0 = (long long)(OPP[i] - 1) * a.qs;
            const long long lo = OPP[i] > i ? up_k0 : own_k0;
            const unsigned d = (unsigned)((OPP[i] > i ? own_k0 - up_k0 : up_k0 - own_k0) * (long long)sizeof(S));
            const bool at_lo = OPP[i] > i ? is_active(nt[i]) : !is_active(nt[i]);
            n.h[i] = T::ld(at(src, lo, at_lo ? kb : kb + d), inv_f);
        }
        n.g[0] = T::ld(at(src, 8 * a.qs, kb), inv_t);
#pragma unroll
        for (int i = 1; i <= 4; i++) {
            const long long up_k0 = (long long)(8 + i) * a.qs - (EY[i] * a.pitch + EX[i]);
            const long long own_k0 = (long long)(8 + OPP[i]) * a.qs;
            const long long lo = OPP[i] > i ? up_k0 : own_k0;
            const unsigned d = (unsigned)((OPP[i] > i ? own_k0 - up_k0 : up_k0 - own_k0) * (long long)sizeof(S));
            const bool at_lo = OPP[i] > i ? is_active(nt[i]) : !is_active(nt[i]);
            n.g[i] = T::ld(at(src, lo, at_lo ? kb : kb + d), inv_t);
        }
        return;
    }
#pragma unroll
    for (int i = 1; i <= 8; i++) {
        const long long off = is_active(nt[i]) ? (long long)(i - 1) * a.qs + (k - EY[i] * a.pitch - EX[i])
                                               : (long long)(OPP[i] - 1) * a.qs + k;
        n.h[i] = T::ld(src + off, inv_f);
    }
    const S* tsrc = src + 8LL * a.qs;
    n.g[0] = T::ld(tsrc + k, inv_t);
#pragma unroll
    for (int i = 1; i <= 4; i++) {
        const long long off = is_active(nt[i]) ? (long long)i * a.qs + (k - EY[i] * a.pitch - EX[i])
                                               : (long long)OPP[i] * a.qs + k;
        n.g[i] = T::ld(tsrc + off, inv_t);
    }
}

// Interpolated bounce-back (Bouzidi et al.; the paper's wall scheme, section 2.3) for link
// i of node k, whose upstream node x - e_i = x + e_o is a wall the link from x along e_o
// meets at the fraction q; v = h*_o(x) (the half-way value), `own_i` = h*_i(x) and
// `behind` = h*_o(x + e_i) (the node behind x, used for q < 1/2).
template <typename R>
__device__ __forceinline__ R bouzidi(R q, R v, R own_i, R behind)
{
    if (q >= R(0.5)) return v / (R(2) * q) + (R(2) * q - R(1)) / (R(2) * q) * own_i;
    return R(2) * q * v + (R(1) - R(2) * q) * behind;
}

// Deviation-form equilibria (eq. 7-8 and eq. 12) for the extrapolated boundaries.
template <typename R>
__device__ __forceinline__ R heq_dev(int i, R dp, R ux, R uy)
{
    const R eu = R(EX[i]) * ux + R(EY[i]) * uy;
    return lam<R>(i) * dp + wflow<R>(i) * (R(3) * eu + R(4.5) * eu * eu - R(1.5) * (ux * ux + uy * uy));
}

// T_abs = T_ref + th
template <typename R>
__device__ __forceinline__ R geq_dev(const StepArgs& a, int i, R th, R T_abs, R ux, R uy)
{
    const R eu = R(EX[i]) * ux + R(EY[i]) * uy;
    return cst<R>(a.wT, a.wT32) * (th + T_abs * eu * cst<R>(a.inv_cs2T, a.inv_cs2T32));
}

// Does node (type t, neighbour types nt) have a link that the paper's extrapolation
// handles: from an INLET / OUTLET node (flow) or a Dirichlet wall or INLET (thermal)?
__device__ __forceinline__ bool needs_extrapolation(const StepArgs& a, const uint8_t* nt)
{
    bool e = false;
#pragma unroll
    for (int i = 1; i <= 8; i++) {
        const uint8_t c = nt[i] & CLS_MASK;
        if (is_active(nt[i])) continue;
        if (c == INLET || c == OUTLET) e = true;
        if (i <= 4 && c == SOLID && ((nt[i] >> WALL_SHIFT) & 3) != WALL_BOX) e = true;
    }
    return a.bc_paper && e;
}

// The extrapolated boundary values (Guo et al.'s non-equilibrium extrapolation; section
// 2.3's inlet/outlet and thermal-wall schemes): for flow link i from an INLET / OUTLET
// node, h_i = h^eq_i(p_b, u_b) + (h*_i(x) - h^eq_i(p*, u*)); for thermal link i from a
// Dirichlet wall or INLET, g_i = g^eq_i(T_w, u_b) + (g*_i(x) - g^eq_i(T*, u*)).  `own`
// holds x's post-collision populations and `ms` their moments.  Returns the flow mass the
// link brings in (for the inflow / outflow sums) through `net`.
template <typename R>
__device__ __forceinline__ void extrapolate_links(const StepArgs& a, const uint8_t* nt, const Node<R>& own,
                                                  const Moments<R>& ms, Node<R>& n)
{
#pragma unroll
    for (int i = 1; i <= 8; i++) {
        if (is_active(nt[i])) continue;
        const uint8_t c = nt[i] & CLS_MASK;
        if (c != INLET && c != OUTLET) continue;
        R dpb = ms.dp, uxb = ms.ux, uyb = ms.uy;
        if (c == INLET) {
            uxb = R(a.uin_x);
            uyb = R(a.uin_y);
        } else if (a.lumped) {
            const int d = ((nt[i] >> WALL_SHIFT) & 3) + 1;
            uxb = R(EX[d]) * R(*a.useep);
            uyb = R(EY[d]) * R(*a.useep);
        } else {
            dpb = R(a.dp_out);
        }
        const R v = n.h[i];
        n.h[i] = heq_dev(i, dpb, uxb, uyb) + (own.h[i] - heq_dev(i, ms.dp, ms.ux, ms.uy));
        if (c == INLET) n.qin += n.h[i] - v;
        else n.qout += v - n.h[i];
    }
    const R T_abs = cst<R>(a.T_ref, a.T_ref32) + ms.th;
#pragma unroll
    for (int i = 1; i <= 4; i++) {
        if (is_active(nt[i])) continue;
        const uint8_t c = nt[i] & CLS_MASK;
        const uint8_t wall = (nt[i] >> WALL_SHIFT) & 3;
        if (!(c == INLET || (c == SOLID && wall != WALL_BOX))) continue;
        const double tw = c == INLET ? a.tw_inlet : (wall == WALL_CORNEA ? a.tw_cornea : a.tw_iris);
        const R uxb = c == INLET ? R(a.uin_x) : R(0), uyb = c == INLET ? R(a.uin_y) : R(0);
        n.g[i] = geq_dev(a, i, R(tw), cst<R>(a.T_ref, a.T_ref32) + R(tw), uxb, uyb) + (own.g[i] - geq_dev(a, i, ms.th, T_abs, ms.ux, ms.uy));
    }
}

// extrapolate_links in physical units: F16S nodes (stored units) are scaled down, the
// links extrapolated, and the node scaled back up (both exact).
template <int MODE, typename R>
__device__ __forceinline__ void extrapolate_physical(const StepArgs& a, const uint8_t* nt, Node<R> own, Node<R>& n)
{
    if constexpr (MODE == 2) {
        const R uf = R(a.inv_sf32), ut = R(a.inv_st32), f = R(a.sf32), t = R(a.st32);
#pragma unroll
        for (int i = 1; i <= 8; i++) {
            own.h[i] *= uf;
            n.h[i] *= uf;
        }
#pragma unroll
        for (int i = 0; i <= 4; i++) {
            own.g[i] *= ut;
            n.g[i] *= ut;
        }
        n.qin *= uf;
        n.qout *= uf;
        const Moments<R> ms = moments(own);
        extrapolate_links(a, nt, own, ms, n);
#pragma unroll
        for (int i = 1; i <= 8; i++) n.h[i] *= f;
#pragma unroll
        for (int i = 0; i <= 4; i++) n.g[i] *= t;
        n.qin *= f;
        n.qout *= f;
    } else {
        const Moments<R> ms = moments(own);
        extrapolate_links(a, nt, own, ms, n);
    }
}

// Link fraction of the wall that link i's upstream solid presents to wall-list node w
// (q of the link toward it, -1 if none).
__device__ __forceinline__ double wall_fraction(const StepArgs& a, int w, int i)
{
    return w < 0 ? -1.0 : a.wall_q[8LL * w + (OPP[i] - 1)];
}

// (3) The link rules on the loaded values of links into non-active nodes.  `t` is the
// node's type byte; the paper's wall scheme loads the extra population it needs here.
template <int MODE, bool BC>
__device__ __forceinline__ void pull_rules(const StepArgs& a, const typename Traits<MODE>::S* src, int k, uint8_t t,
                                           const uint8_t* nt, Node<typename Traits<MODE>::R>& n)
{
    using T = Traits<MODE>;
    using R = typename T::R;
    n.qin = R(0);
    n.qout = R(0);
    if (!(t & F_BOUNDARY)) return;
    const int w = (BC && (t & F_WSS)) ? a.widx[k] : -1;
    const bool extra = BC && needs_extrapolation(a, nt);
#pragma unroll
    for (int i = 1; i <= 8; i++) {
        if (is_active(nt[i])) continue;
        const uint8_t c = nt[i] & CLS_MASK;
        const R v = n.h[i];
        if (extra && (c == INLET || c == OUTLET)) {
            // extrapolated below
        } else if (c == INLET) {                               // moving wall at u_in
            const R corr = R(6.0) * wflow<R>(i) * (R(EX[i]) * cst<R>(a.uin_x, a.uin_x32) + R(EY[i]) * cst<R>(a.uin_y, a.uin_y32)) *
                             fscale<MODE, R>(a);
            n.h[i] = v + corr;
            n.qin += corr;
        } else if (c == OUTLET) {
            if (a.lumped) {                                    // wall moving at u_s n (meshwork)
                const int d = ((nt[i] >> WALL_SHIFT) & 3) + 1;
                const R corr = R(6.0) * wflow<R>(i) * (R(EX[i] * EX[d] + EY[i] * EY[d]) * R(*a.useep)) *
                               fscale<MODE, R>(a);
                n.h[i] = v + corr;
                n.qout -= corr;
            } else {                                           // pressure anti-bounce-back
                const R out = -v + R(2.0) * lam<R>(i) * cst<R>(a.dp_out, a.dp_out32) * fscale<MODE, R>(a);
                n.qout += v - out;
                n.h[i] = out;
            }
        } else if (BC && w >= 0) {                             // SOLID on the wall list
            const double q = wall_fraction(a, w, i);
            const R inv_f = cst<R>(a.inv_sf, a.inv_sf32);
            if (q >= 0.5) {
                n.h[i] = bouzidi(R(q), v, T::ld(src + (long long)(i - 1) * a.qs + k, inv_f), R(0));
            } else if (q > 0.0 && is_active(nt[OPP[i]])) {
                const R behind = T::ld(src + (long long)(OPP[i] - 1) * a.qs + (k + EY[i] * a.pitch + EX[i]), inv_f);
                n.h[i] = bouzidi(R(q), v, R(0), behind);
            }
        }                                                      // else half-way bounce-back
    }
#pragma unroll
    for (int i = 1; i <= 4; i++) {
        if (extra || is_active(nt[i])) continue;
        const uint8_t c = nt[i] & CLS_MASK;
        const uint8_t wall = (nt[i] >> WALL_SHIFT) & 3;
        if (c == INLET || (c == SOLID && wall != WALL_BOX)) {  // Dirichlet anti-bounce-back
            const R tw = c == INLET ? cst<R>(a.tw_inlet, a.tw_inlet32)
                                    : (wall == WALL_CORNEA ? cst<R>(a.tw_cornea, a.tw_cornea32)
                                                           : cst<R>(a.tw_iris, a.tw_iris32));
            n.g[i] = -n.g[i] + R(2.0) * cst<R>(a.wT, a.wT32) * tw * tscale<MODE, R>(a);
        }                                                      // else adiabatic bounce-back
    }
    if constexpr (BC) {
        if (!extra) return;
        // the node's own post-collision populations and their moments
        Node<R> own;
        const R inv_f = cst<R>(a.inv_sf, a.inv_sf32), inv_t = cst<R>(a.inv_st, a.inv_st32);
#pragma unroll
        for (int i = 1; i <= 8; i++) own.h[i] = T::ld(src + (long long)(i - 1) * a.qs + k, inv_f);
#pragma unroll
        for (int i = 0; i <= 4; i++) own.g[i] = T::ld(src + (8LL + i) * a.qs + k, inv_t);
        extrapolate_physical<MODE>(a, nt, own, n);
    }
}

template <int MODE, bool BC>
__device__ __forceinline__ void pull_all(const StepArgs& a, const typename Traits<MODE>::S* src, int k, uint8_t t,
                                         Node<typename Traits<MODE>::R>& n)
{
    uint8_t nt[9];
    const bool boundary = (t & F_BOUNDARY) != 0;
    pull_types(a, k, boundary, nt);
    pull_loads<MODE>(a, src, k, boundary, nt, n);
    pull_rules<MODE, BC>(a, src, k, t, nt, n);
}

// ------------------------------------------------------------------------------ collide
// eq. 7-8 for one link: w_i [3 e_i.u + 4.5 (e_i.u)^2 - 1.5 |u|^2] + lambda_i (p - p_ref),
// with u15 = 1.5 |u|^2 and l = lambda_i (p - p_ref)
template <typename R>
__device__ __forceinline__ R heq_link(R w, R eu, R u15, R l)
{
    return fma(w, fma(R(4.5) * eu, eu, R(3) * eu) - u15, l);
}

template <int MODE, typename R>
__device__ __forceinline__ void collide(const StepArgs& a, bool porous, const Node<R>& n,
                                        const Moments<R>& m, R* hs, R* gs)
{
    const R om = cst<R>(a.omega_f, a.omega_f32), omc = R(1) - om;
    // buoyancy, eq. 15-16 (F16S: th in thermal and the force in flow compute units)
    const R th = MODE == 2 ? m.th * R(a.inv_st32) : m.th;  // T - T_ref
    const R tm = th + cst<R>(a.dT0, a.dT032);                // T - T0
    const R Bx = cst<R>(a.bx, a.bx32) * fscale<MODE, R>(a) * tm, By = cst<R>(a.by, a.by32) * fscale<MODE, R>(a) * tm;
    R Dx = R(0), Dy = R(0);
    if (porous) {                              // Darcy drag on the mid-step velocity, eq. 4
        const R dd = cst<R>(a.drag_den, a.drag_den32), nk = cst<R>(a.nuK, a.nuK32);
        Dx = -nk * ((m.ux + R(0.5) * Bx) * dd);
        Dy = -nk * ((m.uy + R(0.5) * By) * dd);
    }
    const R ux = m.ux, uy = m.uy;
    if constexpr (MODE == 1 || MODE == 2) {
        // FP32 arithmetic whose constants keep the collision's conservation laws exact.
        // Rounded to single precision one by one, the weights of eq. 8 no longer satisfy
        // the discrete identities: 9 fl(1/9) = 1 + 7.5e-9, so sum_i e_i h^eq_i = u (1 +
        // 7.5e-9) and every collision adds omega 7.5e-9 u of momentum, an anti-friction
        // that the chamber's slowest modes (damped by nu k^2 ~ 1e-5 per step) amplify to a
        // ~1e-3 relative velocity error at steady state; the mass identity breaks the same
        // way (by ~7e-8 of sum h per step).  Written out, eq. 7-9 give
        //   h^eq_i = A_i S + B_i (e_i.u) + C_i (e_i.u)^2 - D_i |u|^2,  S = sum_{j>=1} h_j,
        // with A = 3/5 lambda_i, B = 3 w_i, C = 9/2 w_i, D = 3/2 w_i + 2/5 lambda_i
        // (A_1 = 1/5, B_1 = 1/3, C_1 = 1/2, D_1 = 3/10 on the axis links, a quarter of each
        // on the diagonals).  The single-precision constants below satisfy, exactly in
        // real arithmetic, sum_i A_i = 1 and 2 C_1 + 4 C_5 = 4 D_1 + 4 D_5 (mass) and
        // 2 B_1 + 4 B_5 = 1 (momentum); each subtraction forming them is exact.  What is
        // left is the rounding of individual operations, without a sign of its own.
        constexpr float A1 = 0.2f, A5 = 0.25f - A1;
        constexpr float B1 = 1.0f / 3.0f, B5 = (1.0f - 2.0f * B1) * 0.25f;
        constexpr float D1 = 0.3f, D5 = 0.375f - D1;
        // quadratic terms in compute units: F16S's u carries the scale, so C and D take
        // its inverse (exact)
        const float q = MODE == 2 ? a.inv_sf32 : 1.0f;
        const float e1 = fma(A1, m.sum, -((D1 * q) * m.uu)), e5 = fma(A5, m.sum, -((D5 * q) * m.uu));
        // link forces: eq. 17 buoyancy on the axis links, the drag with weights B_i
        const float Fx = fma(0.5f, Bx, B1 * Dx), Fy = fma(0.5f, By, B1 * Dy);
        const float Fp = B5 * (Dx + Dy), Fm = B5 * (Dy - Dx);
        // eq. 6 as h + omega (h^eq - h) + F: near equilibrium h^eq - h is exact, and no
        // rounded 1 - omega enters
        auto pair = [&](float eu, float C, float B, float base, float F, float hi, float ho, float& si, float& so) {
            const float even = fma(C * eu, eu, base), odd = B * eu;
            si = hi + fma(om, (even + odd) - hi, F);
            so = ho + fma(om, (even - odd) - ho, -F);
        };
        pair(ux, 0.5f * q, B1, e1, Fx, n.h[1], n.h[3], hs[1], hs[3]);
        pair(uy, 0.5f * q, B1, e1, Fy, n.h[2], n.h[4], hs[2], hs[4]);
        pair(ux + uy, 0.125f * q, B5, e5, Fp, n.h[5], n.h[7], hs[5], hs[7]);
        pair(uy - ux, 0.125f * q, B5, e5, Fm, n.h[6], n.h[8], hs[6], hs[8]);
        // eq. 11-12 with w0T + 4 wT = 1 exactly (set on the host) and the advective part
        // w_i T (e_i.u)/c_sT^2 = T (e_i.u)/2 (c_sT^2 = 2 wT), whose sum is T u exactly
        // (F16S: the advective part takes the thermal scale over the flow scale)
        const float omT = a.omega_t32;
        const float T = a.T_ref32 + th;
        const float ev = a.wT32 * m.th, k = (MODE == 2 ? 0.5f * (a.st32 * a.inv_sf32) : 0.5f) * T;
        gs[0] = n.g[0] + omT * (a.w0T32 * m.th - n.g[0]);
        gs[1] = n.g[1] + omT * (fma(k, ux, ev) - n.g[1]);
        gs[3] = n.g[3] + omT * (fma(-k, ux, ev) - n.g[3]);
        gs[2] = n.g[2] + omT * (fma(k, uy, ev) - n.g[2]);
        gs[4] = n.g[4] + omT * (fma(-k, uy, ev) - n.g[4]);
    } else {
        // each link on its own: in FP64 this order's rounding stays close to the plain
        // per-link definition (1e-12), in FP32 it keeps the steady-state error lower
        const R u15 = R(1.5) * m.uu;
        const R w1 = R(1.0 / 9.0), w5 = R(1.0 / 36.0);
        const R l1 = R(1.0 / 3.0) * m.dp, l5 = R(1.0 / 12.0) * m.dp;
        const R d3 = R(1.0 / 3.0), d12 = R(1.0 / 12.0);
        // eq. 7-8 equilibria, eq. 6 relaxation, eq. 17 / drag force terms
        hs[1] = fma(omc, n.h[1], fma(om, heq_link(w1, ux, u15, l1), R(0.5) * Bx + d3 * Dx));
        hs[2] = fma(omc, n.h[2], fma(om, heq_link(w1, uy, u15, l1), R(0.5) * By + d3 * Dy));
        hs[3] = fma(omc, n.h[3], fma(om, heq_link(w1, -ux, u15, l1), -(R(0.5) * Bx + d3 * Dx)));
        hs[4] = fma(omc, n.h[4], fma(om, heq_link(w1, -uy, u15, l1), -(R(0.5) * By + d3 * Dy)));
        hs[5] = fma(omc, n.h[5], fma(om, heq_link(w5, ux + uy, u15, l5), d12 * (Dx + Dy)));
        hs[6] = fma(omc, n.h[6], fma(om, heq_link(w5, uy - ux, u15, l5), d12 * (Dy - Dx)));
        hs[7] = fma(omc, n.h[7], fma(om, heq_link(w5, -ux - uy, u15, l5), -(d12 * (Dx + Dy))));
        hs[8] = fma(omc, n.h[8], fma(om, heq_link(w5, ux - uy, u15, l5), d12 * (Dx - Dy)));
        // eq. 11-12: thermal relaxation toward w_i [(T - T_ref) + T e_i.u / c_sT^2]
        const R omT = cst<R>(a.omega_t, a.omega_t32), omTc = R(1) - omT;
        const R T = cst<R>(a.T_ref, a.T_ref32) + m.th;
        const R wT = cst<R>(a.wT, a.wT32), k2 = cst<R>(a.inv_cs2T, a.inv_cs2T32) * T;
        gs[0] = fma(omTc, n.g[0], omT * (cst<R>(a.w0T, a.w0T32) * m.th));
        gs[1] = fma(omTc, n.g[1], omT * (wT * fma(k2, ux, m.th)));
        gs[2] = fma(omTc, n.g[2], omT * (wT * fma(k2, uy, m.th)));
        gs[3] = fma(omTc, n.g[3], omT * (wT * fma(-k2, ux, m.th)));
        gs[4] = fma(omTc, n.g[4], omT * (wT * fma(-k2, uy, m.th)));
    }
}

// Write the 13 encoded values of a node.  Past the last-level cache (working sets larger
// than the 256 MB MALL) non-temporal stores keep the written stream from evicting the data
// the step still has to read; below it, ordinary stores keep the next step's reads cached.
template <int MODE, bool NT>
__device__ __forceinline__ void put_all(const StepArgs& a, typename Traits<MODE>::S* dst, int k,
                                        const typename Traits<MODE>::S* e)
{
    const unsigned kb = (unsigned)k * (unsigned)sizeof(typename Traits<MODE>::S);
    // FP64 addresses each store in 64 bits, the FP32-compute storages as the loads do
    if (MODE == 0) {
#pragma unroll
        for (int i = 0; i < NPOP; i++) {
            typename Traits<MODE>::S* p = dst + (long long)i * a.qs + k;
            if (NT) __builtin_nontemporal_store(e[i], p);
            else *p = e[i];
        }
    } else {
#pragma unroll
        for (int i = 0; i < NPOP; i++) {
            typename Traits<MODE>::S* p = at(dst, i * a.qs, kb);
            if (NT) __builtin_nontemporal_store(e[i], p);
            else *p = e[i];
        }
    }
}

template <int MODE, bool NT>
__device__ __forceinline__ void store_all(const StepArgs& a, typename Traits<MODE>::S* dst, int k,
                                          const typename Traits<MODE>::R* hs,
                                          const typename Traits<MODE>::R* gs)
{
    using T = Traits<MODE>;
    using R = typename T::R;
    const R sf = cst<R>(a.sf, a.sf32), st = cst<R>(a.st, a.st32);
    typename T::S e[NPOP];
#pragma unroll
    for (int i = 1; i <= 8; i++) e[i - 1] = T::enc((typename T::Acc)hs[i], sf);
#pragma unroll
    for (int i = 0; i <= 4; i++) e[8 + i] = T::enc((typename T::Acc)gs[i], st);
    put_all<MODE, NT>(a, dst, k, e);
}

// Reduced-precision store that keeps the node's mass exact.  Collision conserves sum h and
// sum g, but rounding each post-collision value to the storage format does not, and at a
// steady state the same rounding repeats every step: a persistent mass source that shifts
// the pressure level (the IOP) by the source over the outflow resistance.  Here the
// rounded values are decoded, their sum is compared with the sum of the node's incoming
// values (F32 and F32X: in double, exactly for these few terms; F16S: in single precision,
// far finer than binary16's ulp, in stored units like the whole F16S step), and the
// difference r is added to the value where the format resolves finest, which is rounded
// again.  That value must be among the smallest: on a larger one a correction below half
// its ulp rounds away (with the flow residual on the larger-valued h_2 or h_4 the steady
// velocity error of F32X grew 40-fold; with the thermal residual on g_0 the F16S IOP error
// 15-fold).  The flow search covers all eight links in F16S, where binary16's coarse ulp
// makes the difference (on the smallest diagonal only, the F16S steady velocity error grew
// 4-fold), and the four diagonals in single precision, whose pressure part is a quarter of
// the axis links' (no measurable difference: F32X 9.1e-6 against 8.9e-6).  The
// mirror x -> -x maps the links onto each other (flow 1 <-> 3, 5 <-> 6, 7 <-> 8; heat
// 1 <-> 3; the others onto themselves); a mirror-symmetric state stays symmetric because
// ties are never broken by link order between mirror images: the links that are their
// own image come first (flow 2, 4; heat 0, 2, 4), then the pairs in a fixed order, and
// when both links of the pair holding the minimum have it, the one with the larger
// incoming (pre-collision) value takes r, a choice the mirror maps onto its image; only
// when those are equal too (on a symmetry axis) does each take r/2.  (Splitting every tie
// loses the correction at twice the threshold, and binary16 values tie often.)
// Shares of the residual for the two links a, b of a mirror pair, `fa` / `fb`: the link
// holds the minimum (and its pair was chosen); on a tie the larger incoming value ia / ib
// decides, and equal incoming values split it.
template <typename Acc, typename R>
__device__ __forceinline__ void pair_weights(bool fa, bool fb, R ia, R ib, Acc& wa, Acc& wb)
{
    const bool tie = fa && fb;
    const bool ta = ia > ib, tb = ib > ia;
    wa = fa ? (tie ? (ta ? Acc(1) : (tb ? Acc(0) : Acc(0.5))) : Acc(1)) : Acc(0);
    wb = fb ? (tie ? (tb ? Acc(1) : (ta ? Acc(0) : Acc(0.5))) : Acc(1)) : Acc(0);
}

template <int MODE, int N>
__device__ __forceinline__ void conserve_encode(const typename Traits<MODE>::R* in,
                                                const typename Traits<MODE>::R* out,
                                                typename Traits<MODE>::S* enc, typename Traits<MODE>::R sc,
                                                typename Traits<MODE>::R inv)
{
    using T = Traits<MODE>;
    using Acc = typename T::Acc;
    using L = typename T::L;   // exact for a decoded stored value
    Acc target = (Acc)in[0];
#pragma unroll
    for (int i = 1; i < N; i++) target += (Acc)in[i];
    L d[N];
    Acc sum = 0;
#pragma unroll
    for (int i = 0; i < N; i++) {
        enc[i] = T::enc((Acc)out[i], sc);
        d[i] = (L)T::ldv(enc[i], inv);
        sum = i == 0 ? (Acc)d[0] : sum + (Acc)d[i];
    }
    const Acc r = target - sum;
    if constexpr (N == 5 && MODE == 2) {
        // binary16: every link is encoded again with its share (one mixed-precision fma
        // each, cheaper than selecting the links that take r)
        const L a0 = fabs(d[0]), a1 = fabs(d[1]), a2 = fabs(d[2]), a3 = fabs(d[3]), a4 = fabs(d[4]);
        const L mn = fmin(fmin(fmin(a0, a2), a4), fmin(a1, a3));
        const bool f0 = a0 == mn, f1 = a1 == mn, f2 = a2 == mn, f3 = a3 == mn, f4 = a4 == mn;
        const bool self = f0 || f2 || f4;
        const Acc w0 = f0 ? Acc(1) : Acc(0);
        const Acc w2 = !f0 && f2 ? Acc(1) : Acc(0);
        const Acc w4 = !f0 && !f2 && f4 ? Acc(1) : Acc(0);
        Acc w1, w3;
        pair_weights(!self && f1, !self && f3, in[1], in[3], w1, w3);
        enc[0] = T::enc(fma(w0, r, (Acc)d[0]), sc);
        enc[1] = T::enc(fma(w1, r, (Acc)d[1]), sc);
        enc[2] = T::enc(fma(w2, r, (Acc)d[2]), sc);
        enc[3] = T::enc(fma(w3, r, (Acc)d[3]), sc);
        enc[4] = T::enc(fma(w4, r, (Acc)d[4]), sc);
        return;
    }
    if constexpr (N == 5) {
        // the storages with single-precision values and double sums encode again only the
        // one or two links that take r (fewer registers live across the double arithmetic);
        // a zero share would give every other link back its own encoding
        const L a0 = fabs(d[0]), a1 = fabs(d[1]), a2 = fabs(d[2]), a3 = fabs(d[3]), a4 = fabs(d[4]);
        const L mn = fmin(fmin(fmin(a0, a2), a4), fmin(a1, a3));
        const bool f0 = a0 == mn, f1 = a1 == mn, f2 = a2 == mn, f3 = a3 == mn, f4 = a4 == mn;
        const bool self = f0 || f2 || f4;
        const bool s2 = !f0 && f2, s4 = !f0 && !f2 && f4;
        Acc wa, wb;
        pair_weights(!self && f1, !self && f3, in[1], in[3], wa, wb);
        if (self) wa = Acc(1);
        const L da = f0 ? d[0] : s2 ? d[2] : s4 ? d[4] : d[1];
        const typename T::S ea = T::enc(fma(wa, r, (Acc)da), sc), eb = T::enc(fma(wb, r, (Acc)d[3]), sc);
        enc[0] = f0 ? ea : enc[0];
        enc[2] = s2 ? ea : enc[2];
        enc[4] = s4 ? ea : enc[4];
        enc[1] = self ? enc[1] : ea;
        enc[3] = self ? enc[3] : eb;
        return;
    }
    if constexpr (MODE == 2) {
        // links 1..8 are entries 0..7: h_2, h_4 first, then the pairs (1,3), (5,6), (7,8)
        L m[8];
#pragma unroll
        for (int i = 0; i < 8; i++) m[i] = fabs(d[i]);
        const L mn = fmin(fmin(fmin(m[1], m[3]), fmin(m[0], m[2])), fmin(fmin(m[4], m[5]), fmin(m[6], m[7])));
        bool f[8];
#pragma unroll
        for (int i = 0; i < 8; i++) f[i] = m[i] == mn;
        const bool self = f[1] || f[3];
        const bool p13 = !self && (f[0] || f[2]);
        const bool p56 = !self && !p13 && (f[4] || f[5]);
        const bool p78 = !self && !p13 && !p56;
        Acc w[8];
        w[1] = f[1] ? Acc(1) : Acc(0);
        w[3] = !f[1] && f[3] ? Acc(1) : Acc(0);
        pair_weights(p13 && f[0], p13 && f[2], in[0], in[2], w[0], w[2]);
        pair_weights(p56 && f[4], p56 && f[5], in[4], in[5], w[4], w[5]);
        pair_weights(p78 && f[6], p78 && f[7], in[6], in[7], w[6], w[7]);
#pragma unroll
        for (int i = 0; i < 8; i++) enc[i] = T::enc(fma(w[i], r, (Acc)d[i]), sc);
    } else {
        // the diagonals 5..8 (entries 4..7): the pair (5, 6) first, then (7, 8); only the
        // pair that takes r is encoded again, as for the thermal links above
        const L a5 = fabs(d[4]), a6 = fabs(d[5]), a7 = fabs(d[6]), a8 = fabs(d[7]);
        const L mn = fmin(fmin(a5, a6), fmin(a7, a8));
        const bool f5 = a5 == mn, f6 = a6 == mn, f7 = a7 == mn, f8 = a8 == mn;
        const bool p56 = f5 || f6;
        Acc wa, wb;
        pair_weights(p56 ? f5 : f7, p56 ? f6 : f8, p56 ? in[4] : in[6], p56 ? in[5] : in[7], wa, wb);
        const L da = p56 ? d[4] : d[6], db = p56 ? d[5] : d[7];
        const typename T::S ea = T::enc(fma(wa, r, (Acc)da), sc), eb = T::enc(fma(wb, r, (Acc)db), sc);
        enc[4] = p56 ? ea : enc[4];
        enc[5] = p56 ? eb : enc[5];
        enc[6] = p56 ? enc[6] : ea;
        enc[7] = p56 ? enc[7] : eb;
    }
}

template <int MODE, bool NT>
__device__ __forceinline__ void store_conserving(const StepArgs& a, typename Traits<MODE>::S* dst, int k,
                                                 const Node<typename Traits<MODE>::R>& n,
                                                 const typename Traits<MODE>::R* hs,
                                                 const typename Traits<MODE>::R* gs)
{
    using T = Traits<MODE>;
    using R = typename T::R;
    if (MODE == 0) {
        store_all<MODE, NT>(a, dst, k, hs, gs);
        return;
    }
    typename T::S e[NPOP];
    conserve_encode<MODE, 8>(n.h + 1, hs + 1, e, cst<R>(a.sf, a.sf32), cst<R>(a.inv_sf, a.inv_sf32));
    conserve_encode<MODE, 5>(n.g, gs, e + 8, cst<R>(a.st, a.st32), cst<R>(a.inv_st, a.inv_st32));
    put_all<MODE, NT>(a, dst, k, e);
}

// ------------------------------------------------------------------------------ reduction
__device__ __forceinline__ bool red_is_max(int j) { return j == R_WSS_C_MAX || j == R_WSS_I_MAX || j == R_UMAX; }

// Block-level part of the check-step reduction: wavefront shuffles, then one partial
// per block.  The fixed-order sum over blocks is a separate one-block kernel, so no
// fence or atomic is needed and the result is deterministic.
__device__ void block_reduce_store(double* r, double* out)
{
    __shared__ double sm[16][NRED];
#pragma unroll
    for (int j = 0; j < NRED; j++) {
        double v = r[j];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const double o = __shfl_xor(v, off, 64);
            v = red_is_max(j) ? fmax(v, o) : v + o;
        }
        r[j] = v;
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < NRED; j++) sm[w][j] = r[j];
    }
    __syncthreads();
    if (threadIdx.x < NRED) {
        const int j = threadIdx.x;
        double acc = sm[0][j];
        for (int q = 1; q < nw; q++) acc = red_is_max(j) ? fmax(acc, sm[q][j]) : acc + sm[q][j];
        out[j] = acc;
    }
}

// Sum n tile partials in a fixed order (thread t takes t, t+256, ...; then shuffles and
// the 4 waves in order) and append the result to an observables ring.  Called by one
// block of 256 threads.  Single-lattice and batched runs use this same function, so an
// instance gives bitwise the same observables alone or in a batch.
__device__ void finish_sum(const StepArgs& a, const double* partials, int n, double* latest)
{
    double* obs = a.obs;
    unsigned int* obs_count = a.obs_count;
    __shared__ double sm[4][NRED];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double acc[NRED];
#pragma unroll
    for (int j = 0; j < NRED; j++) acc[j] = 0.0;
    // four partials per pass, loaded before any is added (same order of additions)
    int b = threadIdx.x;
    for (; b + 3 * 256 < n; b += 4 * 256) {
        double v[4][NRED];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const double* pb = partials + (long long)(b + u * 256) * NRED;
#pragma unroll
            for (int j = 0; j < NRED; j++) v[u][j] = pb[j];
        }
#pragma unroll
        for (int u = 0; u < 4; u++) {
#pragma unroll
            for (int j = 0; j < NRED; j++) acc[j] = red_is_max(j) ? fmax(acc[j], v[u][j]) : acc[j] + v[u][j];
        }
    }
    for (; b < n; b += 256) {
        const double* pb = partials + (long long)b * NRED;
#pragma unroll
        for (int j = 0; j < NRED; j++) acc[j] = red_is_max(j) ? fmax(acc[j], pb[j]) : acc[j] + pb[j];
    }
#pragma unroll
    for (int j = 0; j < NRED; j++) {
        double v = acc[j];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const double o = __shfl_xor(v, off, 64);
            v = red_is_max(j) ? fmax(v, o) : v + o;
        }
        acc[j] = v;
    }
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < NRED; j++) sm[w][j] = acc[j];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned int c = *obs_count;
        double* o = obs + (long long)(c % OBS_RING) * NRED;
        for (int j = 0; j < NRED; j++) {
            double v = sm[0][j];
            for (int q = 1; q < 4; q++) v = red_is_max(j) ? fmax(v, sm[q][j]) : v + sm[q][j];
            o[j] = v;
            if (latest) latest[j] = v;
        }
        *obs_count = c + 1;
        if (a.lumped) {
            // Darcy seepage across the meshwork from this check step's IOP, in effect from
            // the next step on; the previous value stays readable for the read-out pull
            const double p_iop = a.p_ref + (a.n_fluid > 0 ? o[R_DP_FLUID] / a.n_fluid : 0.0);
            a.useep_state[1] = a.useep_state[0];
            a.useep_state[0] = a.k_mu * ((p_iop - a.p_sc) / a.h_tm);   // eq. 4 across h_TM
        }
    }
    __syncthreads();
}

__global__ __launch_bounds__(256) void finish_kernel(StepArgs a)
{
    finish_sum(a, a.partials, a.n_tiles, nullptr);
}

// Wall-shear stress |t - (t.n) n| with t = sigma n, sigma = -(1 - omega/2) Pi^neq.
template <typename R>
__device__ __forceinline__ double wall_stress(const StepArgs& a, const Node<R>& n, const Moments<R>& m,
                                              double nxw, double nyw)
{
    double pxx = 0, pxy = 0, pyy = 0;
    const double ux = m.ux, uy = m.uy, uu = m.uu, dp = m.dp;
#pragma unroll
    for (int i = 1; i <= 8; i++) {
        const double ex = EX[i], ey = EY[i];
        const double eu = ex * ux + ey * uy;
        const double w = i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0;
        const double l = i <= 4 ? 1.0 / 3.0 : 1.0 / 12.0;
        const double neq = (double)n.h[i] - (l * dp + w * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu));
        pxx += ex * ex * neq;
        pxy += ex * ey * neq;
        pyy += ey * ey * neq;
    }
    const double f = -(1.0 - 0.5 * a.omega_f);
    const double tx = f * (pxx * nxw + pxy * nyw), ty = f * (pxy * nxw + pyy * nyw);
    const double tn = tx * nxw + ty * nyw;
    const double sx = tx - tn * nxw, sy = ty - tn * nyw;
    return sqrt(sx * sx + sy * sy);
}

// ------------------------------------------------------------------------------ step
__device__ __forceinline__ int tile_of_block(const StepArgs& a)
{
    const int G = gridDim.x, b = blockIdx.x;
    if (!a.xcd_remap || G < 8) return b;
    // consecutive tiles to the same XCD (blocks are dealt round-robin over 8 XCDs), so
    // neighbouring tiles share that XCD's L2
    const int xcd = b & 7, seq = b >> 3, q = G >> 3, r = G & 7;
    return xcd * q + min(xcd, r) + seq;
}

// The instance table and the work list do not change during a launch: read them through
// the constant address space so they land in scalar registers (the host compilation pass
// only needs a declaration-compatible body).
__device__ __forceinline__ StepArgs load_desc(const InstDesc* table, int i)
{
#if defined(__HIP_DEVICE_COMPILE__)
    typedef const __attribute__((address_space(4))) InstDesc ConstDesc;
    return ((ConstDesc*)table)[i].a;
#else
    return table[i].a;
#endif
}

__device__ __forceinline__ StepArgs load_desc2(const InstDesc* table, int i)
{
#if defined(__HIP_DEVICE_COMPILE__)
    typedef const __attribute__((address_space(4))) InstDesc ConstDesc;
    return ((ConstDesc*)table)[i].a2;
#else
    return table[i].a2;
#endif
}

__device__ __forceinline__ int2 load_item(const int2* work, int w)
{
#if defined(__HIP_DEVICE_COMPILE__)
    typedef const __attribute__((address_space(4))) int2 ConstItem;
    return ((ConstItem*)work)[w];
#else
    return work[w];
#endif
}

// Work item of this block in a batched launch (one block per item): the XCD-aware order of
// tile_of_block, so neighbouring tiles of an instance share an L2.
__device__ __forceinline__ int batch_item()
{
    const int G = gridDim.x, b = blockIdx.x;
    if (G < 8) return b;
    const int xcd = b & 7, seq = b >> 3, q = G >> 3, r = G & 7;
    return xcd * q + min(xcd, r) + seq;
}

// The step arguments of the instance in `slot` (its descriptor in the instance table), with
// the buffers swapped on odd launches.
template <bool FUSED>
__device__ __forceinline__ StepArgs batch_desc(const BatchArgs& b, int slot)
{
    StepArgs a = FUSED ? load_desc2(b.inst, slot) : load_desc(b.inst, slot);
    if (b.parity) {
        void* t = (void*)a.src;
        a.src = a.dst;
        a.dst = t;
    }
    return a;
}

// One tile of one time step: pull, moments, forces, both collisions, store; on check
// steps also this tile's partial sums (written to `partial`).
template <int MODE, bool REDUCE, bool NT, bool BC>
__device__ __forceinline__ void process_tile(const StepArgs& a, int tile, double* partial)
{
    using T = Traits<MODE>;
    using R = typename T::R;
    const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
    // tile_x is 64, 128 or 256: a mask and a shift, not a division per thread
    const int lx = threadIdx.x & (a.tile_x - 1), ly = threadIdx.x >> __builtin_ctz((unsigned)a.tile_x);
    const int x = tx * a.tile_x + lx, y = ty * a.tile_y + ly;
    const bool inb = x < a.nx && y < a.ny;
    const int k = y * a.pitch + x;
    const uint8_t t = inb ? *at(a.type, 0, (unsigned)k) : (uint8_t)0;
    const bool act = is_active(t);
    if (!REDUCE && !act) return;

    const typename T::S* src = (const typename T::S*)a.src;
    typename T::S* dst = (typename T::S*)a.dst;
    double r[NRED];
    if (REDUCE) {
#pragma unroll
        for (int j = 0; j < NRED; j++) r[j] = 0.0;
    }
    if (act) {
        Node<R> n;
        pull_all<MODE, BC>(a, src, k, t, n);
        const Moments<R> m = moments(n);
        R hs[9], gs[5];
        collide<MODE>(a, (t & CLS_MASK) == POROUS, n, m, hs, gs);
        store_conserving<MODE, NT>(a, dst, k, n, hs, gs);
        if (REDUCE) {
            Node<double> nw;
            const Moments<double> mw = wide_moments<MODE>(a, n, nw);
            const double ux = mw.ux, uy = mw.uy, th = mw.th, dp = mw.dp;
            const double Tabs = a.T_ref + th;
            if ((t & CLS_MASK) == FLUID) r[R_DP_FLUID] = dp;
            r[R_QOUT] = nw.qout;
            r[R_QIN] = nw.qin;
            if (t & F_WSS) {
                const int wi = a.widx[k];
                if (wi >= 0) {
                    const double tw = wall_stress(a, nw, mw, a.wall_n[2 * wi], a.wall_n[2 * wi + 1]);
                    if (a.wall_id[wi] == WALL_CORNEA) { r[R_WSS_C_SUM] = tw; r[R_WSS_C_MAX] = tw; }
                    else { r[R_WSS_I_SUM] = tw; r[R_WSS_I_MAX] = tw; }
                }
            }
            double* up = a.uprev;
            const double pux = up[k], puy = up[a.qs + k], pT = up[2 * a.qs + k];
            r[R_DU2] = (ux - pux) * (ux - pux) + (uy - puy) * (uy - puy);
            r[R_U2] = ux * ux + uy * uy;
            r[R_DT2] = (Tabs - pT) * (Tabs - pT);
            r[R_T2] = th * th;
            up[k] = ux;
            up[a.qs + k] = uy;
            up[2 * a.qs + k] = Tabs;
            r[R_MASS_F] = mw.sum;
            r[R_MASS_T] = th;
            r[R_UMAX] = sqrt(ux * ux + uy * uy);
            r[R_NONFINITE] = (isfinite(dp) && isfinite(ux) && isfinite(uy) && isfinite(th)) ? 0.0 : 1.0;
        }
    }
    if (REDUCE) block_reduce_store(r, partial);
}

// One time step of one lattice: one block per active tile.  The partial of a tile is
// stored at its index in the tile list.
template <int MODE, bool REDUCE, bool NT, bool BC>
__global__ __launch_bounds__(256) void step_kernel(StepArgs a)
{
    const int ti = tile_of_block(a);
    process_tile<MODE, REDUCE, NT, BC>(a, a.tiles[ti], a.partials + (long long)ti * NRED);
}

// One time step of every running instance of a batch in kernel class b.kind: one block per
// (slot, tile) item of the work list (the grid is the list's length); the block reads its
// instance's arguments from the device instance table.
template <int MODE, bool REDUCE, bool NT, bool BC>
__global__ __launch_bounds__(256) void batch_step_kernel(BatchArgs b)
{
    const int w = batch_item();
    if (w >= *b.n_work) return;
    const int2 it = load_item(b.work, w);
    process_tile<MODE, REDUCE, NT, BC>(batch_desc<false>(b, it.x), it.y, b.partials + (long long)w * NRED);
}

// Per-instance fixed-order sums of the batch's check step (one block per instance).
__global__ __launch_bounds__(256) void batch_finish_kernel(BatchArgs b)
{
    for (int sl = blockIdx.x; sl < b.max_slots; sl += gridDim.x) {
        const InstDesc* d = b.inst + sl;
        if (!d->running || d->mode != b.kind) continue;
        finish_sum(d->a, b.partials + (long long)d->work_start * NRED, d->work_count, b.latest + (long long)sl * NRED);
    }
}

// ------------------------------------------------------------------------------ two steps per launch
// Temporal blocking: one launch advances a 64 x TY tile by two time steps.  Step A
// computes step n+1 on the tile plus a one-node halo (pulling from global memory), keeps
// it in LDS, and step B computes step n+2 on the tile from LDS and stores it.  In F64, F32
// and F32X the intermediate values are rounded to the storage format exactly as a store
// and reload through HBM would round them (including the mass-conserving encode), so two
// fused steps are bitwise identical to two single-step launches while the intermediate
// state never travels to HBM.  In F16S the intermediate stays in single precision, the
// compute type: binary16 is a storage format, and the state is rounded (mass-conserving)
// where it is stored.  That skips the encode, the smallest-magnitude search and the decode
// for every step-A node, a quarter of the kernel's VALU instructions, and the steady-state
// IOP error against FP64 stays within 0.1% (smaller than with rounding every step on three
// of four cases).
// TYv: output rows per tile.  64 x 8 everywhere; F32 and F16S also come in 64 x 4 (more
// blocks for mid-size lattices, which 64 x 8 tiles leave partly idle).
template <int MODE, int TYv = 8> struct Fuse {
    static constexpr int TY = TYv;
    // threads per block: the FP64-compute forms take two step-A nodes per thread
    static constexpr int THREADS = (MODE == 0 || MODE == 3) ? 512 : 256;
    static constexpr int EW = 66, EH = TY + 2;        // tile plus a one-node halo
    static constexpr int EN = EW * EH;                // step-A nodes
    // Step A takes a thread's tile nodes first, each the node step B gives the same thread
    // (NT passes), then the halo ring (NH nodes); so g_0, which only its own node reads, stays
    // in the thread's registers between the steps and is not in the LDS image.
    static constexpr int NT = TY * 64 / THREADS;
    static constexpr int NH = 2 * EW + 2 * TY;
    static constexpr int NA = NT + (NH + THREADS - 1) / THREADS;   // step-A nodes per thread
    // LDS image: h_1..h_8 and g_1..g_4 over tile + halo (planes 0..11): 63 KB in FP64, two
    // blocks (16 waves) per CU; 31 KB in the single-precision image, five blocks (20 waves).
    static constexpr int PLANES = 12;
    static constexpr int WORDS = PLANES * EN;
    // resident blocks per CU the register budget is sized for (the LDS image allows it)
    static constexpr int BLOCKS = (MODE == 0 || MODE == 3) ? 2 : TY == 4 ? 6 : 5;
    static_assert((TY * 64) % THREADS == 0, "step B covers the tile in whole passes");
    static_assert(NT * THREADS + NH == EN, "the tile and its ring are the step-A nodes");
};

// Step-A node j of the calling thread in E coordinates (the tile is 1..64 x 1..TY);
// false past the halo ring.
template <int MODE, int TY>
__device__ __forceinline__ bool step_a_node(int j, int& ex, int& ey)
{
    using F = Fuse<MODE, TY>;
    const int t = threadIdx.x;
    if (j < F::NT) {
        ex = (t & 63) + 1;
        ey = (t >> 6) + (F::THREADS / 64) * j + 1;
        return true;
    }
    const int h = t + F::THREADS * (j - F::NT);
    if (h >= F::NH) return false;
    if (h < F::EW) {
        ex = h;
        ey = 0;
    } else if (h < 2 * F::EW) {
        ex = h - F::EW;
        ey = F::EH - 1;
    } else if (h < 2 * F::EW + F::TY) {
        ex = 0;
        ey = h - 2 * F::EW + 1;
    } else {
        ex = F::EW - 1;
        ey = h - 2 * F::EW - F::TY + 1;
    }
    return true;
}

template <int MODE, int TY>
__device__ __forceinline__ int lds_at(int q, int ly, int lx)
{
    return (q * Fuse<MODE, TY>::EH + ly) * Fuse<MODE, TY>::EW + lx;
}

// Pull from the LDS image of step n+1 (E coordinates: the tile node is (ex, ey)); g0 is
// the node's own g_0 of step n+1, kept by the thread.
template <int MODE, bool BC, int TY>
__device__ __forceinline__ void pull_lds(const StepArgs& a, const typename Traits<MODE>::L* lds, int k, int ex,
                                         int ey, uint8_t t, typename Traits<MODE>::L g0,
                                         Node<typename Traits<MODE>::R>& n)
{
    using R = typename Traits<MODE>::R;
    n.qin = R(0);
    n.qout = R(0);
    n.g[0] = R(g0);
    if (!(t & F_BOUNDARY)) {
        // every neighbour active: each link pulls from upstream at a fixed offset
#pragma unroll
        for (int i = 1; i <= 8; i++) n.h[i] = lds[lds_at<MODE, TY>(i - 1, ey - EY[i], ex - EX[i])];
#pragma unroll
        for (int i = 1; i <= 4; i++) n.g[i] = lds[lds_at<MODE, TY>(7 + i, ey - EY[i], ex - EX[i])];
        return;
    }
    uint8_t nt[9];
    pull_types(a, k, true, nt);
    bool up[9];
#pragma unroll
    for (int i = 1; i <= 8; i++) up[i] = is_active(nt[i]);
#pragma unroll
    for (int i = 1; i <= 8; i++)
        n.h[i] = up[i] ? lds[lds_at<MODE, TY>(i - 1, ey - EY[i], ex - EX[i])] : lds[lds_at<MODE, TY>(OPP[i] - 1, ey, ex)];
#pragma unroll
    for (int i = 1; i <= 4; i++)
        n.g[i] = up[i] ? lds[lds_at<MODE, TY>(7 + i, ey - EY[i], ex - EX[i])] : lds[lds_at<MODE, TY>(7 + OPP[i], ey, ex)];
    const int w = (BC && (t & F_WSS)) ? a.widx[k] : -1;
    const bool extra = BC && needs_extrapolation(a, nt);
#pragma unroll
    for (int i = 1; i <= 8; i++) {
        if (up[i]) continue;
        const uint8_t c = nt[i] & CLS_MASK;
        const R v = n.h[i];
        if (extra && (c == INLET || c == OUTLET)) {
            // extrapolated below
        } else if (c == INLET) {
            const R corr = R(6.0) * wflow<R>(i) * (R(EX[i]) * cst<R>(a.uin_x, a.uin_x32) + R(EY[i]) * cst<R>(a.uin_y, a.uin_y32)) *
                             fscale<MODE, R>(a);
            n.h[i] = v + corr;
        } else if (c == OUTLET) {
            if (a.lumped) {
                const int d = ((nt[i] >> WALL_SHIFT) & 3) + 1;
                n.h[i] = v + R(6.0) * wflow<R>(i) * (R(EX[i] * EX[d] + EY[i] * EY[d]) * R(*a.useep)) * fscale<MODE, R>(a);
            } else {
                n.h[i] = -v + R(2.0) * lam<R>(i) * cst<R>(a.dp_out, a.dp_out32) * fscale<MODE, R>(a);
            }
        } else if (BC && w >= 0) {                        // interpolated bounce-back
            const double q = wall_fraction(a, w, i);
            if (q >= 0.5)
                n.h[i] = bouzidi(R(q), v, R(lds[lds_at<MODE, TY>(i - 1, ey, ex)]), R(0));
            else if (q > 0.0 && up[OPP[i]])
                n.h[i] = bouzidi(R(q), v, R(0), R(lds[lds_at<MODE, TY>(OPP[i] - 1, ey + EY[i], ex + EX[i])]));
        }
    }
#pragma unroll
    for (int i = 1; i <= 4; i++) {
        if (extra || up[i]) continue;
        const uint8_t c = nt[i] & CLS_MASK;
        const uint8_t wall = (nt[i] >> WALL_SHIFT) & 3;
        if (c == INLET || (c == SOLID && wall != WALL_BOX)) {
            const R tw = c == INLET ? cst<R>(a.tw_inlet, a.tw_inlet32)
                                    : (wall == WALL_CORNEA ? cst<R>(a.tw_cornea, a.tw_cornea32)
                                                           : cst<R>(a.tw_iris, a.tw_iris32));
            n.g[i] = -n.g[i] + R(2.0) * cst<R>(a.wT, a.wT32) * tw * tscale<MODE, R>(a);
        }
    }
    if constexpr (BC) {
        if (!extra) return;
        Node<R> own;
#pragma unroll
        for (int i = 1; i <= 8; i++) own.h[i] = R(lds[lds_at<MODE, TY>(i - 1, ey, ex)]);
        own.g[0] = R(g0);
#pragma unroll
        for (int i = 1; i <= 4; i++) own.g[i] = R(lds[lds_at<MODE, TY>(7 + i, ey, ex)]);
        extrapolate_physical<MODE>(a, nt, own, n);
    }
}

// Encode the post-collision values exactly as the single-step store would (the same
// mass-conserving rounding), and return them decoded, as the next step would load them.
template <int MODE>
__device__ __forceinline__ void encode_decoded(const StepArgs& a, const Node<typename Traits<MODE>::R>& n,
                                               const typename Traits<MODE>::R* hs, const typename Traits<MODE>::R* gs,
                                               typename Traits<MODE>::S* e)
{
    using T = Traits<MODE>;
    using R = typename T::R;
    if (MODE == 0) {
#pragma unroll
        for (int i = 1; i <= 8; i++) e[i - 1] = T::enc((typename T::Acc)hs[i], cst<R>(a.sf, a.sf32));
#pragma unroll
        for (int i = 0; i <= 4; i++) e[8 + i] = T::enc((typename T::Acc)gs[i], cst<R>(a.st, a.st32));
    } else {
        conserve_encode<MODE, 8>(n.h + 1, hs + 1, e, cst<R>(a.sf, a.sf32), cst<R>(a.inv_sf, a.inv_sf32));
        conserve_encode<MODE, 5>(n.g, gs, e + 8, cst<R>(a.st, a.st32), cst<R>(a.inv_st, a.inv_st32));
    }
}

// Step A of one node (E coordinates ex, ey): collide, round as a store would (F16S: keep the
// single-precision values), and keep the values in LDS; returns g_0, which only the node
// itself reads.
template <int MODE, int TY>
__device__ __forceinline__ typename Traits<MODE>::L step_a_store(const StepArgs& a,
                                                                 const Node<typename Traits<MODE>::R>& n, bool porous,
                                                                 int ex, int ey, typename Traits<MODE>::L* lds)
{
    using T = Traits<MODE>;
    using R = typename T::R;
    const Moments<R> m = moments(n);
    R hs[9], gs[5];
    collide<MODE>(a, porous, n, m, hs, gs);
    if constexpr (MODE == 2) {
        // F16S: the intermediate step stays in single precision
#pragma unroll
        for (int q = 0; q < 8; q++) lds[lds_at<MODE, TY>(q, ey, ex)] = hs[q + 1];
#pragma unroll
        for (int i = 1; i <= 4; i++) lds[lds_at<MODE, TY>(7 + i, ey, ex)] = gs[i];
        return gs[0];
    }
    typename T::S enc[NPOP];
    encode_decoded<MODE>(a, n, hs, gs, enc);
    using L = typename T::L;   // exact: the decoded values of the storage
#pragma unroll
    for (int q = 0; q < 8; q++) lds[lds_at<MODE, TY>(q, ey, ex)] = (L)T::ldv(enc[q], cst<R>(a.inv_sf, a.inv_sf32));
#pragma unroll
    for (int i = 1; i <= 4; i++) lds[lds_at<MODE, TY>(7 + i, ey, ex)] = (L)T::ldv(enc[8 + i], cst<R>(a.inv_st, a.inv_st32));
    return (L)T::ldv(enc[8], cst<R>(a.inv_st, a.inv_st32));
}

// PF: step A issues the loads of all of a thread's nodes before computing any (more bytes
// in flight, more registers).
template <int MODE, bool NT, bool PF, bool BC, int TY>
__device__ __forceinline__ void process_tile2(const StepArgs& a, int tile, typename Traits<MODE>::L* lds)
{
    using T = Traits<MODE>;
    using R = typename T::R;
    using F = Fuse<MODE, TY>;
    const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
    const int x0 = tx * 64, y0 = ty * F::TY;
    const typename T::S* src = (const typename T::S*)a.src;
    typename T::S* dst = (typename T::S*)a.dst;
    // step A: step n+1 on the tile and its halo, into LDS (g_0 of the tile nodes kept)
    using L = typename T::L;
    L g0A[F::NT];
#pragma unroll
    for (int j = 0; j < F::NT; j++) g0A[j] = L(0);
    if constexpr (PF) {
        // each thread owns NA nodes and issues the loads of all of them before computing
        int kA[F::NA], exA[F::NA], eyA[F::NA];
        uint8_t tA[F::NA];
#pragma unroll
        for (int j = 0; j < F::NA; j++) {
            int ex = 0, ey = 0;
            const bool node = step_a_node<MODE, TY>(j, ex, ey);
            exA[j] = ex;
            eyA[j] = ey;
            const int x = x0 - 1 + ex, y = y0 - 1 + ey;
            const bool in = node && x >= 0 && y >= 0 && x < a.nx && y < a.ny;
            kA[j] = in ? y * a.pitch + x : 0;
            // unconditional (node 0 when outside), so the node offset stays a plain 32-bit
            // value and every load takes the scalar-base-plus-offset form
            const uint8_t tk = *at(a.type, 0, (unsigned)kA[j]);
            tA[j] = in ? tk : (uint8_t)0;   // 0 = SOLID: not active
        }
        Node<R> nA[F::NA];
        uint8_t ntA[F::NA][9];
#pragma unroll
        for (int j = 0; j < F::NA; j++) pull_types(a, kA[j], is_active(tA[j]) && (tA[j] & F_BOUNDARY), ntA[j]);
#pragma unroll
        for (int j = 0; j < F::NA; j++)
            if (is_active(tA[j])) pull_loads<MODE>(a, src, kA[j], (tA[j] & F_BOUNDARY) != 0, ntA[j], nA[j]);
#pragma unroll
        for (int j = 0; j < F::NA; j++) pull_rules<MODE, BC>(a, src, kA[j], tA[j], ntA[j], nA[j]);
#pragma unroll
        for (int j = 0; j < F::NA; j++) {
            if (!is_active(tA[j])) continue;
            const L g0 = step_a_store<MODE, TY>(a, nA[j], (tA[j] & CLS_MASK) == POROUS, exA[j], eyA[j], lds);
            if (j < F::NT) g0A[j] = g0;
        }
    } else {
        // one node at a time (fewer registers)
#pragma unroll
        for (int j = 0; j < F::NA; j++) {
            int ex = 0, ey = 0;
            if (!step_a_node<MODE, TY>(j, ex, ey)) continue;
            const int x = x0 - 1 + ex, y = y0 - 1 + ey;
            if (x < 0 || y < 0 || x >= a.nx || y >= a.ny) continue;
            const int k = y * a.pitch + x;
            const uint8_t t = *at(a.type, 0, (unsigned)k);
            if (!is_active(t)) continue;
            Node<R> n;
            pull_all<MODE, BC>(a, src, k, t, n);
            const L g0 = step_a_store<MODE, TY>(a, n, (t & CLS_MASK) == POROUS, ex, ey, lds);
            if (j < F::NT) g0A[j] = g0;
        }
    }
    __syncthreads();
    // step B: step n+2 on the tile, from LDS, to global memory
#pragma unroll
    for (int r = 0; r < F::TY * 64 / F::THREADS; r++) {
        const int lx = threadIdx.x & 63, ly = (threadIdx.x >> 6) + (F::THREADS / 64) * r;
        const int x = x0 + lx, y = y0 + ly;
        if (x >= a.nx || y >= a.ny) continue;
        const int k = y * a.pitch + x;
        const uint8_t t = *at(a.type, 0, (unsigned)k);
        if (!is_active(t)) continue;
        Node<R> n;
        pull_lds<MODE, BC, TY>(a, lds, k, lx + 1, ly + 1, t, g0A[r], n);
        const Moments<R> m = moments(n);
        R hs[9], gs[5];
        collide<MODE>(a, (t & CLS_MASK) == POROUS, n, m, hs, gs);
        store_conserving<MODE, NT>(a, dst, k, n, hs, gs);
    }
}

// Two time steps of one lattice; one block per active 64 x TY tile (tile list in
// a.tiles, laid out with a.tiles_x = ceil(nx / 64) tiles per row).
template <int MODE, bool NT, bool BC, int TY>
__global__ __launch_bounds__((Fuse<MODE, TY>::THREADS), (Fuse<MODE, TY>::BLOCKS)) void step2_kernel(StepArgs a)
{
    __shared__ typename Traits<MODE>::L lds[Fuse<MODE, TY>::WORDS];
    // all of a thread's loads first, except in the paper-scheme variants of the single-
    // precision storages, which would spill (as in batch_step2_kernel)
    process_tile2<MODE, NT, !(MODE != 0 && BC), BC, TY>(a, a.tiles[tile_of_block(a)], lds);
}

// a.tile_y selects the tile rows: 4 (F32 and F16S) or 8
template <int MODE, bool NT, bool BC>
static hipError_t launch_step2_t(const StepArgs& a, hipStream_t s)
{
    if (a.n_tiles == 0) return hipSuccess;
    if constexpr (MODE == 1 || MODE == 2) {
        if (a.tile_y == 4) {
            hipLaunchKernelGGL((step2_kernel<MODE, NT, BC, 4>), dim3(a.n_tiles), dim3(Fuse<MODE, 4>::THREADS), 0, s, a);
            return hipGetLastError();
        }
    }
    if (a.tile_y != 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL((step2_kernel<MODE, NT, BC, 8>), dim3(a.n_tiles), dim3(Fuse<MODE, 8>::THREADS), 0, s, a);
    return hipGetLastError();
}

template <int MODE, bool NT>
static hipError_t launch_step2_bc(const StepArgs& a, hipStream_t s)
{
    return a.bc_paper ? launch_step2_t<MODE, NT, true>(a, s) : launch_step2_t<MODE, NT, false>(a, s);
}

hipError_t launch_step2(int mode, const StepArgs& a, hipStream_t s)
{
    switch (mode * 2 + (a.nt_store ? 1 : 0)) {
    case 0: return launch_step2_bc<0, false>(a, s);
    case 1: return launch_step2_bc<0, true>(a, s);
    case 2: return launch_step2_bc<1, false>(a, s);
    case 3: return launch_step2_bc<1, true>(a, s);
    case 4: return launch_step2_bc<2, false>(a, s);
    case 5: return launch_step2_bc<2, true>(a, s);
    case 6: return launch_step2_bc<3, false>(a, s);
    case 7: return launch_step2_bc<3, true>(a, s);
    }
    return hipErrorInvalidValue;
}

int fused_tile_rows(int mode)
{
    return mode == 0 ? Fuse<0>::TY : mode == 1 ? Fuse<1>::TY : mode == 2 ? Fuse<2>::TY : Fuse<3>::TY;
}

bool fused_rows_supported(int mode, int rows)
{
    return rows == 8 || (rows == 4 && (mode == 1 || mode == 2));
}

// Two time steps of every running instance of a batch in kernel class b.kind (fused tile
// work list of 64 x TY tiles; the same item assignment and argument loads as
// batch_step_kernel).
template <int MODE, bool NT, bool BC, int TY>
__global__ __launch_bounds__((Fuse<MODE, TY>::THREADS), (Fuse<MODE, TY>::BLOCKS)) void batch_step2_kernel(BatchArgs b)
{
    __shared__ typename Traits<MODE>::L lds[Fuse<MODE, TY>::WORDS];
    const int w = batch_item();
    if (w >= *b.n_work2) return;
    const int2 it = load_item(b.work2, w);
    // step A issues all of a thread's loads first (512-instance sweep, FP32: 60.4 against 55.9
    // GLUPS one node at a time; F16S: 69.3 against 61.2), except in the paper-scheme variants
    // of the single-precision storages (F32, F16S, F32X), which would spill
    process_tile2<MODE, NT, !(MODE != 0 && BC), BC, TY>(batch_desc<true>(b, it.x), it.y, lds);
}

// b.tile_y selects the tile rows: 4 (F32 and F16S) or 8; every instance of the launch
// has its fused tile list in rows of that height
template <int MODE, bool NT, bool BC>
static hipError_t launch_batch2_k(const BatchArgs& b, int grid, hipStream_t s)
{
    if (grid <= 0) return hipSuccess;
    if constexpr (MODE == 1 || MODE == 2) {
        if (b.tile_y == 4) {
            hipLaunchKernelGGL((batch_step2_kernel<MODE, NT, BC, 4>), dim3(grid), dim3(Fuse<MODE, 4>::THREADS), 0, s, b);
            return hipGetLastError();
        }
    }
    if (b.tile_y != 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL((batch_step2_kernel<MODE, NT, BC, 8>), dim3(grid), dim3(Fuse<MODE, 8>::THREADS), 0, s, b);
    return hipGetLastError();
}

template <int MODE, bool NT>
static hipError_t launch_batch2_t(const BatchArgs& b, int grid, hipStream_t s)
{
    return b.bc ? launch_batch2_k<MODE, NT, true>(b, grid, s) : launch_batch2_k<MODE, NT, false>(b, grid, s);
}

hipError_t launch_batch_step2(int mode, const BatchArgs& b, int grid, hipStream_t s)
{
    switch (mode * 2 + (b.nt_store ? 1 : 0)) {
    case 0: return launch_batch2_t<0, false>(b, grid, s);
    case 1: return launch_batch2_t<0, true>(b, grid, s);
    case 2: return launch_batch2_t<1, false>(b, grid, s);
    case 3: return launch_batch2_t<1, true>(b, grid, s);
    case 4: return launch_batch2_t<2, false>(b, grid, s);
    case 5: return launch_batch2_t<2, true>(b, grid, s);
    case 6: return launch_batch2_t<3, false>(b, grid, s);
    case 7: return launch_batch2_t<3, true>(b, grid, s);
    }
    return hipErrorInvalidValue;
}

// ------------------------------------------------------------------------------ scatter / unpack
// The state after step N is kept as two buffers: `cur` holds the post-collision
// populations of step N, and `prev` (the buffer step N read) pulls back to the
// pre-collision populations F^N of step N.  To set the state to a given F (the initial
// equilibrium, or caller-given populations) this kernel writes into `dst` the unique
// pre-image X with pull(X) = F: every slot of X is read by exactly one link of the pull,
// so each F_i(x) is placed either at the upstream node's slot or, for a boundary link,
// at the node's own opposite slot with the link rule inverted.  A regular step kernel
// from X then produces cur = collide(F).
template <int MODE>
__global__ __launch_bounds__(256) void scatter_kernel(StepArgs a, const double* pops, double dp0, double th0)
{
    using T = Traits<MODE>;
    using R = typename T::R;
    const int x = blockIdx.x * 64 + (threadIdx.x & 63), y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= a.nx || y >= a.ny) return;
    const int k = y * a.pitch + x;
    const uint8_t t = a.type[k];
    if (!is_active(t)) return;
    typename T::S* X = (typename T::S*)a.dst;
    const long long n2 = (long long)a.nx * a.ny, d = (long long)y * a.nx + x;
    const R sf = R(a.sf), st = R(a.st);
    // flow, q = 1..8
    for (int i = 1; i <= 8; i++) {
        const R f = pops ? R(pops[(i - 1) * n2 + d]) : lam<R>(i) * R(dp0);   // eq. 7 at u = 0
        const int ks = k - EY[i] * a.pitch - EX[i];
        const uint8_t c = a.type[ks] & CLS_MASK;
        if (c == FLUID || c == POROUS) {
            T::st(X + (long long)(i - 1) * a.qs + ks, f, sf);
        } else if (a.bc_paper && (c == INLET || c == OUTLET)) {
            // the extrapolation reads this slot as the node's own post-collision value
            const R own = pops ? R(pops[(OPP[i] - 1) * n2 + d]) : lam<R>(OPP[i]) * R(dp0);
            T::st(X + (long long)(OPP[i] - 1) * a.qs + k, own, sf);
        } else {
            R v;
            if (c == SOLID) v = f;
            else if (c == INLET) v = f - R(6.0) * wflow<R>(i) * (R(EX[i]) * R(a.uin_x) + R(EY[i]) * R(a.uin_y));
            else if (a.lumped) {
                const int dd = ((a.type[ks] >> WALL_SHIFT) & 3) + 1;
                v = f - R(6.0) * wflow<R>(i) * (R(EX[i] * EX[dd] + EY[i] * EY[dd]) * R(*a.useep));
            } else v = R(2.0) * lam<R>(i) * R(a.dp_out) - f;
            T::st(X + (long long)(OPP[i] - 1) * a.qs + k, v, sf);
        }
    }
    // thermal, q = 0..4
    const R g0 = pops ? R(pops[8 * n2 + d]) : R(a.w0T) * R(th0);              // eq. 12 at u = 0
    T::st(X + 8LL * a.qs + k, g0, st);
    for (int i = 1; i <= 4; i++) {
        const R f = pops ? R(pops[(8 + i) * n2 + d]) : R(a.wT) * R(th0);
        const int ks = k - EY[i] * a.pitch - EX[i];
        const uint8_t tn = a.type[ks];
        const uint8_t c = tn & CLS_MASK;
        if (c == FLUID || c == POROUS) {
            T::st(X + (8LL + i) * a.qs + ks, f, st);
        } else {
            const uint8_t wall = (tn >> WALL_SHIFT) & 3;
            R v;
            if (a.bc_paper && (c == INLET || (c == SOLID && wall != WALL_BOX))) {
                v = pops ? R(pops[(8 + OPP[i]) * n2 + d]) : R(a.wT) * R(th0);   // own value (extrapolation)
            } else if (c == INLET || (c == SOLID && wall != WALL_BOX)) {
                const double tw = c == INLET ? a.tw_inlet : (wall == WALL_CORNEA ? a.tw_cornea : a.tw_iris);
                v = R(2.0) * R(a.wT) * R(tw) - f;
            } else {
                v = f;
            }
            T::st(X + (8LL + OPP[i]) * a.qs + k, v, st);
        }
    }
}

// Fields of the current state: pull `src` (the `prev` buffer) to the pre-collision
// populations of the current step and take their moments; NaN at non-active nodes.
// Output is dense [ny][nx].  field 6 instead resets the residual reference (u, T).
template <int MODE>
__global__ __launch_bounds__(256) void unpack_kernel(StepArgs a, int field, int q, double p_ref, double* out)
{
    using T = Traits<MODE>;
    using R = typename T::R;
    const int x = blockIdx.x * 64 + (threadIdx.x & 63), y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= a.nx || y >= a.ny) return;
    const int k = y * a.pitch + x;
    const long long d = (long long)y * a.nx + x;
    const uint8_t t = a.type[k];
    if (!is_active(t)) {
        if (field == 7 || field == 8) {
            const long long n2 = (long long)a.nx * a.ny;
            for (int i = 0; i < (field == 7 ? NPOP : 2); i++) out[i * n2 + d] = __builtin_nan("");
        } else if (field != 6) {
            out[d] = __builtin_nan("");
        }
        return;
    }
    Node<R> n;
    if (a.bc_paper) pull_all<MODE, true>(a, (const typename T::S*)a.src, k, t, n);
    else pull_all<MODE, false>(a, (const typename T::S*)a.src, k, t, n);
    Node<double> nw;
    const Moments<double> m = wide_moments<MODE>(a, n, nw);
    if (field == 7) {                        // all 13 populations, dense [13][ny][nx]
        const long long n2 = (long long)a.nx * a.ny;
        for (int i = 1; i <= 8; i++) out[(i - 1) * n2 + d] = nw.h[i];
        for (int i = 0; i <= 4; i++) out[(8 + i) * n2 + d] = nw.g[i];
        return;
    }
    if (field == 8) {                        // u_x then u_y, dense [2][ny][nx]
        const long long n2 = (long long)a.nx * a.ny;
        out[d] = m.ux;
        out[n2 + d] = m.uy;
        return;
    }
    if (field == 6) {
        a.uprev[k] = m.ux;
        a.uprev[a.qs + k] = m.uy;
        a.uprev[2 * a.qs + k] = a.T_ref + (double)m.th;
        return;
    }
    double v;
    switch (field) {
    case 0: v = p_ref + (double)m.dp; break;
    case 1: v = m.ux; break;
    case 2: v = m.uy; break;
    case 3: v = a.T_ref + (double)m.th; break;
    case 4: v = nw.h[q < 1 ? 1 : (q > 8 ? 8 : q)]; break;
    default: v = nw.g[q < 0 ? 0 : (q > 4 ? 4 : q)]; break;
    }
    out[d] = v;
}

// ------------------------------------------------------------------------------ launchers
template <int MODE, bool NT>
static hipError_t launch_step_t(bool reduce, const StepArgs& a, hipStream_t s)
{
    const dim3 grid(a.n_tiles), block(a.tile_x * a.tile_y);
    if (a.n_tiles == 0) return hipSuccess;
    if (reduce) {
        if (a.bc_paper) hipLaunchKernelGGL((step_kernel<MODE, true, NT, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((step_kernel<MODE, true, NT, false>), grid, block, 0, s, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(256), 0, s, a);
    } else {
        if (a.bc_paper) hipLaunchKernelGGL((step_kernel<MODE, false, NT, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((step_kernel<MODE, false, NT, false>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_step(int mode, bool reduce, const StepArgs& a, hipStream_t s)
{
    switch (mode * 2 + (a.nt_store ? 1 : 0)) {
    case 0: return launch_step_t<0, false>(reduce, a, s);
    case 1: return launch_step_t<0, true>(reduce, a, s);
    case 2: return launch_step_t<1, false>(reduce, a, s);
    case 3: return launch_step_t<1, true>(reduce, a, s);
    case 4: return launch_step_t<2, false>(reduce, a, s);
    case 5: return launch_step_t<2, true>(reduce, a, s);
    case 6: return launch_step_t<3, false>(reduce, a, s);
    case 7: return launch_step_t<3, true>(reduce, a, s);
    }
    return hipErrorInvalidValue;
}

template <int MODE, bool REDUCE, bool NT, bool BC>
static hipError_t launch_batch_k(const BatchArgs& b, int grid, hipStream_t s)
{
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL((batch_step_kernel<MODE, REDUCE, NT, BC>), dim3(grid), dim3(256), 0, s, b);
    return hipGetLastError();
}

template <int MODE, bool NT>
static hipError_t launch_batch_t(bool reduce, const BatchArgs& b, int grid, hipStream_t s)
{
    if (reduce) return b.bc ? launch_batch_k<MODE, true, NT, true>(b, grid, s) : launch_batch_k<MODE, true, NT, false>(b, grid, s);
    return b.bc ? launch_batch_k<MODE, false, NT, true>(b, grid, s) : launch_batch_k<MODE, false, NT, false>(b, grid, s);
}

hipError_t launch_batch_step(int mode, bool reduce, const BatchArgs& b, int grid, hipStream_t s)
{
    switch (mode * 2 + (b.nt_store ? 1 : 0)) {
    case 0: return launch_batch_t<0, false>(reduce, b, grid, s);
    case 1: return launch_batch_t<0, true>(reduce, b, grid, s);
    case 2: return launch_batch_t<1, false>(reduce, b, grid, s);
    case 3: return launch_batch_t<1, true>(reduce, b, grid, s);
    case 4: return launch_batch_t<2, false>(reduce, b, grid, s);
    case 5: return launch_batch_t<2, true>(reduce, b, grid, s);
    case 6: return launch_batch_t<3, false>(reduce, b, grid, s);
    case 7: return launch_batch_t<3, true>(reduce, b, grid, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_batch_finish(const BatchArgs& b, hipStream_t s)
{
    hipLaunchKernelGGL(batch_finish_kernel, dim3(256), dim3(256), 0, s, b);
    return hipGetLastError();
}

static dim3 lattice_grid(const StepArgs& a) { return dim3((a.nx + 63) / 64, (a.ny + 3) / 4); }

hipError_t launch_scatter(int mode, const StepArgs& a, const double* pops, double dp0, double th0,
                          hipStream_t s)
{
    switch (mode) {
    case 0: hipLaunchKernelGGL(scatter_kernel<0>, lattice_grid(a), dim3(256), 0, s, a, pops, dp0, th0); break;
    case 1: hipLaunchKernelGGL(scatter_kernel<1>, lattice_grid(a), dim3(256), 0, s, a, pops, dp0, th0); break;
    case 2: hipLaunchKernelGGL(scatter_kernel<2>, lattice_grid(a), dim3(256), 0, s, a, pops, dp0, th0); break;
    case 3: hipLaunchKernelGGL(scatter_kernel<3>, lattice_grid(a), dim3(256), 0, s, a, pops, dp0, th0); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_unpack(int mode, const StepArgs& a, int field, int q, double p_ref, double* out,
                         hipStream_t s)
{
    switch (mode) {
    case 0: hipLaunchKernelGGL(unpack_kernel<0>, lattice_grid(a), dim3(256), 0, s, a, field, q, p_ref, out); break;
    case 1: hipLaunchKernelGGL(unpack_kernel<1>, lattice_grid(a), dim3(256), 0, s, a, field, q, p_ref, out); break;
    case 2: hipLaunchKernelGGL(unpack_kernel<2>, lattice_grid(a), dim3(256), 0, s, a, field, q, p_ref, out); break;
    case 3: hipLaunchKernelGGL(unpack_kernel<3>, lattice_grid(a), dim3(256), 0, s, a, field, q, p_ref, out); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------------------ diagnostics
// Vortex diagnostics of section 3.5 (Table 3, Figs. 6-7) on the dense velocity planes
// u[0] = u_x, u[1] = u_y ([ny][nx], written by unpack field 8).
//
// omega_z = (d u_y/dx - d u_x/dy) / 2 (eq. 18); a derivative is the central difference
// when both neighbours along the axis are active, the one-sided difference toward the
// active one when only one is, and 0 otherwise.  Vortex intensity I = 2 sum |omega_z| over
// FLUID nodes (unit cell area; the magnitude, since the signed integral of eq. 18 is the
// circulation around the no-slip boundary, i.e. zero).  Also max |u| over FLUID nodes.
__device__ __forceinline__ bool act_at(const StepArgs& a, int x, int y)
{
    return x >= 0 && y >= 0 && x < a.nx && y < a.ny && is_active(a.type[y * a.pitch + x]);
}

__device__ __forceinline__ double axis_derivative(const StepArgs& a, const double* f, int x, int y, int dx, int dy)
{
    const bool up = act_at(a, x + dx, y + dy), dn = act_at(a, x - dx, y - dy);
    const long long c = (long long)y * a.nx + x, o = (long long)dy * a.nx + dx;
    if (up && dn) return (f[c + o] - f[c - o]) / 2.0;
    if (up) return f[c + o] - f[c];
    if (dn) return f[c] - f[c - o];
    return 0.0;
}

__global__ __launch_bounds__(256) void diag_vorticity_kernel(StepArgs a, const double* u, double* partial)
{
    __shared__ double sm[2][4];
    const int x = blockIdx.x * 64 + (threadIdx.x & 63), y = blockIdx.y * 4 + (threadIdx.x >> 6);
    double w = 0.0, um = 0.0;
    if (x < a.nx && y < a.ny && (a.type[y * a.pitch + x] & CLS_MASK) == FLUID) {
        const long long n2 = (long long)a.nx * a.ny;
        const double dvdx = axis_derivative(a, u + n2, x, y, 1, 0);
        const double dudy = axis_derivative(a, u, x, y, 0, 1);
        w = 2.0 * fabs(0.5 * (dvdx - dudy));
        const long long c = (long long)y * a.nx + x;
        um = sqrt(u[c] * u[c] + u[n2 + c] * u[n2 + c]);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        w += __shfl_xor(w, off, 64);
        um = fmax(um, __shfl_xor(um, off, 64));
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sm[0][wv] = w;
        sm[1][wv] = um;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const long long b = (long long)blockIdx.y * gridDim.x + blockIdx.x;
        partial[2 * b] = ((sm[0][0] + sm[0][1]) + sm[0][2]) + sm[0][3];
        partial[2 * b + 1] = fmax(fmax(sm[1][0], sm[1][1]), fmax(sm[1][2], sm[1][3]));
    }
}

// Stream function psi(x, y) = sum over y' <= y of u_x(x, y') along each column (non-active
// nodes carry no flux), so u_x = d psi/dy; one thread per column keeps the column's largest
// and smallest psi over FLUID nodes (first occurrence from the bottom on ties).  The loads of
// PSI_ROWS rows are issued before any of them is summed (the sum keeps the row order): one
// memory round trip per PSI_ROWS rows instead of per row.
constexpr int PSI_ROWS = 16;
__device__ __forceinline__ void psi_row(uint8_t t, double v, int y, double& psi, double& vmax, int& ymax,
                                        double& vmin, int& ymin)
{
    if (!is_active(t)) return;
    psi += v;
    if ((t & CLS_MASK) != FLUID) return;
    if (psi > vmax) { vmax = psi; ymax = y; }
    if (psi < vmin) { vmin = psi; ymin = y; }
}

__global__ __launch_bounds__(256) void diag_psi_kernel(StepArgs a, const double* u, double* col)
{
    const int x = blockIdx.x * 256 + threadIdx.x;
    if (x >= a.nx) return;
    double psi = 0.0, vmax = -__builtin_huge_val(), vmin = __builtin_huge_val();
    int ymax = -1, ymin = -1;
    int y0 = 0;
    for (; y0 + PSI_ROWS <= a.ny; y0 += PSI_ROWS) {
        uint8_t t[PSI_ROWS];
        double v[PSI_ROWS];
#pragma unroll
        for (int j = 0; j < PSI_ROWS; j++) {
            t[j] = a.type[(y0 + j) * a.pitch + x];
            v[j] = u[(long long)(y0 + j) * a.nx + x];
        }
#pragma unroll
        for (int j = 0; j < PSI_ROWS; j++) psi_row(t[j], v[j], y0 + j, psi, vmax, ymax, vmin, ymin);
    }
    for (int y = y0; y < a.ny; y++)
        psi_row(a.type[y * a.pitch + x], u[(long long)y * a.nx + x], y, psi, vmax, ymax, vmin, ymin);
    col[4LL * x] = vmax;
    col[4LL * x + 1] = ymax;
    col[4LL * x + 2] = vmin;
    col[4LL * x + 3] = ymin;
}

// One block: fixed-order sum of the vorticity partials, max of the speed partials, and the
// extrema of psi over columns (smallest node index y * nx + x on ties).  out[0] = I,
// out[1] = max |u|, out[2..4] = psi_max, x, y, out[5..7] = psi_min, x, y.
__global__ __launch_bounds__(256) void diag_finish_kernel(const double* partial, int n_part, const double* col, int nx,
                                                          double* out)
{
    __shared__ double s_w[256], s_u[256], s_mx[256], s_mxi[256], s_mn[256], s_mni[256];
    const int t = threadIdx.x;
    double w = 0.0, um = 0.0;
    for (int b = t; b < n_part; b += 256) {
        w += partial[2 * b];
        um = fmax(um, partial[2 * b + 1]);
    }
    double mx = -__builtin_huge_val(), mn = __builtin_huge_val(), mxi = -1.0, mni = -1.0;   // index y * nx + x
    for (int x = t; x < nx; x += 256) {
        const double* c = col + 4LL * x;
        if (c[1] >= 0) {
            const double i = c[1] * nx + x;
            if (c[0] > mx || (c[0] == mx && i < mxi)) { mx = c[0]; mxi = i; }
        }
        if (c[3] >= 0) {
            const double i = c[3] * nx + x;
            if (c[2] < mn || (c[2] == mn && i < mni)) { mn = c[2]; mni = i; }
        }
    }
    s_w[t] = w; s_u[t] = um; s_mx[t] = mx; s_mxi[t] = mxi; s_mn[t] = mn; s_mni[t] = mni;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if (t < h) {
            s_w[t] += s_w[t + h];
            s_u[t] = fmax(s_u[t], s_u[t + h]);
            const double v = s_mx[t + h], vi = s_mxi[t + h];
            if (vi >= 0 && (s_mxi[t] < 0 || v > s_mx[t] || (v == s_mx[t] && vi < s_mxi[t]))) { s_mx[t] = v; s_mxi[t] = vi; }
            const double m2 = s_mn[t + h], mi = s_mni[t + h];
            if (mi >= 0 && (s_mni[t] < 0 || m2 < s_mn[t] || (m2 == s_mn[t] && mi < s_mni[t]))) { s_mn[t] = m2; s_mni[t] = mi; }
        }
        __syncthreads();
    }
    if (t == 0) {
        out[0] = s_w[0];
        out[1] = s_u[0];
        const long long im = (long long)s_mxi[0], in = (long long)s_mni[0];
        out[2] = s_mx[0];
        out[3] = im >= 0 ? (double)(im % nx) : -1.0;
        out[4] = im >= 0 ? (double)(im / nx) : -1.0;
        out[5] = s_mn[0];
        out[6] = in >= 0 ? (double)(in % nx) : -1.0;
        out[7] = in >= 0 ? (double)(in / nx) : -1.0;
    }
}

size_t diagnostics_words(int nx, int ny)
{
    const size_t n2 = (size_t)nx * ny;
    const size_t nb = (size_t)((nx + 63) / 64) * ((ny + 3) / 4);
    return 2 * n2 + 2 * nb + 4 * (size_t)nx + 8;
}

// ws: diagnostics_words(nx, ny) doubles.  Reads the state through `a` (a read-out pull)
// and leaves the 8 results in ws[2 n2 + 2 nb + 4 nx ...].
hipError_t launch_diagnostics(int mode, const StepArgs& a, double* ws, hipStream_t s)
{
    const long long n2 = (long long)a.nx * a.ny;
    const dim3 g = lattice_grid(a);
    const int nb = (int)(g.x * g.y);
    double* part = ws + 2 * n2;
    double* col = part + 2LL * nb;
    double* out = col + 4LL * a.nx;
    hipError_t e = launch_unpack(mode, a, 8, 0, 0.0, ws, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(diag_vorticity_kernel, g, dim3(256), 0, s, a, (const double*)ws, part);
    hipLaunchKernelGGL(diag_psi_kernel, dim3((a.nx + 255) / 256), dim3(256), 0, s, a, (const double*)ws, col);
    hipLaunchKernelGGL(diag_finish_kernel, dim3(1), dim3(256), 0, s, (const double*)part, nb, (const double*)col, a.nx, out);
    return hipGetLastError();
}

}  // namespace aq
