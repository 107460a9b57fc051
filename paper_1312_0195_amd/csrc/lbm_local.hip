// lbm_local.hip -- batched local problems of Sec. 3 in one persistent launch.
//
// Work item = (patch, drive). A patch is a periodic side x side window of the
// fine permeability field; the drive is G1 = (g, 0) or G2 = (0, g). Each item
// runs the time stepping of Sec. 2.2 from rest until its own volume-averaged
// velocity converges, then writes its column of Eq. tensor-kappa:
//   drive x: kxx = nu ubar_x / g, kyx = nu ubar_y / g
//   drive y: kxy = nu ubar_x / g, kyy = nu ubar_y / g.
//
// On-chip design (gfx950: 160 KB LDS per CU, wave64):
//  * A workgroup of T threads is split into slots of G threads; each slot
//    runs one item. Items of one side share a launch-wide tile choice (G per
//    side) and run side by side, so small patches still fill the CU.
//  * Populations 1..8 of an item live in LDS (8 planes of side^2 FP32
//    values, 32 B per cell, or FP64 with 64 B per cell: deviations from the
//    rest state moving with the item's mean momentum, see collide); the rest
//    population and the drag coefficient stay in registers of the thread that
//    owns the cell. FP32 items use FP32 arithmetic; FP64 items FP64 throughout,
//    for regimes where a step changes the state by less than half an FP32 ulp
//    (tau near 1/2 with weak drag: FP32 state then stops short of the fixed
//    point).
//  * Streaming in place ("AA" order): on even steps a cell reads its own
//    slots and writes the post-collision values back reversed
//    (A[opp(a)][x] = f*_a); on odd steps it reads f_a from A[opp(a)][x - e_a]
//    and writes f*_a to A[a][x + e_a]. In both cases the slots a cell reads are
//    exactly the slots it writes, and different cells own disjoint slots, so a
//    step needs no barrier between its reads and writes: one workgroup barrier
//    per step, and a single LDS copy of the state.
//  * Every check_every steps (even, so the state is back in even order) each
//    slot sums u (Eq. u-of-S-C) over its cells in FP64: wavefront shuffles,
//    then the wave partials of the slot in a fixed order. The relative change
//    of the mean against the previous check decides convergence.
//  * Items are taken from per-side queues (largest side first) with a global
//    atomic counter; a slot whose item finished takes the next one. When a
//    side's queue is empty and all slots are idle the workgroup moves on to
//    the next side. Every item runs at most max_steps steps, so every
//    workgroup reaches the end of the queues and exits.
//  * The largest sides (one item per workgroup, more than one cell per
//    thread) share one queue; each item takes its own side from its entry.
//  * Within a queue, items start in the order given or (LBM_SCHEDULE_COST)
//    longest predicted first: step counts span orders of magnitude, and a
//    long item that starts late sets the end of the whole batch. The
//    prediction adds the patch's two slowest relaxation times, the drag
//    relaxation of a permeable patch and the pressure diffusion of a nearly
//    impermeable one, and weighs in the spread of ln kappa (k_local_cost); a
//    pre-pass bins it and counting-sorts the item list on the device.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "lbm_internal.h"

namespace lbm {
namespace {

constexpr int kMaxSide = 64;
constexpr int kMaxClasses = kMaxSide;  // one class per distinct side
constexpr int kCPT = 4;                // max cells per thread
constexpr int kEscThreads = 512;       // workgroup size of the FP64 re-run

struct ClassDesc {
    int side;
    int slot_threads;  // G
    int nslots;        // slots in use: T / G (capped by LDS)
    int cells_per_thread;
    int begin, count;  // item range in the sorted item list
    int esc_ok;        // FP32 items of this side may be handed to the FP64 re-run
    int merged;        // items of several sides (side: the largest); each item's own side in its int4
};

struct LocalArgs {
    const int4 *__restrict__ items;      // {x0, y0, side, out = patch * 2 + drive}
    const ClassDesc *__restrict__ classes;
    int nclasses;
    int *__restrict__ counters;          // one per class
    const double *__restrict__ field;
    int fnx, fny;
    double *__restrict__ keff;
    int *__restrict__ steps_out;
    int *__restrict__ flags_out;
    float om, omc, twotau, omtt;         // 1/tau, 1 - 1/tau, 2 tau, 1 - 2 tau
    float heg;                           // eps g / 2
    double om_d, omc_d, twotau_d, omtt_d;
    double heg_d;
    double h;                            // eps nu / 2
    double nu_over_g;
    double tol;
    int check_every;
    int max_steps;
    int margin;                          // cells left out of the average at each side
    // FP32 items still running after esc_steps steps stop and are queued for a
    // re-run with FP64 state (0: never): esc_classes[c] (device table whose
    // count the kernel increments) and esc_items (same item ranges as classes)
    int esc_steps;
    ClassDesc *esc_classes;
    int4 *esc_items;
};

__device__ __forceinline__ int wrapm(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// The reference momentum of a rebased item, rounded to 16 significant bits:
// the mean it comes from is an FP64 sum whose rounding depends on how the
// item's cells are spread over waves, and the coarse rounding makes the
// reference (and so the whole FP32 state) the same for every tile layout
// unless that sum lies within ~1e-15 of a rounding boundary. 16 bits keep the
// stored non-uniform part within 2^-16 of the uniform flow, far below what
// the rebasing needs.
template <typename P>
__device__ __forceinline__ P reference_momentum(double v)
{
    const unsigned b = __float_as_uint((float)v);
    return (P)__uint_as_float((b + 0x40u) & ~0x7Fu);
}

// Relaxation constants in the arithmetic type P.
template <typename P> struct Consts;
template <> struct Consts<float> {
    float om, omc, twotau, omtt, heg;
    __device__ explicit Consts(const struct LocalArgs &a);
};
template <> struct Consts<double> {
    double om, omc, twotau, omtt, heg;
    __device__ explicit Consts(const struct LocalArgs &a);
};
__device__ inline Consts<float>::Consts(const LocalArgs &a)
    : om(a.om), omc(a.omc), twotau(a.twotau), omtt(a.omtt), heg(a.heg) {}
__device__ inline Consts<double>::Consts(const LocalArgs &a)
    : om(a.om_d), omc(a.omc_d), twotau(a.twotau_d), omtt(a.omtt_d), heg(a.heg_d) {}

// One collision of a cell, f[0..8] in, post-collision values out in f.
//
// The state is stored rebased: f_a = w_a rho0 + 3 w_a e_a . U + f'_a, where
// U is a momentum uniform over the item (the mean momentum at the last
// check, kept in the storage type) and f' is what is stored. The uniform
// part is a rest state moving with U: streaming leaves it unchanged, and
// since the step is linear in f (with the force entering through rho), the
// collision of the rebased state needs U only inside the drag term. A
// permeable patch converges slowly (relaxation time ~ kappa / (eps nu)) and
// its flow is nearly uniform; stored as plain deviations f - w rho0, a step's
// change to the populations falls below half an FP32 ulp of the values long
// before the fixed point (measured: K_eff short by ~7e-9 per step of the run,
// 2.6e-4 at 39 000 steps), while f' holds only the non-uniform part of the
// flow, so the stall moves down by the ratio of the two.
//
// The drag enters through its deficit E = 1 - D = h / (kappa + h),
// h = eps nu / 2; with j' = sum e f', rho = rho0 + sum f':
//   rho u_eq - U = 2 tau D (U + j' + rho eps G / 2) + (1 - 2 tau)(U + j') - U
//               = j' + 2 tau (rho eps G / 2 - E (U + j' + rho eps G / 2)),
// every term of which is as small as the non-uniform flow or the drag.
// FP64 items take cE = 2 tau E per cell and tgx, tgy = 2 tau eps G / 2 of
// the item's drive; FP32 items take cE = 2 E, tgx, tgy = 2 eps G / 2 and
// form om (rho u_eq - U) as om j' + 2 (rho eps G / 2 - E (...)), with the
// exact factor 2 = om 2 tau,
// and weights that sum exactly (the rest weight and the diagonal momentum
// weight as remainders): with rounded FP32 weights, and with (1/tau) (2 tau)
// as a product of two rounded constants, every step would add a fixed
// fraction (~3e-8) of the mass and momentum terms, a bias the slow relaxation
// of a permeable patch accumulates. Ux, Uy: the reference U.
template <typename P>
__device__ __forceinline__ void collide(P f[9], P cE, P hegx, P hegy, P tgx, P tgy, P Ux, P Uy,
                                        const Consts<P> &k)
{
    const P dr = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
    const P jx = (f[1] - f[3]) + ((f[5] - f[6]) + (f[8] - f[7]));
    const P jy = (f[2] - f[4]) + ((f[5] + f[6]) - (f[7] + f[8]));
    const P rho = P(1) + dr;
    const P om = k.om, omc = k.omc;
    if constexpr (sizeof(P) == 8) {
        const P mx = (jx + tgx * rho) - cE * (jx + (hegx * rho + Ux));
        const P my = (jy + tgy * rho) - cE * (jy + (hegy * rho + Uy));
        const P s0 = (P(4) / P(9)) * om * dr;
        const P b = (P(1) / P(9)) * om * dr;
        const P bx = (P(1) / P(3)) * om * mx;
        const P by = (P(1) / P(3)) * om * my;
        const P cc = (P(1) / P(36)) * om * dr;
        const P cx = (P(1) / P(12)) * om * mx;
        const P cy = (P(1) / P(12)) * om * my;
        const P pp = cx + cy, qq = cx - cy;
        f[0] = omc * f[0] + s0;
        f[1] = omc * f[1] + (b + bx);
        f[2] = omc * f[2] + (b + by);
        f[3] = omc * f[3] + (b - bx);
        f[4] = omc * f[4] + (b - by);
        f[5] = omc * f[5] + (cc + pp);
        f[6] = omc * f[6] + (cc - qq);
        f[7] = omc * f[7] + (cc - pp);
        f[8] = omc * f[8] + (cc + qq);
    } else {
        // every fused multiply-add written out and no other contraction, so
        // the launches compiled for 1, 2 or 4 cells per thread round alike
#pragma clang fp contract(off)
        // cE = 2 E, tgx = 2 eps G / 2 here (doublings are exact), so
        // t = 2 (rho eps G / 2 - E (j' + rho eps G / 2 + U)) in one rounding
        const P tx = __builtin_fmaf(-cE, jx + __builtin_fmaf(hegx, rho, Ux), tgx * rho);
        const P ty = __builtin_fmaf(-cE, jy + __builtin_fmaf(hegy, rho, Uy), tgy * rho);
        const P Mx = __builtin_fmaf(om, jx, tx), My = __builtin_fmaf(om, jy, ty);
        const P D = om * dr;
        const P b = D * (P(1) / P(9));
        const P cc = D * (P(1) / P(36));
        const P s0 = __builtin_fmaf(P(-4), b + cc, D);
        // momentum: 2 t3 M on the axes and 4 c12 M on the diagonals, with t3
        // = fl(1/3) and c12 = (1 - 2 t3) / 4 exact in FP32: they sum to M
        // exactly, each term rounded once
        constexpr P t3 = P(1) / P(3), c12 = (P(1) - P(2) * t3) * P(0.25);
        const P cx = Mx * c12, cy = My * c12;
        const P pp = cx + cy, qq = cx - cy;
        f[0] = __builtin_fmaf(omc, f[0], s0);
        f[1] = __builtin_fmaf(omc, f[1], __builtin_fmaf(Mx, t3, b));
        f[2] = __builtin_fmaf(omc, f[2], __builtin_fmaf(My, t3, b));
        f[3] = __builtin_fmaf(omc, f[3], __builtin_fmaf(-Mx, t3, b));
        f[4] = __builtin_fmaf(omc, f[4], __builtin_fmaf(-My, t3, b));
        f[5] = __builtin_fmaf(omc, f[5], cc + pp);
        f[6] = __builtin_fmaf(omc, f[6], cc - qq);
        f[7] = __builtin_fmaf(omc, f[7], cc - pp);
        f[8] = __builtin_fmaf(omc, f[8], cc + qq);
    }
}

// CPT: the most cells any thread of this launch owns (1, 2 or 4); the
// register arrays are sized by it, so launches of small patches keep fewer
// registers live and fit more workgroups per CU.
template <int T, typename P, int CPT>
__global__ __launch_bounds__(T, (CPT == 1 && sizeof(P) == 4 ? 8 : 1)) void k_local(LocalArgs a)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    P *lds = reinterpret_cast<P *>(lds_raw);
    const Consts<P> kc(a);
    constexpr int NW = T / 64;
    __shared__ double red[NW][4];
    __shared__ int ctrl[NW];  // item index per slot (at most NW slots), -1 = none

    const int tid = threadIdx.x;
    int cls = 0;

    // per-slot state (uniform over the threads of a slot)
    int item = -1;
    int steps = 0;
    bool have_prev = false;
    bool over_budget = false;  // FP32 item past esc_steps that cannot be re-run in FP64
    double prev_x = 0.0, prev_y = 0.0;
    int out = 0, x0 = 0, y0 = 0;
    int item_side = 0;  // side of the slot's item (classes of merged sides)
    P hegx = 0, hegy = 0, tgx = 0, tgy = 0;
    P Ux = 0, Uy = 0;  // reference momentum of the rebased state
    double hegx_d = 0.0, hegy_d = 0.0;
    // per-cell registers
    P f0[CPT], tE[CPT];  // rest population and scaled drag deficit of each owned cell (cE of collide)
    int xy[CPT];

    bool need_item = true;
    __syncthreads();

    while (true) {
        const ClassDesc cd = a.classes[cls];
        const int G = cd.slot_threads, C = cd.cells_per_thread;
        // a merged class has one slot (G = T), so the slot's LDS starts at 0
        // whatever the side, and the side is the item's from its claim on
        int S = cd.merged ? item_side : cd.side;
        int S2 = S * S;
        const int slot = tid / G, lt = tid - slot * G;
        const bool in_slot = slot < cd.nslots;
        P *A = lds + (size_t)(in_slot ? slot : 0) * 8 * S2;

        // ---- control: claim items for slots that need one -------------------
        if (in_slot && lt == 0 && need_item) {
            const int k = atomicAdd(&a.counters[cls], 1);
            ctrl[slot] = (k < cd.count) ? cd.begin + k : -1;
        }
        __syncthreads();
        if (in_slot && need_item) {
            item = ctrl[slot];
            need_item = false;
            if (item >= 0) {
                const int4 it = a.items[item];
                x0 = it.x;
                y0 = it.y;
                out = it.w;
                item_side = it.z;
                if (cd.merged) {
                    S = it.z;
                    S2 = S * S;
                }
                const int drive = out & 1;
                hegx = drive == 0 ? kc.heg : P(0);
                hegy = drive == 1 ? kc.heg : P(0);
                hegx_d = drive == 0 ? a.heg_d : 0.0;
                hegy_d = drive == 1 ? a.heg_d : 0.0;
                tgx = (P)((sizeof(P) == 8 ? a.twotau_d : 2.0) * hegx_d);
                tgy = (P)((sizeof(P) == 8 ? a.twotau_d : 2.0) * hegy_d);
                Ux = Uy = P(0);
                steps = 0;
                have_prev = false;
                over_budget = false;
#pragma unroll
                for (int k = 0; k < CPT; ++k) {
                    const int c = lt + k * G;
                    if (k < C && c < S2) {
                        const int x = c % S, y = c / S;
                        xy[k] = x | (y << 8);
                        const int fx = (x0 + x) % a.fnx, fy = (y0 + y) % a.fny;
                        const double kap = a.field[(size_t)fy * a.fnx + fx];
                        // kappa <= 0 or NaN poisons the item: it ends flagged non-finite
                        tE[k] = (kap > 0.0) ? (P)((sizeof(P) == 8 ? a.twotau_d : 2.0) * a.h / (kap + a.h))
                                            : (P)__longlong_as_double(0x7ff8000000000000LL);
                        f0[k] = P(0);
#pragma unroll
                        for (int q = 0; q < 8; ++q) A[q * S2 + c] = P(0);
                    }
                }
            }
        }
        // ---- all slots idle: next side class, or done -----------------------
        int busy = 0;
        __syncthreads();
        for (int s = 0; s < cd.nslots; ++s) busy |= (ctrl[s] >= 0);
        if (!busy) {
            __syncthreads();
            if (cls + 1 >= a.nclasses) break;
            ++cls;
            need_item = true;
            continue;
        }

        // ---- check_every steps ----------------------------------------------
        const bool active = in_slot && item >= 0;
        for (int st = 0; st < a.check_every; ++st) {
            if (active) {
                const bool odd = ((steps + st) & 1) != 0;
#pragma unroll
                for (int k = 0; k < CPT; ++k) {
                    const int c = lt + k * G;
                    if (k < C && c < S2) {
                        const int x = xy[k] & 255, y = xy[k] >> 8;
                        P f[9];
                        f[0] = f0[k];
                        if (!odd) {
                            // own slots, in order; written back reversed
#pragma unroll
                            for (int q = 1; q < 9; ++q) f[q] = A[(q - 1) * S2 + c];
                            collide<P>(f, tE[k], hegx, hegy, tgx, tgy, Ux, Uy, kc);
                            A[(3 - 1) * S2 + c] = f[1];
                            A[(4 - 1) * S2 + c] = f[2];
                            A[(1 - 1) * S2 + c] = f[3];
                            A[(2 - 1) * S2 + c] = f[4];
                            A[(7 - 1) * S2 + c] = f[5];
                            A[(8 - 1) * S2 + c] = f[6];
                            A[(5 - 1) * S2 + c] = f[7];
                            A[(6 - 1) * S2 + c] = f[8];
                        } else {
                            const int xm = x == 0 ? S - 1 : x - 1, xp = x == S - 1 ? 0 : x + 1;
                            const int rm = (y == 0 ? S - 1 : y - 1) * S, rp = (y == S - 1 ? 0 : y + 1) * S;
                            const int r0 = y * S;
                            // f_a(x) = A[opp a][x - e_a]
                            f[1] = A[(3 - 1) * S2 + r0 + xm];
                            f[2] = A[(4 - 1) * S2 + rm + x];
                            f[3] = A[(1 - 1) * S2 + r0 + xp];
                            f[4] = A[(2 - 1) * S2 + rp + x];
                            f[5] = A[(7 - 1) * S2 + rm + xm];
                            f[6] = A[(8 - 1) * S2 + rm + xp];
                            f[7] = A[(5 - 1) * S2 + rp + xp];
                            f[8] = A[(6 - 1) * S2 + rp + xm];
                            collide<P>(f, tE[k], hegx, hegy, tgx, tgy, Ux, Uy, kc);
                            // f*_a goes to A[a][x + e_a]
                            A[(1 - 1) * S2 + r0 + xp] = f[1];
                            A[(2 - 1) * S2 + rp + x] = f[2];
                            A[(3 - 1) * S2 + r0 + xm] = f[3];
                            A[(4 - 1) * S2 + rm + x] = f[4];
                            A[(5 - 1) * S2 + rp + xp] = f[5];
                            A[(6 - 1) * S2 + rp + xm] = f[6];
                            A[(7 - 1) * S2 + rm + xm] = f[7];
                            A[(8 - 1) * S2 + rm + xp] = f[8];
                        }
                        f0[k] = f[0];
                    }
                    __builtin_amdgcn_sched_barrier(0);  // one cell at a time: bounded register use
                }
            }
            __syncthreads();
        }
        if (active) steps += a.check_every;

        // ---- convergence check: FP64 mean velocity of each slot --------------
        double sx = 0.0, sy = 0.0, qx = 0.0, qy = 0.0;  // sums of u (inner window) and of j'
        if (active) {
#pragma unroll
            for (int k = 0; k < CPT; ++k) {
                const int c = lt + k * G;
                if (k < C && c < S2) {
                    // even order: A[a - 1][c] holds f_a(x) before collision
                    double fd[9];
                    fd[0] = f0[k];
#pragma unroll
                    for (int q = 1; q < 9; ++q) fd[q] = (double)A[(q - 1) * S2 + c];
                    const double dr = ((fd[0] + fd[1]) + (fd[2] + fd[3])) + ((fd[4] + fd[5]) + (fd[6] + fd[7])) + fd[8];
                    const double jpx = (fd[1] - fd[3]) + ((fd[5] - fd[6]) + (fd[8] - fd[7]));
                    const double jpy = (fd[2] - fd[4]) + ((fd[5] + fd[6]) - (fd[7] + fd[8]));
                    qx += jpx;
                    qy += jpy;
                    const double jx = (double)Ux + jpx, jy = (double)Uy + jpy;
                    const double rho = 1.0 + dr;
                    const double D = 1.0 - (double)tE[k] / (sizeof(P) == 8 ? a.twotau_d : 2.0);
                    // oversampling: only the inner window enters the average
                    const int x = xy[k] & 255, y = xy[k] >> 8;
                    const int m = a.margin;
                    if (x >= m && x < S - m && y >= m && y < S - m) {
                        sx += D * (jx + hegx_d * rho) / rho;
                        sy += D * (jy + hegy_d * rho) / rho;
                    }
                }
            }
        }
        sx = wave_sum(sx);
        sy = wave_sum(sy);
        qx = wave_sum(qx);
        qy = wave_sum(qy);
        if ((tid & 63) == 0) {
            red[tid >> 6][0] = sx;
            red[tid >> 6][1] = sy;
            red[tid >> 6][2] = qx;
            red[tid >> 6][3] = qy;
        }
        __syncthreads();
        if (active) {
            const int w0 = (slot * G) >> 6, nw = G >> 6;
            double tx = 0.0, ty = 0.0, tqx = 0.0, tqy = 0.0;
            for (int w = 0; w < nw; ++w) {
                tx += red[w0 + w][0];
                ty += red[w0 + w][1];
                tqx += red[w0 + w][2];
                tqy += red[w0 + w][3];
            }
            const double inner = (double)(S - 2 * a.margin) * (double)(S - 2 * a.margin);
            const double ux = tx / inner, uy = ty / inner;
            int flag = -2;  // -2: keep going
            if (!isfinite(ux) || !isfinite(uy)) {
                flag = 2;
            } else if (have_prev) {
                const double dx = ux - prev_x, dy = uy - prev_y;
                if (sqrt(dx * dx + dy * dy) <= a.tol * sqrt(ux * ux + uy * uy)) flag = 0;
            }
            if (flag == -2 && steps >= a.max_steps) flag = 1;
            // Past the FP32 step budget: a slowly converging item whose FP32
            // state would stop short of the fixed point by more than the
            // target (the stall grows with the relaxation time). Hand it to
            // the FP64 re-run, or, where FP64 state does not fit, finish in
            // FP32 and say so in the flag.
            if (flag == -2 && a.esc_steps > 0 && steps >= a.esc_steps) {
                if (cd.esc_ok)
                    flag = 4;
                else
                    over_budget = true;
            }
            if (flag == 0 && over_budget) flag = 3;
            prev_x = ux;
            prev_y = uy;
            have_prev = true;
            if (flag == 4) {
                if (lt == 0) {
                    const int pos = atomicAdd(&a.esc_classes[cls].count, 1);
                    a.esc_items[a.esc_classes[cls].begin + pos] = make_int4(x0, y0, S, out);
                }
                need_item = true;
            } else if (flag != -2) {
                if (lt == 0) {
                    const int patch = out >> 1, drive = out & 1;
                    a.keff[4 * (size_t)patch + drive] = a.nu_over_g * ux;
                    a.keff[4 * (size_t)patch + 2 + drive] = a.nu_over_g * uy;
                    if (a.steps_out) a.steps_out[2 * patch + drive] = steps;
                    if (a.flags_out) a.flags_out[2 * patch + drive] = flag;
                }
                need_item = true;
            } else {
                // rebase on the item's current mean momentum U + mean j':
                // f' -= 3 w_a e_a . (U_new - U); U_new is kept in the storage
                // type, so the stored state and U describe the same f
                const P nUx = reference_momentum<P>((double)Ux + tqx / (double)S2);
                const P nUy = reference_momentum<P>((double)Uy + tqy / (double)S2);
                const P dUx = nUx - Ux, dUy = nUy - Uy;
                Ux = nUx;
                Uy = nUy;
                const P ax = P(1) / P(3) * dUx, ay = P(1) / P(3) * dUy;              // 3 w_a e_a . dU, axes
                const P dp = P(1) / P(12) * (dUx + dUy), dm = P(1) / P(12) * (dUx - dUy);  // diagonals
#pragma unroll
                for (int k = 0; k < CPT; ++k) {
                    const int c = lt + k * G;
                    if (k < C && c < S2) {
                        // even order: A[a - 1][c] holds f'_a of cell c
                        A[0 * S2 + c] -= ax;
                        A[1 * S2 + c] -= ay;
                        A[2 * S2 + c] += ax;
                        A[3 * S2 + c] += ay;
                        A[4 * S2 + c] -= dp;
                        A[5 * S2 + c] += dm;
                        A[6 * S2 + c] += dp;
                        A[7 * S2 + c] -= dm;
                    }
                }
            }
        }
        __syncthreads();  // red[] and ctrl[] are reused
    }
}

// Entries of skipped drives: NaN K_eff, flag -1, 0 steps.
__global__ void k_local_prefill(int n, const int *__restrict__ mask, double *__restrict__ keff,
                                int *__restrict__ steps, int *__restrict__ flags,
                                int *__restrict__ counters, int ncounters)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ncounters) counters[i] = 0;  // item counters and the schedule histogram
    if (i >= n) return;
    const double qnan = __longlong_as_double(0x7ff8000000000000LL);
    for (int d = 0; d < 2; ++d) {
        if (!(mask[i] & (1 << d))) {
            keff[4 * (size_t)i + d] = qnan;
            keff[4 * (size_t)i + 2 + d] = qnan;
            if (steps) steps[2 * i + d] = 0;
            if (flags) flags[2 * i + d] = -1;
        }
    }
}

// ---- start order (LBM_SCHEDULE_COST) --------------------------------------
// Key of an item: its side class in the high part (classes keep their
// ranges), then the bin of its predicted cost, largest first. The prediction
// is the logarithm of the sum of the two slowest relaxation times of the
// Brinkman flow in the patch, plus the spread sd(ln kappa):
//  * the drag relaxation of the mean flow, kappa / (eps nu), with the
//    arithmetic mean of kappa: a permeable patch relaxes slowly;
//  * the diffusion of pressure across the patch. Where the drag dominates,
//    the momentum follows the pressure gradient, j = -(kappa / (eps nu))
//    c_s^2 grad rho, so the density obeys a diffusion equation with
//    coefficient c_s^2 kappa / (eps nu), and its slowest mode on a side S
//    decays on the time scale S^2 eps nu / (pi^2 c_s^2 kappa), with the
//    geometric mean of kappa: a nearly impermeable patch relaxes slowly too;
//  * strong heterogeneity adds nearly blocked directions whose tiny
//    velocities converge slowly.
// kCostBins bins of width 1/4.
constexpr int kCostBins = 64;

__global__ __launch_bounds__(256) void k_local_cost(const int4 *__restrict__ items,
                                                    const ClassDesc *__restrict__ classes, int nclasses,
                                                    const double *__restrict__ field, int fnx, int fny,
                                                    double inv_eps_nu, double pdiff,
                                                    int *__restrict__ keys, int *__restrict__ hist)
{
    __shared__ double red[3][4];
    const int item = blockIdx.x;
    const int4 it = items[item];
    const int S = it.z, n = S * S;
    double sum = 0.0, sl = 0.0, sl2 = 0.0;
    for (int c = threadIdx.x; c < n; c += 256) {
        const int fx = (it.x + c % S) % fnx, fy = (it.y + c / S) % fny;
        const double k = field[(size_t)fy * fnx + fx];
        const double l = log(k);
        sum += k;
        sl += l;
        sl2 += l * l;
    }
    sum = wave_sum(sum);
    sl = wave_sum(sl);
    sl2 = wave_sum(sl2);
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = sum;
        red[1][threadIdx.x >> 6] = sl;
        red[2][threadIdx.x >> 6] = sl2;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double inv = 1.0 / (double)n;
    const double mean = ((red[0][0] + red[0][1]) + (red[0][2] + red[0][3])) * inv;
    const double ml = ((red[1][0] + red[1][1]) + (red[1][2] + red[1][3])) * inv;
    const double var = ((red[2][0] + red[2][1]) + (red[2][2] + red[2][3])) * inv - ml * ml;
    // relaxation times: drag of the mean flow, pressure diffusion (pdiff =
    // eps nu / (pi^2 c_s^2))
    const double t_drag = mean * inv_eps_nu;
    const double t_pres = (double)n * pdiff / exp(ml);
    int cls = 0;
    for (int c = 0; c < nclasses; ++c)
        if (item >= classes[c].begin && item < classes[c].begin + classes[c].count) cls = c;
    // in a class of merged sides a step of a smaller side costs less, in
    // proportion to its cells
    const double score = log(t_drag + t_pres) + sqrt(fmax(var, 0.0)) +
                         (classes[cls].merged ? 2.0 * log((double)S / (double)classes[cls].side) : 0.0);
    int bin;
    if (isfinite(score))
        bin = max(0, min(kCostBins - 1, (int)(4.0 * score)));
    else
        bin = (score > 0.0) ? kCostBins - 1 : 0;  // +inf: a cell without drag, slowest; NaN: negative mean,
                                                  // the item ends at its first check (non-finite)
    const int key = cls * kCostBins + (kCostBins - 1 - bin);
    keys[item] = key;
    atomicAdd(&hist[key], 1);
}

// Exclusive scan of the key histogram (one workgroup of 256 threads): the
// first position of each key in the ordered item list.
__global__ __launch_bounds__(256) void k_local_scan(const int *__restrict__ hist, int *__restrict__ cursor,
                                                    int nh)
{
    __shared__ int part[256];
    const int t = threadIdx.x;
    const int chunk = (nh + 255) / 256, lo = min(t * chunk, nh), hi = min(lo + chunk, nh);
    int own = 0;
    for (int i = lo; i < hi; ++i) own += hist[i];
    part[t] = own;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int pos = part[t] - own;
    for (int i = lo; i < hi; ++i) {
        cursor[i] = pos;
        pos += hist[i];
    }
}

__global__ void k_local_scatter(int n, const int4 *__restrict__ items, const int *__restrict__ keys,
                                int *__restrict__ cursor, int4 *__restrict__ sorted)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    sorted[atomicAdd(&cursor[keys[i]], 1)] = items[i];
}

struct LocalLayout {
    size_t off_items, off_classes, off_counters, off_mask, off_sorted, off_keys, off_esc_items, off_esc_classes,
        off_esc_counters, total;
};

// counters: kMaxClasses item counters, then the schedule histogram and its
// cursors (kMaxClasses x kCostBins each)
constexpr int kHist = kMaxClasses * kCostBins;
constexpr int kNumCounters = kMaxClasses + 2 * kHist;

LocalLayout local_layout(int n_patches)
{
    LocalLayout L{};
    size_t off = 0;
    const size_t items = 2 * (size_t)std::max(n_patches, 1);
    L.off_items = off;    off = align_up(off + sizeof(int4) * items);
    L.off_classes = off;  off = align_up(off + sizeof(ClassDesc) * 2 * kMaxClasses);
    L.off_counters = off; off = align_up(off + sizeof(int) * kNumCounters);
    L.off_mask = off;     off = align_up(off + sizeof(int) * (size_t)std::max(n_patches, 1));
    L.off_sorted = off;   off = align_up(off + sizeof(int4) * items);
    L.off_keys = off;     off = align_up(off + sizeof(int) * items);
    L.off_esc_items = off;    off = align_up(off + sizeof(int4) * items);
    L.off_esc_classes = off;  off = align_up(off + sizeof(ClassDesc) * kMaxClasses);
    L.off_esc_counters = off; off = align_up(off + sizeof(int) * kMaxClasses);
    L.total = off;
    return L;
}

int lds_budget_bytes()
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
        return v;
    return 64 * 1024;
}

int pow2_at_least(int v)
{
    int p = 64;
    while (p < v) p <<= 1;
    return p;
}

// A second stream per device (default priority, created on first use) for
// running two launches of one call side by side.
hipStream_t side_stream()
{
    static std::mutex mu;
    static hipStream_t streams[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    if (!streams[dev] && hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking) != hipSuccess)
        streams[dev] = nullptr;
    return streams[dev];
}

// Two streams per device with complementary CU masks, for running the two
// launches of a mixed call on disjoint sets of CUs: a launch of one
// workgroup per CU (the largest sides) otherwise takes every CU at the start,
// and the single-cell launch beside it only gets the CUs it frees at its end.
// On a 256-CU part the mask bits interleave the eight XCDs (CU i lies on XCD
// i % 8), and a mask that leaves an XCD without CUs makes launches fail; the
// single-cell stream therefore gets k of the 32 CUs of every XCD, spread
// evenly over them (k a multiple of kSplitStep), the other stream the rest.
// Created on first use of each k and kept for the life of the process.
constexpr int kSplitStep = 4;

bool split_streams(int k, hipStream_t *multi, hipStream_t *single)
{
    static std::mutex mu;
    static hipStream_t streams[64][32 / kSplitStep][2] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return false;
    if (device_cu_count() != 256 || k < kSplitStep || k > 32 - kSplitStep || k % kSplitStep) return false;
    const int slot = k / kSplitStep - 1;
    std::lock_guard<std::mutex> lock(mu);
    if (!streams[dev][slot][0]) {
        uint32_t mm[8] = {}, ms[8] = {};
        for (int i = 0; i < 256; ++i) {
            const int l = i / 8;  // position of CU i within its XCD
            const bool to_single = ((l + 1) * k) / 32 != (l * k) / 32;
            (to_single ? ms : mm)[i / 32] |= 1u << (i % 32);
        }
        hipStream_t a = nullptr, b = nullptr;
        if (hipExtStreamCreateWithCUMask(&a, 8, mm) != hipSuccess) return false;
        if (hipExtStreamCreateWithCUMask(&b, 8, ms) != hipSuccess) {
            (void)hipStreamDestroy(a);
            return false;
        }
        streams[dev][slot][0] = a;
        streams[dev][slot][1] = b;
    }
    *multi = streams[dev][slot][0];
    *single = streams[dev][slot][1];
    return true;
}

// cu_budget: the CUs the launch's stream may use (0: all of them); the grid
// holds no more workgroups than fit on them at once.
template <int T, typename P, int CPT>
lbm_status launch_local_c(const LocalArgs &a, size_t lds_bytes, int grid, hipStream_t stream, int cu_budget)
{
    if (lds_bytes > 64 * 1024)
        LBM_HIP(hipFuncSetAttribute((const void *)k_local<T, P, CPT>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes));
    int occ = 0;
    LBM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_local<T, P, CPT>, T, lds_bytes));
    if (occ < 1) return set_error(LBM_EINVAL, "lbm_local_keff: tile does not fit on a CU");
    const int blocks = std::min(grid, (cu_budget > 0 ? cu_budget : device_cu_count()) * occ);
    hipLaunchKernelGGL((k_local<T, P, CPT>), dim3(blocks), dim3(T), lds_bytes, stream, a);
    LBM_HIP(hipGetLastError());
    return LBM_OK;
}

template <int T, typename P>
lbm_status launch_local(const LocalArgs &a, size_t lds_bytes, int grid, int cpt, hipStream_t stream,
                        int cu_budget = 0)
{
    if (cpt <= 1) return launch_local_c<T, P, 1>(a, lds_bytes, grid, stream, cu_budget);
    if (cpt <= 2) return launch_local_c<T, P, 2>(a, lds_bytes, grid, stream, cu_budget);
    return launch_local_c<T, P, kCPT>(a, lds_bytes, grid, stream, cu_budget);
}

}  // namespace
}  // namespace lbm

using namespace lbm;

extern "C" int32_t lbm_local_max_side(void) { return kMaxSide; }

extern "C" size_t lbm_local_workspace_bytes(int32_t n_patches)
{
    if (n_patches < 0) return 0;
    return local_layout(n_patches).total;
}

extern "C" lbm_status lbm_local_keff(const lbm_local_params *lp, int32_t n_patches, const int32_t *h_x0,
                                     const int32_t *h_y0, const int32_t *h_side,
                                     const int32_t *h_drive_mask, const double *d_kappa_field,
                                     int32_t fnx, int32_t fny, double *d_keff, int32_t *d_steps,
                                     int32_t *d_flags, const lbm_local_tile *tiles, int32_t n_tiles,
                                     int32_t block_threads, void *d_ws, size_t ws_bytes,
                                     hipStream_t stream)
{
    const char *fn = "lbm_local_keff: ";
    if (!lp) return set_error(LBM_EINVAL, std::string(fn) + "params is NULL");
    if (!(lp->tau >= 0.5) || !std::isfinite(lp->tau)) return set_error(LBM_EINVAL, std::string(fn) + "tau must be >= 0.5");
    if (!(lp->eps > 0.0 && lp->eps <= 1.0)) return set_error(LBM_EINVAL, std::string(fn) + "eps must lie in (0, 1]");
    if (!(lp->nu > 0.0) || !std::isfinite(lp->nu)) return set_error(LBM_EINVAL, std::string(fn) + "nu must be > 0");
    if (!(lp->g > 0.0) || !std::isfinite(lp->g)) return set_error(LBM_EINVAL, std::string(fn) + "g must be > 0");
    if (!(lp->tol >= 0.0)) return set_error(LBM_EINVAL, std::string(fn) + "tol must be >= 0");
    if (lp->check_every < 2 || (lp->check_every & 1))
        return set_error(LBM_EINVAL, std::string(fn) + "check_every must be even and >= 2");
    if (lp->max_steps < 1 || lp->max_steps > (int64_t)1 << 30)
        return set_error(LBM_EINVAL, std::string(fn) + "max_steps must lie in [1, 2^30]");
    if (lp->pop_dtype != LBM_F32_SHIFTED && lp->pop_dtype != LBM_F64)
        return set_error(LBM_EINVAL, std::string(fn) + "unknown pop_dtype");
    if (lp->avg_margin < 0) return set_error(LBM_EINVAL, std::string(fn) + "avg_margin must be >= 0");
    if (lp->schedule != LBM_SCHEDULE_GIVEN && lp->schedule != LBM_SCHEDULE_COST)
        return set_error(LBM_EINVAL, std::string(fn) + "unknown schedule");
    if (lp->fp32_step_budget < 0) return set_error(LBM_EINVAL, std::string(fn) + "fp32_step_budget must be >= 0");
    if (n_patches < 0) return set_error(LBM_EINVAL, std::string(fn) + "n_patches < 0");
    if (n_patches == 0) return LBM_OK;
    if (!h_x0 || !h_y0 || !h_side || !h_drive_mask || !d_kappa_field || !d_keff)
        return set_error(LBM_EINVAL, std::string(fn) + "NULL array");
    if (fnx < 1 || fny < 1) return set_error(LBM_EINVAL, std::string(fn) + "field sides must be >= 1");
    if (block_threads == 0) block_threads = 1024;
    if (block_threads != 256 && block_threads != 512 && block_threads != 1024)
        return set_error(LBM_EINVAL, std::string(fn) + "block_threads must be 256, 512 or 1024");
    if (n_tiles < 0 || (n_tiles > 0 && !tiles)) return set_error(LBM_EINVAL, std::string(fn) + "bad tile table");
    const LocalLayout L = local_layout(n_patches);
    if (!d_ws || ((uintptr_t)d_ws % kAlign) != 0 || ws_bytes < L.total)
        return set_error(LBM_EWORKSPACE, std::string(fn) + "workspace NULL, misaligned or smaller than " +
                                             std::to_string(L.total));

    // items, grouped by side (largest first), drives of one patch adjacent
    std::vector<int> order(n_patches);
    std::iota(order.begin(), order.end(), 0);
    for (int i = 0; i < n_patches; ++i) {
        if (h_side[i] < 1 || h_side[i] > kMaxSide)
            return set_error(LBM_EINVAL, std::string(fn) + "patch side must lie in [1, 64]");
        if (h_side[i] - 2 * lp->avg_margin < 1)
            return set_error(LBM_EINVAL, std::string(fn) + "avg_margin leaves no inner window");
        if (h_drive_mask[i] < 0 || h_drive_mask[i] > 3)
            return set_error(LBM_EINVAL, std::string(fn) + "drive mask must be 0..3");
    }
    std::stable_sort(order.begin(), order.end(), [&](int p, int q) { return h_side[p] > h_side[q]; });
    std::vector<int4> items;
    items.reserve(2 * (size_t)n_patches);
    std::vector<ClassDesc> classes;
    const bool f64 = lp->pop_dtype == LBM_F64;
    // FP64 state needs twice the registers: at most 512 threads per workgroup
    const int T = f64 ? std::min(block_threads, 512) : block_threads;
    const size_t cb = f64 ? 64 : 32;  // LDS bytes per cell (populations 1..8)
    const int budget = lds_budget_bytes() - 2048;
    for (int i : order) {
        const int s = h_side[i];
        if (classes.empty() || classes.back().side != s) {
            ClassDesc c{};
            c.side = s;
            c.begin = (int)items.size();
            int G = 0;
            for (int t = 0; t < n_tiles; ++t)
                if (tiles[t].side == s && !(f64 && tiles[t].slot_threads > T)) G = tiles[t].slot_threads;
            const int cells = s * s;
            if (G == 0) {
                const int gmin = pow2_at_least((cells + kCPT - 1) / kCPT);
                const int fit = std::max(1, budget / (int)(cb * cells));
                G = std::max(gmin, pow2_at_least((T + fit - 1) / fit));
                G = std::min(G, T);
            }
            if (G < 64 || (G & 63) || G > T || (T % G))
                return set_error(LBM_EINVAL, std::string(fn) + "slot_threads must be a multiple of 64 dividing block_threads");
            c.slot_threads = G;
            c.cells_per_thread = (cells + G - 1) / G;
            if (c.cells_per_thread > kCPT)
                return set_error(LBM_EINVAL, std::string(fn) + "tile leaves more than 4 cells per thread (side " +
                                                     std::to_string(s) + ")");
            c.nslots = T / G;
            while (c.nslots > 1 && (size_t)c.nslots * cb * cells > (size_t)budget) --c.nslots;
            if (cb * cells > (size_t)budget)
                return set_error(LBM_EINVAL, std::string(fn) + "patch of side " + std::to_string(s) +
                                                     " does not fit in LDS");
            classes.push_back(c);
        }
        for (int d = 0; d < 2; ++d)
            if (h_drive_mask[i] & (1 << d)) items.push_back(make_int4(h_x0[i] % fnx, h_y0[i] % fny, s, 2 * i + d));
        classes.back().count = (int)items.size() - classes.back().begin;
    }
    // drop classes without items (all drives masked)
    classes.erase(std::remove_if(classes.begin(), classes.end(), [](const ClassDesc &c) { return c.count == 0; }),
                  classes.end());
    // The largest sides (one item per workgroup over all its threads, more
    // than one cell per thread, never eligible for the FP64 re-run, whose
    // layout cannot hold them) share one queue, so that their items start in
    // one longest-predicted-first order across the sides: in queues of their
    // own, a long item of a smaller side waits until the larger side's queue
    // is empty. Their items lie next to each other in the list (sorted by
    // side), and each takes its own side from its entry.
    if (!f64) {
        std::vector<ClassDesc> m;
        bool prev_whole = false;
        for (const ClassDesc &c : classes) {
            const int cells = c.side * c.side;
            const int ge = std::min(kEscThreads, std::max(64, pow2_at_least(cells)));
            const bool whole = c.nslots == 1 && c.slot_threads == T && c.cells_per_thread > 1 &&
                               ((cells + ge - 1) / ge > kCPT || (size_t)64 * cells > (size_t)budget);
            if (whole && prev_whole) {
                m.back().count += c.count;
                m.back().merged = 1;
                m.back().cells_per_thread = std::max(m.back().cells_per_thread, c.cells_per_thread);
            } else {
                m.push_back(c);
            }
            prev_whole = whole;
        }
        classes.swap(m);
    }
    if ((int)classes.size() > kMaxClasses) return set_error(LBM_EINVAL, std::string(fn) + "too many sides");
    for (const int4 &it : items)
        if (it.x < 0 || it.y < 0) return set_error(LBM_EINVAL, std::string(fn) + "origins must be >= 0");

    char *ws = static_cast<char *>(d_ws);
    int4 *d_items = reinterpret_cast<int4 *>(ws + L.off_items);
    ClassDesc *d_classes = reinterpret_cast<ClassDesc *>(ws + L.off_classes);
    int *d_counters = reinterpret_cast<int *>(ws + L.off_counters);
    int *d_mask = reinterpret_cast<int *>(ws + L.off_mask);
    if (!items.empty())
        LBM_HIP(hipMemcpyAsync(d_items, items.data(), sizeof(int4) * items.size(), hipMemcpyHostToDevice, stream));
    if (!classes.empty())
        LBM_HIP(hipMemcpyAsync(d_classes, classes.data(), sizeof(ClassDesc) * classes.size(),
                               hipMemcpyHostToDevice, stream));
    LBM_HIP(hipMemcpyAsync(d_mask, h_drive_mask, sizeof(int) * n_patches, hipMemcpyHostToDevice, stream));
    const int nfill = std::max(n_patches, kNumCounters);
    hipLaunchKernelGGL(k_local_prefill, dim3((nfill + 255) / 256), dim3(256), 0, stream, n_patches, d_mask,
                       d_keff, d_steps, d_flags, d_counters, kNumCounters);
    LBM_HIP(hipGetLastError());
    if (items.empty()) return LBM_OK;
    const int4 *d_run = d_items;
    if (lp->schedule == LBM_SCHEDULE_COST) {
        const int ni = (int)items.size();
        int *d_hist = d_counters + kMaxClasses, *d_cursor = d_hist + kHist;
        int *d_keys = reinterpret_cast<int *>(ws + L.off_keys);
        int4 *d_sorted = reinterpret_cast<int4 *>(ws + L.off_sorted);
        const double kPi = 3.14159265358979323846;
        hipLaunchKernelGGL(k_local_cost, dim3(ni), dim3(256), 0, stream, d_items, d_classes,
                           (int)classes.size(), d_kappa_field, fnx, fny, 1.0 / (lp->eps * lp->nu),
                           lp->eps * lp->nu * 3.0 / (kPi * kPi), d_keys, d_hist);
        LBM_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_local_scan, dim3(1), dim3(256), 0, stream, d_hist, d_cursor,
                           (int)classes.size() * kCostBins);
        LBM_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_local_scatter, dim3((ni + 255) / 256), dim3(256), 0, stream, ni, d_items, d_keys,
                           d_cursor, d_sorted);
        LBM_HIP(hipGetLastError());
        d_run = d_sorted;
    }

    LocalArgs a{};
    a.items = d_run;
    a.classes = d_classes;
    a.nclasses = (int)classes.size();
    a.counters = d_counters;
    a.field = d_kappa_field;
    a.fnx = fnx;
    a.fny = fny;
    a.keff = d_keff;
    a.steps_out = d_steps;
    a.flags_out = d_flags;
    a.om = (float)(1.0 / lp->tau);
    a.omc = 1.0f - a.om;  // exact for tau in [1/2, 2]: om + omc = 1 in FP32
    a.twotau = (float)(2.0 * lp->tau);
    a.omtt = (float)(1.0 - 2.0 * lp->tau);
    a.heg = (float)(0.5 * lp->eps * lp->g);
    a.heg_d = 0.5 * lp->eps * lp->g;
    a.om_d = 1.0 / lp->tau;
    a.omc_d = 1.0 - 1.0 / lp->tau;
    a.twotau_d = 2.0 * lp->tau;
    a.omtt_d = 1.0 - 2.0 * lp->tau;
    a.h = 0.5 * lp->eps * lp->nu;
    a.nu_over_g = lp->nu / lp->g;
    a.tol = lp->tol;
    a.check_every = lp->check_every;
    a.margin = lp->avg_margin;
    const int64_t ms = (lp->max_steps + lp->check_every - 1) / lp->check_every * lp->check_every;
    a.max_steps = (int)std::min<int64_t>(ms, (int64_t)1 << 30);
    // FP32 step budget (FP32 state only): rounded up to a check; a budget at
    // or beyond the step cap never triggers
    const bool escalate = !f64 && lp->fp32_step_budget > 0 &&
                          (int64_t)lp->fp32_step_budget < (int64_t)a.max_steps;
    a.esc_steps = escalate ? (int)((lp->fp32_step_budget + lp->check_every - 1) / lp->check_every *
                                   lp->check_every)
                           : 0;
    // One persistent launch per register shape: each is compiled for the most
    // cells any of its threads owns (1, 2 or 4), since a launch for single
    // cells keeps fewer registers live and fits two workgroups per CU. When a
    // call mixes single-cell sides with larger ones, the single-cell sides run
    // in a launch of their own on a second stream beside the others (joined
    // back to the caller's stream before the call's later work); run one
    // after the other, the two launches were slower than one launch for all.
    // Within a launch, the classes keep their order (largest side first), and
    // there is one workgroup per concurrent slot-set, no more than the items
    // need.
    std::vector<ClassDesc> grouped;
    grouped.reserve(classes.size());
    for (const ClassDesc &c : classes)
        if (c.cells_per_thread > 1) grouped.push_back(c);
    const int n_multi = (int)grouped.size();
    for (const ClassDesc &c : classes)
        if (c.cells_per_thread <= 1) grouped.push_back(c);
    // The FP64 re-run of items past the FP32 step budget: one class per
    // grouped class (same item ranges, in a queue of its own), laid out for
    // FP64 state on kEscThreads threads with as many threads per item as the
    // side allows (the re-run items are few and long, so per-item latency
    // matters more than items per CU); sides whose FP64 state does not fit
    // stay in FP32.
    std::vector<ClassDesc> esc(grouped.size());
    size_t esc_lds = 0;
    int esc_cpt = 1;
    for (size_t i = 0; i < grouped.size(); ++i) {
        ClassDesc c = grouped[i];
        const int cells = c.side * c.side;
        const int G = std::min(kEscThreads, std::max(64, pow2_at_least(cells)));
        c.slot_threads = G;
        c.cells_per_thread = (cells + G - 1) / G;
        c.nslots = kEscThreads / G;
        c.count = 0;  // filled by the FP32 launch
        c.esc_ok = escalate && c.cells_per_thread <= kCPT && (size_t)64 * cells <= (size_t)budget;
        while (c.nslots > 1 && (size_t)c.nslots * 64 * cells > (size_t)budget) --c.nslots;
        if (c.esc_ok) {
            esc_lds = std::max(esc_lds, (size_t)c.nslots * 64 * cells);
            esc_cpt = std::max(esc_cpt, c.cells_per_thread);
        }
        grouped[i].esc_ok = c.esc_ok;
        esc[i] = c;
    }
    const bool any_esc = std::any_of(esc.begin(), esc.end(), [](const ClassDesc &c) { return c.esc_ok != 0; });
    ClassDesc *d_grouped = d_classes + kMaxClasses;
    LBM_HIP(hipMemcpyAsync(d_grouped, grouped.data(), sizeof(ClassDesc) * grouped.size(), hipMemcpyHostToDevice,
                           stream));
    ClassDesc *d_esc = reinterpret_cast<ClassDesc *>(ws + L.off_esc_classes);
    int *d_esc_counters = reinterpret_cast<int *>(ws + L.off_esc_counters);
    int4 *d_esc_items = reinterpret_cast<int4 *>(ws + L.off_esc_items);
    if (any_esc) {
        LBM_HIP(hipMemcpyAsync(d_esc, esc.data(), sizeof(ClassDesc) * esc.size(), hipMemcpyHostToDevice, stream));
        LBM_HIP(hipMemsetAsync(d_esc_counters, 0, sizeof(int) * esc.size(), stream));
    }
    auto launch_group = [&](int first, int count, hipStream_t st, int cu_budget) -> lbm_status {
        LocalArgs g = a;
        g.classes = d_grouped + first;
        g.nclasses = count;
        g.counters = d_counters + first;
        g.esc_classes = d_esc + first;
        g.esc_items = d_esc_items;
        int cmax = 1, need = 0;
        size_t lds = 0;
        for (int i = first; i < first + count; ++i) {
            const ClassDesc &c = grouped[i];
            cmax = std::max(cmax, c.cells_per_thread);
            need = std::max(need, (c.count + c.nslots - 1) / c.nslots);
            lds = std::max(lds, (size_t)c.nslots * cb * c.side * c.side);
        }
        const int cpt = cmax <= 1 ? 1 : (cmax <= 2 ? 2 : 4);
        const int grid = std::max(1, need);
        if (f64)
            return (T == 256) ? launch_local<256, double>(g, lds, grid, cpt, st, cu_budget)
                              : launch_local<512, double>(g, lds, grid, cpt, st, cu_budget);
        if (T == 256) return launch_local<256, float>(g, lds, grid, cpt, st, cu_budget);
        if (T == 512) return launch_local<512, float>(g, lds, grid, cpt, st, cu_budget);
        return launch_local<1024, float>(g, lds, grid, cpt, st, cu_budget);
    };
    // The FP64 re-run, queued on `stream` after the FP32 launch(es): a
    // persistent launch over the re-run queues, whose workgroups leave at
    // once when the queues are empty.
    auto launch_esc = [&]() -> lbm_status {
        if (!any_esc) return LBM_OK;
        LocalArgs e = a;
        e.items = d_esc_items;
        e.classes = d_esc;
        e.nclasses = (int)esc.size();
        e.counters = d_esc_counters;
        e.esc_steps = 0;
        e.esc_classes = nullptr;
        e.esc_items = nullptr;
        int potential = 0;  // workgroups the queues could use at most
        for (size_t i = 0; i < esc.size(); ++i)
            if (esc[i].esc_ok) potential = std::max(potential, (grouped[i].count + esc[i].nslots - 1) / esc[i].nslots);
        const int cpt = esc_cpt <= 1 ? 1 : (esc_cpt <= 2 ? 2 : 4);
        return launch_local<kEscThreads, double>(e, esc_lds, std::max(1, potential), cpt, stream);
    };
    const int n_single = (int)grouped.size() - n_multi;
    hipStream_t side = (n_multi > 0 && n_single > 0) ? side_stream() : nullptr;
    if (!side) {
        const lbm_status st = launch_group(0, (int)grouped.size(), stream, 0);
        if (st != LBM_OK) return st;
        return launch_esc();
    }
    // CUs for the single-cell launch in proportion to its share of the cells
    // (step counts are not known here); 256-CU parts only, else both launches
    // share all CUs
    double w_multi = 0.0, w_single = 0.0;
    for (int i = 0; i < (int)grouped.size(); ++i)
        for (int j = grouped[i].begin; j < grouped[i].begin + grouped[i].count; ++j)
            (i < n_multi ? w_multi : w_single) += (double)items[j].z * items[j].z;
    const int k = (int)std::lround(w_single / (w_multi + w_single) * (32.0 / kSplitStep)) * kSplitStep;
    hipStream_t s_multi = stream, s_single = side;
    int cu_multi = 0, cu_single = 0;
    if (split_streams(k, &s_multi, &s_single)) {
        cu_single = 8 * k;
        cu_multi = 256 - cu_single;
    } else {
        s_multi = stream;
        s_single = side;
    }
    hipEvent_t fork = nullptr, join = nullptr, join2 = nullptr;
    LBM_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    if (hipEventCreateWithFlags(&join, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&join2, hipEventDisableTiming) != hipSuccess) {
        (void)hipEventDestroy(fork);
        if (join) (void)hipEventDestroy(join);
        return set_error(LBM_EDEVICE, std::string(fn) + "hipEventCreateWithFlags failed");
    }
    lbm_status st = LBM_OK;
    hipError_t e = hipEventRecord(fork, stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(s_single, fork, 0);
    if (e == hipSuccess && s_multi != stream) e = hipStreamWaitEvent(s_multi, fork, 0);
    if (e == hipSuccess) {
        st = launch_group(0, n_multi, s_multi, cu_multi);
        if (st == LBM_OK) st = launch_group(n_multi, n_single, s_single, cu_single);
        // join even after a failed launch, so the caller's stream never runs
        // ahead of work queued on the other streams
        e = hipEventRecord(join, s_single);
        if (e == hipSuccess) e = hipStreamWaitEvent(stream, join, 0);
        if (e == hipSuccess && s_multi != stream) {
            e = hipEventRecord(join2, s_multi);
            if (e == hipSuccess) e = hipStreamWaitEvent(stream, join2, 0);
        }
    }
    (void)hipEventDestroy(fork);
    (void)hipEventDestroy(join);
    (void)hipEventDestroy(join2);
    if (st != LBM_OK) return st;
    if (e != hipSuccess) return hip_check(e, "lbm_local_keff: stream fork/join");
    return launch_esc();
}
