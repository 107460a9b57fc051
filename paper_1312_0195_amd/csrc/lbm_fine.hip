// lbm_fine.hip -- fine-grid solver of liblbm (Sec. 2.2 of the paper).
//
// A time step is a pull: every cell pulls its nine incoming post-collision
// populations from its neighbours (streaming of Eq. f-evolution-of-S-C read
// backwards), collides them in registers and writes the nine new
// post-collision values to its own cell. k_step does one step per pass over
// HBM; k_stepd does D = 2, 4 or 6 steps per pass, the intermediate steps
// staying in LDS (temporal blocking, bit-identical to D single steps).
// The state in memory is therefore the post-collision populations of the
// previous step; the pre-collision populations at the current step are the
// pulled ones, which is what lbm_fields and lbm_get_populations report.
//
// Storage: structure of arrays, plane a holds population a for all cells
// (x fastest), so each of the 9 loads and 9 stores of a wavefront is 64
// consecutive elements. FP32 planes store deviations f_a - w_a rho0 from the
// rest state: the velocity signal is ~1e-5 of a population, and storing the
// deviations keeps FP32 rounding relative to the signal, not to w_a rho0.
//
// Collision in deviation form, with dr = sum f~, j = sum e f~, rho = rho0 + dr:
//   rho u    = D (j + eps rho G / 2)                  Eq. explicit-u-in-Guo
//   rho u_eq = 2 tau rho u + (1 - 2 tau) j            Eq. final-ueq-of-S-C
//   f~eq_a   = w_a (dr + 3 e_a . rho u_eq)            Eq. feq minus w_a rho0
//   f~*_a    = f~_a + (f~eq_a - f~_a) / tau           Eq. f-evolution-of-S-C
// with D = 1 / (1 + eps nu / (2 kappa)) per cell, or, for a tensor
// permeability K, rho u = (K + eps nu I / 2)^{-1} K (j + eps rho G / 2) (Eq.
// u-of-S-C with Eq. f_m-depends-on-u-and-tensor-k). No division is needed in
// the step. The coefficient planes hold the drag deficit E = 1 - D =
// h / (kappa + h), h = eps nu / 2 (tensor: I - M = h (K + h I)^{-1}), not D:
// rounded to FP32, D would lose the relative precision of the drag 1 - D in
// permeable cells (its absolute rounding error 2^-25 is 2e-4 of 1 - D at
// kappa = 130, eps nu = 0.04), E keeps it; D = 1 - E is formed in FP64. The algebra is exact; only the rounding order differs from a
// literal transcription. The collision arithmetic is FP64 for both storage
// types; FP32 storage only rounds the nine values written per cell.
#include <hip/hip_runtime.h>

#include <array>

#include <cmath>
#include <cstring>
#include <algorithm>
#include <new>
#include <type_traits>

#include "lbm_internal.h"

namespace lbm {
namespace {

constexpr int kBlock = 256;
constexpr size_t kPlanePadBytes = 16384;

template <typename R>
struct StepArgs {
    const R *__restrict__ fin;
    R *__restrict__ fout;
    const R *__restrict__ coef;    // perm_kind planes of cstride elements
    const R *__restrict__ hforce;  // 2 planes: eps G / 2 per cell (or null)
    int nx, ny;
    int stride;   // plane stride of the populations, elements
    int cstride;  // plane stride of coef / hforce, elements
    R om;         // 1 / tau
    R omc;        // 1 - 1 / tau
    R twotau;     // 2 tau
    R omtt;       // 1 - 2 tau
    R hegx, hegy; // eps G / 2 for a uniform force
    R rho0;
    // FP64 copies of the constants for the FP64 arithmetic
    double hegx_d, hegy_d, om_d, omc_d, twotau_d, omtt_d, rho0_d;
};

// The relaxation constants in the arithmetic type A of a collision: FP64
// arithmetic uses the FP64 copies, FP32 arithmetic the storage-type ones.
template <typename A, typename R>
struct Kc {
    A om, omc, twotau, omtt, hegx, hegy, rho0;
    A hegx2, hegy2;  // 2 hegx, 2 hegy (exact)
    __device__ explicit Kc(const StepArgs<R> &a)
    {
        if constexpr (sizeof(A) == 8) {
            om = a.om_d; omc = a.omc_d; twotau = a.twotau_d; omtt = a.omtt_d;
            hegx = a.hegx_d; hegy = a.hegy_d; rho0 = a.rho0_d;
        } else {
            om = (A)a.om; omc = (A)a.omc; twotau = (A)a.twotau; omtt = (A)a.omtt;
            hegx = (A)a.hegx; hegy = (A)a.hegy; rho0 = (A)a.rho0;
        }
        hegx2 = hegx + hegx;
        hegy2 = hegy + hegy;
    }
};

// Plane accessors: element i of plane q of an SoA array with a plane stride.
// GMem indexes through a 64-bit pointer per lane. BMem goes through a buffer
// resource per plane, built in scalar registers from the (uniform) plane base,
// so a lane only supplies a 32-bit byte offset: this removes the 64-bit
// address arithmetic from the VALU. An offset past the plane reads zero and a
// store there is dropped (the hardware bounds check of raw buffer accesses).
// Plane bytes stay below 2^31 (the grid-size limit of params_ok).
template <typename R>
struct GMem {
    const R *p;
    R *w;
    int stride;
    __device__ R ld(int q, int i) const { return p[(size_t)q * stride + i]; }
    __device__ void st(int q, int i, R v) const { w[(size_t)q * stride + i] = v; }
};

template <typename R>
struct BMem {
    const R *p;
    R *w;
    int stride;
    static constexpr int kFlags = 0x00020000;  // gfx9 dword 3: 32-bit data format
    __device__ R ld(int q, int i) const
    {
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(p + (size_t)q * stride), 0, stride * (int)sizeof(R), kFlags);
        if constexpr (sizeof(R) == 4)
            return __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b32(r, i * 4, 0, 0));
        else
            return __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b64(r, i * 8, 0, 0));
    }
    __device__ void st(int q, int i, R v) const
    {
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(w + (size_t)q * stride), 0, stride * (int)sizeof(R), kFlags);
        if constexpr (sizeof(R) == 4)
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, i * 4, 0, 0);
        else
            __builtin_amdgcn_raw_buffer_store_b64(
                __builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)), v), r, i * 8, 0, 0);
    }
};

// Pull the nine pre-collision deviations of cell (x, y): f_a(x) = f*_a(x - e_a)
// from the previous step, with periodic wrap in x (and in y without walls)
// and halfway bounce-back f_a(x) = f*_opp(a)(x) where x - e_a is beyond a wall.
template <typename R, bool WALLS>
__device__ __forceinline__ void pull(const R *__restrict__ fin, int stride, int nx, int ny, int x,
                                     int y, R f[9])
{
    const int xm = (x == 0) ? nx - 1 : x - 1;
    const int xp = (x == nx - 1) ? 0 : x + 1;
    const int rc = y * nx;
    const R *p0 = fin;
    const R *p1 = fin + stride;
    const R *p2 = fin + 2 * (size_t)stride;
    const R *p3 = fin + 3 * (size_t)stride;
    const R *p4 = fin + 4 * (size_t)stride;
    const R *p5 = fin + 5 * (size_t)stride;
    const R *p6 = fin + 6 * (size_t)stride;
    const R *p7 = fin + 7 * (size_t)stride;
    const R *p8 = fin + 8 * (size_t)stride;
    f[0] = p0[rc + x];
    f[1] = p1[rc + xm];
    f[3] = p3[rc + xp];
    if (WALLS) {
        const bool lo = (y == 0), hi = (y == ny - 1);
        const int rm = (lo ? y : y - 1) * nx;
        const int rp = (hi ? y : y + 1) * nx;
        f[2] = lo ? p4[rc + x] : p2[rm + x];
        f[5] = lo ? p7[rc + x] : p5[rm + xm];
        f[6] = lo ? p8[rc + x] : p6[rm + xp];
        f[4] = hi ? p2[rc + x] : p4[rp + x];
        f[7] = hi ? p5[rc + x] : p7[rp + xp];
        f[8] = hi ? p6[rc + x] : p8[rp + xm];
    } else {
        const int rm = ((y == 0) ? ny - 1 : y - 1) * nx;
        const int rp = ((y == ny - 1) ? 0 : y + 1) * nx;
        f[2] = p2[rm + x];
        f[5] = p5[rm + xm];
        f[6] = p6[rm + xp];
        f[4] = p4[rp + x];
        f[7] = p7[rp + xp];
        f[8] = p8[rp + xm];
    }
}

// pull through a plane accessor (same indices as pull)
template <typename R, bool WALLS, class M>
__device__ __forceinline__ void pullm(const M &in, int nx, int ny, int x, int y, R f[9])
{
    const int xm = (x == 0) ? nx - 1 : x - 1;
    const int xp = (x == nx - 1) ? 0 : x + 1;
    const int rc = y * nx;
    f[0] = in.ld(0, rc + x);
    f[1] = in.ld(1, rc + xm);
    f[3] = in.ld(3, rc + xp);
    if (WALLS) {
        const bool lo = (y == 0), hi = (y == ny - 1);
        const int rm = (lo ? y : y - 1) * nx;
        const int rp = (hi ? y : y + 1) * nx;
        f[2] = lo ? in.ld(4, rc + x) : in.ld(2, rm + x);
        f[5] = lo ? in.ld(7, rc + x) : in.ld(5, rm + xm);
        f[6] = lo ? in.ld(8, rc + x) : in.ld(6, rm + xp);
        f[4] = hi ? in.ld(2, rc + x) : in.ld(4, rp + x);
        f[7] = hi ? in.ld(5, rc + x) : in.ld(7, rp + xp);
        f[8] = hi ? in.ld(6, rc + x) : in.ld(8, rp + xm);
    } else {
        const int rm = ((y == 0) ? ny - 1 : y - 1) * nx;
        const int rp = ((y == ny - 1) ? 0 : y + 1) * nx;
        f[2] = in.ld(2, rm + x);
        f[5] = in.ld(5, rm + xm);
        f[6] = in.ld(6, rm + xp);
        f[4] = in.ld(4, rp + x);
        f[7] = in.ld(7, rp + xp);
        f[8] = in.ld(8, rp + xm);
    }
}

template <typename R>
__device__ __forceinline__ void moments(const R f[9], R &dr, R &jx, R &jy)
{
    dr = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
    jx = (f[1] - f[3]) + ((f[5] - f[6]) + (f[8] - f[7]));
    jy = (f[2] - f[4]) + ((f[5] + f[6]) - (f[7] + f[8]));
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2). Renumber them so that each XCD gets one contiguous run of row
// segments: the cache lines that neighbouring segments share (x-shifted
// populations) and the rows above and below then stay in one L2.
__device__ __forceinline__ int xcd_block(int bid, int nb)
{
    constexpr int kXcd = 8;
    const int q = nb / kXcd, rem = nb % kXcd;
    const int k = bid % kXcd, slot = bid / kXcd;
    return k * q + (k < rem ? k : rem) + slot;
}

// Post-collision values of cell c in place (FP64 arithmetic): the deviation
// form of Eqs. explicit-u-in-Guo, final-ueq-of-S-C, feq, f-evolution-of-S-C.
// The Guo form (Sec. 2.1) taken literally, for the cost comparison of the two
// forms: u from Eq. explicit-u-in-Guo (one division), the drag force f_m of
// Eq. f_m-depends-on-u, f_eq at u (Eq. feq), the forcing term F_a of Eq.
// Fi-of-Guo and the update of Eq. f-evolution-of-Guo. coef holds eps nu / kappa.
template <typename R, bool FF, class CM, class FM>
__device__ __forceinline__ void collide_guo(const StepArgs<R> &a, double f[9], int c, int cf,
                                            const CM &cm, const FM &fm)
{
    double dr, jx, jy;
    moments(f, dr, jx, jy);
    const double rho = a.rho0_d + dr;
    double hgx, hgy;  // eps G / 2
    if (FF) {
        hgx = (double)fm.ld(0, cf);
        hgy = (double)fm.ld(1, cf);
    } else {
        hgx = a.hegx_d;
        hgy = a.hegy_d;
    }
    const double cnu = (double)cm.ld(0, c);
    const double den = rho * (1.0 + 0.5 * cnu);
    const double ux = (jx + hgx * rho) / den, uy = (jy + hgy * rho) / den;
    // rho f_m = rho (eps G - (eps nu / kappa) u)
    const double fmx = rho * (2.0 * hgx - cnu * ux), fmy = rho * (2.0 * hgy - cnu * uy);
    const double om = a.om_d;
    const double kf = 3.0 * (1.0 - 0.5 * om);  // (1 - 1/(2 tau)) / c_s^2
    const double ru3x = 3.0 * rho * ux, ru3y = 3.0 * rho * uy;
    // deviations: f~eq_a = w_a (dr + 3 rho e_a . u), F_a = w_a kf e_a . rho f_m
    const double w0 = 4.0 / 9.0, w1 = 1.0 / 9.0, w5 = 1.0 / 36.0;
    f[0] = f[0] + om * (w0 * dr - f[0]);
    f[1] = f[1] + om * (w1 * (dr + ru3x) - f[1]) + w1 * kf * fmx;
    f[2] = f[2] + om * (w1 * (dr + ru3y) - f[2]) + w1 * kf * fmy;
    f[3] = f[3] + om * (w1 * (dr - ru3x) - f[3]) - w1 * kf * fmx;
    f[4] = f[4] + om * (w1 * (dr - ru3y) - f[4]) - w1 * kf * fmy;
    f[5] = f[5] + om * (w5 * (dr + ru3x + ru3y) - f[5]) + w5 * kf * (fmx + fmy);
    f[6] = f[6] + om * (w5 * (dr - ru3x + ru3y) - f[6]) + w5 * kf * (fmy - fmx);
    f[7] = f[7] + om * (w5 * (dr - ru3x - ru3y) - f[7]) - w5 * kf * (fmx + fmy);
    f[8] = f[8] + om * (w5 * (dr + ru3x - ru3y) - f[8]) + w5 * kf * (fmx - fmy);
}

// Coefficient sources besides the plane accessors: one value already in a
// register, or an array in LDS indexed like the tile buffer.
template <typename R>
struct OneCoef {
    R v;
    __device__ R ld(int, int) const { return v; }
};
template <typename R>
struct LdsCoef {
    const R *p;
    __device__ R ld(int, int i) const { return p[i]; }
};

// PK: 1 scalar drag deficit E = 1 - D, 4 tensor I - M (Shan-Chen form); 0 the Guo
// form with coef = eps nu / kappa. Coefficients come from cm at index c, the
// per-cell force from fm at index cf.
// E2 (FP32 arithmetic, scalar drag): cm gives 2E, so the exact factor 2 of
// om rho u_eq is folded into the coefficient (2 fma(-E, h, g) = fma(-2E, h,
// 2g) exactly). GY false: no drive along y (hegy = 0), so hy = jy and the
// y terms of g vanish; om rho u_eq is bit for bit the same either way.
template <typename R, int PK, bool FF, bool E2 = false, bool GY = true, class CM, class FM, typename A>
__device__ __forceinline__ void collide_m(const StepArgs<R> &a, A f[9], int c, int cf, const CM &cm,
                                          const FM &fm)
{
    if constexpr (PK == 0) {
        static_assert(sizeof(A) == 8, "the Guo form runs in FP64 arithmetic");
        collide_guo<R, FF>(a, f, c, cf, cm, fm);
        return;
    } else {
    const Kc<A, R> k(a);
    A dr, jx, jy;
    moments(f, dr, jx, jy);
    const A rho = k.rho0 + dr;
    A gx, gy;  // eps rho G / 2
    if (FF) {
        gx = (A)fm.ld(0, cf) * rho;
        gy = (A)fm.ld(1, cf) * rho;
    } else {
        gx = k.hegx * rho;
        gy = k.hegy * rho;
    }
    const A hx = jx + gx, hy = jy + gy;
    const A om = k.om, omc = k.omc;
    if constexpr (sizeof(A) == 8) {
        // rho u_eq = 2 tau M h + (1 - 2 tau) j with M = I - E, formed exactly
        // enough in FP64, then the weights
        A mx, my;
        if (PK == 1) {
            const A tD = k.twotau - k.twotau * (A)cm.ld(0, c);
            mx = tD * hx + k.omtt * jx;
            my = tD * hy + k.omtt * jy;
        } else {
            const A e00 = cm.ld(0, c), e01 = cm.ld(1, c);
            const A e10 = cm.ld(2, c), e11 = cm.ld(3, c);
            mx = k.twotau * ((hx - e00 * hx) - e01 * hy) + k.omtt * jx;
            my = k.twotau * ((hy - e11 * hy) - e10 * hx) + k.omtt * jy;
        }
        // equilibrium terms: w_a om dr and 3 w_a e_a . om rho u_eq
        const A s0 = (A)(4.0 / 9.0) * om * dr;
        const A b = (A)(1.0 / 9.0) * om * dr;
        const A bx = (A)(1.0 / 3.0) * om * mx;
        const A by = (A)(1.0 / 3.0) * om * my;
        const A cc = (A)(1.0 / 36.0) * om * dr;
        const A cx = (A)(1.0 / 12.0) * om * mx;
        const A cy = (A)(1.0 / 12.0) * om * my;
        const A pp = cx + cy, qq = cx - cy;
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
        // FP32: every rounded constant that multiplies a conserved or slowly
        // relaxing quantity would bias it by a fixed fraction each step, which
        // the slow modes of the flow accumulate (measured 6.5e-5 of the
        // velocity after 20 000 steps at tau 0.8). So:
        //  * om rho u_eq = om j + 2 (eps rho G / 2 - E h): (1/tau) (2 tau) is
        //    the exact 2, not a product of two rounded constants;
        //  * the rest weight and the diagonal momentum weight are remainders,
        //    so the nine terms sum to om dr and om rho u_eq up to unbiased
        //    rounding (the subtraction in cx is exact by Sterbenz's lemma);
        //  * omc = 1 - om exactly (set on the host);
        //  * every fused multiply-add written out and no other contraction,
        //    so all kernels that inline this (interior and edge paths, one and
        //    several steps per launch) round alike.
#pragma clang fp contract(off)
        // h = j + eps rho G / 2 with one rounding (g x rho fused into the sum)
        const A gcx = FF ? (A)fm.ld(0, cf) : k.hegx, gcy = FF ? (A)fm.ld(1, cf) : k.hegy;
        const A hxf = __builtin_fmaf(gcx, rho, jx), hyf = __builtin_fmaf(gcy, rho, jy);
        A tx, ty;  // 2 (eps rho G / 2 - E h)
        if constexpr (PK == 1 && E2) {
            static_assert(!FF, "the doubled coefficient is for a uniform drive");
            const A e2 = (A)cm.ld(0, c);  // 2E
            tx = __builtin_fmaf(-e2, hxf, k.hegx2 * rho);
            ty = GY ? __builtin_fmaf(-e2, hyf, k.hegy2 * rho) : -e2 * jy;
        } else if constexpr (PK == 1) {
            const A e = (A)cm.ld(0, c);
            tx = (A)2 * __builtin_fmaf(-e, hxf, gcx * rho);
            ty = (A)2 * __builtin_fmaf(-e, hyf, gcy * rho);
        } else {
            const A e00 = cm.ld(0, c), e01 = cm.ld(1, c);
            const A e10 = cm.ld(2, c), e11 = cm.ld(3, c);
            tx = (A)2 * (gcx * rho - __builtin_fmaf(e00, hxf, e01 * hyf));
            ty = (A)2 * (gcy * rho - __builtin_fmaf(e10, hxf, e11 * hyf));
        }
        const A Mx = __builtin_fmaf(om, jx, tx), My = __builtin_fmaf(om, jy, ty);
        const A D = om * dr;
        const A b = D * (A)(1.0 / 9.0);
        const A cc = D * (A)(1.0 / 36.0);
        const A s0 = __builtin_fmaf((A)-4, b + cc, D);
        // momentum: 2 t3 M on the axes and 4 c12 M on the diagonals, with t3
        // = fl(1/3) and c12 = (1 - 2 t3) / 4 exact in FP32: they sum to M
        // exactly, each term rounded once
        constexpr A t3 = (A)1 / (A)3, c12 = ((A)1 - (A)2 * t3) * (A)0.25;
        const A cx = Mx * c12, cy = My * c12;
        const A pp = cx + cy, qq = cx - cy;
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
}

// Collision of lattice cell c with coefficients and force read through plane
// accessors of type M.
template <typename R, int PK, bool FF, class M = GMem<R>, typename A>
__device__ __forceinline__ void collide_cell(const StepArgs<R> &a, A f[9], int c)
{
    const M cm{a.coef, nullptr, a.cstride}, fm{a.hforce, nullptr, a.cstride};
    collide_m<R, PK, FF>(a, f, c, c, cm, fm);
}

// One time step per launch: pull, collide, store (one HBM pass).
template <typename R, bool WALLS, int PK, bool FF, typename A = double>
__global__ __launch_bounds__(kBlock) void k_step(StepArgs<R> a)
{
    const int bid = xcd_block(blockIdx.x, gridDim.x);
    const int nbx = (a.nx + kBlock - 1) / kBlock;
    const int y = bid / nbx;
    const int x = (bid - y * nbx) * kBlock + threadIdx.x;
    if (x >= a.nx) return;
    R fr[9];
    pull<R, WALLS>(a.fin, a.stride, a.nx, a.ny, x, y, fr);
    const int c = y * a.nx + x;
    // The arithmetic runs in FP64 whatever the storage type (LBM_F32_SHIFTED,
    // LBM_F64), or in FP32 with FP32 storage (LBM_F32_FAST).
    A f[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = (A)fr[i];
    collide_cell<R, PK, FF>(a, f, c);
    R *o = a.fout;
    const size_t S = (size_t)a.stride;
#pragma unroll
    for (int q = 0; q < 9; ++q) o[q * S + c] = (R)f[q];
}

// Tiles of the multi-step kernel, per storage type and depth D (time steps
// per launch): TX x TY output cells per workgroup of BS threads. The LDS
// holds one buffer of 9 x (TX + 2 (D - 1)) x (TY + 2 (D - 1)) values.
#ifndef LBM_DEEP
#define LBM_DEEP 6  // steps per launch of the deepest kernel (FP32 state)
#endif
#ifndef LBM_TILE6
#define LBM_TILE6 48, 24, 512
#endif
#ifndef LBM_TILE4
#define LBM_TILE4 64, 16, 512
#endif
template <int X, int Y, int B> struct TileShape { static constexpr int TX = X, TY = Y, BS = B; };
template <typename R, int D> struct TileD;
template <> struct TileD<float, 2> : TileShape<64, 64, 1024> {};
template <> struct TileD<float, 4> : TileShape<LBM_TILE4> {};
template <> struct TileD<float, LBM_DEEP> : TileShape<LBM_TILE6> {};
constexpr int kDeep = LBM_DEEP;
static_assert(kDeep > 4, "the deepest kernel must take more than 4 steps");
#ifndef LBM_TILE6D
#define LBM_TILE6D 32, 12, 256
#endif
#ifndef LBM_TILE4D
#define LBM_TILE4D 32, 16, 256
#endif
template <> struct TileD<double, 2> : TileShape<32, 16, 256> {};
template <> struct TileD<double, 4> : TileShape<LBM_TILE4D> {};
template <> struct TileD<double, LBM_DEEP> : TileShape<LBM_TILE6D> {};
// Per arithmetic type A: FP32 collision arithmetic needs 61 VGPRs where FP64
// needs 96, so two 768-thread workgroups (24 waves) fit a CU beside each
// other's 80 KB of LDS. Measured per six-step launch on 2048^2 (us): 50 x 24
// on 768 threads 89.8, 48 x 24 90.8, 56 x 20 90.7; 48 x 24 on 512 99.3, on
// 704 103.0, on 640, 832, 896 or 1024 threads 138-153; five steps per launch
// with 56 x 24 on 768 97.6.
#ifndef LBM_TILE6F
#define LBM_TILE6F 50, 24, 768
#endif
#ifndef LBM_TILE4F
#define LBM_TILE4F 64, 20, 768  // four-step launches (us, 2048^2): 81.0 against 88.6 for 64 x 16 on 512
#endif
template <typename R, int D, typename A> struct TileDA : TileD<R, D> {};
template <> struct TileDA<float, LBM_DEEP, float> : TileShape<LBM_TILE6F> {};
template <> struct TileDA<float, 4, float> : TileShape<LBM_TILE4F> {};
#ifndef LBM_TILE2F
#define LBM_TILE2F 96, 18, 768  // two-step launches (us, 2048^2): 66.0 against 74.3 for 64 x 64 on 1024
#endif
template <> struct TileDA<float, 2, float> : TileShape<LBM_TILE2F> {};
// Seven steps per launch, FP32 collision arithmetic only (the depth the
// launch planner takes for most steps of that path): per launch on 2048^2
// (us) 36 x 28 on 768 threads 98.8 (14.1 per step against 14.9 at six
// steps), 48 x 22 99.9, 40 x 26 101.3, 42 x 24 102.7, 44 x 22 104.7,
// 32 x 32 105.4; eight steps with 30 x 30 120.4.
constexpr int kDeeper = 7;
#ifndef LBM_TILE7F
#define LBM_TILE7F 36, 28, 768
#endif
template <> struct TileDA<float, kDeeper, float> : TileShape<LBM_TILE7F> {};

// D time steps per launch (temporal blocking). Phase 1 takes step t on the
// workgroup's tile plus a (D - 1)-cell halo, pulling from HBM and keeping the
// post-collision values in LDS, rounded to the storage type exactly as a
// store to HBM would round them; phases 2 .. D - 1 take the next steps on
// regions that shrink by one cell per step, in place in LDS; phase D takes the
// last step on the tile and writes to HBM. The result is bit-identical to D
// one-step launches while HBM sees one read and one write of the state per D
// steps (plus the halo, which neighbouring tiles mostly find in L2). Loads and
// stores go through BMem (32-bit offsets, plane bases in scalar registers).
template <typename R, bool WALLS, int PK, bool FF, int D, typename A = double, bool GY = true>
__global__ __launch_bounds__((TileDA<R, D, A>::BS)) void k_stepd(StepArgs<R> a)
{
    constexpr int TX = TileDA<R, D, A>::TX, TY = TileDA<R, D, A>::TY, BS = TileDA<R, D, A>::BS;
    constexpr int H = D - 1;
    constexpr int AX = TX + 2 * H, AY = TY + 2 * H, AN = AX * AY;
    constexpr int KM = (D > 2) ? ((AX - 2) * (AY - 2) + BS - 1) / BS : 1;  // cells per thread, phase 2
    // scalar coefficients without a force field are read once from HBM and
    // kept in LDS next to the populations
    constexpr bool CL = (PK != 4) && !FF && 10 * AN * sizeof(R) <= 160 * 1024;
    // FP32 arithmetic keeps 2E there (the exact factor 2 of the collision)
    constexpr bool E2 = CL && PK == 1 && sizeof(A) == 4 && sizeof(R) == 4;
    static_assert(GY || E2, "the variant without a y drive is the FP32 scalar one");
    __shared__ R P[9][AN];
    __shared__ R Dl[CL ? AN : 1];
    const int nx = a.nx, ny = a.ny;
    const int ntx = (nx + TX - 1) / TX;
    const int bid = xcd_block(blockIdx.x, gridDim.x);
    const int y0 = (bid / ntx) * TY, x0 = (bid % ntx) * TX;
    const int tw = min(TX, nx - x0), th = min(TY, ny - y0);  // ragged tiles at the far edges
    const BMem<R> mem{a.fin, a.fout, a.stride};
    // Interior tiles (most of a large grid): every cell the launch touches,
    // including the neighbours phase 1 pulls from, lies inside the grid away
    // from the walls, so no wrap, wall or ragged-edge test is needed.
    const bool interior = tw == TX && th == TY && x0 >= H + 1 && x0 + TX + H <= nx - 1 &&
                          y0 >= H + 1 && y0 + TY + H <= ny - 1;
    // lattice cell of P coordinate (px, py); false beyond a wall
    // (x0 - H + px lies in [-H, nx + H): one wrap suffices unless the grid
    // is narrower than the halo)
    const bool wide = nx > H, tall = ny > H;
    auto cell_of = [&](int px, int py, int &x, int &y) -> bool {
        x = x0 - H + px;
        if (wide) {
            x = x < 0 ? x + nx : (x >= nx ? x - nx : x);
        } else {
            x %= nx;
            x = x < 0 ? x + nx : x;
        }
        y = y0 - H + py;
        if (WALLS) return y >= 0 && y < ny;
        if (tall) {
            y = y < 0 ? y + ny : (y >= ny ? y - ny : y);
        } else {
            y %= ny;
            y = y < 0 ? y + ny : y;
        }
        return true;
    };
    // the nine pre-collision values of P cell c (lattice row y) from the buffer
    auto pull_lds = [&](int c, int y, bool edge, A f[9]) {
        const bool lo = WALLS && edge && y == 0, hi = WALLS && edge && y == ny - 1;
        f[0] = (A)P[0][c];
        f[1] = (A)P[1][c - 1];
        f[3] = (A)P[3][c + 1];
        f[2] = (A)(lo ? P[4][c] : P[2][c - AX]);
        f[5] = (A)(lo ? P[7][c] : P[5][c - AX - 1]);
        f[6] = (A)(lo ? P[8][c] : P[6][c - AX + 1]);
        f[4] = (A)(hi ? P[2][c] : P[4][c + AX]);
        f[7] = (A)(hi ? P[5][c] : P[7][c + AX + 1]);
        f[8] = (A)(hi ? P[6][c] : P[8][c + AX - 1]);
    };
    const int w1 = tw + 2 * H, h1 = th + 2 * H;
    auto body = [&](auto fast_tag) {
        constexpr bool FAST = decltype(fast_tag)::value;
        // phase 1: region [0, tw + 2H) x [0, th + 2H) from HBM
        for (int i = threadIdx.x; i < AN; i += BS) {
            const int px = i % AX, py = i / AX;
            int x, y;
            R fr[9];
            if constexpr (FAST) {
                x = x0 - H + px;
                y = y0 - H + py;
                const int c = y * nx + x;
                fr[0] = mem.ld(0, c);
                fr[1] = mem.ld(1, c - 1);
                fr[3] = mem.ld(3, c + 1);
                fr[2] = mem.ld(2, c - nx);
                fr[5] = mem.ld(5, c - nx - 1);
                fr[6] = mem.ld(6, c - nx + 1);
                fr[4] = mem.ld(4, c + nx);
                fr[7] = mem.ld(7, c + nx + 1);
                fr[8] = mem.ld(8, c + nx - 1);
            } else {
                if (px >= w1 || py >= h1 || !cell_of(px, py, x, y)) continue;
                pullm<R, WALLS>(mem, nx, ny, x, y, fr);
            }
            A f[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) f[q] = (A)fr[q];
            if constexpr (CL) {
                const R d0 = BMem<R>{a.coef, nullptr, a.cstride}.ld(0, y * nx + x);
                const R d = E2 ? d0 + d0 : d0;
                Dl[i] = d;
                collide_m<R, PK, FF, E2, GY>(a, f, 0, 0, OneCoef<R>{d}, OneCoef<R>{d});
            } else {
                collide_cell<R, PK, FF, BMem<R>>(a, f, y * nx + x);
            }
#pragma unroll
            for (int q = 0; q < 9; ++q) P[q][i] = (R)f[q];
        }
        // phases 2 .. D - 1: region [ph, w1 - ph) x [ph, h1 - ph), in place;
        // threads walk the full-tile shape (compile-time divisors) and skip
        // the part a ragged tile lacks
#pragma unroll
        for (int ph = 1; ph < H; ++ph) {
            const int RW = AX - 2 * ph, RN = RW * (AY - 2 * ph);
            __syncthreads();
            R pr[KM][9];
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                const int i = threadIdx.x + k * BS;
                const int px = ph + i % RW, py = ph + i / RW;
                int x = x0 - H + px, y = y0 - H + py;
                const bool in = FAST ? i < RN
                                     : (i < RN && px < w1 - ph && py < h1 - ph && cell_of(px, py, x, y));
                if (in) {
                    A f[9];
                    pull_lds(py * AX + px, y, !FAST, f);
#pragma unroll
                    for (int q = 0; q < 9; ++q) pr[k][q] = (R)f[q];
                }
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                const int i = threadIdx.x + k * BS;
                const int px = ph + i % RW, py = ph + i / RW;
                int x = x0 - H + px, y = y0 - H + py;
                const bool in = FAST ? i < RN
                                     : (i < RN && px < w1 - ph && py < h1 - ph && cell_of(px, py, x, y));
                if (in) {
                    A f[9];
#pragma unroll
                    for (int q = 0; q < 9; ++q) f[q] = (A)pr[k][q];
                    const int c = py * AX + px;
                    if constexpr (CL)
                        collide_m<R, PK, FF, E2, GY>(a, f, c, c, LdsCoef<R>{Dl}, LdsCoef<R>{Dl});
                    else
                        collide_cell<R, PK, FF, BMem<R>>(a, f, y * nx + x);
#pragma unroll
                    for (int q = 0; q < 9; ++q) P[q][c] = (R)f[q];
                }
            }
        }
        __syncthreads();
        // phase D: the tile, from LDS to HBM
        for (int i = threadIdx.x; i < TX * TY; i += BS) {
            const int lx = i % TX, ly = i / TX;
            if (!FAST && (lx >= tw || ly >= th)) continue;
            const int x = x0 + lx, y = y0 + ly;
            A f[9];
            const int c = (ly + H) * AX + (lx + H);
            pull_lds(c, y, !FAST, f);
            const int g = y * nx + x;
            if constexpr (CL)
                collide_m<R, PK, FF, E2, GY>(a, f, c, c, LdsCoef<R>{Dl}, LdsCoef<R>{Dl});
            else
                collide_cell<R, PK, FF, BMem<R>>(a, f, g);
#pragma unroll
            for (int q = 0; q < 9; ++q) mem.st(q, g, (R)f[q]);
        }
    };
    if (interior)
        body(std::true_type{});
    else
        body(std::false_type{});
}

// Flow velocity (Eq. u-of-S-C) and density of the current state in FP64, and
// per-block FP64 partial sums of u for the volume average.
template <typename R, bool WALLS, int PK, bool FF>
__global__ __launch_bounds__(kBlock) void k_fields(StepArgs<R> a, double *__restrict__ u_out,
                                                   double *__restrict__ rho_out,
                                                   double *__restrict__ partials)
{
    __shared__ double red[2][kBlock / 64];
    const int x = blockIdx.x * kBlock + threadIdx.x;
    const int y = blockIdx.y;
    double ux = 0.0, uy = 0.0;
    if (x < a.nx) {
        R fr[9];
        pull<R, WALLS>(a.fin, a.stride, a.nx, a.ny, x, y, fr);
        double f[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i] = (double)fr[i];
        double dr, jx, jy;
        moments(f, dr, jx, jy);
        const double rho = a.rho0_d + dr;
        const int c = y * a.nx + x;
        double hx, hy;
        if (FF) {
            hx = jx + (double)a.hforce[c] * rho;
            hy = jy + (double)a.hforce[a.cstride + c] * rho;
        } else {
            hx = jx + a.hegx_d * rho;
            hy = jy + a.hegy_d * rho;
        }
        if (PK == 1) {
            const double D = 1.0 - (double)a.coef[c];
            ux = D * hx / rho;
            uy = D * hy / rho;
        } else if (PK == 0) {
            const double den = rho * (1.0 + 0.5 * (double)a.coef[c]);
            ux = hx / den;
            uy = hy / den;
        } else {
            const double e00 = a.coef[c], e01 = a.coef[a.cstride + c];
            const double e10 = a.coef[2 * a.cstride + c], e11 = a.coef[3 * a.cstride + c];
            ux = ((hx - e00 * hx) - e01 * hy) / rho;
            uy = ((hy - e11 * hy) - e10 * hx) / rho;
        }
        if (u_out) {
            const size_t N = (size_t)a.nx * a.ny;
            u_out[c] = ux;
            u_out[N + c] = uy;
        }
        if (rho_out) rho_out[c] = rho;
    }
    if (partials) {
        ux = wave_sum(ux);
        uy = wave_sum(uy);
        const int wv = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
            red[0][wv] = ux;
            red[1][wv] = uy;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double sx = 0.0, sy = 0.0;
            for (int w = 0; w < kBlock / 64; ++w) {
                sx += red[0][w];
                sy += red[1][w];
            }
            const int bid = blockIdx.y * gridDim.x + blockIdx.x;
            partials[2 * bid] = sx;
            partials[2 * bid + 1] = sy;
        }
    }
}

// Fixed-order sum of n (x, y) pairs into out[0..1], divided by ncells.
__global__ __launch_bounds__(kBlock) void k_reduce_pairs(const double *__restrict__ partials,
                                                         int n, double inv_cells,
                                                         double *__restrict__ out)
{
    __shared__ double red[2][kBlock / 64];
    double sx = 0.0, sy = 0.0;
    // each thread adds its partials in index order, reading 16 of them ahead
    // (a loop that waited for each read took most of the reduction's time)
    constexpr int kAhead = 16;
    for (int i0 = threadIdx.x; i0 < n; i0 += kAhead * kBlock) {
        double vx[kAhead], vy[kAhead];
#pragma unroll
        for (int u = 0; u < kAhead; ++u) {
            const int i = min(i0 + u * kBlock, n - 1);
            vx[u] = partials[2 * i];
            vy[u] = partials[2 * i + 1];
        }
#pragma unroll
        for (int u = 0; u < kAhead; ++u)
            if (i0 + u * kBlock < n) {
                sx += vx[u];
                sy += vy[u];
            }
    }
    sx = wave_sum(sx);
    sy = wave_sum(sy);
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][wv] = sx;
        red[1][wv] = sy;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tx = 0.0, ty = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) {
            tx += red[0][w];
            ty += red[1][w];
        }
        out[0] = tx * inv_cells;
        out[1] = ty * inv_cells;
    }
}

__global__ void k_zero_i32(int *__restrict__ p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// Per-cell coefficient from the permeability (FP64, rounded once to R),
// eps G / 2 per cell, and the rest state (zero deviations) in buffer fin.
template <typename R, int PK>
__global__ __launch_bounds__(kBlock) void k_init(const double *__restrict__ perm,
                                                 const double *__restrict__ force, int n,
                                                 double eps, double nu, R *__restrict__ coef,
                                                 R *__restrict__ hforce, int cstride,
                                                 R *__restrict__ pops, int stride,
                                                 int *__restrict__ bad)
{
    const int c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= n) return;
    const double h = 0.5 * eps * nu;
    if (PK == 1) {
        const double k = perm[c];
        if (!(k > 0.0)) atomicOr(bad, 1);  // also catches NaN
        // E = 1 - D = h / (kappa + h) with D = 1 / (1 + eps nu / (2 kappa));
        // kappa = +inf gives 0
        coef[c] = (R)(h / (k + h));
    } else if (PK == 0) {
        const double k = perm[c];
        if (!(k > 0.0)) atomicOr(bad, 1);
        coef[c] = (R)(2.0 * h / k);  // eps nu / kappa (Guo form)
    } else {
        const double kxx = perm[4 * c], kxy = perm[4 * c + 1];
        const double kyx = perm[4 * c + 2], kyy = perm[4 * c + 3];
        const double det = kxx * kyy - kxy * kyx;
        // M = (K + h I)^{-1} K
        const double axx = kxx + h, axy = kxy, ayx = kyx, ayy = kyy + h;
        const double adet = axx * ayy - axy * ayx;
        const bool ok = std::isfinite(det) && det != 0.0 && std::isfinite(adet) && adet != 0.0;
        if (!ok) atomicOr(bad, 1);
        // E = I - M = h (K + h I)^{-1}
        const double ia = h / adet;
        coef[c] = (R)(ia * ayy);
        coef[cstride + c] = (R)(-ia * axy);
        coef[2 * cstride + c] = (R)(-ia * ayx);
        coef[3 * cstride + c] = (R)(ia * axx);
    }
    if (force) {
        const double gx = force[2 * c], gy = force[2 * c + 1];
        if (!std::isfinite(gx) || !std::isfinite(gy)) atomicOr(bad, 2);
        hforce[c] = (R)(0.5 * eps * gx);
        hforce[cstride + c] = (R)(0.5 * eps * gy);
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) pops[(size_t)q * stride + c] = (R)0;
}

// Full pre-collision populations of the current state, FP64 [9][ny][nx].
template <typename R, bool WALLS>
__global__ __launch_bounds__(kBlock) void k_get_pops(const R *__restrict__ fin, int stride, int nx,
                                                     int ny, double rho0, double *__restrict__ out)
{
    const int x = blockIdx.x * kBlock + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= nx) return;
    R f[9];
    pull<R, WALLS>(fin, stride, nx, ny, x, y, f);
    const size_t N = (size_t)nx * ny;
    const int c = y * nx + x;
#pragma unroll
    for (int q = 0; q < 9; ++q) out[q * N + c] = (double)f[q] + weight(q) * rho0;
}

// Inverse of the pull: store g with pull(g) = f, i.e. g_b(x) = f_b(x + e_b),
// or f_opp(b)(x) when x + e_b lies beyond a wall.
template <typename R, bool WALLS>
__global__ __launch_bounds__(kBlock) void k_set_pops(const double *__restrict__ in, int nx, int ny,
                                                     double rho0, R *__restrict__ fout, int stride)
{
    const int x = blockIdx.x * kBlock + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= nx) return;
    const size_t N = (size_t)nx * ny;
    const int c = y * nx + x;
#pragma unroll
    for (int b = 0; b < 9; ++b) {
        int xs = x + ex(b);
        int ys = y + ey(b);
        xs = (xs < 0) ? nx - 1 : (xs >= nx ? 0 : xs);
        int src_pop = b;
        if (ys < 0 || ys >= ny) {
            if (WALLS) {
                xs = x;
                ys = y;
                src_pop = opposite(b);
            } else {
                ys = (ys < 0) ? ny - 1 : 0;
            }
        }
        const double v = in[src_pop * N + (size_t)ys * nx + xs] - weight(src_pop) * rho0;
        fout[(size_t)b * stride + c] = (R)v;
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

struct Layout {
    size_t elem;      // bytes per population element
    size_t stride;    // elements per population plane
    size_t cstride;   // elements per coefficient plane
    size_t off_a, off_b, off_coef, off_force, off_part, off_res, off_flag, total;
    int nbx, nby;     // launch grid of the per-cell kernels
};

bool params_ok(const lbm_params *p, std::string &why)
{
    if (!p) { why = "params is NULL"; return false; }
    if (p->nx < 1 || p->ny < 1) { why = "nx and ny must be >= 1"; return false; }
    if (9 * ((int64_t)p->nx * p->ny + 8192) >= (int64_t)1 << 31) { why = "grid too large (9 nx ny must be below 2^31 - 73728)"; return false; }
    if (!(p->tau >= 0.5) || !std::isfinite(p->tau)) { why = "tau must be finite and >= 0.5"; return false; }
    if (!(p->eps > 0.0 && p->eps <= 1.0)) { why = "eps must lie in (0, 1]"; return false; }
    if (!(p->nu > 0.0) || !std::isfinite(p->nu)) { why = "nu must be finite and > 0"; return false; }
    if (!(p->rho0 > 0.0) || !std::isfinite(p->rho0)) { why = "rho0 must be finite and > 0"; return false; }
    if (!std::isfinite(p->gx) || !std::isfinite(p->gy)) { why = "gx, gy must be finite"; return false; }
    if (p->walls_y != 0 && p->walls_y != 1) { why = "walls_y must be 0 or 1"; return false; }
    if (p->pop_dtype != LBM_F32_SHIFTED && p->pop_dtype != LBM_F64 && p->pop_dtype != LBM_F32_FAST) {
        why = "unknown pop_dtype";
        return false;
    }
    if (p->pop_dtype == LBM_F32_FAST && p->scheme == LBM_SCHEME_GUO) {
        why = "the Guo form runs with FP64 arithmetic only (pop_dtype LBM_F32_SHIFTED or LBM_F64)";
        return false;
    }
    if (p->perm_kind != LBM_PERM_SCALAR && p->perm_kind != LBM_PERM_TENSOR) { why = "perm_kind must be 1 or 4"; return false; }
    if (p->scheme != LBM_SCHEME_SHAN_CHEN && p->scheme != LBM_SCHEME_GUO) { why = "scheme must be 0 or 1"; return false; }
    if (p->scheme == LBM_SCHEME_GUO && p->perm_kind != LBM_PERM_SCALAR) { why = "the Guo form takes a scalar permeability"; return false; }
    return true;
}

Layout layout_of(const lbm_params *p)
{
    Layout L{};
    const size_t n = (size_t)p->nx * p->ny;
    L.elem = (p->pop_dtype == LBM_F64) ? 8 : 4;
    // Planes are 16 KB apart beyond their size, so that the ten streams of a
    // step (nine planes and the coefficient) do not start on the same HBM
    // channels when the plane size is a large power of two.
    L.stride = align_up(n, 64) + kPlanePadBytes / L.elem;
    L.cstride = n;
    size_t off = 0;
    L.off_a = off;  off = align_up(off + 9 * L.stride * L.elem);
    L.off_b = off;  off = align_up(off + 9 * L.stride * L.elem);
    L.off_coef = off; off = align_up(off + (size_t)p->perm_kind * L.cstride * L.elem);
    L.off_force = off; off = align_up(off + 2 * L.cstride * L.elem);
    L.nbx = (p->nx + kBlock - 1) / kBlock;
    L.nby = p->ny;
    L.off_part = off; off = align_up(off + 2 * sizeof(double) * (size_t)L.nbx * L.nby);
    L.off_res = off;  off = align_up(off + 4 * sizeof(double));
    L.off_flag = off; off = align_up(off + sizeof(int));
    L.total = off;
    return L;
}

}  // namespace
}  // namespace lbm

struct lbm_handle {
    lbm_params p;
    lbm::Layout L;
    hipStream_t stream;
    char *ws;
    int cur;            // 0: state in buffer A, 1: in buffer B
    bool has_force;
    int64_t steps_total;
    double prev_u[2];
    bool have_prev;
    double *host_res;   // pinned host copy of the reduction result
};

namespace lbm {
namespace {

template <typename R>
StepArgs<R> step_args(const lbm_handle *h)
{
    StepArgs<R> a{};
    const Layout &L = h->L;
    a.fin = reinterpret_cast<const R *>(h->ws + (h->cur ? L.off_b : L.off_a));
    a.fout = reinterpret_cast<R *>(h->ws + (h->cur ? L.off_a : L.off_b));
    a.coef = reinterpret_cast<const R *>(h->ws + L.off_coef);
    a.hforce = h->has_force ? reinterpret_cast<const R *>(h->ws + L.off_force) : nullptr;
    a.nx = h->p.nx;
    a.ny = h->p.ny;
    a.stride = (int)L.stride;
    a.cstride = (int)L.cstride;
    const double tau = h->p.tau;
    a.om = (R)(1.0 / tau);
    // 1 - om formed in the storage type: for tau in [1/2, 2] the subtraction
    // is exact (Sterbenz), so om + omc = 1 and the FP32-arithmetic collision
    // conserves mass without a bias from the rounded 1/tau
    a.omc = (R)1 - a.om;
    a.twotau = (R)(2.0 * tau);
    a.omtt = (R)(1.0 - 2.0 * tau);
    a.hegx = (R)(0.5 * h->p.eps * h->p.gx);
    a.hegy = (R)(0.5 * h->p.eps * h->p.gy);
    a.rho0 = (R)h->p.rho0;
    a.hegx_d = 0.5 * h->p.eps * h->p.gx;
    a.hegy_d = 0.5 * h->p.eps * h->p.gy;
    a.om_d = 1.0 / tau;
    a.omc_d = 1.0 - 1.0 / tau;
    a.twotau_d = 2.0 * tau;
    a.omtt_d = 1.0 - 2.0 * tau;
    a.rho0_d = h->p.rho0;
    return a;
}

template <typename R, bool W, int PK, bool FF>
void launch_step_t(const lbm_handle *h)
{
    const dim3 grid(h->L.nbx * h->L.nby);
    if constexpr (std::is_same<R, float>::value && PK != 0) {
        if (h->p.pop_dtype == LBM_F32_FAST) {
            hipLaunchKernelGGL((k_step<R, W, PK, FF, float>), grid, dim3(kBlock), 0, h->stream, step_args<R>(h));
            return;
        }
    }
    hipLaunchKernelGGL((k_step<R, W, PK, FF>), grid, dim3(kBlock), 0, h->stream, step_args<R>(h));
}

template <typename R, bool W, int PK, bool FF>
void launch_fields_t(const lbm_handle *h, double *u, double *rho, double *part)
{
    const dim3 grid(h->L.nbx, h->L.nby);
    hipLaunchKernelGGL((k_fields<R, W, PK, FF>), grid, dim3(kBlock), 0, h->stream, step_args<R>(h),
                       u, rho, part);
}

// Dispatch on (dtype, walls, perm kind, force field) to one instantiation.
template <template <typename, bool, int, bool> class Fn, typename... Args>
void dispatch(const lbm_handle *h, Args... args)
{
    const bool w = h->p.walls_y != 0, ff = h->has_force;
    const int pk = h->p.scheme == LBM_SCHEME_GUO ? 0 : h->p.perm_kind;
#define LBM_CASE(R, W, PK, FF) \
    if (w == W && pk == PK && ff == FF) { Fn<R, W, PK, FF>::run(h, args...); return; }
    if (h->p.pop_dtype == LBM_F64) {
        LBM_CASE(double, false, 1, false) LBM_CASE(double, false, 1, true)
        LBM_CASE(double, false, 4, false) LBM_CASE(double, false, 4, true)
        LBM_CASE(double, true, 1, false)  LBM_CASE(double, true, 1, true)
        LBM_CASE(double, true, 4, false)  LBM_CASE(double, true, 4, true)
        LBM_CASE(double, false, 0, false) LBM_CASE(double, false, 0, true)
        LBM_CASE(double, true, 0, false)  LBM_CASE(double, true, 0, true)
    } else {
        LBM_CASE(float, false, 1, false) LBM_CASE(float, false, 1, true)
        LBM_CASE(float, false, 4, false) LBM_CASE(float, false, 4, true)
        LBM_CASE(float, true, 1, false)  LBM_CASE(float, true, 1, true)
        LBM_CASE(float, true, 4, false)  LBM_CASE(float, true, 4, true)
        LBM_CASE(float, false, 0, false) LBM_CASE(float, false, 0, true)
        LBM_CASE(float, true, 0, false)  LBM_CASE(float, true, 0, true)
    }
#undef LBM_CASE
}

template <typename R, bool W, int PK, bool FF>
struct StepFn {
    static void run(const lbm_handle *h) { launch_step_t<R, W, PK, FF>(h); }
};
template <typename R, bool W, int PK, bool FF>
struct StepDFn {
    template <int D>
    static void launch(const lbm_handle *h)
    {
        if constexpr (std::is_same<R, float>::value && PK != 0) {
            if (h->p.pop_dtype == LBM_F32_FAST) {
                using TF = TileDA<R, D, float>;
                const int fx = (h->p.nx + TF::TX - 1) / TF::TX, fy = (h->p.ny + TF::TY - 1) / TF::TY;
                const StepArgs<R> sa = step_args<R>(h);
                if constexpr (PK == 1 && !FF) {
                    if ((float)sa.hegy == 0.0f) {  // drive along x only
                        hipLaunchKernelGGL((k_stepd<R, W, PK, FF, D, float, false>), dim3(fx * fy), dim3(TF::BS), 0,
                                           h->stream, sa);
                        return;
                    }
                }
                hipLaunchKernelGGL((k_stepd<R, W, PK, FF, D, float>), dim3(fx * fy), dim3(TF::BS), 0, h->stream, sa);
                return;
            }
        }
        if constexpr (D != kDeeper) {  // seven steps: FP32 collision arithmetic only
            constexpr int TX = TileD<R, D>::TX, TY = TileD<R, D>::TY, BS = TileD<R, D>::BS;
            const int ntx = (h->p.nx + TX - 1) / TX, nty = (h->p.ny + TY - 1) / TY;
            hipLaunchKernelGGL((k_stepd<R, W, PK, FF, D>), dim3(ntx * nty), dim3(BS), 0, h->stream,
                               step_args<R>(h));
        }
    }
    static void run(const lbm_handle *h, int depth)
    {
        if (depth == kDeeper) return launch<kDeeper>(h);
        if (depth == kDeep) return launch<kDeep>(h);
        if (depth == 4) return launch<4>(h);
        launch<2>(h);
    }
};

// Steps per launch before the next check (or the end), `room` steps away; 1
// runs the single-step kernel. Every depth gives the same state bit for bit,
// so the choice is one of time only. With FP32 collision arithmetic, whose
// seven-step kernel takes fewer microseconds per step than the six-step one,
// the plan of launches that covers `room` in the least time by the launch
// costs measured on 2048^2 (us: 1 step 54.5, 2: 66.0, 4: 76.8, 6: 89.2,
// 7: 98.8): seven-step launches while more than 60 steps remain, then the
// best mix for the rest (e.g. 100 = 10 x 7 + 5 x 6, 1434 us against 1505 for
// 16 x 6 + 4; 20 = 7 + 7 + 6, 287 us against 334 for 6 + 6 + 6 + 2).
// Otherwise the deepest depth that fits.
int launch_depth(const lbm_handle *h, int64_t room)
{
    if (h->p.pop_dtype == LBM_F32_FAST) {
        static const std::array<signed char, 61> first = [] {
            const int depth[5] = {kDeeper, kDeep, 4, 2, 1};
            const double cost[5] = {98.8, 89.2, 76.8, 66.0, 54.5};
            std::array<double, 61> best{};
            std::array<signed char, 61> f{};
            for (int r = 1; r <= 60; ++r) {
                best[r] = 1e30;
                for (int i = 0; i < 5; ++i)
                    if (depth[i] <= r && cost[i] + best[r - depth[i]] < best[r]) {
                        best[r] = cost[i] + best[r - depth[i]];
                        f[r] = (signed char)depth[i];
                    }
            }
            return f;
        }();
        if (room > 60) return kDeeper;
        return room >= 1 ? first[room] : 1;
    }
    if (room >= kDeep) return kDeep;
    if (room >= 4) return 4;
    return room >= 2 ? 2 : 1;
}
template <typename R, bool W, int PK, bool FF>
struct FieldsFn {
    static void run(const lbm_handle *h, double *u, double *rho, double *part)
    {
        launch_fields_t<R, W, PK, FF>(h, u, rho, part);
    }
};

lbm_status mean_velocity(lbm_handle *h, double out[2])
{
    double *part = reinterpret_cast<double *>(h->ws + h->L.off_part);
    double *res = reinterpret_cast<double *>(h->ws + h->L.off_res);
    dispatch<FieldsFn>(h, (double *)nullptr, (double *)nullptr, part);
    const int nparts = h->L.nbx * h->L.nby;
    hipLaunchKernelGGL(k_reduce_pairs, dim3(1), dim3(kBlock), 0, h->stream, part, nparts,
                       1.0 / ((double)h->p.nx * h->p.ny), res);
    LBM_HIP(hipGetLastError());
    LBM_HIP(hipMemcpyAsync(h->host_res, res, 2 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    LBM_HIP(hipStreamSynchronize(h->stream));
    out[0] = h->host_res[0];
    out[1] = h->host_res[1];
    return LBM_OK;
}

}  // namespace
}  // namespace lbm

using namespace lbm;

extern "C" size_t lbm_workspace_bytes(const lbm_params *p)
{
    std::string why;
    if (!params_ok(p, why)) return 0;
    return layout_of(p).total;
}

extern "C" lbm_status lbm_init(lbm_handle **out, const lbm_params *p, const double *d_perm,
                               const double *d_force, void *d_ws, size_t ws_bytes,
                               hipStream_t stream)
{
    if (!out) return set_error(LBM_EINVAL, "lbm_init: handle pointer is NULL");
    *out = nullptr;
    std::string why;
    if (!params_ok(p, why)) return set_error(LBM_EINVAL, "lbm_init: " + why);
    if (!d_perm) return set_error(LBM_EINVAL, "lbm_init: permeability pointer is NULL");
    const Layout L = layout_of(p);
    if (!d_ws || ((uintptr_t)d_ws % kAlign) != 0)
        return set_error(LBM_EWORKSPACE, "lbm_init: workspace is NULL or not 256-byte aligned");
    if (ws_bytes < L.total)
        return set_error(LBM_EWORKSPACE, "lbm_init: workspace too small (need " +
                                             std::to_string(L.total) + " bytes)");
    lbm_handle *h = new (std::nothrow) lbm_handle{};
    if (!h) return set_error(LBM_EINVAL, "lbm_init: out of host memory");
    h->p = *p;
    h->L = L;
    h->stream = stream;
    h->ws = static_cast<char *>(d_ws);
    h->cur = 0;
    h->has_force = d_force != nullptr;
    if (hipHostMalloc((void **)&h->host_res, 4 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        delete h;
        return set_error(LBM_EDEVICE, "lbm_init: hipHostMalloc failed");
    }
    int *flag = reinterpret_cast<int *>(h->ws + L.off_flag);
    const int n = p->nx * p->ny;
    const int nb = (n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, stream, flag, 1);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        if (p->pop_dtype == LBM_F64) {
            double *coef = reinterpret_cast<double *>(h->ws + L.off_coef);
            double *hf = reinterpret_cast<double *>(h->ws + L.off_force);
            double *pa = reinterpret_cast<double *>(h->ws + L.off_a);
            if (p->scheme == LBM_SCHEME_GUO)
                hipLaunchKernelGGL((k_init<double, 0>), dim3(nb), dim3(kBlock), 0, stream, d_perm, d_force, n,
                                   p->eps, p->nu, coef, hf, (int)L.cstride, pa, (int)L.stride, flag);
            else if (p->perm_kind == LBM_PERM_SCALAR)
                hipLaunchKernelGGL((k_init<double, 1>), dim3(nb), dim3(kBlock), 0, stream, d_perm, d_force, n,
                                   p->eps, p->nu, coef, hf, (int)L.cstride, pa, (int)L.stride, flag);
            else
                hipLaunchKernelGGL((k_init<double, 4>), dim3(nb), dim3(kBlock), 0, stream, d_perm, d_force, n,
                                   p->eps, p->nu, coef, hf, (int)L.cstride, pa, (int)L.stride, flag);
        } else {
            float *coef = reinterpret_cast<float *>(h->ws + L.off_coef);
            float *hf = reinterpret_cast<float *>(h->ws + L.off_force);
            float *pa = reinterpret_cast<float *>(h->ws + L.off_a);
            if (p->scheme == LBM_SCHEME_GUO)
                hipLaunchKernelGGL((k_init<float, 0>), dim3(nb), dim3(kBlock), 0, stream, d_perm, d_force, n,
                                   p->eps, p->nu, coef, hf, (int)L.cstride, pa, (int)L.stride, flag);
            else if (p->perm_kind == LBM_PERM_SCALAR)
                hipLaunchKernelGGL((k_init<float, 1>), dim3(nb), dim3(kBlock), 0, stream, d_perm, d_force, n,
                                   p->eps, p->nu, coef, hf, (int)L.cstride, pa, (int)L.stride, flag);
            else
                hipLaunchKernelGGL((k_init<float, 4>), dim3(nb), dim3(kBlock), 0, stream, d_perm, d_force, n,
                                   p->eps, p->nu, coef, hf, (int)L.cstride, pa, (int)L.stride, flag);
        }
        e = hipGetLastError();
    }
    int bad = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        (void)hipHostFree(h->host_res);
        delete h;
        return hip_check(e, "lbm_init");
    }
    if (bad) {
        (void)hipHostFree(h->host_res);
        delete h;
        return set_error(LBM_EINVAL, (bad & 1) ? "lbm_init: permeability must be > 0 (or +inf) and "
                                                 "tensors invertible"
                                               : "lbm_init: force field has non-finite values");
    }
    *out = h;
    return LBM_OK;
}

extern "C" lbm_status lbm_step(lbm_handle *h, int64_t max_steps, double tol, int32_t check_every,
                               int64_t *steps_done, double mean_u[2])
{
    if (!h) return set_error(LBM_EINVAL, "lbm_step: handle is NULL");
    if (max_steps < 0) return set_error(LBM_EINVAL, "lbm_step: max_steps must be >= 0");
    if (check_every < 0) return set_error(LBM_EINVAL, "lbm_step: check_every must be >= 0");
    if (tol > 0.0 && check_every == 0)
        return set_error(LBM_EINVAL, "lbm_step: a tolerance needs check_every > 0");
    if (steps_done) *steps_done = 0;
    lbm_status st = (tol > 0.0) ? LBM_ENOTCONV : LBM_OK;
    int64_t done = 0;
    bool last_checked = false;
    double u[2] = {0.0, 0.0};
    while (done < max_steps) {
        // several steps per launch unless a check or the end falls in between
        const int64_t to_check = check_every > 0 ? check_every - done % check_every : max_steps - done;
        const int n = launch_depth(h, std::min<int64_t>(to_check, max_steps - done));
        if (n >= 2)
            dispatch<StepDFn>(h, n);
        else
            dispatch<StepFn>(h);
        h->cur ^= 1;
        done += n;
        h->steps_total += n;
        last_checked = false;
        if (check_every > 0 && done % check_every == 0) {
            LBM_HIP(hipGetLastError());
            lbm_status s = mean_velocity(h, u);
            if (s != LBM_OK) return s;
            last_checked = true;
            if (!std::isfinite(u[0]) || !std::isfinite(u[1])) {
                st = LBM_ENONFINITE;
                break;
            }
            if (tol > 0.0 && h->have_prev) {
                const double dx = u[0] - h->prev_u[0], dy = u[1] - h->prev_u[1];
                if (std::sqrt(dx * dx + dy * dy) <= tol * std::sqrt(u[0] * u[0] + u[1] * u[1])) {
                    h->prev_u[0] = u[0];
                    h->prev_u[1] = u[1];
                    st = LBM_OK;
                    break;
                }
            }
            h->prev_u[0] = u[0];
            h->prev_u[1] = u[1];
            h->have_prev = true;
        }
    }
    LBM_HIP(hipGetLastError());
    if (steps_done) *steps_done = done;
    if (mean_u) {
        if (!last_checked) {
            lbm_status s = mean_velocity(h, u);
            if (s != LBM_OK) return s;
        }
        mean_u[0] = u[0];
        mean_u[1] = u[1];
        if (st == LBM_OK && (!std::isfinite(u[0]) || !std::isfinite(u[1]))) st = LBM_ENONFINITE;
    }
    if (st == LBM_ENOTCONV) return set_error(st, "lbm_step: tolerance not reached within max_steps");
    if (st == LBM_ENONFINITE) return set_error(st, "lbm_step: non-finite mean velocity");
    return LBM_OK;
}

extern "C" lbm_status lbm_fields(lbm_handle *h, double *d_u, double *d_rho)
{
    if (!h) return set_error(LBM_EINVAL, "lbm_fields: handle is NULL");
    if (!d_u && !d_rho) return set_error(LBM_EINVAL, "lbm_fields: no output given");
    if (d_u) {
        dispatch<FieldsFn>(h, d_u, d_rho, (double *)nullptr);
    } else {
        // density only: velocities are still computed, into nowhere
        dispatch<FieldsFn>(h, (double *)nullptr, d_rho, (double *)nullptr);
    }
    LBM_HIP(hipGetLastError());
    return LBM_OK;
}

extern "C" lbm_status lbm_get_populations(lbm_handle *h, double *d_f)
{
    if (!h || !d_f) return set_error(LBM_EINVAL, "lbm_get_populations: NULL argument");
    const dim3 grid(h->L.nbx, h->L.nby);
    const char *cur = h->ws + (h->cur ? h->L.off_b : h->L.off_a);
    const int S = (int)h->L.stride;
    const bool w = h->p.walls_y != 0;
    if (h->p.pop_dtype == LBM_F64) {
        auto *fin = reinterpret_cast<const double *>(cur);
        if (w) hipLaunchKernelGGL((k_get_pops<double, true>), grid, dim3(kBlock), 0, h->stream, fin, S, h->p.nx, h->p.ny, h->p.rho0, d_f);
        else   hipLaunchKernelGGL((k_get_pops<double, false>), grid, dim3(kBlock), 0, h->stream, fin, S, h->p.nx, h->p.ny, h->p.rho0, d_f);
    } else {
        auto *fin = reinterpret_cast<const float *>(cur);
        if (w) hipLaunchKernelGGL((k_get_pops<float, true>), grid, dim3(kBlock), 0, h->stream, fin, S, h->p.nx, h->p.ny, h->p.rho0, d_f);
        else   hipLaunchKernelGGL((k_get_pops<float, false>), grid, dim3(kBlock), 0, h->stream, fin, S, h->p.nx, h->p.ny, h->p.rho0, d_f);
    }
    LBM_HIP(hipGetLastError());
    return LBM_OK;
}

extern "C" lbm_status lbm_set_populations(lbm_handle *h, const double *d_f)
{
    if (!h || !d_f) return set_error(LBM_EINVAL, "lbm_set_populations: NULL argument");
    const dim3 grid(h->L.nbx, h->L.nby);
    char *cur = h->ws + (h->cur ? h->L.off_b : h->L.off_a);
    const int S = (int)h->L.stride;
    const bool w = h->p.walls_y != 0;
    if (h->p.pop_dtype == LBM_F64) {
        auto *fo = reinterpret_cast<double *>(cur);
        if (w) hipLaunchKernelGGL((k_set_pops<double, true>), grid, dim3(kBlock), 0, h->stream, d_f, h->p.nx, h->p.ny, h->p.rho0, fo, S);
        else   hipLaunchKernelGGL((k_set_pops<double, false>), grid, dim3(kBlock), 0, h->stream, d_f, h->p.nx, h->p.ny, h->p.rho0, fo, S);
    } else {
        auto *fo = reinterpret_cast<float *>(cur);
        if (w) hipLaunchKernelGGL((k_set_pops<float, true>), grid, dim3(kBlock), 0, h->stream, d_f, h->p.nx, h->p.ny, h->p.rho0, fo, S);
        else   hipLaunchKernelGGL((k_set_pops<float, false>), grid, dim3(kBlock), 0, h->stream, d_f, h->p.nx, h->p.ny, h->p.rho0, fo, S);
    }
    h->have_prev = false;
    LBM_HIP(hipGetLastError());
    return LBM_OK;
}

extern "C" int64_t lbm_steps_total(const lbm_handle *h) { return h ? h->steps_total : -1; }

extern "C" void lbm_destroy(lbm_handle *h)
{
    if (!h) return;
    if (h->host_res) (void)hipHostFree(h->host_res);
    delete h;
}
