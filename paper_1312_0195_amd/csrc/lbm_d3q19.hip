// lbm_d3q19.hip -- the fine-grid time step on the D3Q19 lattice.
//
// Sec. 2: three-dimensional problems use the D3Q19 lattice, whose velocities
// and weights differ from D2Q9 while the algorithm stays the same. So this is
// the Shan-Chen form of Sec. 2.2 (Eqs. explicit-u-in-Guo, final-ueq-of-S-C,
// feq, f-evolution-of-S-C) with three velocity components, a scalar
// permeability per cell and a uniform body force.
//
// Storage: FP32 deviations from the rest state (f_a - w_a rho0) or FP64
// populations, one plane per population ([19][nz][ny][nx] plus padding), two
// buffers. The buffer holds post-collision values; one launch pulls each
// population from its upstream neighbour, collides in FP64 and stores, so
// every population element is read once and written once per step:
// 19 x 2 x 4 B + 4 B of drag coefficient = 156 B per lattice update (FP32).
// With FP32 state two steps run per launch (k3_step2, below), halving that.
//
// Population order (also the layout of lbm3d_get_populations): rest; +x, -x,
// +y, -y, +z, -z; the diagonals of the xy plane (+x+y, -x-y, +x-y, -x+y), of
// the xz plane (+x+z, -x-z, +x-z, -x+z) and of the yz plane (+y+z, -y-z,
// +y-z, -y+z). Opposite pairs are adjacent (1-2, 3-4, ..., 17-18).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>

#include "lbm_internal.h"

namespace lbm3 {
namespace {

using lbm::kAlign;
using lbm::align_up;
using lbm::set_error;
using lbm::hip_check;
using lbm::wave_sum;

constexpr int Q = 19;
constexpr int kTX = 128, kTY = 2, kBlock3 = kTX * kTY;
constexpr size_t kPlanePad = 16384;  // bytes between planes beyond their size

__host__ __device__ constexpr int cx(int a)
{
    return (a == 1 || a == 7 || a == 9 || a == 11 || a == 13) ? 1
         : (a == 2 || a == 8 || a == 10 || a == 12 || a == 14) ? -1 : 0;
}
__host__ __device__ constexpr int cy(int a)
{
    return (a == 3 || a == 7 || a == 10 || a == 15 || a == 17) ? 1
         : (a == 4 || a == 8 || a == 9 || a == 16 || a == 18) ? -1 : 0;
}
__host__ __device__ constexpr int cz(int a)
{
    return (a == 5 || a == 11 || a == 14 || a == 15 || a == 18) ? 1
         : (a == 6 || a == 12 || a == 13 || a == 16 || a == 17) ? -1 : 0;
}
__host__ __device__ constexpr int opp(int a) { return a == 0 ? 0 : ((a & 1) ? a + 1 : a - 1); }
__host__ __device__ constexpr double wgt(int a) { return a == 0 ? 1.0 / 3.0 : (a <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }

template <typename R>
struct Args3 {
    const R *__restrict__ fin;
    R *__restrict__ fout;
    const R *__restrict__ coef;  // drag deficit E = 1 - D = h / (kappa + h), h = eps nu / 2, per cell
                                 // (D = 1 / (1 + h / kappa) itself would lose the relative
                                 // precision of 1 - D in FP32 for permeable cells)
    int nx, ny, nz;
    size_t stride;               // elements per population plane
    double hegx, hegy, hegz;     // eps G / 2
    double om, omc;              // 1 / tau, 1 - 1 / tau
    double twotau, omtt;         // 2 tau, 1 - 2 tau
    double rho0;
};

// Cell of this thread; false outside the grid. Workgroups are renumbered so
// that each of the 8 XCDs gets one contiguous run of tiles (a slab in z).
__device__ __forceinline__ bool cell_of(int nx, int ny, int &x, int &y, int &z)
{
    constexpr int kXcd = 8;
    const int nb = gridDim.x, bid = blockIdx.x;
    const int q = nb / kXcd, rem = nb % kXcd;
    const int k = bid % kXcd, slot = bid / kXcd;
    const int t = k * q + (k < rem ? k : rem) + slot;
    const int ntx = (nx + kTX - 1) / kTX, nty = (ny + kTY - 1) / kTY;
    const int tx = t % ntx, rest = t / ntx;
    const int ty = rest % nty;
    z = rest / nty;
    x = tx * kTX + (threadIdx.x & (kTX - 1));
    y = ty * kTY + (int)(threadIdx.x / kTX);
    return x < nx && y < ny;
}

// Pre-collision populations of cell (x, y, z): f_a from the upstream cell
// (x, y, z) - e_a, periodic in x and y; in z periodic, or, with walls, the
// opposite population of the cell itself where the upstream cell lies
// beyond a wall (halfway bounce-back).
template <typename R, bool WALLS>
__device__ __forceinline__ void pull3(const R *__restrict__ in, size_t S, int nx, int ny, int nz,
                                      int x, int y, int z, R f[Q])
{
    const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
    const bool zlo = z == 0, zhi = z == nz - 1;
    const int zm = zlo ? nz - 1 : z - 1, zp = zhi ? 0 : z + 1;
    const unsigned pn = (unsigned)nx * (unsigned)ny;
    const unsigned p0 = (unsigned)z * pn, pm = (unsigned)zm * pn, pp = (unsigned)zp * pn;
    const unsigned r0 = (unsigned)y * nx, rm = (unsigned)ym * nx, rp = (unsigned)yp * nx;
    const unsigned c = p0 + r0 + x;
    // plane base (uniform, in scalar registers) plus a 32-bit byte offset per
    // lane: global loads in their scalar-base form, no 64-bit address adds
    auto ld = [&](int a, unsigned i) {
        const char *base = reinterpret_cast<const char *>(in + (size_t)a * S);
        return *reinterpret_cast<const R *>(base + i * (unsigned)sizeof(R));
    };
    f[0] = ld(0, c);
    f[1] = ld(1, p0 + r0 + xm);
    f[2] = ld(2, p0 + r0 + xp);
    f[3] = ld(3, p0 + rm + x);
    f[4] = ld(4, p0 + rp + x);
    f[7] = ld(7, p0 + rm + xm);
    f[8] = ld(8, p0 + rp + xp);
    f[9] = ld(9, p0 + rp + xm);
    f[10] = ld(10, p0 + rm + xp);
    if (WALLS && zlo) {
        // upstream of +z populations lies below the bottom wall
        f[5] = ld(6, c);
        f[11] = ld(12, c);
        f[14] = ld(13, c);
        f[15] = ld(16, c);
        f[18] = ld(17, c);
    } else {
        f[5] = ld(5, pm + r0 + x);
        f[11] = ld(11, pm + r0 + xm);
        f[14] = ld(14, pm + r0 + xp);
        f[15] = ld(15, pm + rm + x);
        f[18] = ld(18, pm + rp + x);
    }
    if (WALLS && zhi) {
        f[6] = ld(5, c);
        f[12] = ld(11, c);
        f[13] = ld(14, c);
        f[16] = ld(15, c);
        f[17] = ld(18, c);
    } else {
        f[6] = ld(6, pp + r0 + x);
        f[12] = ld(12, pp + r0 + xp);
        f[13] = ld(13, pp + r0 + xm);
        f[16] = ld(16, pp + rp + x);
        f[17] = ld(17, pp + rm + x);
    }
}

// Density deviation and momentum of 19 populations (FP64).
__device__ __forceinline__ void moments3(const double f[Q], double &dr, double &jx, double &jy,
                                         double &jz)
{
    const double sxy = (f[7] + f[8]) + (f[9] + f[10]);
    const double sxz = (f[11] + f[12]) + (f[13] + f[14]);
    const double syz = (f[15] + f[16]) + (f[17] + f[18]);
    dr = ((f[0] + (f[1] + f[2])) + ((f[3] + f[4]) + (f[5] + f[6]))) + ((sxy + sxz) + syz);
    jx = (f[1] - f[2]) + (((f[7] - f[8]) + (f[9] - f[10])) + ((f[11] - f[12]) + (f[13] - f[14])));
    jy = (f[3] - f[4]) + (((f[7] - f[8]) - (f[9] - f[10])) + ((f[15] - f[16]) + (f[17] - f[18])));
    jz = (f[5] - f[6]) + (((f[11] - f[12]) - (f[13] - f[14])) + ((f[15] - f[16]) - (f[17] - f[18])));
}

// Post-collision deviations in place: rho u_eq = 2 tau D (j + rho eps G / 2)
// + (1 - 2 tau) j and f~_a <- (1 - 1/tau) f~_a + (w_a / tau)(dr + 3 e_a . rho u_eq).
// E: the cell's drag deficit 1 - D as stored (full relative precision in FP32).
template <typename R>
__device__ __forceinline__ void collide3(const Args3<R> &a, double f[Q], double E)
{
    double dr, jx, jy, jz;
    moments3(f, dr, jx, jy, jz);
    const double rho = a.rho0 + dr;
    const double tD = a.twotau - a.twotau * E;
    const double mx = tD * (jx + a.hegx * rho) + a.omtt * jx;
    const double my = tD * (jy + a.hegy * rho) + a.omtt * jy;
    const double mz = tD * (jz + a.hegz * rho) + a.omtt * jz;
    const double om = a.om, omc = a.omc;
    const double s0 = (1.0 / 3.0) * om * dr;
    const double b = (1.0 / 18.0) * om * dr;
    const double bx = (1.0 / 6.0) * om * mx, by = (1.0 / 6.0) * om * my, bz = (1.0 / 6.0) * om * mz;
    const double c = (1.0 / 36.0) * om * dr;
    const double gx = (1.0 / 12.0) * om * mx, gy = (1.0 / 12.0) * om * my, gz = (1.0 / 12.0) * om * mz;
    f[0] = omc * f[0] + s0;
    f[1] = omc * f[1] + (b + bx);
    f[2] = omc * f[2] + (b - bx);
    f[3] = omc * f[3] + (b + by);
    f[4] = omc * f[4] + (b - by);
    f[5] = omc * f[5] + (b + bz);
    f[6] = omc * f[6] + (b - bz);
    const double xyp = gx + gy, xym = gx - gy;
    f[7] = omc * f[7] + (c + xyp);
    f[8] = omc * f[8] + (c - xyp);
    f[9] = omc * f[9] + (c + xym);
    f[10] = omc * f[10] + (c - xym);
    const double xzp = gx + gz, xzm = gx - gz;
    f[11] = omc * f[11] + (c + xzp);
    f[12] = omc * f[12] + (c - xzp);
    f[13] = omc * f[13] + (c + xzm);
    f[14] = omc * f[14] + (c - xzm);
    const double yzp = gy + gz, yzm = gy - gz;
    f[15] = omc * f[15] + (c + yzp);
    f[16] = omc * f[16] + (c - yzp);
    f[17] = omc * f[17] + (c + yzm);
    f[18] = omc * f[18] + (c - yzm);
}

template <typename R, bool WALLS>
__global__ __launch_bounds__(kBlock3) void k3_step(Args3<R> a)
{
    int x, y, z;
    if (!cell_of(a.nx, a.ny, x, y, z)) return;
    R fr[Q];
    pull3<R, WALLS>(a.fin, a.stride, a.nx, a.ny, a.nz, x, y, z, fr);
    const unsigned c = ((unsigned)z * a.ny + y) * (unsigned)a.nx + x;
    double f[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) f[q] = (double)fr[q];
    collide3(a, f, (double)*reinterpret_cast<const R *>(reinterpret_cast<const char *>(a.coef) + c * (unsigned)sizeof(R)));
#pragma unroll
    for (int q = 0; q < Q; ++q)
        *reinterpret_cast<R *>(reinterpret_cast<char *>(a.fout + (size_t)q * a.stride) + c * (unsigned)sizeof(R)) = (R)f[q];
}

// ---------------------------------------------------------------------------
// Two time steps per launch (FP32 state): each workgroup owns an IX x IY tile
// of (x, y) columns and a run of zc planes, and marches up z. For every
// plane p it takes step 1 on the tile plus a one-cell halo, (IX + 2) x
// (IY + 2) cells (pulled from HBM, collided in FP64, rounded to FP32 as a
// stored step would be), into LDS, then step 2 on the IX x IY cells of plane
// p - 1, pulling from the step-1 planes p - 2, p - 1 and p, and stores that
// to HBM. The state passes through HBM once per two steps (156 B per two
// lattice updates) and the result is bit-identical to two single steps.
// Extra work: the halo cells and two step-1 planes per chunk.
//
// LDS keeps each population only as long as step 2 needs it: the in-plane
// populations of the last two planes, the +z populations of the last three
// (read by the plane above) and the -z populations of the last two (read by
// the plane below, and by the bounce-back of the bottom plane): 43 planes of
// the halo tile. The loads of the next plane's step 1 are issued before
// step 2 and stay in flight across the barrier, which orders LDS operations
// only.
//
// Tile 64 x 8 (66 x 10 with the halo: 29% extra step-1 cells), 512 threads,
// 113.5 KB of LDS: one workgroup per CU. Measured on 256^3 against 32 x 8,
// 30 x 6, 32 x 4, 64 x 4, 32 x 16, 62 x 6, 64 x 6, 96 x 4 and 128 x 4 tiles,
// without the prefetch, and with z runs of 16 to 128 planes (all
// bit-identical): 64 x 8 with runs of 128 planes was the fastest. The run
// length zc is chosen per grid on the host (launch_step2).
// ---------------------------------------------------------------------------
constexpr int k2IX = 64, k2IY = 8, k2T = 512;

// Barrier that orders LDS only: global loads in flight stay in flight.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// populations by role in step 2: in the plane (0..4, 7..10), +z, -z
__device__ constexpr int kIn[9] = {0, 1, 2, 3, 4, 7, 8, 9, 10};
__device__ constexpr int kUp[5] = {5, 11, 14, 15, 18};
__device__ constexpr int kDn[5] = {6, 12, 13, 16, 17};

template <int IX, int IY, int T>
struct Tile2 {
    static constexpr int EX = IX + 2, EY = IY + 2, NE = EX * EY;  // halo tile
    static constexpr int R1 = (NE + T - 1) / T;                    // step-1 cells per thread
    static_assert(IX * IY <= T, "one step-2 cell per thread");
    static_assert(R1 <= 2, "at most two step-1 cells per thread");
};
using Tl2 = Tile2<k2IX, k2IY, k2T>;

template <bool WALLS>
__global__ __launch_bounds__(k2T) void k3_step2(Args3<float> a, int zc)
{
    constexpr bool PF = true;
    constexpr int IX = k2IX, IY = k2IY, T = k2T;
    constexpr int EX = Tl2::EX, NE = Tl2::NE, R1 = Tl2::R1;
    __shared__ float sin_[2][9][NE];  // in-plane populations, planes p - 1, p
    __shared__ float sup[3][5][NE];   // +z populations, planes p - 2 .. p
    __shared__ float sdn[2][5][NE];   // -z populations, planes p - 1, p
    constexpr int kXcd = 8;
    const int nb = gridDim.x, bid = blockIdx.x;
    const int qq = nb / kXcd, rem = nb % kXcd;
    const int k = bid % kXcd, slot = bid / kXcd;
    const int t = k * qq + (k < rem ? k : rem) + slot;
    const int ntx = (a.nx + IX - 1) / IX, nty = (a.ny + IY - 1) / IY;
    const int tx = t % ntx, rest = t / ntx;
    const int ty = rest % nty, tz = rest / nty;
    const int x0 = tx * IX, y0 = ty * IY, z0 = tz * zc;
    const int zend = min(z0 + zc, a.nz);  // step-2 planes [z0, zend)
    const int tid = threadIdx.x;
    // step-1 cells of this thread: halo-tile index e1[r], grid column (gx1, gy1)
    int e1[R1], gx1[R1], gy1[R1];
#pragma unroll
    for (int r = 0; r < R1; ++r) {
        const int e = tid + r * T;
        e1[r] = e;
        const int lx = e % EX, ly = e / EX;
        int gx = (x0 - 1 + lx) % a.nx, gy = (y0 - 1 + ly) % a.ny;
        gx1[r] = gx < 0 ? gx + a.nx : gx;
        gy1[r] = gy < 0 ? gy + a.ny : gy;
    }
    // step-2 cell of this thread
    const int ix = tid % IX, iy = tid / IX;
    const int e2 = (iy + 1) * EX + ix + 1;
    const int gx2 = x0 + ix, gy2 = y0 + iy;
    const bool act2 = tid < IX * IY && gx2 < a.nx && gy2 < a.ny;
    const unsigned pn = (unsigned)a.nx * (unsigned)a.ny;
    auto plane_of = [&](int p) {
        int pz = p % a.nz;
        return pz < 0 ? pz + a.nz : pz;
    };
    auto have1 = [&](int p) { return WALLS ? (p >= 0 && p < a.nz) : true; };
    auto load1 = [&](int r, int pz, float fr[Q], float &D) {
        pull3<float, WALLS>(a.fin, a.stride, a.nx, a.ny, a.nz, gx1[r], gy1[r], pz, fr);
        D = *reinterpret_cast<const float *>(reinterpret_cast<const char *>(a.coef) +
                                             ((unsigned)pz * pn + (unsigned)gy1[r] * a.nx + gx1[r]) * 4u);
    };

    float fr[R1][Q];
    float Dn[R1];
    if (PF && have1(z0 - 1)) {
#pragma unroll
        for (int r = 0; r < R1; ++r)
            if (e1[r] < NE) load1(r, plane_of(z0 - 1), fr[r], Dn[r]);
    }
    for (int p = z0 - 1; p <= zend; ++p) {
        const int rr = p - z0 + 1;  // >= 0
        const int s2 = rr & 1, s3 = rr % 3;
        // ---- step 1 on plane p
        if (have1(p)) {
#pragma unroll
            for (int r = 0; r < R1; ++r) {
                if (e1[r] < NE) {
                    if (!PF) load1(r, plane_of(p), fr[r], Dn[r]);
                    double f[Q];
#pragma unroll
                    for (int q = 0; q < Q; ++q) f[q] = (double)fr[r][q];
                    collide3(a, f, (double)Dn[r]);
                    const int e = e1[r];
#pragma unroll
                    for (int i = 0; i < 9; ++i) sin_[s2][i][e] = (float)f[kIn[i]];
#pragma unroll
                    for (int i = 0; i < 5; ++i) sup[s3][i][e] = (float)f[kUp[i]];
#pragma unroll
                    for (int i = 0; i < 5; ++i) sdn[s2][i][e] = (float)f[kDn[i]];
                }
            }
        }
        lds_barrier();
        // ---- loads for the next plane's step 1, in flight during step 2
        if (PF && p + 1 <= zend && have1(p + 1)) {
#pragma unroll
            for (int r = 0; r < R1; ++r)
                if (e1[r] < NE) load1(r, plane_of(p + 1), fr[r], Dn[r]);
        }
        // ---- step 2 on plane p - 1
        const int qz = p - 1;
        if (qz >= z0 && qz < zend && act2) {
            const int i0 = (rr - 1) & 1;       // plane qz: in-plane and -z slots
            const int um = (rr + 1) % 3;       // plane qz - 1: +z slot
            const int u0 = (rr + 2) % 3;       // plane qz: +z slot (top wall)
            const int dp = rr & 1;             // plane qz + 1: -z slot
            const bool blo = WALLS && qz == 0, bhi = WALLS && qz == a.nz - 1;
            const int e = e2;
            float g[Q];
            g[0] = sin_[i0][0][e];
            g[1] = sin_[i0][1][e - 1];
            g[2] = sin_[i0][2][e + 1];
            g[3] = sin_[i0][3][e - EX];
            g[4] = sin_[i0][4][e + EX];
            g[7] = sin_[i0][5][e - EX - 1];
            g[8] = sin_[i0][6][e + EX + 1];
            g[9] = sin_[i0][7][e + EX - 1];
            g[10] = sin_[i0][8][e - EX + 1];
            if (blo) {  // +z populations come back from the wall below as -z ones
                g[5] = sdn[i0][0][e];
                g[11] = sdn[i0][1][e];
                g[14] = sdn[i0][2][e];
                g[15] = sdn[i0][3][e];
                g[18] = sdn[i0][4][e];
            } else {
                g[5] = sup[um][0][e];
                g[11] = sup[um][1][e - 1];
                g[14] = sup[um][2][e + 1];
                g[15] = sup[um][3][e - EX];
                g[18] = sup[um][4][e + EX];
            }
            if (bhi) {
                g[6] = sup[u0][0][e];
                g[12] = sup[u0][1][e];
                g[13] = sup[u0][2][e];
                g[16] = sup[u0][3][e];
                g[17] = sup[u0][4][e];
            } else {
                g[6] = sdn[dp][0][e];
                g[12] = sdn[dp][1][e + 1];
                g[13] = sdn[dp][2][e - 1];
                g[16] = sdn[dp][3][e + EX];
                g[17] = sdn[dp][4][e - EX];
            }
            const unsigned c = (unsigned)qz * pn + (unsigned)gy2 * a.nx + gx2;
            double f[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) f[q] = (double)g[q];
            collide3(a, f, (double)*reinterpret_cast<const float *>(
                               reinterpret_cast<const char *>(a.coef) + c * 4u));
#pragma unroll
            for (int q = 0; q < Q; ++q)
                *reinterpret_cast<float *>(reinterpret_cast<char *>(a.fout + (size_t)q * a.stride) + c * 4u) =
                    (float)f[q];
        }
        // the next step 1 overwrites the slots of planes p - 1 (two-slot
        // rings) and p - 2 (+z ring)
        lds_barrier();
    }
}

// Flow velocity and density of the current state (FP64), and per-block FP64
// partial sums of u for the volume average.
template <typename R, bool WALLS>
__global__ __launch_bounds__(kBlock3) void k3_fields(Args3<R> a, double *__restrict__ u_out,
                                                     double *__restrict__ rho_out,
                                                     double *__restrict__ partials)
{
    __shared__ double red[3][kBlock3 / 64];
    int x, y, z;
    double ux = 0.0, uy = 0.0, uz = 0.0;
    if (cell_of(a.nx, a.ny, x, y, z)) {
        R fr[Q];
        pull3<R, WALLS>(a.fin, a.stride, a.nx, a.ny, a.nz, x, y, z, fr);
        double f[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) f[q] = (double)fr[q];
        double dr, jx, jy, jz;
        moments3(f, dr, jx, jy, jz);
        const double rho = a.rho0 + dr;
        const size_t c = ((size_t)z * a.ny + y) * a.nx + x;
        const double D = 1.0 - (double)a.coef[c];
        ux = D * (jx + a.hegx * rho) / rho;
        uy = D * (jy + a.hegy * rho) / rho;
        uz = D * (jz + a.hegz * rho) / rho;
        const size_t N = (size_t)a.nx * a.ny * a.nz;
        if (u_out) {
            u_out[c] = ux;
            u_out[N + c] = uy;
            u_out[2 * N + c] = uz;
        }
        if (rho_out) rho_out[c] = rho;
    }
    if (partials) {
        ux = wave_sum(ux);
        uy = wave_sum(uy);
        uz = wave_sum(uz);
        const int wv = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
            red[0][wv] = ux;
            red[1][wv] = uy;
            red[2][wv] = uz;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double s[3] = {0.0, 0.0, 0.0};
            for (int k = 0; k < 3; ++k)
                for (int w = 0; w < kBlock3 / 64; ++w) s[k] += red[k][w];
            // partials are indexed by the tile, not the dispatch order
            int tx, ty, tz;
            cell_of(a.nx, a.ny, tx, ty, tz);
            const int ntx = (a.nx + kTX - 1) / kTX, nty = (a.ny + kTY - 1) / kTY;
            const int t = (tz * nty + ty / kTY) * ntx + tx / kTX;
            partials[3 * t] = s[0];
            partials[3 * t + 1] = s[1];
            partials[3 * t + 2] = s[2];
        }
    }
}

// Fixed-order sum of n triples, divided by the number of cells.
__global__ __launch_bounds__(256) void k3_reduce(const double *__restrict__ partials, int n,
                                                 double inv_cells, double *__restrict__ out)
{
    __shared__ double red[3][4];
    double s[3] = {0.0, 0.0, 0.0};
    // each thread adds its partials in index order, reading 8 of them ahead
    constexpr int kAhead = 8;
    for (int i0 = threadIdx.x; i0 < n; i0 += kAhead * 256) {
        double v[kAhead][3];
#pragma unroll
        for (int u = 0; u < kAhead; ++u) {
            const int i = min(i0 + u * 256, n - 1);
#pragma unroll
            for (int k = 0; k < 3; ++k) v[u][k] = partials[3 * i + k];
        }
#pragma unroll
        for (int u = 0; u < kAhead; ++u)
            if (i0 + u * 256 < n)
#pragma unroll
                for (int k = 0; k < 3; ++k) s[k] += v[u][k];
    }
    for (int k = 0; k < 3; ++k) s[k] = wave_sum(s[k]);
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < 3; ++k) red[k][wv] = s[k];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) out[k] = (((red[k][0] + red[k][1]) + red[k][2]) + red[k][3]) * inv_cells;
}

__global__ void k3_zero_flag(int *p)
{
    if (threadIdx.x == 0) p[0] = 0;
}

// Drag coefficient D per cell from kappa (FP64, rounded once to R), and the
// rest state (zero deviations).
template <typename R>
__global__ __launch_bounds__(256) void k3_init(const double *__restrict__ kappa, size_t n, double h,
                                               R *__restrict__ coef, R *__restrict__ pops,
                                               size_t stride, int *__restrict__ bad)
{
    const size_t c = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= n) return;
    const double k = kappa[c];
    if (!(k > 0.0)) atomicOr(bad, 1);  // also NaN; +inf gives E = 0 (no drag)
    coef[c] = (R)(h / (k + h));         // E = 1 - D, D = 1 / (1 + h / kappa)
#pragma unroll
    for (int q = 0; q < Q; ++q) pops[(size_t)q * stride + c] = (R)0;
}

// Full pre-collision populations, FP64 [19][nz][ny][nx].
template <typename R, bool WALLS>
__global__ __launch_bounds__(kBlock3) void k3_get(const R *__restrict__ fin, size_t S, int nx, int ny,
                                                  int nz, double rho0, double *__restrict__ out)
{
    int x, y, z;
    if (!cell_of(nx, ny, x, y, z)) return;
    R f[Q];
    pull3<R, WALLS>(fin, S, nx, ny, nz, x, y, z, f);
    const size_t N = (size_t)nx * ny * nz, c = ((size_t)z * ny + y) * nx + x;
#pragma unroll
    for (int q = 0; q < Q; ++q) out[q * N + c] = (double)f[q] + wgt(q) * rho0;
}

// Inverse of the pull: stored g_b(x) = f_b(x + e_b), or f_opp(b)(x) where
// x + e_b lies beyond a wall.
template <typename R, bool WALLS>
__global__ __launch_bounds__(kBlock3) void k3_set(const double *__restrict__ in, int nx, int ny, int nz,
                                                  double rho0, R *__restrict__ fout, size_t S)
{
    int x, y, z;
    if (!cell_of(nx, ny, x, y, z)) return;
    const size_t N = (size_t)nx * ny * nz, c = ((size_t)z * ny + y) * nx + x;
#pragma unroll
    for (int b = 0; b < Q; ++b) {
        int xs = x + cx(b), ys = y + cy(b), zs = z + cz(b);
        xs = xs < 0 ? nx - 1 : (xs >= nx ? 0 : xs);
        ys = ys < 0 ? ny - 1 : (ys >= ny ? 0 : ys);
        int src = b;
        if (zs < 0 || zs >= nz) {
            if (WALLS) {
                xs = x;
                ys = y;
                zs = z;
                src = opp(b);
            } else {
                zs = zs < 0 ? nz - 1 : 0;
            }
        }
        const double v = in[src * N + ((size_t)zs * ny + ys) * nx + xs] - wgt(src) * rho0;
        fout[(size_t)b * S + c] = (R)v;
    }
}

struct Layout3 {
    size_t elem, stride, n;
    size_t off_a, off_b, off_coef, off_part, off_res, off_flag, total;
    int ntiles;
};

bool params_ok(const lbm3d_params *p, std::string &why)
{
    if (!p) { why = "params is NULL"; return false; }
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) { why = "nx, ny and nz must be >= 1"; return false; }
    // byte offsets within a plane are 32-bit
    const int64_t n = (int64_t)p->nx * p->ny * p->nz;
    const int64_t elem = p->pop_dtype == LBM_F64 ? 8 : 4;
    if ((n + 65536) * elem >= ((int64_t)1 << 32)) { why = "grid too large (nx ny nz times the population size must be below 4 GiB)"; return false; }
    if (!(p->tau >= 0.5) || !std::isfinite(p->tau)) { why = "tau must be finite and >= 0.5"; return false; }
    if (!(p->eps > 0.0 && p->eps <= 1.0)) { why = "eps must lie in (0, 1]"; return false; }
    if (!(p->nu > 0.0) || !std::isfinite(p->nu)) { why = "nu must be finite and > 0"; return false; }
    if (!(p->rho0 > 0.0) || !std::isfinite(p->rho0)) { why = "rho0 must be finite and > 0"; return false; }
    if (!std::isfinite(p->gx) || !std::isfinite(p->gy) || !std::isfinite(p->gz)) { why = "gx, gy, gz must be finite"; return false; }
    if (p->walls_z != 0 && p->walls_z != 1) { why = "walls_z must be 0 or 1"; return false; }
    if (p->pop_dtype != LBM_F32_SHIFTED && p->pop_dtype != LBM_F64) { why = "unknown pop_dtype"; return false; }
    return true;
}

Layout3 layout_of(const lbm3d_params *p)
{
    Layout3 L{};
    L.n = (size_t)p->nx * p->ny * p->nz;
    L.elem = p->pop_dtype == LBM_F64 ? 8 : 4;
    L.stride = align_up(L.n, 64) + kPlanePad / L.elem;
    L.ntiles = ((p->nx + kTX - 1) / kTX) * ((p->ny + kTY - 1) / kTY) * p->nz;
    size_t off = 0;
    L.off_a = off;    off = align_up(off + Q * L.stride * L.elem);
    L.off_b = off;    off = align_up(off + Q * L.stride * L.elem);
    L.off_coef = off; off = align_up(off + L.n * L.elem);
    L.off_part = off; off = align_up(off + 3 * sizeof(double) * (size_t)L.ntiles);
    L.off_res = off;  off = align_up(off + 4 * sizeof(double));
    L.off_flag = off; off = align_up(off + sizeof(int));
    L.total = off;
    return L;
}

}  // namespace
}  // namespace lbm3

struct lbm3d_handle {
    lbm3d_params p;
    lbm3::Layout3 L;
    hipStream_t stream;
    char *ws;
    int cur;
    int64_t steps_total;
    double prev_u[3];
    bool have_prev;
    double *host_res;
    int zchunk;         // planes per workgroup run of the two-step kernel
};

namespace lbm3 {
namespace {

template <typename R>
Args3<R> args_of(const lbm3d_handle *h)
{
    Args3<R> a{};
    a.fin = reinterpret_cast<const R *>(h->ws + (h->cur ? h->L.off_b : h->L.off_a));
    a.fout = reinterpret_cast<R *>(h->ws + (h->cur ? h->L.off_a : h->L.off_b));
    a.coef = reinterpret_cast<const R *>(h->ws + h->L.off_coef);
    a.nx = h->p.nx;
    a.ny = h->p.ny;
    a.nz = h->p.nz;
    a.stride = h->L.stride;
    a.hegx = 0.5 * h->p.eps * h->p.gx;
    a.hegy = 0.5 * h->p.eps * h->p.gy;
    a.hegz = 0.5 * h->p.eps * h->p.gz;
    a.om = 1.0 / h->p.tau;
    a.omc = 1.0 - 1.0 / h->p.tau;
    a.twotau = 2.0 * h->p.tau;
    a.omtt = 1.0 - 2.0 * h->p.tau;
    a.rho0 = h->p.rho0;
    return a;
}

template <typename R, bool W>
void launch_step(const lbm3d_handle *h)
{
    hipLaunchKernelGGL((k3_step<R, W>), dim3(h->L.ntiles), dim3(kBlock3), 0, h->stream, args_of<R>(h));
}

template <typename R, bool W>
void launch_fields(const lbm3d_handle *h, double *u, double *rho, double *part)
{
    hipLaunchKernelGGL((k3_fields<R, W>), dim3(h->L.ntiles), dim3(kBlock3), 0, h->stream, args_of<R>(h),
                       u, rho, part);
}

// Planes per workgroup run: the number of runs per column that minimises
// (waves of workgroups over the CUs, one resident per CU) x (planes per run
// + the two extra step-1 planes), so the grid neither leaves CUs idle in its
// last wave nor repeats many halo planes.
int zchunk_for(int nx, int ny, int nz)
{
    const int64_t cols = (int64_t)((nx + k2IX - 1) / k2IX) * ((ny + k2IY - 1) / k2IY);
    const int64_t slots = std::max(1, lbm::device_cu_count());
    int best_zc = nz;
    int64_t best = -1;
    for (int runs = 1; runs <= nz; ++runs) {
        const int zc = (nz + runs - 1) / runs;
        if (runs > 1 && (nz + zc - 1) / zc != runs) continue;  // same zc as a smaller count
        const int64_t waves = (cols * runs + slots - 1) / slots;
        const int64_t cost = waves * (zc + 2);
        if (best < 0 || cost < best) {
            best = cost;
            best_zc = zc;
        }
        if (zc <= 8) break;
    }
    return best_zc;
}

template <bool W>
void launch_step2(const lbm3d_handle *h)
{
    const int zc = h->zchunk;
    const int nt = ((h->p.nx + k2IX - 1) / k2IX) * ((h->p.ny + k2IY - 1) / k2IY) *
                   ((h->p.nz + zc - 1) / zc);
    hipLaunchKernelGGL((k3_step2<W>), dim3(nt), dim3(k2T), 0, h->stream, args_of<float>(h), zc);
}

// Two steps in one launch (FP32 state only).
void step_twice(const lbm3d_handle *h)
{
    if (h->p.walls_z != 0) launch_step2<true>(h); else launch_step2<false>(h);
}

void step_once(const lbm3d_handle *h)
{
    const bool w = h->p.walls_z != 0;
    if (h->p.pop_dtype == LBM_F64) {
        if (w) launch_step<double, true>(h); else launch_step<double, false>(h);
    } else {
        if (w) launch_step<float, true>(h); else launch_step<float, false>(h);
    }
}

void fields(const lbm3d_handle *h, double *u, double *rho, double *part)
{
    const bool w = h->p.walls_z != 0;
    if (h->p.pop_dtype == LBM_F64) {
        if (w) launch_fields<double, true>(h, u, rho, part); else launch_fields<double, false>(h, u, rho, part);
    } else {
        if (w) launch_fields<float, true>(h, u, rho, part); else launch_fields<float, false>(h, u, rho, part);
    }
}

lbm_status mean_velocity(lbm3d_handle *h, double out[3])
{
    double *part = reinterpret_cast<double *>(h->ws + h->L.off_part);
    double *res = reinterpret_cast<double *>(h->ws + h->L.off_res);
    fields(h, nullptr, nullptr, part);
    hipLaunchKernelGGL(k3_reduce, dim3(1), dim3(256), 0, h->stream, part, h->L.ntiles,
                       1.0 / (double)h->L.n, res);
    LBM_HIP(hipGetLastError());
    LBM_HIP(hipMemcpyAsync(h->host_res, res, 3 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    LBM_HIP(hipStreamSynchronize(h->stream));
    for (int k = 0; k < 3; ++k) out[k] = h->host_res[k];
    return LBM_OK;
}

}  // namespace
}  // namespace lbm3

using namespace lbm3;

extern "C" size_t lbm3d_workspace_bytes(const lbm3d_params *p)
{
    std::string why;
    if (!params_ok(p, why)) return 0;
    return layout_of(p).total;
}

extern "C" lbm_status lbm3d_init(lbm3d_handle **out, const lbm3d_params *p, const double *d_kappa,
                                 void *d_ws, size_t ws_bytes, hipStream_t stream)
{
    if (!out) return set_error(LBM_EINVAL, "lbm3d_init: handle pointer is NULL");
    *out = nullptr;
    std::string why;
    if (!params_ok(p, why)) return set_error(LBM_EINVAL, "lbm3d_init: " + why);
    if (!d_kappa) return set_error(LBM_EINVAL, "lbm3d_init: permeability pointer is NULL");
    const Layout3 L = layout_of(p);
    if (!d_ws || ((uintptr_t)d_ws % kAlign) != 0)
        return set_error(LBM_EWORKSPACE, "lbm3d_init: workspace is NULL or not 256-byte aligned");
    if (ws_bytes < L.total)
        return set_error(LBM_EWORKSPACE, "lbm3d_init: workspace too small (need " +
                                             std::to_string(L.total) + " bytes)");
    lbm3d_handle *h = new (std::nothrow) lbm3d_handle{};
    if (!h) return set_error(LBM_EINVAL, "lbm3d_init: out of host memory");
    h->p = *p;
    h->L = L;
    h->stream = stream;
    h->ws = static_cast<char *>(d_ws);
    h->zchunk = zchunk_for(p->nx, p->ny, p->nz);
    if (hipHostMalloc((void **)&h->host_res, 4 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        delete h;
        return set_error(LBM_EDEVICE, "lbm3d_init: hipHostMalloc failed");
    }
    int *flag = reinterpret_cast<int *>(h->ws + L.off_flag);
    const double hh = 0.5 * p->eps * p->nu;
    const unsigned nb = (unsigned)((L.n + 255) / 256);
    hipLaunchKernelGGL(k3_zero_flag, dim3(1), dim3(64), 0, stream, flag);
    if (p->pop_dtype == LBM_F64)
        hipLaunchKernelGGL((k3_init<double>), dim3(nb), dim3(256), 0, stream, d_kappa, L.n, hh,
                           reinterpret_cast<double *>(h->ws + L.off_coef),
                           reinterpret_cast<double *>(h->ws + L.off_a), L.stride, flag);
    else
        hipLaunchKernelGGL((k3_init<float>), dim3(nb), dim3(256), 0, stream, d_kappa, L.n, hh,
                           reinterpret_cast<float *>(h->ws + L.off_coef),
                           reinterpret_cast<float *>(h->ws + L.off_a), L.stride, flag);
    hipError_t e = hipGetLastError();
    int bad = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess || bad) {
        (void)hipHostFree(h->host_res);
        delete h;
        if (e != hipSuccess) return hip_check(e, "lbm3d_init");
        return set_error(LBM_EINVAL, "lbm3d_init: permeability must be > 0 (or +inf)");
    }
    *out = h;
    return LBM_OK;
}

extern "C" lbm_status lbm3d_step(lbm3d_handle *h, int64_t max_steps, double tol, int32_t check_every,
                                 int64_t *steps_done, double mean_u[3])
{
    if (!h) return set_error(LBM_EINVAL, "lbm3d_step: handle is NULL");
    if (max_steps < 0) return set_error(LBM_EINVAL, "lbm3d_step: max_steps must be >= 0");
    if (check_every < 0) return set_error(LBM_EINVAL, "lbm3d_step: check_every must be >= 0");
    if (tol > 0.0 && check_every == 0)
        return set_error(LBM_EINVAL, "lbm3d_step: a tolerance needs check_every > 0");
    if (steps_done) *steps_done = 0;
    lbm_status st = tol > 0.0 ? LBM_ENOTCONV : LBM_OK;
    int64_t done = 0;
    bool last_checked = false;
    double u[3] = {0.0, 0.0, 0.0};
    while (done < max_steps) {
        // two steps per launch unless a check or the end falls in between
        const int64_t to_check = check_every > 0 ? check_every - done % check_every : max_steps - done;
        const int n = (h->p.pop_dtype == LBM_F32_SHIFTED &&
                       std::min<int64_t>(to_check, max_steps - done) >= 2) ? 2 : 1;
        if (n == 2)
            step_twice(h);
        else
            step_once(h);
        h->cur ^= 1;
        done += n;
        h->steps_total += n;
        last_checked = false;
        if (check_every > 0 && done % check_every == 0) {
            LBM_HIP(hipGetLastError());
            lbm_status s = mean_velocity(h, u);
            if (s != LBM_OK) return s;
            last_checked = true;
            if (!std::isfinite(u[0]) || !std::isfinite(u[1]) || !std::isfinite(u[2])) {
                st = LBM_ENONFINITE;
                break;
            }
            if (tol > 0.0 && h->have_prev) {
                double d2 = 0.0, n2 = 0.0;
                for (int k = 0; k < 3; ++k) {
                    d2 += (u[k] - h->prev_u[k]) * (u[k] - h->prev_u[k]);
                    n2 += u[k] * u[k];
                }
                if (std::sqrt(d2) <= tol * std::sqrt(n2)) {
                    for (int k = 0; k < 3; ++k) h->prev_u[k] = u[k];
                    st = LBM_OK;
                    break;
                }
            }
            for (int k = 0; k < 3; ++k) h->prev_u[k] = u[k];
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
        for (int k = 0; k < 3; ++k) mean_u[k] = u[k];
        if (st == LBM_OK && !(std::isfinite(u[0]) && std::isfinite(u[1]) && std::isfinite(u[2])))
            st = LBM_ENONFINITE;
    }
    if (st == LBM_ENOTCONV) return set_error(st, "lbm3d_step: tolerance not reached within max_steps");
    if (st == LBM_ENONFINITE) return set_error(st, "lbm3d_step: non-finite mean velocity");
    return LBM_OK;
}

extern "C" lbm_status lbm3d_fields(lbm3d_handle *h, double *d_u, double *d_rho)
{
    if (!h) return set_error(LBM_EINVAL, "lbm3d_fields: handle is NULL");
    if (!d_u && !d_rho) return set_error(LBM_EINVAL, "lbm3d_fields: no output given");
    fields(h, d_u, d_rho, nullptr);
    LBM_HIP(hipGetLastError());
    return LBM_OK;
}

extern "C" lbm_status lbm3d_get_populations(lbm3d_handle *h, double *d_f)
{
    if (!h || !d_f) return set_error(LBM_EINVAL, "lbm3d_get_populations: NULL argument");
    const char *cur = h->ws + (h->cur ? h->L.off_b : h->L.off_a);
    const bool w = h->p.walls_z != 0;
    const dim3 g(h->L.ntiles), b(kBlock3);
    const size_t S = h->L.stride;
    const int nx = h->p.nx, ny = h->p.ny, nz = h->p.nz;
    if (h->p.pop_dtype == LBM_F64) {
        auto *fin = reinterpret_cast<const double *>(cur);
        if (w) hipLaunchKernelGGL((k3_get<double, true>), g, b, 0, h->stream, fin, S, nx, ny, nz, h->p.rho0, d_f);
        else   hipLaunchKernelGGL((k3_get<double, false>), g, b, 0, h->stream, fin, S, nx, ny, nz, h->p.rho0, d_f);
    } else {
        auto *fin = reinterpret_cast<const float *>(cur);
        if (w) hipLaunchKernelGGL((k3_get<float, true>), g, b, 0, h->stream, fin, S, nx, ny, nz, h->p.rho0, d_f);
        else   hipLaunchKernelGGL((k3_get<float, false>), g, b, 0, h->stream, fin, S, nx, ny, nz, h->p.rho0, d_f);
    }
    LBM_HIP(hipGetLastError());
    return LBM_OK;
}

extern "C" lbm_status lbm3d_set_populations(lbm3d_handle *h, const double *d_f)
{
    if (!h || !d_f) return set_error(LBM_EINVAL, "lbm3d_set_populations: NULL argument");
    char *cur = h->ws + (h->cur ? h->L.off_b : h->L.off_a);
    const bool w = h->p.walls_z != 0;
    const dim3 g(h->L.ntiles), b(kBlock3);
    const size_t S = h->L.stride;
    const int nx = h->p.nx, ny = h->p.ny, nz = h->p.nz;
    if (h->p.pop_dtype == LBM_F64) {
        auto *fo = reinterpret_cast<double *>(cur);
        if (w) hipLaunchKernelGGL((k3_set<double, true>), g, b, 0, h->stream, d_f, nx, ny, nz, h->p.rho0, fo, S);
        else   hipLaunchKernelGGL((k3_set<double, false>), g, b, 0, h->stream, d_f, nx, ny, nz, h->p.rho0, fo, S);
    } else {
        auto *fo = reinterpret_cast<float *>(cur);
        if (w) hipLaunchKernelGGL((k3_set<float, true>), g, b, 0, h->stream, d_f, nx, ny, nz, h->p.rho0, fo, S);
        else   hipLaunchKernelGGL((k3_set<float, false>), g, b, 0, h->stream, d_f, nx, ny, nz, h->p.rho0, fo, S);
    }
    h->have_prev = false;
    LBM_HIP(hipGetLastError());
    return LBM_OK;
}

extern "C" int64_t lbm3d_steps_total(const lbm3d_handle *h) { return h ? h->steps_total : -1; }

extern "C" void lbm3d_destroy(lbm3d_handle *h)
{
    if (!h) return;
    if (h->host_res) (void)hipHostFree(h->host_res);
    delete h;
}
