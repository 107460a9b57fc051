// lbm_coarse.hip -- coarse-grid solve of the upscaled scheme (Sec. 3, Sec. 4.3).
//
// Each coarse cell stands for an r x r subdomain of the fine grid and carries
// the effective permeability found by the local problems. The coarse run uses
// the same scheme as the fine grid with the same physical rho0, nu_eff, eps,
// nu and G, while dx and dt both grow by r (Sec. 4.3: dx 0.0025 -> 0.025 m and
// dt 2.5e-5 -> 2.5e-4 s, tau 0.50012 -> 0.500012). In lattice units:
//   tau_c = 1/2 + (tau_f - 1/2) / r,  nu_c = nu_f / r,
//   kappa_c = kappa_f / r^2,           G_c = r G_f,   u_c = u_f.
// The drag uses either the scalar kappa* = (kxx + kyy) / 2 (Sec. 4.3) or the
// full tensor (Eq. f_m-depends-on-u-and-tensor-k), through the per-cell matrix
// M = (K + eps nu I / 2)^{-1} K with rho u = M (j + eps rho G / 2).
//
// Coarse grids that fit in one CU's LDS (8 planes x 4 B x cells) run in a
// single persistent workgroup with the in-place AA streaming of the local
// solver, so a coarse step costs no kernel launch; larger coarse grids run on
// the HBM fine-grid path with a tensor permeability.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "lbm_internal.h"

namespace lbm {
namespace {

constexpr int kT = 1024;
constexpr int kCPT32 = 4;  // cells per thread, FP32 populations (4096 cells)
constexpr int kCPT64 = 2;  // cells per thread, FP64 populations (2048 cells)

template <typename R>
struct CoarseArgs {
    int nx, ny;
    const R *__restrict__ M;         // [4][N] per-cell drag deficit E = I - M (e00, e01, e10, e11),
                                     // M = (K + h I)^{-1} K; E keeps its relative precision in FP32
    const R *__restrict__ heg;       // [2][N] eps G_c / 2 per cell
    double om, omc, twotau, omtt;
    double tol;
    int check_every;
    int max_steps;
    double *__restrict__ u_out;      // [2][N]
    double *__restrict__ rho_out;    // [N] or null
    long long *__restrict__ status;  // [0] steps, [1] flag
};

// Coefficients of the coarse lattice from the effective permeability (FP64),
// rounded once to the storage type R.
template <typename R>
__global__ void k_coarse_coef(const double *__restrict__ keff, const double *__restrict__ force, int n,
                              int tensor, double r, double eps, double nu_c, double gxf, double gyf,
                              R *__restrict__ M, R *__restrict__ heg, double *__restrict__ perm_c,
                              double *__restrict__ force_c, int *__restrict__ bad)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const double s = 1.0 / (r * r);  // kappa_c = kappa_f / r^2
    double kxx = keff[4 * c] * s, kxy = keff[4 * c + 1] * s, kyx = keff[4 * c + 2] * s, kyy = keff[4 * c + 3] * s;
    if (!tensor) {
        const double k = 0.5 * (kxx + kyy);
        kxx = kyy = k;
        kxy = kyx = 0.0;
    }
    const double h = 0.5 * eps * nu_c;
    const double det = kxx * kyy - kxy * kyx;
    const double axx = kxx + h, ayy = kyy + h;
    const double adet = axx * ayy - kxy * kyx;
    if (!(std::isfinite(det) && det > 0.0 && std::isfinite(adet) && adet != 0.0 && kxx > 0.0 && kyy > 0.0))
        atomicOr(bad, 1);
    // E = I - M = h (K + h I)^{-1}: rounded to FP32, M itself would lose the
    // relative precision of the drag I - M of permeable cells
    const double ia = h / adet;
    const int N = n;
    M[c] = (R)(ia * ayy);
    M[N + c] = (R)(-ia * kxy);
    M[2 * N + c] = (R)(-ia * kyx);
    M[3 * N + c] = (R)(ia * axx);
    const double gx = r * (force ? force[2 * c] : gxf), gy = r * (force ? force[2 * c + 1] : gyf);
    heg[c] = (R)(0.5 * eps * gx);
    heg[N + c] = (R)(0.5 * eps * gy);
    if (perm_c) {
        perm_c[4 * c] = kxx;
        perm_c[4 * c + 1] = kxy;
        perm_c[4 * c + 2] = kyx;
        perm_c[4 * c + 3] = kyy;
        force_c[2 * c] = gx;
        force_c[2 * c + 1] = gy;
    }
}

// Collision in FP64 (deviation form, tensor drag), f in and out.
template <typename R>
__device__ __forceinline__ void collide_t(double f[9], const R m[4], R hx0, R hy0, const CoarseArgs<R> &a)
{
    const double dr = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
    const double jx = (f[1] - f[3]) + ((f[5] - f[6]) + (f[8] - f[7]));
    const double jy = (f[2] - f[4]) + ((f[5] + f[6]) - (f[7] + f[8]));
    const double rho = 1.0 + dr;
    const double hx = jx + (double)hx0 * rho, hy = jy + (double)hy0 * rho;
    // M h = h - E h
    const double mx = a.twotau * ((hx - (double)m[0] * hx) - (double)m[1] * hy) + a.omtt * jx;
    const double my = a.twotau * ((hy - (double)m[3] * hy) - (double)m[2] * hx) + a.omtt * jy;
    const double om = a.om, omc = a.omc;
    const double s0 = (4.0 / 9.0) * om * dr;
    const double b = (1.0 / 9.0) * om * dr;
    const double bx = (1.0 / 3.0) * om * mx;
    const double by = (1.0 / 3.0) * om * my;
    const double cc = (1.0 / 36.0) * om * dr;
    const double cx = (1.0 / 12.0) * om * mx;
    const double cy = (1.0 / 12.0) * om * my;
    const double pp = cx + cy, qq = cx - cy;
    f[0] = omc * f[0] + s0;
    f[1] = omc * f[1] + (b + bx);
    f[2] = omc * f[2] + (b + by);
    f[3] = omc * f[3] + (b - bx);
    f[4] = omc * f[4] + (b - by);
    f[5] = omc * f[5] + (cc + pp);
    f[6] = omc * f[6] + (cc - qq);
    f[7] = omc * f[7] + (cc - pp);
    f[8] = omc * f[8] + (cc + qq);
}

// Velocity of a cell in FP64 from its pre-collision deviations.
template <typename R>
__device__ __forceinline__ void cell_velocity(const double fd[9], const R m[4], R hx0, R hy0, double &ux,
                                              double &uy, double &rho)
{
    const double dr = ((fd[0] + fd[1]) + (fd[2] + fd[3])) + ((fd[4] + fd[5]) + (fd[6] + fd[7])) + fd[8];
    const double jx = (fd[1] - fd[3]) + ((fd[5] - fd[6]) + (fd[8] - fd[7]));
    const double jy = (fd[2] - fd[4]) + ((fd[5] + fd[6]) - (fd[7] + fd[8]));
    rho = 1.0 + dr;
    const double hx = jx + (double)hx0 * rho, hy = jy + (double)hy0 * rho;
    ux = ((hx - (double)m[0] * hx) - (double)m[1] * hy) / rho;
    uy = ((hy - (double)m[3] * hy) - (double)m[2] * hx) / rho;
}

// One workgroup runs the whole periodic coarse lattice to steady state.
// Convergence: relative L2 change of the velocity field between checks. The
// previous field is kept in the storage type R, and the new field is rounded
// to R before the difference, so a state that no longer changes gives
// exactly zero.
template <typename R, int CPT>
__global__ __launch_bounds__(kT) void k_coarse_onchip(CoarseArgs<R> a)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    R *A = reinterpret_cast<R *>(lds_raw);
    __shared__ double red[kT / 64][2];
    const int tid = threadIdx.x;
    const int nx = a.nx, ny = a.ny, N = nx * ny;
    const int C = (N + kT - 1) / kT;
    R f0[CPT], m[CPT][4], hg[CPT][2], upx[CPT], upy[CPT];
    int xy[CPT];
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
        const int c = tid + k * kT;
        if (k < C && c < N) {
            xy[k] = (c % nx) | ((c / nx) << 16);
            f0[k] = (R)0;
            m[k][0] = a.M[c];
            m[k][1] = a.M[N + c];
            m[k][2] = a.M[2 * N + c];
            m[k][3] = a.M[3 * N + c];
            hg[k][0] = a.heg[c];
            hg[k][1] = a.heg[N + c];
            upx[k] = (R)0;
            upy[k] = (R)0;
#pragma unroll
            for (int q = 0; q < 8; ++q) A[q * N + c] = (R)0;
        }
    }
    __syncthreads();
    int steps = 0, flag = 1;
    bool have_prev = false;
    while (true) {
        for (int st = 0; st < a.check_every; ++st) {
            const bool odd = (st & 1) != 0;
#pragma unroll
            for (int k = 0; k < CPT; ++k) {
                const int c = tid + k * kT;
                if (k < C && c < N) {
                    double f[9];
                    f[0] = (double)f0[k];
                    if (!odd) {
#pragma unroll
                        for (int q = 1; q < 9; ++q) f[q] = (double)A[(q - 1) * N + c];
                        collide_t(f, m[k], hg[k][0], hg[k][1], a);
                        A[2 * N + c] = (R)f[1];
                        A[3 * N + c] = (R)f[2];
                        A[0 * N + c] = (R)f[3];
                        A[1 * N + c] = (R)f[4];
                        A[6 * N + c] = (R)f[5];
                        A[7 * N + c] = (R)f[6];
                        A[4 * N + c] = (R)f[7];
                        A[5 * N + c] = (R)f[8];
                    } else {
                        const int x = xy[k] & 0xffff, y = xy[k] >> 16;
                        const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
                        const int rm = (y == 0 ? ny - 1 : y - 1) * nx, rp = (y == ny - 1 ? 0 : y + 1) * nx;
                        const int r0 = y * nx;
                        f[1] = (double)A[2 * N + r0 + xm];
                        f[2] = (double)A[3 * N + rm + x];
                        f[3] = (double)A[0 * N + r0 + xp];
                        f[4] = (double)A[1 * N + rp + x];
                        f[5] = (double)A[6 * N + rm + xm];
                        f[6] = (double)A[7 * N + rm + xp];
                        f[7] = (double)A[4 * N + rp + xp];
                        f[8] = (double)A[5 * N + rp + xm];
                        collide_t(f, m[k], hg[k][0], hg[k][1], a);
                        A[0 * N + r0 + xp] = (R)f[1];
                        A[1 * N + rp + x] = (R)f[2];
                        A[2 * N + r0 + xm] = (R)f[3];
                        A[3 * N + rm + x] = (R)f[4];
                        A[4 * N + rp + xp] = (R)f[5];
                        A[5 * N + rp + xm] = (R)f[6];
                        A[6 * N + rm + xm] = (R)f[7];
                        A[7 * N + rm + xp] = (R)f[8];
                    }
                    f0[k] = (R)f[0];
                }
                __builtin_amdgcn_sched_barrier(0);  // one cell at a time: bounded register use
            }
            __syncthreads();
        }
        steps += a.check_every;
        double d2 = 0.0, u2 = 0.0;
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int c = tid + k * kT;
            if (k < C && c < N) {
                double fd[9];
                fd[0] = (double)f0[k];
#pragma unroll
                for (int q = 1; q < 9; ++q) fd[q] = (double)A[(q - 1) * N + c];
                double ux, uy, rho;
                cell_velocity(fd, m[k], hg[k][0], hg[k][1], ux, uy, rho);
                const R rx = (R)ux, ry = (R)uy;
                const double dx = (double)rx - (double)upx[k], dy = (double)ry - (double)upy[k];
                d2 += dx * dx + dy * dy;
                u2 += ux * ux + uy * uy;
                upx[k] = rx;
                upy[k] = ry;
            }
        }
        d2 = wave_sum(d2);
        u2 = wave_sum(u2);
        if ((tid & 63) == 0) {
            red[tid >> 6][0] = d2;
            red[tid >> 6][1] = u2;
        }
        __syncthreads();
        double td = 0.0, tu = 0.0;
        for (int w = 0; w < kT / 64; ++w) {
            td += red[w][0];
            tu += red[w][1];
        }
        bool stop = false;
        if (!isfinite(td) || !isfinite(tu)) {
            flag = 2;
            stop = true;
        } else if (have_prev && a.tol > 0.0 && sqrt(td) <= a.tol * sqrt(tu)) {
            flag = 0;
            stop = true;
        } else if (steps >= a.max_steps) {
            flag = (a.tol > 0.0) ? 1 : 0;
            stop = true;
        }
        have_prev = true;
        __syncthreads();
        if (stop) break;
    }
    // final fields (state is in even order after an even number of steps)
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
        const int c = tid + k * kT;
        if (k < C && c < N) {
            double fd[9];
            fd[0] = (double)f0[k];
#pragma unroll
            for (int q = 1; q < 9; ++q) fd[q] = (double)A[(q - 1) * N + c];
            double ux, uy, rho;
            cell_velocity(fd, m[k], hg[k][0], hg[k][1], ux, uy, rho);
            a.u_out[c] = ux;
            a.u_out[N + c] = uy;
            if (a.rho_out) a.rho_out[c] = rho;
        }
    }
    if (tid == 0) {
        a.status[0] = steps;
        a.status[1] = flag;
    }
}

__global__ void k_zero_i32c(int *p) { p[0] = 0; }

// Mean of each r x r block of nplanes fields [plane][ny][nx]: one workgroup
// per output value, fixed-order FP64 sum.
__global__ __launch_bounds__(256) void k_block_average(const double *__restrict__ in, int nx, int ny, int r,
                                                       double *__restrict__ out)
{
    __shared__ double red[4];
    const int ncx = nx / r, ncy = ny / r;
    const int o = blockIdx.x;  // plane * ncx * ncy + J * ncx + I
    const int plane = o / (ncx * ncy), rem = o % (ncx * ncy);
    const int J = rem / ncx, I = rem % ncx;
    const double *f = in + (size_t)plane * nx * ny;
    double s = 0.0;
    for (int k = threadIdx.x; k < r * r; k += 256) {
        const int y = J * r + k / r, x = I * r + k % r;
        s += f[(size_t)y * nx + x];
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[o] = ((red[0] + red[1]) + (red[2] + red[3])) / ((double)r * r);
}

struct CoarseLayout {
    bool onchip;
    size_t lds;
    size_t off_M, off_heg, off_status, off_flag, off_perm, off_force, off_fine, fine_bytes, total;
};

int lds_budget()
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
        return v;
    return 64 * 1024;
}

CoarseLayout coarse_layout(int ncx, int ncy, bool f64, bool query_device)
{
    CoarseLayout L{};
    const size_t n = (size_t)ncx * ncy;
    const size_t es = f64 ? 8 : 4;
    L.lds = 8 * es * n;
    const size_t budget = query_device ? (size_t)lds_budget() - 2048 : 160 * 1024 - 2048;
    L.onchip = (n <= (size_t)kT * (f64 ? kCPT64 : kCPT32)) && L.lds <= budget;
    size_t off = 0;
    L.off_M = off;      off = align_up(off + 4 * n * sizeof(double));
    L.off_heg = off;    off = align_up(off + 2 * n * sizeof(double));
    L.off_status = off; off = align_up(off + 2 * sizeof(long long));
    L.off_flag = off;   off = align_up(off + sizeof(int));
    // the HBM path needs the coarse tensor, force and a fine-solver workspace;
    // size for it always, so the workspace does not depend on the device
    L.off_perm = off;   off = align_up(off + 4 * n * sizeof(double));
    L.off_force = off;  off = align_up(off + 2 * n * sizeof(double));
    lbm_params q{};
    q.nx = ncx; q.ny = ncy; q.tau = 0.75; q.eps = 0.5; q.nu = 0.1; q.rho0 = 1.0;
    q.walls_y = 0; q.pop_dtype = LBM_F64; q.perm_kind = LBM_PERM_TENSOR;
    L.fine_bytes = lbm_workspace_bytes(&q);
    L.off_fine = off;   off = align_up(off + L.fine_bytes);
    L.total = off;
    return L;
}

template <typename R, int CPT>
lbm_status launch_onchip(const lbm_params &pc, char *ws, const CoarseLayout &L, double tol, int check_every,
                         int64_t max_steps, double *d_u, double *d_rho, hipStream_t stream)
{
    CoarseArgs<R> a{};
    a.nx = pc.nx;
    a.ny = pc.ny;
    a.M = reinterpret_cast<const R *>(ws + L.off_M);
    a.heg = reinterpret_cast<const R *>(ws + L.off_heg);
    a.om = 1.0 / pc.tau;
    a.omc = 1.0 - 1.0 / pc.tau;
    a.twotau = 2.0 * pc.tau;
    a.omtt = 1.0 - 2.0 * pc.tau;
    a.tol = tol;
    a.check_every = check_every;
    a.max_steps = (int)std::min<int64_t>(max_steps, (int64_t)1 << 30);
    a.u_out = d_u;
    a.rho_out = d_rho;
    a.status = reinterpret_cast<long long *>(ws + L.off_status);
    if (L.lds > 64 * 1024)
        LBM_HIP(hipFuncSetAttribute((const void *)k_coarse_onchip<R, CPT>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.lds));
    hipLaunchKernelGGL((k_coarse_onchip<R, CPT>), dim3(1), dim3(kT), L.lds, stream, a);
    LBM_HIP(hipGetLastError());
    return LBM_OK;
}

}  // namespace
}  // namespace lbm

using namespace lbm;

extern "C" lbm_status lbm_coarse_params(const lbm_params *fine, int32_t r, lbm_params *coarse)
{
    if (!fine || !coarse) return set_error(LBM_EINVAL, "lbm_coarse_params: NULL argument");
    if (r < 1) return set_error(LBM_EINVAL, "lbm_coarse_params: r must be >= 1");
    if (fine->nx % r || fine->ny % r) return set_error(LBM_EINVAL, "lbm_coarse_params: r must divide nx and ny");
    if (fine->walls_y != 0) return set_error(LBM_EINVAL, "lbm_coarse_params: the coarse grid is periodic (walls_y = 0)");
    if (lbm_workspace_bytes(fine) == 0) return set_error(LBM_EINVAL, "lbm_coarse_params: invalid fine parameters");
    *coarse = *fine;
    coarse->nx = fine->nx / r;
    coarse->ny = fine->ny / r;
    coarse->tau = 0.5 + (fine->tau - 0.5) / r;
    coarse->nu = fine->nu / r;
    coarse->gx = fine->gx * r;
    coarse->gy = fine->gy * r;
    return LBM_OK;
}

extern "C" size_t lbm_coarse_workspace_bytes(int32_t ncx, int32_t ncy)
{
    if (ncx < 1 || ncy < 1) return 0;
    return coarse_layout(ncx, ncy, true, false).total;
}

extern "C" lbm_status lbm_coarse_solve(const lbm_params *fine, int32_t r, const double *d_keff, int32_t keff_mode,
                                       const double *d_force, int64_t max_steps, double tol, int32_t check_every,
                                       double *d_u, double *d_rho, int64_t *steps_done, void *d_ws,
                                       size_t ws_bytes, hipStream_t stream)
{
    const std::string fn = "lbm_coarse_solve: ";
    lbm_params pc{};
    lbm_status s = lbm_coarse_params(fine, r, &pc);
    if (s != LBM_OK) return s;
    if (fine->scheme != LBM_SCHEME_SHAN_CHEN) return set_error(LBM_EINVAL, fn + "the coarse solver runs the Shan-Chen form (scheme 0)");
    if (!d_keff || !d_u) return set_error(LBM_EINVAL, fn + "NULL keff or u");
    if (keff_mode != LBM_KEFF_SCALAR && keff_mode != LBM_KEFF_TENSOR) return set_error(LBM_EINVAL, fn + "bad keff_mode");
    if (check_every < 2 || (check_every & 1)) return set_error(LBM_EINVAL, fn + "check_every must be even and >= 2");
    if (max_steps < 1 || max_steps > (int64_t)1 << 30) return set_error(LBM_EINVAL, fn + "max_steps must lie in [1, 2^30]");
    if (!(tol >= 0.0)) return set_error(LBM_EINVAL, fn + "tol must be >= 0");
    const int ncx = pc.nx, ncy = pc.ny, n = ncx * ncy;
    const bool f64 = fine->pop_dtype == LBM_F64;
    const CoarseLayout L = coarse_layout(ncx, ncy, f64, true);
    const size_t need = coarse_layout(ncx, ncy, true, false).total;
    if (!d_ws || ((uintptr_t)d_ws % kAlign) != 0 || ws_bytes < need)
        return set_error(LBM_EWORKSPACE, fn + "workspace NULL, misaligned or smaller than " + std::to_string(need));
    char *ws = static_cast<char *>(d_ws);
    long long *status = reinterpret_cast<long long *>(ws + L.off_status);
    int *flag = reinterpret_cast<int *>(ws + L.off_flag);
    double *perm_c = reinterpret_cast<double *>(ws + L.off_perm);
    double *force_c = reinterpret_cast<double *>(ws + L.off_force);
    hipLaunchKernelGGL(k_zero_i32c, dim3(1), dim3(1), 0, stream, flag);
    const int tensor = keff_mode == LBM_KEFF_TENSOR ? 1 : 0;
    const dim3 cg((n + 255) / 256), cb(256);
    if (f64)
        hipLaunchKernelGGL(k_coarse_coef<double>, cg, cb, 0, stream, d_keff, d_force, n, tensor, (double)r, pc.eps, pc.nu,
                           fine->gx, fine->gy, reinterpret_cast<double *>(ws + L.off_M),
                           reinterpret_cast<double *>(ws + L.off_heg), L.onchip ? nullptr : perm_c,
                           L.onchip ? nullptr : force_c, flag);
    else
        hipLaunchKernelGGL(k_coarse_coef<float>, cg, cb, 0, stream, d_keff, d_force, n, tensor, (double)r, pc.eps, pc.nu,
                           fine->gx, fine->gy, reinterpret_cast<float *>(ws + L.off_M),
                           reinterpret_cast<float *>(ws + L.off_heg), L.onchip ? nullptr : perm_c,
                           L.onchip ? nullptr : force_c, flag);
    LBM_HIP(hipGetLastError());
    int bad = 0;
    LBM_HIP(hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, stream));
    LBM_HIP(hipStreamSynchronize(stream));
    if (bad) return set_error(LBM_EINVAL, fn + "effective permeability must be positive definite");

    if (L.onchip) {
        const int64_t ms = (max_steps + check_every - 1) / check_every * check_every;
        lbm_status ls = f64 ? launch_onchip<double, kCPT64>(pc, ws, L, tol, check_every, ms, d_u, d_rho, stream)
                            : launch_onchip<float, kCPT32>(pc, ws, L, tol, check_every, ms, d_u, d_rho, stream);
        if (ls != LBM_OK) return ls;
        long long hs[2] = {0, 0};
        LBM_HIP(hipMemcpyAsync(hs, status, sizeof(hs), hipMemcpyDeviceToHost, stream));
        LBM_HIP(hipStreamSynchronize(stream));
        if (steps_done) *steps_done = hs[0];
        if (hs[1] == 2) return set_error(LBM_ENONFINITE, fn + "non-finite velocity");
        if (hs[1] == 1) return set_error(LBM_ENOTCONV, fn + "tolerance not reached within max_steps");
        return LBM_OK;
    }

    // HBM path: the fine-grid solver with the coarse tensor permeability
    pc.perm_kind = LBM_PERM_TENSOR;
    pc.pop_dtype = f64 ? LBM_F64 : LBM_F32_SHIFTED;
    lbm_handle *h = nullptr;
    s = lbm_init(&h, &pc, perm_c, force_c, ws + L.off_fine, L.fine_bytes, stream);
    if (s != LBM_OK) return s;
    int64_t done = 0;
    double mu[2];
    s = lbm_step(h, max_steps, tol, check_every, &done, mu);
    if (steps_done) *steps_done = done;
    if (s == LBM_OK || s == LBM_ENOTCONV) {
        lbm_status s2 = lbm_fields(h, d_u, d_rho);
        if (s2 != LBM_OK) s = s2;
        else {
            hipError_t e = hipStreamSynchronize(stream);
            if (e != hipSuccess) s = hip_check(e, "lbm_coarse_solve");
        }
    }
    lbm_destroy(h);
    return s;
}

extern "C" lbm_status lbm_block_average(const double *d_in, int32_t nx, int32_t ny, int32_t nplanes, int32_t r,
                                        double *d_out, hipStream_t stream)
{
    if (!d_in || !d_out || nx < 1 || ny < 1 || nplanes < 1 || r < 1 || nx % r || ny % r)
        return set_error(LBM_EINVAL, "lbm_block_average: NULL pointer, or r does not divide nx and ny");
    const int64_t nout = (int64_t)nplanes * (nx / r) * (ny / r);
    if (nout >= (int64_t)1 << 31) return set_error(LBM_EINVAL, "lbm_block_average: too many blocks");
    hipLaunchKernelGGL(k_block_average, dim3((unsigned)nout), dim3(256), 0, stream, d_in, nx, ny, r, d_out);
    LBM_HIP(hipGetLastError());
    return LBM_OK;
}
