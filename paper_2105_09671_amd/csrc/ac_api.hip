// libac C ABI: argument validation, parameter derivation and launch planning
// for the 2D and 3D steppers.  Declarations and semantics: include/ac.h.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "ac_internal.h"
#include "reg2d.h"

namespace ac {

thread_local std::string g_err;

ac_status fail(ac_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

ac_status hip_fail(hipError_t e, const char *what) {
    return fail(AC_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

size_t elem_size(int32_t dtype) { return dtype == AC_F64 ? 8 : 4; }

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Checks shared by every stepping entry point.  Makes no HIP call.
ac_status validate(const void *phi, const void *work, int64_t ncells, int dim, double h,
                   double dt, double eps, int64_t nsteps, int32_t dtype, double *alpha,
                   double *r) {
    if (dtype != AC_F32 && dtype != AC_F64)
        return fail(AC_ERR_INVALID_ARG, "dtype must be AC_F32 (0) or AC_F64 (1), got %d", dtype);
    if (!phi || !work) return fail(AC_ERR_INVALID_ARG, "phi and work must be non-null");
    if ((reinterpret_cast<uintptr_t>(phi) | reinterpret_cast<uintptr_t>(work)) & 15u)
        return fail(AC_ERR_INVALID_ARG, "phi and work must be 16-byte aligned");
    const size_t bytes = (size_t)ncells * elem_size(dtype);
    const uintptr_t a = reinterpret_cast<uintptr_t>(phi), b = reinterpret_cast<uintptr_t>(work);
    if (a < b + bytes && b < a + bytes)
        return fail(AC_ERR_INVALID_ARG, "phi and work overlap");
    if (!finite_pos(h) || !finite_pos(dt) || !finite_pos(eps))
        return fail(AC_ERR_INVALID_ARG, "h, dt and eps must be finite and > 0 (h=%g dt=%g eps=%g)",
                    h, dt, eps);
    if (nsteps < 0) return fail(AC_ERR_INVALID_ARG, "nsteps must be >= 0, got %lld", (long long)nsteps);
    *alpha = dt / (eps * eps);
    *r = dt / (h * h);
    if (*r > 1.0 / (2.0 * dim))
        return fail(AC_ERR_UNSTABLE, "r = dt/h^2 = %g exceeds 1/(2d) = %g", *r, 1.0 / (2.0 * dim));
    const double amax = (1.0 - 2.0 * dim * *r) / 2.0;
    if (*alpha > amax)
        return fail(AC_ERR_UNSTABLE, "alpha = dt/eps^2 = %g exceeds (1 - 2d r)/2 = %g", *alpha, amax);
    return AC_OK;
}

// Split nsteps into launches of at most k steps such that the number of
// launches is even (ping-pong then ends in phi).  Returns false if that is
// impossible (every launch is a single step and the count is odd): the caller
// then copies work back into phi at the end.
Chunks plan_chunks(int64_t nsteps, int64_t k) {
    Chunks c{};
    if (nsteps <= 0 || k <= 0) return c;   // no launch (a plan query may ask for 0 steps)
    c.n = (nsteps + k - 1) / k;
    c.copy_back = false;
    if (c.n & 1) {
        if (nsteps >= c.n + 1) c.n += 1;
        else c.copy_back = true;
    }
    c.base = nsteps / c.n;
    c.rem = nsteps % c.n;
    return c;
}

// ------------------------------------------------------------ planning ----
// A plan fixes the kernel, its launch shape and the launch sequence of one
// call.  Built on the host from the device limits; executing it makes no other
// decision, so ac_plan_* reports exactly what ac_step_* will launch.
// Launch time of the 2D register-tile kernels on MI355X by depth K and tile
// height LY: about a + b * ceil(tiles / CUs) microseconds.  b is one tile's
// share of a CU's time while every CU streams tiles (two resident per CU); a
// is the rest of a launch (its start, the first loads that no step overlaps,
// the last stores).  Fitted by least squares in relative error to launches
// timed on FP32 grids 512^2 .. 16384^2 (with 2048 x 1024 and 4096 x 2048) and
// FP64 grids 512^2 .. 16384 x 8192, every pair on each grid in one run.  A small
// grid's launch is mostly a, so deep steps and few tiles win there; a large
// grid's is mostly b per tile.  Register tiles of 6 or 10 waves (64 x
// 96, 64 x 160) measured 10-25 % slower than 4, 8 or 12 and are left out, as
// are 128 x 128 FP64 tiles (16 waves), slower than 128 x 64 on every grid.
struct TileTime { int K, LY; double a, b; };
static const TileTime kRegF32[] = {
    {5, 64, 3.16, 1.624}, {5, 128, 2.33, 3.540}, {5, 192, 1.94, 5.460},
    {6, 64, 3.79, 1.676}, {6, 128, 3.09, 3.521}, {6, 192, 2.82, 5.391},
    {7, 64, 4.18, 1.752}, {7, 128, 3.38, 3.800}, {7, 192, 3.34, 5.602},
    {8, 64, 4.52, 1.951}, {8, 128, 3.96, 3.906}, {8, 192, 3.36, 5.891}};
static const TileTime kRegF64[] = {
    {5, 64, 2.74, 2.768}, {5, 128, 2.10, 5.931}, {5, 192, 1.41, 9.449},
    {6, 64, 3.49, 2.750}, {6, 128, 2.87, 6.165}, {6, 192, 2.85, 9.403},
    {7, 64, 3.93, 2.959}, {7, 128, 3.46, 6.514}, {7, 192, 3.67, 9.905},
    {8, 64, 4.34, 3.204}, {8, 128, 4.20, 6.662}, {8, 192, 3.74, 10.211}};
// 128-wide register tiles (two columns per lane)
static const TileTime kRegWF32[] = {
    {5, 32, 3.59, 1.417}, {5, 64, 2.79, 3.274}, {5, 96, 2.37, 5.398}, {5, 128, 1.44, 7.557},
    {6, 32, 3.97, 1.497}, {6, 64, 3.60, 3.147}, {6, 96, 3.10, 5.065}, {6, 128, 2.46, 7.239},
    {7, 32, 4.08, 1.636}, {7, 64, 3.73, 3.607}, {7, 96, 3.60, 5.407}, {7, 128, 2.85, 7.961},
    {8, 32, 4.53, 1.778}, {8, 64, 4.13, 3.735}, {8, 96, 3.91, 5.655}, {8, 128, 3.68, 7.760}};
static const TileTime kRegWF64[] = {
    {5, 32, 3.00, 2.407}, {5, 64, 1.73, 5.657},
    {6, 32, 3.33, 2.358}, {6, 64, 2.39, 5.487},
    {7, 32, 3.55, 2.627}, {7, 64, 2.81, 6.005},
    {8, 32, 3.82, 2.621}, {8, 64, 3.20, 5.882}};
// in place in LDS: GLUPS of the whole chip (256 CUs) streaming tiles
struct TileRate { int K, LY; double rate; };
static const TileRate kInplaceF32[] = {{6, 64, 1603}, {7, 64, 1617}, {8, 64, 1645},
                                       {6, 128, 1682}, {7, 128, 1707}, {8, 128, 1732}};
static const TileRate kInplaceF64[] = {{3, 32, 666}, {4, 32, 749}, {5, 32, 758}, {6, 32, 730},
                                       {3, 64, 661}, {4, 64, 719}, {5, 64, 731}, {6, 64, 725}};

// 3D: the register kernel is the default from half a round of resident
// workgroups on (measured on MI355X with flush tiles: 256^3 FP32, 0.57 rounds,
// 740 GLUPS against 715 on the LDS kernel; 192^3, 0.25 rounds, 387 against
// 509; 512^3 FP32 1254 against 817, 1024^3 1288 against 970)
static const int64_t kReg3dMinRoundsNum = 1, kReg3dMinRoundsDen = 2;

// The (depth, tile height) with the shortest predicted time per cell-step on
// this grid: ceil(tiles / CUs) is the busiest CU's tile count (the dispatcher
// spreads workgroups evenly), so a grid whose tile count just exceeds a
// multiple of the CU count gives some CUs one tile more, and the choice is
// made per grid.  Returns the predicted GLUPS.
double choose_tile2d(int nx, int ny, size_t elem, int kernel, const ac::DevInfo &dev, int *K,
                     int *LY) {
    const bool f64 = elem == 8;
    const bool reg = kernel == AC_KERNEL_2D_REG, wide = kernel == AC_KERNEL_2D_REGW;
    const int LX = wide ? 128 : 64;
    const int64_t cus = std::max(dev.cus, 1);
    // (K, LY, a, b) rows: the register tables as they are, the in-place table
    // as a streaming rate (a = 0, b = a tile's share of the chip's rate)
    struct Row { int K, LY; double a, b; };
    Row rows[24];
    int n = 0;
    if (reg || wide) {
        const auto put = [&](const auto &t) {
            for (const TileTime &r : t) rows[n++] = Row{r.K, r.LY, r.a, r.b};
        };
        if (wide) f64 ? put(kRegWF64) : put(kRegWF32);
        else f64 ? put(kRegF64) : put(kRegF32);
    } else {
        const auto put = [&](const auto &t) {
            for (const TileRate &r : t)
                rows[n++] = Row{r.K, r.LY, 0.0,
                                (double)(LX - 2 * r.K) * (r.LY - 2 * r.K) * r.K * 256 / r.rate * 1e-3};
        };
        f64 ? put(kInplaceF64) : put(kInplaceF32);
    }
    double best = -1.0;
    *K = rows[0].K;
    *LY = rows[0].LY;
    for (int i = 0; i < n; ++i) {
        const int k = rows[i].K, ly = rows[i].LY;
        const int OX = LX - 2 * k, OY = ly - 2 * k;
        if ((ny + OY - 1) / OY > 65535) continue;
        // register tiles sit flush against the domain edges (reg2d.h)
        const int64_t tiles = reg || wide ? (int64_t)ac::reg2d_tiles_1d(nx, LX, k) * ac::reg2d_tiles_1d(ny, ly, k)
                                          : (int64_t)((nx + OX - 1) / OX) * ((ny + OY - 1) / OY);
        const double t = rows[i].a + rows[i].b * (double)((tiles + cus - 1) / cus);
        const double rate = (double)nx * ny * k / t * 1e-3;
        if (rate > best) {
            best = rate;
            *K = k;
            *LY = ly;
        }
    }
    return best;
}

ac_status make_plan2d(int nx, int ny, int64_t nsteps, size_t elem, const ac_tune *tune,
                      const ac::DevInfo &dev, ac_plan *p) {
    std::memset(p, 0, sizeof *p);
    const bool force_tiled = tune && (tune->tile_x < 0 || tune->tile_y < 0);
    const int want = tune ? tune->kernel : 0;
    if (!force_tiled && nx <= 64 && ny <= ac::kRegRows * 16 &&
        (want == 0 || want == AC_KERNEL_2D_REG) &&
        (!tune || (!tune->tb_depth && !tune->tile_x && !tune->tile_y))) {
        // the whole grid as one register tile (every tile edge a domain edge, no
        // halo): all steps in one launch, phi -> work, copied back at the end
        // (64^2 FP64, 500 steps: 0.30 ms against 0.47 ms in LDS)
        const int nw = (ny + ac::kRegRows - 1) / ac::kRegRows;
        p->kernel = AC_KERNEL_2D_REG;
        p->tb_depth = 0;
        p->tile_x = 64;
        p->tile_y = nw * ac::kRegRows;
        p->threads = 64 * nw;
        p->launches = nsteps > 0 ? (nsteps + INT_MAX - 1) / INT_MAX : 0;
        p->copy_back = (int)(p->launches & 1);
        p->lds_bytes = (int64_t)ac::tile2d_reg_lds_bytes(p->tile_y, elem);
        return AC_OK;
    }
    if (!force_tiled && ac::tile2d_lds_bytes(nx, ny, elem) <= dev.lds_per_block) {
        p->kernel = AC_KERNEL_2D_RESIDENT;
        p->tb_depth = 0;
        p->tile_x = nx;
        p->tile_y = ny;
        p->threads = 1024;
        p->launches = nsteps > 0 ? (nsteps + INT_MAX - 1) / INT_MAX : 0;
        p->lds_bytes = (int64_t)ac::tile2d_lds_bytes(nx, ny, elem);
        return AC_OK;
    }
    int K = 0, LX = 0, LY = 0, kern = 0;
    if (tune) {
        K = tune->tb_depth;
        if (tune->tile_x > 0) LX = tune->tile_x;
        if (tune->tile_y > 0) LY = tune->tile_y;
        kern = tune->kernel;
    }
    if (kern != 0 && kern != AC_KERNEL_2D_TILED && kern != AC_KERNEL_2D_INPLACE &&
        kern != AC_KERNEL_2D_REG && kern != AC_KERNEL_2D_REGW)
        return fail(AC_ERR_UNSUPPORTED, "kernel %d is not a tiled 2D kernel", kern);
    if (kern == AC_KERNEL_2D_REGW && LX == 0) LX = 128;
    if (LX == 0) {
        // default: the register tile, 128 wide where the grid is and the
        // predicted time is shorter (every shape free), else 64 wide
        LX = 64;
        int k1, l1, k2, l2;
        if (kern == 0 && !K && !LY && nx >= 128 &&
            choose_tile2d(nx, ny, elem, AC_KERNEL_2D_REGW, dev, &k2, &l2) >
                choose_tile2d(nx, ny, elem, AC_KERNEL_2D_REG, dev, &k1, &l1)) {
            LX = 128;
            kern = AC_KERNEL_2D_REGW;
        }
    }
    if (!K || !LY) {
        // default: the (depth, tile height) with the best predicted time on
        // this grid, for the register kernel unless another one is asked for
        int dK = 0, dLY = 0;
        const int kind = kern == AC_KERNEL_2D_REGW             ? AC_KERNEL_2D_REGW
                         : kern == 0 || kern == AC_KERNEL_2D_REG ? AC_KERNEL_2D_REG
                                                                 : AC_KERNEL_2D_INPLACE;
        choose_tile2d(nx, ny, elem, kind, dev, &dK, &dLY);
        if (!K) K = dK;
        if (!LY) LY = dLY;
    }
    if (K < 1 || K > 8) return fail(AC_ERR_UNSUPPORTED, "tb_depth must be 1..8, got %d", K);
    if (LX < 2 * K + 1 || LY < 2 * K + 1 || LX > 4096 || LY > 4096)
        return fail(AC_ERR_UNSUPPORTED, "tile %dx%d too small/large for depth %d", LX, LY, K);
    const int rch = ac::rows_per_chunk(elem);
    // 64-wide tiles of whole 16-row wave blocks (at most 16 waves) run from
    // registers; other 64-wide tiles of at most 16 row chunks in place in LDS;
    // 128-wide tiles of whole 8-row wave blocks from registers, two columns
    // per lane, on grids at least 128 wide
    const bool reg_ok = LX == 64 && LY % ac::kRegRows == 0 && LY / ac::kRegRows <= 16;
    const bool regw_ok = LX == 128 && nx >= 128 && LY % ac::kRegWRows == 0 &&
                         LY / ac::kRegWRows <= 16;
    const bool inplace_ok = LX == 64 && (LY + rch - 1) / rch <= 16;
    int kernel = AC_KERNEL_2D_TILED;
    if (kern == AC_KERNEL_2D_REG || kern == AC_KERNEL_2D_INPLACE || kern == AC_KERNEL_2D_REGW) {
        const bool ok = kern == AC_KERNEL_2D_REG ? reg_ok : kern == AC_KERNEL_2D_REGW ? regw_ok : inplace_ok;
        if (!ok)
            return fail(AC_ERR_UNSUPPORTED, "tile %dx%d does not fit kernel %d on a %dx%d grid", LX,
                        LY, kern, nx, ny);
        kernel = kern;
    } else if (kern == 0) {
        kernel = reg_ok ? AC_KERNEL_2D_REG : inplace_ok ? AC_KERNEL_2D_INPLACE : AC_KERNEL_2D_TILED;
    }
    const size_t lds = kernel == AC_KERNEL_2D_REG      ? ac::tile2d_reg_lds_bytes(LY, elem)
                       : kernel == AC_KERNEL_2D_REGW    ? ac::tile2d_regw_lds_bytes(LY, elem)
                       : kernel == AC_KERNEL_2D_INPLACE ? ac::tile2d_inplace_lds_bytes(LY, elem)
                                                        : ac::tile2d_lds_bytes(LX, LY, elem);
    if (lds > dev.lds_per_block)
        return fail(AC_ERR_UNSUPPORTED, "tile %dx%d needs %zu B LDS > %zu", LX, LY, lds,
                    dev.lds_per_block);
    const int64_t gy = (ny + (LY - 2 * K) - 1) / (LY - 2 * K);
    if (gy > 65535) return fail(AC_ERR_UNSUPPORTED, "grid of %lld tile rows exceeds 65535", (long long)gy);
    const Chunks c = plan_chunks(nsteps, K);
    p->kernel = kernel;
    p->tb_depth = K;
    p->tile_x = LX;
    p->tile_y = LY;
    // register kernels: one wave per 16 (64 wide) or 8 (128 wide) rows; in
    // place: one wave per row chunk
    // of the tile; two buffers: per row chunk of the widest sub-step, at most 16
    p->threads = kernel == AC_KERNEL_2D_REG       ? 64 * (LY / ac::kRegRows)
                 : kernel == AC_KERNEL_2D_REGW    ? 64 * (LY / ac::kRegWRows)
                 : kernel == AC_KERNEL_2D_INPLACE ? ac::tile2d_inplace_threads(LY, elem)
                                                  : 64 * std::max(1, std::min(16, (LY - 2 + rch - 1) / rch));
    p->launches = nsteps > 0 ? c.n : 0;
    p->copy_back = nsteps > 0 && c.copy_back;
    p->lds_bytes = (int64_t)lds;
    return AC_OK;
}

ac_status make_plan3d(int nx, int ny, int nz, int64_t nsteps, size_t elem, const ac_tune *tune,
                      const ac::DevInfo &dev, ac_plan *p) {
    std::memset(p, 0, sizeof *p);
    const bool f64 = elem == 8;
    const int kern = tune ? tune->kernel : 0;
    if (kern != 0 && kern != AC_KERNEL_3D_STREAM && kern != AC_KERNEL_3D_REG)
        return fail(AC_ERR_UNSUPPORTED, "kernel %d is not a 3D kernel", kern);
    const bool shape_given = tune && (tune->tile_x > 0 || tune->tile_y > 0);
    // the register kernel (64 x 32 tiles: 8 waves of 4 rows) is the default when
    // the grid yields at least half a round of its workgroups (z segments of
    // 32 planes); smaller grids keep the LDS kernel's 32-wide tiles, which make
    // more workgroups of the same grid
    bool reg = kern == AC_KERNEL_3D_REG;
    const bool plane32 = (int64_t)nx * ny <= INT_MAX;   // the register kernel's in-plane offsets
    if (reg && !plane32)
        return fail(AC_ERR_UNSUPPORTED, "3D register tiles need nx * ny < 2^31 (%d x %d)", nx, ny);
    if (kern == 0 && !shape_given && plane32) {
        const int rk = tune && tune->tb_depth ? tune->tb_depth : (f64 ? 3 : 4);
        if (rk <= ac::reg3d_max_depth(elem)) {
            const int64_t wgs = (int64_t)ac::reg2d_tiles_1d(nx, 64, rk) *
                                ac::reg2d_tiles_1d(ny, 32, rk) * ((nz + 31) / 32);
            const int per_cu =
                ac::reg3d_blocks_per_cu(rk, 32, elem, ac::reg3d_select_reads(nx, ny, nz, elem));
            reg = wgs * kReg3dMinRoundsDen >=
                  kReg3dMinRoundsNum * (int64_t)std::max(per_cu, 1) * std::max(dev.cus, 1);
        }
    }
    // LDS-kernel defaults measured on MI355X at 256^3: depth 4 / 32x32x32 in
    // FP32, depth 3 / 32x16x32 in FP64; register kernel: depth 4 FP32, 3 FP64
    int K = f64 ? 3 : 4, LX = reg ? 64 : 32, LY = reg ? 32 : (f64 ? 16 : 32), LZ = 32;
    int threads = f64 ? 256 : 512;
    if (reg && !f64 && !(tune && (tune->tb_depth || tune->tile_y > 0)) &&
        (int64_t)ac::reg2d_tiles_1d(nx, 64, 4) * ac::reg2d_tiles_1d(ny, 32, 4) * ((nz + 31) / 32) <
            4LL * std::max(dev.cus, 1)) {
        // FP32 register tiles on a grid of less than two rounds of depth-4
        // segments (the short-segment regime below): depth 3 recomputes less
        // halo per segment.  Measured at 256^3 (A/B on one box): 1255-1258
        // GLUPS at depth 3 (26-plane segments) against 1208 at depth 4; at
        // 512^3, outside the regime, depth 3 runs 1086 against 1623-1632
        K = 3;
    }
    if (tune) {
        if (tune->tb_depth) K = tune->tb_depth;
        if (tune->tile_x > 0) LX = tune->tile_x;
        if (tune->tile_y > 0) LY = tune->tile_y;
        if (tune->tile_z > 0) LZ = tune->tile_z;
    }
    if (K < 1 || K > 8) return fail(AC_ERR_UNSUPPORTED, "tb_depth must be 1..8, got %d", K);
    if (LX < 2 * K + 1 || LY < 2 * K + 1 || LZ < 1)
        return fail(AC_ERR_UNSUPPORTED, "tile %dx%dx%d too small for depth %d", LX, LY, LZ, K);
    if (reg) {
        if (LX != 64 || LY % ac::kReg3dRows || LY / ac::kReg3dRows > ac::kReg3dMaxWaves ||
            K > ac::reg3d_max_depth(elem))
            return fail(AC_ERR_UNSUPPORTED,
                        "3D register tiles need tile_x 64, tile_y a multiple of %d up to %d and "
                        "depth <= %d (got %dx%d, depth %d)",
                        ac::kReg3dRows, ac::kReg3dRows * ac::kReg3dMaxWaves, ac::reg3d_max_depth(elem),
                        LX, LY, K);
        threads = 64 * (LY / ac::kReg3dRows);
    }
    if (!tune || tune->tile_z <= 0) {
        // longer z segments re-stream fewer halo planes (2K per segment) but
        // leave fewer workgroups.  LDS tiles: lengthen them only while the grid
        // still has about eight rounds of resident workgroups (measured: 1024^3
        // gains 15 % at 128 planes, 256^3 loses at anything above 32).
        // FP32 register tiles: below.  FP64 register tiles (2 per CU) keep the
        // eight-round rule (512^3: 697 GLUPS at 32 planes, 598 at 128).
        const int64_t xy = reg ? (int64_t)ac::reg2d_tiles_1d(nx, 64, K) * ac::reg2d_tiles_1d(ny, LY, K)
                               : (int64_t)((nx + LX - 2 * K - 1) / (LX - 2 * K)) *
                                     ((ny + LY - 2 * K - 1) / (LY - 2 * K));
        const int64_t want = reg && !f64
                                 ? (int64_t)std::max(ac::reg3d_blocks_per_cu(
                                                         K, LY, elem, ac::reg3d_select_reads(nx, ny, nz, elem)),
                                                     1) *
                                       dev.cus
                                 : 32LL * dev.cus;
        const int64_t two_per_cu = 2LL * std::max(dev.cus, 1);
        if (reg && !f64 && xy * ((nz + 31) / 32) < 2 * two_per_cu) {
            // FP32 register tiles on a grid of less than two rounds of
            // 32-plane segments: S = floor(2 CUs / xy) segments of about equal
            // length, so that (with each XCD taking a contiguous eighth of the
            // items) no CU takes more than two segments.  Measured on MI355X at
            // 256^3, depth 4 (S = 9): 29 planes 1208 GLUPS against 1124 at 32
            // (eight segments), 876 at 28 (ten: nine long ones crowd seven
            // XCDs' ranges) and 913 at 43; depth 5 (S = 8): 32 planes, its best.
            const int64_t S = std::max<int64_t>(1, two_per_cu / std::max<int64_t>(xy, 1));
            LZ = (int)std::max<int64_t>(16, std::min<int64_t>(128, (nz + S - 1) / S));
        } else if (reg && !f64) {
            // longer segments re-stream fewer halo planes, but the last round
            // of resident workgroups may run part-empty: the length in {32, 64,
            // 128} with the least (rounds, rounded up) x (LZ + 1.5 K).
            // Measured: 512^3 64 planes (1506 GLUPS against 1468 at 128, which
            // leaves 1.5 rounds; 1607 with the XCD-aware numbering), 1024^3
            // 128 (+2 % over 64; 1555 with the XCD-aware numbering)
            double best = 0;
            for (int lz = 32; lz <= 128; lz *= 2) {
                const int64_t rounds = (xy * ((nz + lz - 1) / lz) + want - 1) / want;
                const double cost = (double)rounds * (lz + 1.5 * K);
                if (lz == 32 || cost < best) {
                    best = cost;
                    LZ = lz;
                }
            }
        } else {
            while (LZ < 128 && xy * ((nz + 2 * LZ - 1) / (2 * LZ)) >= want) LZ *= 2;
        }
    }
    ac::Tile3D t{LX, LY, LZ, K, threads};
    if (!reg && ac::stream3d_cells_per_thread(t) > 4)
        return fail(AC_ERR_UNSUPPORTED, "tile %dx%d has more than 4 cells per thread", LX, LY);
    const size_t lds = reg ? ac::reg3d_lds_bytes(K, LY, elem) : ac::stream3d_lds_bytes(t, elem);
    if (lds > dev.lds_per_block)
        return fail(AC_ERR_UNSUPPORTED, "3D tile needs %zu B LDS > %zu", lds, dev.lds_per_block);
    const int64_t gz = (nz + LZ - 1) / LZ;
    if (gz > 65535) return fail(AC_ERR_UNSUPPORTED, "%lld z segments exceed 65535", (long long)gz);
    const Chunks c = plan_chunks(nsteps, K);
    p->kernel = reg ? AC_KERNEL_3D_REG : AC_KERNEL_3D_STREAM;
    p->tb_depth = K;
    p->tile_x = LX;
    p->tile_y = LY;
    p->tile_z = LZ;
    p->threads = threads;
    p->launches = nsteps > 0 ? c.n : 0;
    p->copy_back = nsteps > 0 && c.copy_back;
    p->lds_bytes = (int64_t)lds;
    return AC_OK;
}

template <typename T>
ac_status run2d(T *phi, T *work, int nx, int ny, double alpha_d, double r_d, int64_t nsteps,
                const ac_plan &p, hipStream_t stream) {
    const T alpha = (T)alpha_d, r = (T)r_d;
    hipError_t e;
    if (p.kernel == AC_KERNEL_2D_RESIDENT) {
        // whole grid in one workgroup: all steps in LDS, in place in phi
        ac::Tile2D t{nx, ny, 0, p.threads};
        for (int64_t done = 0; done < nsteps;) {
            const int k = (int)std::min<int64_t>(nsteps - done, INT_MAX);
            e = ac::launch_tile2d<T>(phi, phi, nx, ny, alpha, r, t, k, stream);
            if (e != hipSuccess) return hip_fail(e, "resident 2D launch");
            done += k;
        }
        return AC_OK;
    }
    if (p.kernel == AC_KERNEL_2D_REG && p.tb_depth == 0) {
        // whole grid in one register tile (halo 0): all steps per launch
        ac::Tile2D t{64, p.tile_y, 0, p.threads};
        T *src = phi, *dst = work;
        for (int64_t done = 0; done < nsteps;) {
            const int k = (int)std::min<int64_t>(nsteps - done, INT_MAX);
            e = ac::launch_tile2d_reg<T>(src, dst, nx, ny, alpha, r, t, k, stream);
            if (e != hipSuccess) return hip_fail(e, "whole-grid register launch");
            T *tmp = src; src = dst; dst = tmp;
            done += k;
        }
        if (src != phi) {
            e = hipMemcpyAsync(phi, src, (size_t)nx * ny * sizeof(T), hipMemcpyDeviceToDevice, stream);
            if (e != hipSuccess) return hip_fail(e, "copy back");
        }
        return AC_OK;
    }
    ac::Tile2D t{p.tile_x, p.tile_y, p.tb_depth, p.threads};
    const Chunks c = plan_chunks(nsteps, p.tb_depth);
    T *src = phi, *dst = work;
    for (int64_t i = 0; i < c.n; ++i) {
        const int k = (int)(c.base + (i < c.rem ? 1 : 0));
        e = p.kernel == AC_KERNEL_2D_REG ? ac::launch_tile2d_reg<T>(src, dst, nx, ny, alpha, r, t, k, stream)
            : p.kernel == AC_KERNEL_2D_REGW
                ? ac::launch_tile2d_regw<T>(src, dst, nx, ny, alpha, r, t, k, stream)
            : p.kernel == AC_KERNEL_2D_INPLACE
                ? ac::launch_tile2d_inplace<T>(src, dst, nx, ny, alpha, r, t, k, stream)
                : ac::launch_tile2d<T>(src, dst, nx, ny, alpha, r, t, k, stream);
        if (e != hipSuccess) return hip_fail(e, "tiled 2D launch");
        T *tmp = src; src = dst; dst = tmp;
    }
    if (c.copy_back) {
        e = hipMemcpyAsync(phi, src, (size_t)nx * ny * sizeof(T), hipMemcpyDeviceToDevice, stream);
        if (e != hipSuccess) return hip_fail(e, "copy back");
    }
    return AC_OK;
}

template <typename T>
ac_status run3d(T *phi, T *work, int nx, int ny, int nz, double alpha_d, double r_d,
                int64_t nsteps, const ac_plan &p, hipStream_t stream) {
    const T alpha = (T)alpha_d, r = (T)r_d;
    ac::Tile3D t{p.tile_x, p.tile_y, p.tile_z, p.tb_depth, p.threads};
    const Chunks c = plan_chunks(nsteps, p.tb_depth);
    T *src = phi, *dst = work;
    hipError_t e;
    for (int64_t i = 0; i < c.n; ++i) {
        t.K = (int)(c.base + (i < c.rem ? 1 : 0));
        e = p.kernel == AC_KERNEL_3D_REG
                ? ac::launch_reg3d<T>(src, dst, nx, ny, nz, alpha, r, t, stream)
                : ac::launch_stream3d<T>(src, dst, nx, ny, nz, alpha, r, t, stream);
        if (e != hipSuccess) return hip_fail(e, "3D launch");
        T *tmp = src; src = dst; dst = tmp;
    }
    if (c.copy_back) {
        e = hipMemcpyAsync(phi, src, (size_t)nx * ny * nz * sizeof(T), hipMemcpyDeviceToDevice,
                           stream);
        if (e != hipSuccess) return hip_fail(e, "copy back");
    }
    return AC_OK;
}

hipError_t device_info(DevInfo *out) {
    static std::mutex mu;
    static DevInfo cache[64];
    static bool have[64];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!have[dev]) {
        int cus = 0, lds = 0;
        if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
            return e;
        if ((e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev)) != hipSuccess)
            return e;
        cache[dev].cus = cus;
        cache[dev].lds_per_block = (size_t)lds;
        cache[dev].xcds = 8;
        have[dev] = true;
    }
    *out = cache[dev];
    return hipSuccess;
}

}  // namespace ac

using namespace ac;

// The plan of a 2D call: an explicit tune, else the tuning table's entry for
// the grid's size class, else the built-in choice.  A table entry is shared by
// every grid of the class, so it can fail to fit one of them (a 128-wide tile
// on a grid narrower than 128); that grid then takes the built-in choice.
static ac_status plan2d_with_table(int nx, int ny, int64_t nsteps, int32_t dtype,
                                   const ac_tune *tune, const ac::DevInfo &dev, ac_plan *p) {
    ac_tune tabled;
    const bool from_table = !tune && tuned_lookup(AC_TUNE_2D, dtype, nx, ny, 1, &tabled);
    ac_status s = make_plan2d(nx, ny, nsteps, elem_size(dtype), from_table ? &tabled : tune, dev, p);
    if (s != AC_OK && from_table) {
        s = make_plan2d(nx, ny, nsteps, elem_size(dtype), nullptr, dev, p);
        if (s == AC_OK) g_err.clear();
    }
    return s;
}

// The same for 3D (an entry can fail a grid of its class by, e.g., giving it
// more than 65535 z segments).
static ac_status plan3d_with_table(int nx, int ny, int nz, int64_t nsteps, int32_t dtype,
                                   const ac_tune *tune, const ac::DevInfo &dev, ac_plan *p) {
    ac_tune tabled;
    const bool from_table = !tune && tuned_lookup(AC_TUNE_3D, dtype, nx, ny, nz, &tabled);
    ac_status s = make_plan3d(nx, ny, nz, nsteps, elem_size(dtype), from_table ? &tabled : tune, dev, p);
    if (s != AC_OK && from_table) {
        s = make_plan3d(nx, ny, nz, nsteps, elem_size(dtype), nullptr, dev, p);
        if (s == AC_OK) g_err.clear();
    }
    return s;
}

extern "C" {

ac_status ac_step_2d_tuned(void *phi, void *work, int32_t nx, int32_t ny, double h, double dt,
                           double eps, int64_t nsteps, int32_t dtype, const ac_tune *tune,
                           void *stream) {
    g_err.clear();
    if (nx < 1 || ny < 1) return fail(AC_ERR_INVALID_ARG, "nx, ny must be >= 1 (%d x %d)", nx, ny);
    double alpha, r;
    ac_status s = validate(phi, work, (int64_t)nx * ny, 2, h, dt, eps, nsteps, dtype, &alpha, &r);
    if (s != AC_OK || nsteps == 0) return s;
    ac::DevInfo dev;
    hipError_t e = ac::device_info(&dev);
    if (e != hipSuccess) return hip_fail(e, "device query");
    ac_plan p;
    if ((s = plan2d_with_table(nx, ny, nsteps, dtype, tune, dev, &p)) != AC_OK) return s;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (dtype == AC_F64)
        return run2d<double>((double *)phi, (double *)work, nx, ny, alpha, r, nsteps, p, st);
    return run2d<float>((float *)phi, (float *)work, nx, ny, alpha, r, nsteps, p, st);
}

ac_status ac_step_2d(void *phi, void *work, int32_t nx, int32_t ny, double h, double dt,
                     double eps, int64_t nsteps, int32_t dtype, void *stream) {
    return ac_step_2d_tuned(phi, work, nx, ny, h, dt, eps, nsteps, dtype, nullptr, stream);
}

ac_status ac_step_3d_tuned(void *phi, void *work, int32_t nx, int32_t ny, int32_t nz, double h,
                           double dt, double eps, int64_t nsteps, int32_t dtype,
                           const ac_tune *tune, void *stream) {
    g_err.clear();
    if (nx < 1 || ny < 1 || nz < 1)
        return fail(AC_ERR_INVALID_ARG, "nx, ny, nz must be >= 1 (%d x %d x %d)", nx, ny, nz);
    double alpha, r;
    ac_status s = validate(phi, work, (int64_t)nx * ny * nz, 3, h, dt, eps, nsteps, dtype, &alpha, &r);
    if (s != AC_OK || nsteps == 0) return s;
    ac::DevInfo dev;
    hipError_t e = ac::device_info(&dev);
    if (e != hipSuccess) return hip_fail(e, "device query");
    ac_plan p;
    if ((s = plan3d_with_table(nx, ny, nz, nsteps, dtype, tune, dev, &p)) != AC_OK) return s;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (dtype == AC_F64)
        return run3d<double>((double *)phi, (double *)work, nx, ny, nz, alpha, r, nsteps, p, st);
    return run3d<float>((float *)phi, (float *)work, nx, ny, nz, alpha, r, nsteps, p, st);
}

ac_status ac_step_3d(void *phi, void *work, int32_t nx, int32_t ny, int32_t nz, double h,
                     double dt, double eps, int64_t nsteps, int32_t dtype, void *stream) {
    return ac_step_3d_tuned(phi, work, nx, ny, nz, h, dt, eps, nsteps, dtype, nullptr, stream);
}

ac_status ac_plan_2d(int32_t nx, int32_t ny, int64_t nsteps, int32_t dtype, const ac_tune *tune,
                     ac_plan *out) {
    g_err.clear();
    if (!out) return fail(AC_ERR_INVALID_ARG, "out must be non-null");
    if (nx < 1 || ny < 1 || nsteps < 0 || (dtype != AC_F32 && dtype != AC_F64))
        return fail(AC_ERR_INVALID_ARG, "bad grid, step count or dtype");
    ac::DevInfo dev;
    hipError_t e = ac::device_info(&dev);
    if (e != hipSuccess) return hip_fail(e, "device query");
    return plan2d_with_table(nx, ny, nsteps, dtype, tune, dev, out);
}

ac_status ac_plan_3d(int32_t nx, int32_t ny, int32_t nz, int64_t nsteps, int32_t dtype,
                     const ac_tune *tune, ac_plan *out) {
    g_err.clear();
    if (!out) return fail(AC_ERR_INVALID_ARG, "out must be non-null");
    if (nx < 1 || ny < 1 || nz < 1 || nsteps < 0 || (dtype != AC_F32 && dtype != AC_F64))
        return fail(AC_ERR_INVALID_ARG, "bad grid, step count or dtype");
    ac::DevInfo dev;
    hipError_t e = ac::device_info(&dev);
    if (e != hipSuccess) return hip_fail(e, "device query");
    return plan3d_with_table(nx, ny, nz, nsteps, dtype, tune, dev, out);
}

ac_status ac_check(void *stream) {
    hipError_t e = hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "ac_check");
    return batched_check_errors();
}

const char *ac_status_string(int32_t s) {
    switch (s) {
    case AC_OK: return "ok";
    case AC_ERR_INVALID_ARG: return "invalid argument";
    case AC_ERR_UNSTABLE: return "time step outside the stability bounds";
    case AC_ERR_UNSUPPORTED: return "unsupported configuration";
    case AC_ERR_HIP: return "HIP runtime error";
    case AC_ERR_NOMEM: return "out of memory";
    default: return "unknown status";
    }
}

const char *ac_last_error(void) { return g_err.c_str(); }

int32_t ac_version(void) { return 100; }

}  // extern "C"
