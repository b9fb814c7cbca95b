/*
 * ac.h -- C ABI of libac, an MI355X (gfx950) stepper for the Allen-Cahn
 * equation by the explicit finite-difference method of
 * Kim, "Fast Numerical Simulation of Allen-Cahn Equation".
 *
 * The operation (section 2.1, Eq. pytorchACeq, with the zero-Neumann boundary
 * of section 2):
 *
 *   phi_{c}^{n+1} = phi_c^n + dt * ( (phi_c^n - (phi_c^n)^3) / eps^2 + Lap_h phi_c^n )
 *   Lap_h phi_c  = ( sum of the 2d axis neighbours of c  -  2d * phi_c ) / h^2
 *
 * where a neighbour outside the grid is replaced by phi_c itself (the ghost
 * layer equals the adjacent interior cell).  d = 2 uses the 5-point stencil,
 * d = 3 the 7-point one.  The library evaluates it as
 *   phi + alpha*(phi - phi^3) + r*(S - 2d*phi),   alpha = dt/eps^2, r = dt/h^2,
 * with alpha and r derived once on the host in double precision (rounded once
 * to float for AC_F32).
 *
 * Conventions shared by every call:
 *   - phi and work are device pointers to contiguous row-major arrays, x
 *     fastest: 2D index j*nx + i, 3D index (k*ny + j)*nx + i.  Both hold
 *     nx*ny[*nz] elements of the given dtype and are owned by the caller; the
 *     library keeps no pointer after the call returns.
 *   - On return the state after nsteps steps is (will be, in stream order) in
 *     phi; work is clobbered.  phi and work must not overlap.
 *   - Calls are asynchronous on `stream` (a hipStream_t; NULL = the null
 *     stream).  Argument errors are reported before any HIP call is made.
 *     Kernel faults surface at the caller's next synchronisation; ac_check()
 *     synchronises the stream and maps a HIP error to AC_ERR_HIP.
 *   - The return value is an ac_status; ac_last_error() gives a thread-local
 *     message for the last failing call.
 *   - Stability: the call is refused with AC_ERR_UNSTABLE unless
 *       r <= 1/(2d)  and  alpha <= (1 - 2 d r)/2,
 *     the conditions under which |phi| <= 1 is preserved (maximum principle)
 *     for the scheme above.  dt = 0.1 h^2 (section 2) gives r = 0.1, so any
 *     eps_m with m >= 3 passes in 2D and 3D.
 */
#ifndef AC_H
#define AC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AC_OK = 0,
    AC_ERR_INVALID_ARG = 1, /* null/overlapping/misaligned pointer, bad size, non-finite or <= 0 h/dt/eps */
    AC_ERR_UNSTABLE = 2,    /* r or alpha outside the maximum-principle bounds above */
    AC_ERR_UNSUPPORTED = 3, /* a tuning request the library cannot honour */
    AC_ERR_HIP = 4,         /* a HIP runtime call failed */
    AC_ERR_NOMEM = 5        /* device or host allocation failed */
} ac_status;

typedef enum { AC_F32 = 0, AC_F64 = 1 } ac_dtype;

/* Optional launch shape for the tiled kernels.  Zero fields mean "choose":
 * the library then uses its tuning table (ac_autotune) or a built-in default.
 *   tb_depth  time steps fused per launch (temporal blocking), 1..8
 *   tile_x/y  loaded tile extent in cells, including the tb_depth halo
 *   tile_z    2D: unused; 3D: z-extent of one streamed column segment
 *   kernel    0 = choose; 2D: AC_KERNEL_2D_TILED / _INPLACE / _REG / _REGW
 *             (_REG needs tile_x = 64 and tile_y a multiple of 16 up to 256,
 *             _REGW tile_x = 128 (its default), tile_y a multiple of 8 up to
 *             128 and nx >= 128, _INPLACE tile_x = 64; in a batch, _REGW
 *             gives the instances at least 128 wide 128 x tile_y tiles and
 *             the others 64 x 2*tile_y ones, every other kernel 64-wide
 *             tiles); 3D: AC_KERNEL_3D_STREAM / _REG (_REG needs tile_x =
 *             64, tile_y a multiple of 4 up to 32 and tb_depth <= 8 in
 *             FP32, <= 6 in FP64)
 * Any valid choice gives bitwise the same result: every cell is always
 * updated by the same expression from the same neighbour values. */
typedef struct {
    int32_t tb_depth;
    int32_t tile_x;
    int32_t tile_y;
    int32_t tile_z;
    int32_t kernel;   /* 2D tiled: 0 = choose, or AC_KERNEL_2D_TILED / _INPLACE / _REG / _REGW */
} ac_tune;

/* 2D step, 5-point stencil (section 2.1, Eq. pytorchACeq).  phi, work: nx*ny
 * elements of dtype (AC_F32 or AC_F64), 16-byte aligned.  nsteps = 0 is a
 * no-op.  Grids up to 64 wide and 256 tall run all steps in one launch as one
 * register tile (plan: AC_KERNEL_2D_REG with tb_depth 0); other grids whose
 * state fits one workgroup's LDS run all steps in one launch in LDS; larger
 * grids run ceil(nsteps / tb_depth) tiled launches. */
ac_status ac_step_2d(void *phi, void *work, int32_t nx, int32_t ny,
                     double h, double dt, double eps, int64_t nsteps,
                     int32_t dtype, void *stream);

/* As ac_step_2d with an explicit launch shape (NULL = as ac_step_2d).
 * tune->tile_x/y = -1 forces the tiled path even for small grids; a tune with
 * tb_depth or tile_y set, or a kernel other than AC_KERNEL_2D_REG, skips the
 * whole-grid register tile. */
ac_status ac_step_2d_tuned(void *phi, void *work, int32_t nx, int32_t ny,
                           double h, double dt, double eps, int64_t nsteps,
                           int32_t dtype, const ac_tune *tune, void *stream);

/* 3D step, 7-point stencil: the extension of the 2D scheme the paper calls
 * immediate (section 2).  phi, work: nx*ny*nz elements, 16-byte aligned. */
ac_status ac_step_3d(void *phi, void *work, int32_t nx, int32_t ny, int32_t nz,
                     double h, double dt, double eps, int64_t nsteps,
                     int32_t dtype, void *stream);

ac_status ac_step_3d_tuned(void *phi, void *work, int32_t nx, int32_t ny, int32_t nz,
                           double h, double dt, double eps, int64_t nsteps,
                           int32_t dtype, const ac_tune *tune, void *stream);

/* Kernels a plan can use. */
enum {
    AC_KERNEL_2D_RESIDENT = 0, /* whole grid in one workgroup's LDS, all steps in one launch */
    AC_KERNEL_2D_TILED = 1,    /* LDS tiles, tb_depth steps per launch */
    AC_KERNEL_3D_STREAM = 2,   /* z-streamed tiles, tb_depth levels per launch */
    AC_KERNEL_2D_INPLACE = 3,  /* 64-wide LDS tiles updated in place, tb_depth steps per launch */
    AC_KERNEL_2D_REG = 4,      /* 64-wide tiles held in registers (16 rows per wave), x
                                * neighbours by cross-lane shifts, tb_depth steps per launch */
    AC_KERNEL_3D_REG = 5,      /* z-streamed 64-wide tiles held in registers (4 rows per
                                * wave), tb_depth 1..8 (FP64 1..6) levels per launch */
    AC_KERNEL_2D_REGW = 6      /* 128-wide tiles held in registers, two adjacent columns
                                * per lane (8 rows per wave), tb_depth steps per launch;
                                * needs nx >= 128 */
};

/* What a stepping call with the same arguments launches (filled by ac_plan_*). */
typedef struct {
    int32_t kernel;     /* AC_KERNEL_* */
    int32_t tb_depth;   /* steps fused per launch (0: all steps in one launch, whole grid) */
    int32_t tile_x, tile_y, tile_z;
    int32_t threads;    /* workgroup size */
    int64_t launches;   /* kernel launches for nsteps */
    int32_t copy_back;  /* 1 if the result is copied from work into phi at the end */
    int64_t lds_bytes;  /* dynamic LDS per workgroup */
} ac_plan;

/* Report the plan ac_step_2d_tuned / ac_step_3d_tuned would execute for these
 * sizes on the current device.  Queries device limits (a HIP call) but
 * launches nothing.  Errors as the stepping calls (AC_ERR_UNSUPPORTED for an
 * impossible tune). */
ac_status ac_plan_2d(int32_t nx, int32_t ny, int64_t nsteps, int32_t dtype,
                     const ac_tune *tune, ac_plan *out);
ac_status ac_plan_3d(int32_t nx, int32_t ny, int32_t nz, int64_t nsteps, int32_t dtype,
                     const ac_tune *tune, ac_plan *out);

/* ------------------------------------------------------------- batched ----
 * Many independent 2D grids, each with its own size and (h, dt, eps), advanced
 * by the same number of steps in ONE persistent kernel launch replayed from a
 * hipGraph.  This batching is not in the paper; each instance computes exactly
 * what ac_step_2d computes for it (section 2.1, Eq. pytorchACeq), bitwise. */
typedef struct {
    void *phi;          /* device pointer, nx*ny elements, 16-byte aligned */
    void *work;         /* device scratch of the same size */
    int32_t nx, ny;
    double h, dt, eps;
} ac_instance2d;

/* What the persistent launch of a batched call looks like. */
typedef struct {
    int32_t grid;       /* workgroups of the persistent launch (all resident) */
    int32_t items;      /* tiles over all instances, processed per temporal block */
    int32_t tb_depth;   /* steps per temporal block */
    int32_t tile_x, tile_y;
    int32_t blocks;     /* temporal blocks = grid barriers + 1 */
    int32_t copy_back;
    int64_t lds_bytes;
} ac_batch_info;

/* Advance every instance by nsteps.  Every instance is validated as in
 * ac_step_2d (argument errors name the instance index) and no two buffers of
 * the batch may overlap.  On first use of an instance table the library
 * uploads it and its tile list, captures the whole call into a hipGraph on a
 * private stream and caches it (the 64 most recent tables are kept); calls
 * with the same table (same pointers, sizes and parameters) and nsteps replay
 * the graph on `stream`.  By default the graph holds one launch per temporal
 * block, one workgroup per tile of every instance; ac_batched_set_persistent
 * switches to one persistent launch (workgroups sized to what the device
 * holds, tiles taken from ticket counters, a bounded-wait phase barrier per
 * temporal block; a timeout ends the kernel early and is reported by
 * ac_check).  The launch shape comes from `tune`, else from the autotuner's
 * table (ac_autotune_batched), else depth 8 with 128-wide register tiles of
 * 96 rows (FP64: 64) for instances at least 128 cells wide and 64-wide ones
 * of twice the height for narrower instances.  A call
 * longer than 2048 temporal blocks runs, in the graph mode, as repeated
 * 2048-block graphs plus a remainder.  Each instance gets exactly what
 * ac_step_2d computes for it, bit for bit. */
ac_status ac_step_batched(const ac_instance2d *inst, int32_t n_inst, int64_t nsteps,
                          int32_t dtype, void *stream);
ac_status ac_step_batched_tuned(const ac_instance2d *inst, int32_t n_inst, int64_t nsteps,
                                int32_t dtype, const ac_tune *tune, ac_batch_info *info,
                                void *stream);

/* As ac_step_batched_tuned, stepping only the instances i with active[i] != 0;
 * the others are left untouched (phi and work).  active is a device array of
 * n_inst int32 read by the kernel at run time, so its contents may change
 * between calls without a new plan (the plan is keyed by the pointer). */
ac_status ac_step_batched_masked(const ac_instance2d *inst, int32_t n_inst, int64_t nsteps,
                                 int32_t dtype, const ac_tune *tune, const int32_t *active,
                                 ac_batch_info *info, void *stream);

/* A 3D instance: its own grid nx x ny x nz (x fastest), h, dt and eps. */
typedef struct {
    void *phi, *work;
    int32_t nx, ny, nz;
    double h, dt, eps;
} ac_instance3d;

/* Advance every 3D instance by nsteps in one persistent launch (the
 * z-streamed 7-point tile of ac_step_3d, one item per (instance, xy tile, z
 * segment)), captured in a hipGraph and cached like the 2D batch.  Validation
 * as in ac_step_3d per instance, no two buffers may overlap.  The launch shape
 * comes from `tune` (tb_depth 1..4, tile_x, tile_y, tile_z), else the batch
 * defaults (FP32: depth 2, segments of about 24 planes; FP64: the 3D
 * defaults); nsteps not divisible by tb_depth adds one shorter phase.  With
 * no tile_x / tile_y given, each instance gets its own LDS tile shape (the
 * one of at most two cells per thread that computes the fewest cells over
 * its xy extent), and each instance's depth is cut into z segments of equal
 * length near tile_z.  Every instance runs the LDS tile body, except with
 * tune->kernel = AC_KERNEL_3D_REG in FP32, where instances at least 64 cells
 * wide run the register tile body on flush 64 x 32 tiles and 32-plane
 * segments.  Result in each phi.  Each instance is stepped exactly as ac_step_3d steps it, bit
 * for bit (the update of a cell does not depend on tile shape or depth). */
ac_status ac_step_batched_3d(const ac_instance3d *inst, int32_t n_inst, int64_t nsteps,
                             int32_t dtype, const ac_tune *tune, ac_batch_info *info,
                             void *stream);

/* Free every cached batched plan (synchronises the device). */
ac_status ac_batched_release(void);

/* How batched calls execute (drops cached plans).  on = 0 (the default): the
 * cached hipGraph holds one launch per temporal block (one workgroup per tile,
 * the ordering between blocks is the kernel boundary).  on != 0: one
 * persistent launch whose workgroups take tiles from ticket counters and meet
 * at a phase barrier per temporal block.  Same results bit for bit; on
 * MI355X the barrier's per-workgroup device-scope cache release and acquire
 * cost more than the launch boundaries (measured figures in the design
 * notes). */
void ac_batched_set_persistent(int32_t on);

/* Polls a grid barrier makes before giving up (default 2e7, about 2 s;
 * negative restores the default).  Drops cached plans.  A diagnostic control:
 * a tiny limit forces the timeout path. */
void ac_batched_set_spin_limit(int64_t polls);

/* ----------------------------------------------------------- autotuner ----
 * Time candidate launch shapes (tb_depth x tile) on scratch buffers of the
 * given size, store the fastest in a process-wide table keyed by (kind,
 * dtype, size class = floor(log2(cells))) and return it in *best.  Stepping
 * calls made with tune == NULL use a matching table entry.  The caller's data
 * is never touched.  Every candidate gives bitwise the same results. */
enum { AC_TUNE_2D = 2, AC_TUNE_3D = 3, AC_TUNE_BATCHED = 4 };
ac_status ac_autotune_2d(int32_t nx, int32_t ny, int32_t dtype, int64_t probe_steps,
                         ac_tune *best, void *stream);
ac_status ac_autotune_3d(int32_t nx, int32_t ny, int32_t nz, int32_t dtype,
                         int64_t probe_steps, ac_tune *best, void *stream);
ac_status ac_autotune_batched(const ac_instance2d *inst, int32_t n_inst, int32_t dtype,
                              int64_t probe_steps, ac_tune *best, void *stream);
/* The autotuner in one call: fill the table for representative grids of
 * dimension dim (2: 512^2, 2048^2, 4096^2; 3: 128^3, 256^3 -- one size class
 * each) in dtype, timing every candidate on scratch buffers on the null stream.
 * cache_json_path may be NULL (no persistence).  If the file exists its entries
 * are loaded first and every size whose class they already cover is skipped,
 * so a complete cache times nothing and makes no HIP call; the whole table is
 * then written back to the file.  Errors: AC_ERR_INVALID_ARG for dim outside
 * {2, 3} or a bad dtype (before any HIP call) and for an existing file that
 * does not parse (it is left untouched); otherwise as ac_autotune_2d/3d and
 * ac_tune_save. */
ac_status ac_autotune(int32_t dim, int32_t dtype, const char *cache_json_path);
/* Persist / restore / clear the tuning table (a small JSON file). */
ac_status ac_tune_save(const char *path);
ac_status ac_tune_load(const char *path);
void ac_tune_clear(void);
int32_t ac_tune_count(void);

/* --------------------------------------------------- learned surrogate ----
 * A small conv network that advances phi by K explicit steps per call
 * (phi -> phi + U(phi)); not in the paper.  Architecture (all 3x3 convs are
 * replicate padded, matching the zero-Neumann boundary):
 *   e1a = relu conv3(phi; 1->32)   e1 = relu conv3(e1a; 32->32)     H x W
 *   e2a = relu conv3(pool e1; 32->64)   e2 = relu conv3(e2a; 64->64)  H/2
 *   bt  = relu conv3(pool e2; 64->128)                               H/4
 *   u2  = conv1(up bt; 128->64)   d2 = relu conv3(cat(u2, e2); 128->64)
 *   u1  = conv1(up d2; 64->32)    d1 = relu conv3(cat(u1, e1); 64->32)
 *   out = phi + conv1(d1; 32->1)
 * pool = 2x2 average, up = 2x nearest.  241,473 parameters, flat in that
 * layer order: weights [Cout][ky][kx][Cin] (1x1: [Cout][Cin]), then bias.
 * Kernels: BF16 operands on v_mfma_f32_16x16x32_bf16 with FP32 accumulation;
 * FP32 master weights, FP32 Adam.  The handle owns all device state; inputs
 * and outputs are device pointers to [batch][hw][hw] FP32 fields.  Calls are
 * asynchronous on the handle's stream. */
typedef struct ac_sur ac_sur;
int64_t ac_sur_num_params(void);
/* batch_max >= 1; hw >= 8 and a multiple of 4.  Weights start at zero. */
ac_status ac_sur_create(ac_sur **out, int32_t batch_max, int32_t hw, void *stream);
void ac_sur_destroy(ac_sur *s);
ac_status ac_sur_set_stream(ac_sur *s, void *stream);
/* host FP32 arrays of ac_sur_num_params() values; set also resets Adam state */
ac_status ac_sur_set_weights(ac_sur *s, const float *host, int64_t n);
ac_status ac_sur_get_weights(ac_sur *s, float *host, int64_t n);
/* phi_out (may be NULL: kept internally) = phi_in + U(phi_in) */
ac_status ac_sur_forward(ac_sur *s, const float *phi_in, float *phi_out, int32_t batch);
/* inference only: phi_out (required, device, batch*H*W floats, not aliasing
 * phi_in) = phi_in + U(phi_in), the same network as ac_sur_forward with the
 * 1x1 head and the residual fused into the last 3x3 layer's epilogue (equal to
 * ac_sur_forward up to FP32 summation order).  Keeps no activations for a
 * backward pass: ac_sur_loss after it fails until the next ac_sur_forward. */
ac_status ac_sur_infer(ac_sur *s, const float *phi_in, float *phi_out, int32_t batch);
/* after ac_sur_forward on the same batch: mean squared error against target;
 * stores d loss / d out for the backward pass; loss_dev (may be NULL) receives
 * the loss as a device float */
ac_status ac_sur_loss(ac_sur *s, const float *target, int32_t batch, float *loss_dev);
/* after ac_sur_forward on the same batch: gradients with respect to every
 * parameter of a loss whose gradient with respect to phi_out is dloss_dout
 * (device, batch*H*W floats, [batch][hw][hw]; read before the call returns in
 * stream order).  dloss_dout = NULL takes the gradient ac_sur_loss stored, and
 * then requires ac_sur_loss on that batch first. */
ac_status ac_sur_backward(ac_sur *s, const float *dloss_dout, int32_t batch);
ac_status ac_sur_get_grads(ac_sur *s, float *host, int64_t n);
/* one Adam update (bias-corrected, step t >= 1) of the FP32 master weights */
ac_status ac_sur_adam_step(ac_sur *s, float lr, float b1, float b2, float eps_adam, int64_t t);

/* ------------------------------------------------------- precision trace ----
 * The paper's Err (section 2, Eq. ERReq) between FP32 and FP64 runs of the
 * explicit step: both fields advance nsteps steps together (one launch per
 * step, no temporal blocking), and after step t (t = 1..nsteps)
 *   rms[t-1] = sqrt(mean over cells of (phi32 - phi64)^2)   (FP64)
 * and *err = the mean of rms over the nsteps steps.  phi32/work32 (float) and
 * phi64/work64 (double) are caller-owned device buffers of nx*ny(*nz) cells,
 * pairwise disjoint and 16-byte aligned; the final states end in phi32 and
 * phi64.  rms (nsteps doubles) and err (one double) are device memory.  The
 * FP32 path computes exactly what ac_step_2d / ac_step_3d compute in FP32 (the
 * same update, bit for bit); the FP64 path that of the FP64 call.  h, dt, eps
 * are validated as for the stepping calls; nsteps = 0 sets *err = 0. */
ac_status ac_err_2d(float *phi32, float *work32, double *phi64, double *work64, int32_t nx,
                    int32_t ny, double h, double dt, double eps, int64_t nsteps, double *rms,
                    double *err, void *stream);
ac_status ac_err_3d(float *phi32, float *work32, double *phi64, double *work64, int32_t nx,
                    int32_t ny, int32_t nz, double h, double dt, double eps, int64_t nsteps,
                    double *rms, double *err, void *stream);

/* ---------------------------------------------------------------- judge ----
 * Per grid of a batch of 2D FP32 fields a (candidate) and b (reference), both
 * [batch][ny][nx] on the device: iface_err[n] = Hausdorff distance between the
 * zero-crossing sets of a[n] and b[n] (crossings located by linear
 * interpolation on the edges between adjacent cell centres; physical units via
 * h), searched within +-window cells, exact when <= (window - 1) h and +inf
 * beyond; 0 when neither field has a crossing, +inf when only one has.
 * l2_err[n] = root mean square of a[n] - b[n].  workspace: device scratch of
 * ac_judge_workspace_bytes(batch) bytes owned by the caller.  1 <= window <= 16. */
ac_status ac_judge_2d(const float *a, const float *b, int32_t batch, int32_t nx, int32_t ny,
                      double h, int32_t window, float *iface_err, float *l2_err,
                      void *workspace, void *stream);
int64_t ac_judge_workspace_bytes(int32_t batch);

/* ac_judge_2d without a workspace and without allocating, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, results and
 * kernels as ac_judge_2d; the per-grid scratch lives in a fixed device array
 * of the library (196,608 bytes, kept on each device it runs on until the
 * process ends), cleared by a kernel at the start of every call.  batch is
 * limited to 16384: larger batches return AC_ERR_INVALID_ARG before any HIP
 * call.  Every call on one device shares that array, so calls that overlap on
 * one GPU (concurrent streams, or host threads) race and must be ordered by
 * the caller. */
ac_status ac_judge_2d_noalloc(const float *a, const float *b, int32_t batch, int32_t nx, int32_t ny,
                              double h, int32_t window, float *iface_err, float *l2_err, void *stream);

/* Synchronise `stream` and report any pending HIP error, or a batched grid
 * barrier timeout, as AC_ERR_HIP. */
ac_status ac_check(void *stream);

/* Static description of a status code. */
const char *ac_status_string(int32_t status);

/* Thread-local message describing the last failing call ("" if none). */
const char *ac_last_error(void);

/* Library version, major*10000 + minor*100 + patch. */
int32_t ac_version(void);

#ifdef __cplusplus
}
#endif

#endif /* AC_H */
