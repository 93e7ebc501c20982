/*
 * qla.h - C ABI of the MI355X (gfx950) qubit lattice algorithm (QLA) library for
 * the 2D Maxwell equations in an isotropic inhomogeneous dielectric n(x, y).
 *
 * Method: Soe, Ram, Koukoutsis, Vahala, Vahala & Hizanidis, "Quantum Computing
 * Framework for Transient Scattering of Electromagnetic Waves by Dielectric
 * Structures". One time step is Eq. (2e14): Q(t + dt) = V_y V_x U_y U_x Q(t),
 * with the collide-stream sequences U_x (Eq. 2e6) and U_y (Eq. 2e9) built from
 * the collisions C_x (Eq. 2e3), C_y (Eq. 2e8) and the streaming operators of
 * Eq. (2e5), and the refractive-index potentials V_x, V_y (Eqs. 2e11-2e13).
 *
 * State. The qubit vector is Q = (n Ex, n Ey, n Ez, Bx, By, Bz) = (q0..q5)
 * (Eq. 3b3, c = 1, t -> ct). The operators of Eq. (2e14) never couple the
 * triple (q2, q3, q4) = (n Ez, Bx, By) to (q0, q1, q5) = (n Ex, n Ey, Bz); a context
 * evolves one of them (the E_z triple unless created with qla_create_triple). Every
 * field array that crosses this ABI is a set of 3 planes ordered (q2, q3, q4) - or
 * (Ez, Bx, By) for physical readout - for the E_z triple, (q0, q1, q5) - or
 * (Ex, Ey, Bz) - for the B_z triple, each plane row-major [y][x] with x fastest,
 * nx * ny doubles, planes contiguous one after another.
 *
 * Lattice. nx * ny sites, periodic in x and y, spacing delta (physical units);
 * one step advances time by delta^2 (Section IV, "diffusion ordering"), so light
 * in vacuum crosses delta cells per step. Collision angle theta = delta / (4 n)
 * (Eq. 2e4); potential angles beta = delta^2 (dn/dx) / n^2 (Eq. 2e13) with
 * centred differences of the sampled n.
 *
 * Ownership. A context owns all device memory it allocates; host arrays passed
 * in are copied and remain owned by the caller; device pointers passed in
 * (the *_device calls) are read or written on the context's stream and remain
 * owned by the caller.
 *
 * Errors. Every call returns a qla_status. Nothing throws across the ABI. On an
 * error the context's state is unchanged, except QLA_EDEVICE, after which the
 * context should be destroyed. qla_last_error() gives a message for the last
 * failing call on the calling thread.
 *
 * Streams. Work is enqueued on the context's HIP stream (given at creation, or a
 * library-owned stream). qla_advance, qla_init_packet, qla_set_index_device,
 * qla_get_fields_device and qla_energy_device are asynchronous; the calls that
 * return host data synchronise the stream. One context must not be used from
 * two threads at once.
 */
#ifndef QLA_H
#define QLA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qla_ctx qla_ctx;

typedef enum {
    QLA_OK = 0,
    QLA_EINVAL = -1,   /* bad argument (size, pointer, value); nothing was changed */
    QLA_ENOMEM = -2,   /* device or host allocation failed */
    QLA_EDEVICE = -3,  /* a HIP runtime call or kernel launch failed */
    QLA_ESTATE = -4    /* call out of order (e.g. advance before the index is set) */
} qla_status;

typedef enum {
    QLA_F64 = 0,  /* amplitudes stored and stepped in FP64 */
    QLA_F32 = 1   /* amplitudes stored and stepped in FP32; energy always in FP64 */
} qla_precision;

/* Potential operators V_x, V_y of Eq. (2e14). */
typedef enum {
    /* Default. Unitary half-angle rotations V_x = C_x(theta2 -> -beta2/2),
     * V_y = C_y(theta2 -> -beta3/2): with site-dependent collision angles the
     * unitary U_x, U_y recover the symmetrised operator (1/2)[(1/n)d + d(1/n)];
     * these rotations add the skew remainder that yields Eqs. (2d3)-(2d5)
     * exactly to second order, and conserve the energy of Eq. (A13). */
    QLA_V_SKEW_HALF = 0,
    /* Eqs. (2e11)-(2e12) as printed, with V_y's q3 row read as
     * (0, 0, sin b3, cos b3, 0, 0) so that V_y = I when n is uniform. Not
     * unitary; kept for comparison. */
    QLA_V_PAPER = 1,
    /* Potentials off: the homogeneous-medium scheme of Eq. (2e10). */
    QLA_V_NONE = 2,
    /* A scheme beyond the paper (E_z triple only): no potentials, and U_x, U_y built
     * only from the sets of Eqs. (2e6), (2e9) that stream the B-qubit of each pair
     * (S_14 along x, S_03 along y), each used twice. Every neighbour pair then takes
     * the angle of its E site, which gives the Maxwell form of Eqs. (2d3)-(2d5)
     * without a potential: fully unitary, second order in delta. */
    QLA_V_BSTREAM = 3
} qla_potential;

/* Which polarisation a context evolves. The operators of Eq. (2e14) never couple the
 * triple (q2, q3, q4) = (n Ez, Bx, By) to (q0, q1, q5) = (n Ex, n Ey, Bz). */
typedef enum {
    QLA_TRIPLE_EZ = 0,  /* (q2, q3, q4): field arrays are planes (q2, q3, q4) */
    QLA_TRIPLE_BZ = 1   /* (q0, q1, q5): field arrays are planes (q0, q1, q5) */
} qla_triple;

/* Gaussian-envelope plane-wave packet in E_z (Section V, initial conditions):
 * Ez0 = amp * exp(-r^2 / (2 sigma^2)) * cos(2 pi s / lambda), where s is the
 * minimum-image displacement from (x0, y0) (cells) projected on the direction of
 * travel phi (radians, 0 = +x) and r = s if planar != 0 (uniform across the
 * direction of travel, the paper's 1D packet), else the full minimum-image
 * distance. The paired magnetic field is that of a wave travelling one way along
 * phi in a uniform medium: q2 = n Ez0, q3 = q2 sin(phi), q4 = -q2 cos(phi).
 * In a B_z-triple context the same envelope is the B_z packet of the other
 * polarisation: q5 = Bz0 and, from E = -(1/n) k x B, (q0, q1) = n (Ex, Ey) =
 * Bz0 (-sin(phi), cos(phi)). */
typedef struct {
    double x0, y0, sigma, lambda, phi, amp;
    int planar;
} qla_packet;

/* Create a context for an nx-by-ny periodic lattice with spacing delta.
 * nx, ny >= 8 (the step reads 4 neighbours on each side), nx < 2^28 (a row below
 * 2 GiB); the lattice size is bounded only by device memory (80 bytes per site
 * in FP64, 60 in FP32; planes beyond 2 GiB are addressed row by row),
 * delta > 0 and finite. hip_stream: a hipStream_t to enqueue on, or NULL for a
 * library-owned stream. Allocates the amplitude planes (two buffers), the index
 * planes and small scratch; the state starts at zero with no index set. */
qla_status qla_create(int nx, int ny, double delta, qla_precision precision,
                      qla_potential potential, void *hip_stream, qla_ctx **out);

/* As qla_create for either triple (qla_create is the E_z triple). The B_z triple is
 * stepped with the same operators of Eq. (2e14) acting on (q0, q1, q5): C_x (Eq. 2e3)
 * on (q1, q5), C_y (Eq. 2e8) on (q0, q5), streaming S_14, S_03 and S_25 (Eq. 2e5).
 * Its field arrays are planes (q0, q1, q5), or (Ex, Ey, Bz) = (q0 / n, q1 / n, q5) for
 * physical readout. QLA_V_PAPER and QLA_V_BSTREAM are implemented for the E_z triple
 * only (QLA_EINVAL). */
qla_status qla_create_triple(int nx, int ny, double delta, qla_precision precision,
                             qla_potential potential, qla_triple triple, void *hip_stream,
                             qla_ctx **out);

/* Set n(x, y) from a host array of ny rows of nx doubles, row stride ld >= nx
 * (elements). Computes the coefficients of Eqs. (2e4) and (2e13) in FP64 on the
 * GPU and checks them: every n must be finite and > 0, and the collision and
 * potential rotation angles must not exceed 0.5 rad (QLA_EINVAL otherwise).
 * Synchronises. Resets the step counter; the amplitudes are kept. */
qla_status qla_set_index(qla_ctx *ctx, const double *n_host, size_t ld);

/* As qla_set_index, from device memory (ny rows of nx doubles, stride ld). */
qla_status qla_set_index_device(qla_ctx *ctx, const double *n_device, size_t ld);

/* Elliptical dielectric (or bubble) of the paper's scattering experiments (Section V,
 * initial conditions), in cells and radians: semi-axis a along the x' axis rotated by
 * rot about (xc, yc), b along y'; n_in inside, n_out outside, joined by a boundary
 * layer about `width` cells thick. */
typedef struct {
    double xc, yc, a, b, rot, n_in, n_out, width;
} qla_ellipse;

/* Set n(x, y) from an ellipse, computed on the GPU in FP64:
 * n = n_out + (n_in - n_out) (1 - tanh(d / width)) / 2 with d = (rho^2 - 1) / |grad rho^2|
 * the first-order signed distance to rho^2 = (x'/a)^2 + (y'/b)^2 = 1 (n = n_in at the
 * exact centre). Then as qla_set_index (checks, coefficients, step counter reset).
 * QLA_EINVAL unless a, b, width > 0 and every field is finite. Synchronises. */
qla_status qla_set_index_ellipse(qla_ctx *ctx, const qla_ellipse *ellipse);

/* Fill the amplitudes with the packet of qla_packet on the current n
 * (QLA_ESTATE if no index is set). Resets the step counter. Asynchronous. */
qla_status qla_init_packet(qla_ctx *ctx, const qla_packet *packet);

/* Replace the amplitudes by 3 host planes (q2, q3, q4), or (q0, q1, q5) for the B_z
 * triple, in FP64 (rounded to FP32 in QLA_F32 mode): checkpoint restore. Resets the
 * step counter to `step`. */
qla_status qla_set_fields(qla_ctx *ctx, const double *q_host, int64_t step);

/* Advance k >= 0 full steps of Eq. (2e14). Asynchronous. */
qla_status qla_advance(qla_ctx *ctx, int64_t k);

/* Copy the state to 3 host planes in FP64: (q2, q3, q4) if physical == 0,
 * else (Ez, Bx, By) = (q2 / n, q3, q4); for the B_z triple (q0, q1, q5), else
 * (Ex, Ey, Bz) = (q0 / n, q1 / n, q5). Synchronises. */
qla_status qla_get_fields(qla_ctx *ctx, double *out_host, int physical);

/* As qla_get_fields into 3 device planes (3 * nx * ny doubles). Asynchronous. */
qla_status qla_get_fields_device(qla_ctx *ctx, double *out_device, int physical);

/* Energy of Eq. (A13): the sum over sites of q2^2 + q3^2 + q4^2 (q0^2 + q1^2 + q5^2
 * for the B_z triple), accumulated in FP64 in a fixed order (bitwise reproducible).
 * Synchronises. */
qla_status qla_energy(qla_ctx *ctx, double *energy);

/* As qla_energy, written to one device double. Asynchronous. */
qla_status qla_energy_device(qla_ctx *ctx, double *energy_device);

/* Divergence diagnostic (Section V: the paper monitors div D and div B). The in-plane
 * field F is B = (q3, q4) for the E_z triple and D = n^2 E = n (q0, q1) for the B_z
 * triple (whose other divergence is zero in 2D); with centred periodic differences
 * dF/dx = (F[x+1] - F[x-1]) / (2 delta), div = dFx/dx + dFy/dy at every site. Writes
 * through the non-NULL pointers: l2 = sqrt(sum div^2), max_abs = max |div| and
 * scale = sqrt(sum (dFx/dx)^2 + (dFy/dy)^2), so l2 / scale is a relative divergence
 * (0 for a divergence-free field, order 1 for a generic one). FP64, fixed order.
 * Synchronises. QLA_ESTATE for the B_z triple without an index. */
qla_status qla_divergence(qla_ctx *ctx, double *l2, double *max_abs, double *scale);

/* Per-site FP64 coefficients the step uses, copied to host arrays of nx * ny
 * (any pointer may be NULL): theta = delta / (4 n) (Eq. 2e4) and
 * beta_x, beta_y = delta^2 (dn/dx, dn/dy) / n^2 (Eq. 2e13), centred differences.
 * Synchronises. QLA_ESTATE if no index is set. */
qla_status qla_get_coefficients(qla_ctx *ctx, double *theta, double *beta_x, double *beta_y);

/* Number of steps taken since the last reset. */
qla_status qla_step_count(const qla_ctx *ctx, int64_t *steps);

/* Tuning of the step kernel (results do not depend on it, bit for bit):
 * rows_per_segment = output rows each wavefront marches through (rounded up so
 * that the rows plus the halo rows fill whole unrolled loop trips; 0 = default);
 * prefetch_rows = how many rows ahead its loads run (2 or 3; 0 = default);
 * steps_per_pass = steps of Eq. (2e14) applied per pass over HBM (1 or 2,
 * temporal blocking; 0 = default). */
qla_status qla_set_tuning(qla_ctx *ctx, int rows_per_segment, int prefetch_rows,
                          int steps_per_pass);

/* Lattice columns each lane of the step kernel holds: 1, or 2 (FP32 contexts of
 * even nx only: a wavefront then covers 128 columns, so fewer of its lanes are
 * halo, and every load and store moves 8 bytes per lane). Each column goes
 * through the same arithmetic either way, so results are bitwise the same.
 * 0 restores the default (1). QLA_EINVAL for other values, for 2 on an FP64
 * context or on odd nx. */
qla_status qla_set_lane_columns(qla_ctx *ctx, int columns);
qla_status qla_get_lane_columns(const qla_ctx *ctx, int *columns);

/* Pick the tuning of the step kernel for this context's lattice by timing
 * candidate segment heights, prefetch depths, steps per pass and (FP32, even nx)
 * columns per lane on it (tens of milliseconds to seconds, growing with the
 * lattice). The fastest four are timed twice more; among those within 3% of the
 * best, the one that recomputes the fewest halo sites is kept. The state and step
 * counter are saved and restored, so results are unaffected; the chosen values are
 * kept and returned through the non-NULL pointers (columns per lane:
 * qla_get_lane_columns). Synchronises. QLA_ESTATE if no index is set. */
qla_status qla_autotune(qla_ctx *ctx, int *rows_per_segment, int *prefetch_rows,
                        int *steps_per_pass);

/* The tuning currently in use (see qla_set_tuning). */
qla_status qla_get_tuning(const qla_ctx *ctx, int *rows_per_segment, int *prefetch_rows,
                          int *steps_per_pass);

/* Release every resource of the context (NULL is accepted). Synchronises. */
qla_status qla_destroy(qla_ctx *ctx);

/* The energy of Eq. (A13), sum over sites of q_a^2 + q_b^2 + q_c^2 in FP64, of three
 * caller-owned device planes, WITHOUT ALLOCATING: for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid it). The same kernels and summation order as qla_energy_device, so on a
 * context's planes it returns the same bits. Planes: ny rows of nx values of the given
 * precision (FP64 or FP32), row stride `pitch` >= nx elements, read on hip_stream (NULL:
 * the null stream); the result is written to the device double energy_device
 * (asynchronous). nx, ny >= 1; QLA_EINVAL otherwise. Scratch: the 1024 FP64 partial
 * sums live in a file-scope device array of this library (8 KiB on each GPU it runs on,
 * held until the process ends), whatever the lattice size; every call overwrites them
 * all, and calls that overlap on one GPU (two streams, two threads) race on them. The
 * array's address is looked up once per device on the first call there. */
qla_status qla_energy_noalloc(const void *q_a, const void *q_b, const void *q_c, int nx, int ny,
                              size_t pitch, qla_precision precision, double *energy_device,
                              void *hip_stream);

/* ---------------------------------------------------------------------------
 * Batches: many independent lattices (sizes, media and packets of their own)
 * advanced together. Each pass (2 steps, or 1 if some step count is odd) is one
 * persistent launch whose wavefronts stride over the tiles of every lattice still
 * running; the whole run is captured once into a hipGraph.
 * --------------------------------------------------------------------------- */
typedef struct qla_batch qla_batch;

/* Create `count` (1..4095) lattices nx[i] x ny[i] with spacing delta[i], all in one
 * precision and potential mode, on one stream (NULL = library-owned). Each lattice
 * is an ordinary context (see qla_batch_context); each amplitude plane must fit in
 * 2 GiB (QLA_EINVAL otherwise). */
qla_status qla_batch_create(int count, const int *nx, const int *ny, const double *delta,
                            qla_precision precision, qla_potential potential,
                            void *hip_stream, qla_batch **out);

/* Borrow lattice i's context to set its index, packet or fields and to read its
 * fields or energy with the single-lattice calls. It must not be destroyed and
 * must not be advanced on its own while the batch has a plan. */
qla_status qla_batch_context(qla_batch *batch, int i, qla_ctx **ctx);

/* Plan a run in which lattice i advances steps[i] steps (every index must be set):
 * autotune the segment height (one for all lattices, or fitted to each lattice's
 * height around it), prefetch depth and steps per pass on the batch itself (the
 * states are saved and restored), build the tile tables and capture the run (one
 * persistent launch per pass) into a hipGraph. mode: 0 or 1 (one launch per pass);
 * 2 (one cooperative launch per run) is not available (QLA_EINVAL). Synchronises. */
qla_status qla_batch_plan(qla_batch *batch, const int64_t *steps, int mode);

/* As qla_batch_plan with a given tuning instead of the autotuned one: segment
 * height rows_per_segment (>= 1; fit = 1: fitted to each lattice's height around
 * it), prefetch_rows 2 or 3, steps_per_pass 1 or 2 (2 needs every step count even).
 * QLA_EINVAL for values outside these ranges. Synchronises. */
qla_status qla_batch_plan_fixed(qla_batch *batch, const int64_t *steps, int rows_per_segment,
                                int prefetch_rows, int steps_per_pass, int fit);

/* Replay the planned run (asynchronous). Runs can be repeated; each continues
 * from the previous one's result. A lattice's index may be set again between runs,
 * but the run evaluates rotation angles with the series range (up to 1/16 rad, or
 * up to 1/2 rad) of the indices set when it was planned: if a new index needs the
 * wider range, QLA_ESTATE (plan again) and nothing is launched. */
qla_status qla_batch_run(qla_batch *batch);

/* The plan's choices: tuning, mode (1), passes, and the lattice-site updates of
 * one run. */
qla_status qla_batch_plan_info(const qla_batch *batch, int *rows_per_segment,
                               int *prefetch_rows, int *steps_per_pass, int *mode,
                               int *passes, int64_t *site_updates);

/* The segment height (output rows per wavefront tile) the plan gives lattice i. */
qla_status qla_batch_segment_rows(const qla_batch *batch, int i, int *rows);

/* Release the batch and every lattice in it (NULL is accepted). Synchronises. */
qla_status qla_batch_destroy(qla_batch *batch);

/* ---------------------------------------------------------------------------
 * Learned surrogate: a Fourier neural operator (FNO) that maps the medium and the
 * initial fields of a lattice to its fields a fixed number of steps later. QLA stays
 * the reference and the fallback: a caller accepts a prediction only if its energy
 * (Eq. A13, qla_fno_output_energy) is within a tolerance of the initial energy that
 * QLA conserves, and advances the lattice with QLA otherwise.
 *
 * Network (all sizes fixed at creation):
 *   v0 = P u + p                                    (lift, Cin -> C channels)
 *   v_{l+1} = act(IDFT_m[R_l . DFT_m(v_l)] + W_l v_l + b_l),   l = 0 .. L-1
 *   out = Q2 GELU(Q1 v_L + q1) + q2                 (projection C -> C2 -> Cout)
 * act is GELU, x Phi(x) (erf by Abramowitz & Stegun 7.1.26, |error| <= 1.5e-7), except
 * after the last Fourier layer (identity).
 * DFT_m keeps the modes ky in [0, m) U [H - m, H), kx in [0, m) of the real 2D
 * transform over the periodic H x W grid; R_l holds a complex C x C matrix per kept
 * mode. Activations are stored in BF16 and every contraction runs on the matrix
 * cores in BF16 with FP32 accumulation; parameters, gradients and Adam moments are
 * FP32.
 *
 * Tensors are [batch][channel][y][x] with x fastest (H rows of W). The network input
 * is BF16 [B][Cin][H][W]; the output FP32 [B][Cout][H][W]; targets BF16
 * [B][Cout][H][W]. BF16 values are raw 16-bit patterns (the upper half of an
 * IEEE-754 binary32, rounded to nearest even). All tensor pointers are device
 * pointers owned by the caller; work is enqueued on the surrogate's stream.
 *
 * Parameter vector (FP32, qla_fno_param_count entries), in this order:
 *   P [C][Cin], p [C];
 *   for each layer: W [C][C] (out, in), b [C], R [ky index][kx][c_in][c_out][re, im]
 *     with ky index 0 .. 2m-1 for ky = 0 .. m-1, H-m .. H-1;
 *   Q1 [C2][C], q1 [C2], Q2 [Cout][C2], q2 [Cout].
 * --------------------------------------------------------------------------- */
typedef struct qla_fno qla_fno;

/* Create a surrogate for an H x W grid (2m <= H, 2m <= W) with the given channel
 * counts (width C <= 64), m kept modes per axis, L Fourier layers and batches up to
 * max_batch (max_batch * max(C, C2) * H * W < 2^31); QLA_EINVAL otherwise. Allocates the parameters, optimiser state
 * and the activations of a max_batch batch. Weights are initialised from `seed`:
 * linear maps uniform in +-1/sqrt(fan_in), spectral weights uniform in [0, 1/C^2).
 * hip_stream: the stream to use, or NULL for a library-owned one. Synchronises. */
qla_status qla_fno_create(int height, int width, int in_channels, int out_channels,
                          int channels, int modes, int layers, int proj_channels,
                          int max_batch, uint64_t seed, void *hip_stream, qla_fno **out);

/* Release the surrogate (NULL is accepted). Synchronises. */
qla_status qla_fno_destroy(qla_fno *fno);

/* Number of FP32 parameters. */
qla_status qla_fno_param_count(const qla_fno *fno, int64_t *count);

/* Copy the parameters to / from a host array of qla_fno_param_count floats
 * (layout above). Setting refreshes the BF16 weight copies. Synchronise. */
qla_status qla_fno_get_params(qla_fno *fno, float *params_host);
qla_status qla_fno_set_params(qla_fno *fno, const float *params_host);

/* Gradient of the last qla_fno_loss_grad / qla_fno_train_step call, to a host array
 * of qla_fno_param_count floats. Synchronises. */
qla_status qla_fno_get_grads(qla_fno *fno, float *grads_host);

/* Forward pass of `batch` (1..max_batch) inputs; writes the FP32 output (device,
 * batch * Cout * H * W floats). The output also stays inside the surrogate for
 * qla_fno_output_energy. Asynchronous. */
qla_status qla_fno_forward(qla_fno *fno, const uint16_t *input_device, int batch,
                           float *output_device);

/* Forward and backward pass of the loss mean_b ||out_b - target_b|| / ||target_b||
 * (relative L2 per sample, averaged over the batch); the gradient replaces the
 * stored one. If loss_host is not NULL the loss is copied there (synchronises),
 * else the call is asynchronous. */
qla_status qla_fno_loss_grad(qla_fno *fno, const uint16_t *input_device,
                             const uint16_t *target_device, int batch, float *loss_host);

/* One Adam update of the parameters from the stored gradient (bias-corrected,
 * step counter kept by the surrogate). lr >= 0, 0 <= beta1, beta2 < 1, eps > 0.
 * Asynchronous. */
qla_status qla_fno_adam_step(qla_fno *fno, float lr, float beta1, float beta2, float eps);

/* qla_fno_loss_grad then qla_fno_adam_step(lr, 0.9, 0.999, 1e-8); the loss is
 * written to one device float if loss_device is not NULL. Asynchronous. */
qla_status qla_fno_train_step(qla_fno *fno, const uint16_t *input_device,
                              const uint16_t *target_device, int batch, float lr,
                              float *loss_device);

/* Energy sum over the Cout output planes of out^2, per sample of the last forward
 * pass of `batch` samples, to `batch` device doubles (Eq. A13 when the outputs are
 * (q2, q3, q4)). Asynchronous. */
qla_status qla_fno_output_energy(qla_fno *fno, int batch, double *energy_device);

/* Share of each input sample's energy that the Fourier layers can carry: for the
 * `channels` input planes from `first_channel` on (0 <= first_channel,
 * 1 <= channels <= C, first_channel + channels <= Cin) of `batch` BF16 samples laid
 * out as for qla_fno_forward, the energy in the kept modes of their 2D DFT (ky in
 * [0, m) U [H - m, H), kx in [0, m), each kx > 0 mode counted with its Hermitian
 * partner (-ky, -kx)) over the planes' energy sum of squares, by Parseval; 0 for a
 * zero sample. Written to `batch` device doubles. A caller can send samples whose
 * fields lie mostly outside the kept band straight to QLA instead of predicting them.
 * The transforms run in BF16 on the matrix cores (about 1e-2 relative accuracy) and
 * use the forward pass's scratch, so the call must not overlap another call on the
 * same surrogate. Asynchronous. */
qla_status qla_fno_band_fraction(qla_fno *fno, const uint16_t *input_device, int batch,
                                 int first_channel, int channels, double *fraction_device);

/* Build one sample from a lattice's state: q_device = 3 FP64 planes (q2, q3, q4)
 * (as qla_get_fields_device writes them), n_device = the nx * ny index (FP64).
 * input_device (may be NULL) receives 4 BF16 planes (n - n_shift, q2, q3, q4);
 * target_device (may be NULL) receives 3 BF16 planes (q2, q3, q4). Asynchronous on
 * hip_stream (NULL = the null stream). */
qla_status qla_fno_pack(const double *q_device, const double *n_device, int nx, int ny,
                        double n_shift, uint16_t *input_device, uint16_t *target_device,
                        void *hip_stream);

const char *qla_strerror(qla_status status);
const char *qla_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* QLA_H */
