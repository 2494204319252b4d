/*
 * qla.h -- C ABI of libqla, a gfx950 (MI355X) implementation of the qubit
 * lattice algorithm (QLA) for the 2D curl-Maxwell equations in a diagonal
 * tensor dielectric, after G. Vahala et al., "Qubit Lattice Algorithm
 * Simulations of Maxwell's Equations for Scattering from Anisotropic
 * Dielectric Objects", arXiv:2301.13601 (2023).
 *
 * The library advances the Dyson-mapped field
 *     Q = (n_x E_x, n_y E_y, n_z E_z, B_x, B_y, B_z)            (Eq. (15))
 * on a periodic nx-by-ny lattice with the collide-stream sequences U_X,
 * U_Y (Eq. (17)-(20)) and the refractive-index potentials V_X, V_Y
 * (Eq. (21), (22)), in the arrangement of Eq. (23) or Eq. (28), with the
 * angles of Eq. (24) and (25). One call to qla_step performs whole time
 * steps; every sub-operator of a step runs in one fused kernel pass, for
 * one lattice or for a batch of lattices of uneven sizes.
 *
 * Conventions shared by every entry point:
 *  - Arrays are structure-of-arrays FP32 planes in device memory,
 *    component-major, then row (y), then column (x), x fastest:
 *    element (c, y, x) is at index (c * ny + y) * nx + x.
 *    Q has 6 planes (q0..q5 as above), n has 3 planes (n_x, n_y, n_z).
 *  - Streaming pulls: S^{+x}_{ab} replaces q_a, q_b at column x by their
 *    values at column x+1 (S^{-x}: x-1); likewise along y. This is the
 *    direction under which Eq. (17)-(20) reproduce the signs of Eq. (16).
 *  - Eq. (19) row 2 is read with sin(theta_2) in column 3; Eq. (22) is read
 *    with 0 for the "o" of row 0 and q3' = sin(b3) q2 + cos(b3) q3.
 *  - Eq. (25) derivatives are periodic central differences in cells, times
 *    kappa (see qla_beta_scale).
 *  - The library never allocates or frees device memory: the caller owns
 *    every buffer (n, both state buffers, the workspace) and keeps them
 *    alive until qla_free. All device work is enqueued on the caller's HIP
 *    stream. No entry point throws; each returns a qla_status and records
 *    a message retrievable with qla_last_error() (per thread).
 */
#ifndef QLA_H
#define QLA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QLA_OK = 0,
    QLA_EINVAL = -1,   /* bad argument: null pointer, size, delta, mode, n <= 0 or not finite */
    QLA_ENOMEM = -2,   /* host-side allocation failed, or the workspace is too small */
    QLA_EDEVICE = -3,  /* a HIP call failed; the message holds hipGetErrorString */
    QLA_ESTATE = -4    /* context unusable (null, freed, or poisoned by an earlier device error) */
} qla_status;

/* Placement of the potentials: Eq. (23) applies V_X(beta) then V_Y(beta)
 * after U_Y U_X; Eq. (28) applies V_X(beta/2) after the 8th and after the
 * 16th operator of U_X, and V_Y(beta/2) likewise within U_Y. */
typedef enum { QLA_POT_EQ23 = 0, QLA_POT_EQ28 = 1 } qla_pot_mode;

/* Scale kappa of the index derivative in Eq. (25):
 *   PHYS:    kappa = delta   (lattice spacing delta in the coordinates of
 *                             Eq. (25); the reading consistent with Eq. (26))
 *   LATTICE: kappa = delta^2 (derivative taken per cell)
 *   OFF:     kappa = 0       (no potentials: the unitary collide-stream
 *                             sequence alone) */
typedef enum { QLA_BETA_PHYS = 0, QLA_BETA_LATTICE = 1, QLA_BETA_OFF = 2 } qla_beta_scale;

/* Field triple a context advances. C_X, C_Y, V_X and V_Y (Eq. (17), (19),
 * (21), (22)) couple q0, q1, q5 only among themselves and q2, q3, q4 only
 * among themselves, so a state with one triple zero keeps it zero (the
 * polarisations of Sec. 4.1 and 4.2).
 *   BOTH: all six components (any state)
 *   TM:   (q2, q3, q4) = (n_z E_z, B_x, B_y); the step reads n_z only
 *   TE:   (q0, q1, q5) = (n_x E_x, n_y E_y, B_z); the step reads n_x, n_y
 * A TM or TE context holds the other triple at zero: qla_init clears its
 * three planes in both state buffers, qla_load_at in the loaded state, and
 * the step neither reads nor writes them. On the live triple the results are
 * bitwise those of a BOTH context. */
typedef enum { QLA_POL_BOTH = 0, QLA_POL_TM = 1, QLA_POL_TE = 2 } qla_polarisation;

/* Form of the potential operators.
 *   PRINTED: V_X, V_Y as Eq. (21), (22) (the paper's method)
 *   SKEW:    the exponential of the antisymmetric part of their generator:
 *            a rotation by beta/2 in each coupled pair, in the sense of the
 *            printed coupling -- V_X rotates (q4, q2) by beta_2/2 and
 *            (q1, q5) by beta_0/2; V_Y rotates (q2, q3) by beta_3/2 and
 *            (q5, q0) by beta_1/2 (a' = cos a - sin b, b' = sin a + cos b
 *            for the pair (a, b)). Orthogonal, so every step conserves
 *            Eq. (27). The paper leaves a unitary potential to future work
 *            without specifying one; this variant is the library's own
 *            construction, not a formula of the paper. */
typedef enum { QLA_V_PRINTED = 0, QLA_V_SKEW = 1 } qla_v_form;

typedef struct {
    int32_t nx, ny;       /* lattice size, each >= 1 */
    double delta;         /* the perturbation parameter delta > 0 (Sec. 3) */
    int32_t pot_mode;     /* qla_pot_mode */
    int32_t beta_scale;   /* qla_beta_scale */
    int32_t polarisation; /* qla_polarisation (0: all six components) */
    int32_t v_form;       /* qla_v_form (0: as printed) */
} qla_params;

/* Diagnostics of the current state (Sec. 3.1 and 4), all accumulated in FP64.
 *   energy   = (1/(nx ny)) sum over sites of Q.Q                     (Eq. (27))
 *   divB     = D_x B_x + D_y B_y,  D the periodic central difference in cells
 *   divD     = D_x (n_x q0) + D_y (n_y q1)   (D_c = eps_c E_c = n_c q_c)
 *   *_max are maxima of absolute values over the lattice, *_l2 Euclidean
 *   norms over the lattice; B_max, D_max are max |B| and max |D|. */
typedef struct {
    int64_t step;         /* whole steps taken since qla_init */
    double energy;
    double divB_max, divB_l2, B_max, B_l2;
    double divD_max, divD_l2, D_max;
} qla_diag;

typedef struct qla_ctx qla_ctx;   /* opaque */

/* Launch geometry of the fused step kernel (a tuning knob, not part of the
 * method; results are bitwise identical for every geometry). A wave owns 128
 * lattice columns (120 of them output; 112 when a launch advances two
 * steps) and a segment of seg_rows rows. A field set to 0 asks for the
 * library's default.
 *   seg_rows         rows per wave segment for every lattice, rounded up
 *                    to a multiple of 4 (default: per lattice, segments of
 *                    about equal height across the batch, the height picked
 *                    by simulating the block schedule; qla_get_launch then
 *                    reports the tallest)
 *   waves_per_block  1..4 waves (vertically adjacent segments) per block of
 *                    a one-step launch (default 1); a two-step block is
 *                    always one producer/consumer pair of waves
 *   graph_steps      steps per replayed HIP graph (rounded up to a multiple
 *                    of 2 * steps_per_pass); 1 launches every pass on its
 *                    own (default 32)
 *   steps_per_pass   1 or 2 time steps per launch (default 2). With 2, each
 *                    wave runs the step twice in one march over its rows
 *                    (temporal blocking: Q and n cross HBM once per two
 *                    steps); an odd remainder of a qla_step call runs as one
 *                    one-step launch.
 *   stream_loads     1: read the state rows with the non-temporal cache
 *                    policy, 2: with the default policy (the default).
 *                    Six-component contexts only; TM and TE contexts
 *                    always use the default policy (reported 2).
 *   vacuum_rows      1 (default): a wave does not fetch the index row of
 *                    its 128 columns when every index there that the step
 *                    uses is exactly 1 (vacuum; qla_init records, per row,
 *                    the columns where it is not), 2: every index row is
 *                    fetched. */
typedef struct {
    int32_t seg_rows;
    int32_t waves_per_block;
    int32_t graph_steps;
    int32_t steps_per_pass;
    int32_t stream_loads;
    int32_t vacuum_rows;
} qla_launch;

/* One lattice of a batch: its parameters and caller-owned device buffers
 * (layouts as for qla_init). Every lattice of a batch must use the same
 * pot_mode, beta_scale, polarisation and v_form; sizes and delta may
 * differ. */
typedef struct {
    qla_params p;
    const float *d_n;
    float *d_q;
    float *d_q_pong;
} qla_instance;

/* Bytes of device workspace qla_init needs for these parameters. */
qla_status qla_workspace_size(const qla_params *p, size_t *bytes);

/* Bytes of device workspace qla_init_batch needs for this batch. */
qla_status qla_batch_workspace_size(int32_t count, const qla_instance *inst, size_t *bytes);

/* Bind the caller's buffers and validate n.
 *   d_n        3*ny*nx FP32, n_x, n_y, n_z; read by every step, never
 *              written, and not to be changed by the caller while the
 *              context lives (qla_init records its angle ranges and, per
 *              row, the columns where it differs from 1, in d_work)
 *   d_q        6*ny*nx FP32, holds Q at step 0 on entry
 *   d_q_pong   6*ny*nx FP32 scratch state; steps alternate between the two
 *   d_work     qla_workspace_size() bytes, 256-byte aligned
 *   hip_stream a hipStream_t (NULL: the default stream); all work is
 *              enqueued on it
 * Every n must be > 0 and finite (QLA_EINVAL otherwise). Synchronises the
 * stream once (to read the validation result). On success *out owns only
 * host memory. */
qla_status qla_init(const qla_params *p, const float *d_n, float *d_q, float *d_q_pong,
                    void *d_work, void *hip_stream, qla_ctx **out);

/* A batch of count >= 1 independent lattices of uneven sizes (many
 * scattering instances): every qla_step advances all of them, with one
 * kernel launch per step covering the whole batch. inst is read during the
 * call only; the buffers it names must outlive the context. d_work is
 * qla_batch_workspace_size() bytes, 256-byte aligned. qla_init is the batch
 * of one. */
qla_status qla_init_batch(int32_t count, const qla_instance *inst, void *d_work, void *hip_stream,
                          qla_ctx **out);

/* Number of lattices the context steps. */
qla_status qla_count(qla_ctx *ctx, int32_t *count);

/* Enqueue nsteps >= 0 whole time steps (Eq. (23) or Eq. (28)) of every
 * lattice on the context's stream. Runs of graph_steps steps are replayed
 * from a HIP graph built on first use. Asynchronous; launch errors are
 * reported. */
qla_status qla_step(qla_ctx *ctx, int64_t nsteps);

/* Compute qla_diag for the current state of each lattice: out holds one
 * entry per lattice, in batch order. Synchronises the stream. */
qla_status qla_energy(qla_ctx *ctx, qla_diag *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * diagnostics of qla_energy for one state given by its buffers, with no
 * context and no workspace. p gives the lattice (nx, ny; the other fields
 * are checked as for qla_init but not used); d_n (3*ny*nx FP32) and d_q
 * (6*ny*nx FP32) are laid out as for qla_init; d_out is device memory,
 * 8-byte aligned, that receives one qla_diag with its step field set to
 * `step`. Enqueued on hip_stream: two kernel launches, no synchronisation,
 * no allocation, no memset, no copy. The per-block partial sums go to a
 * static device buffer of 64 KiB per GPU (1024 blocks of partials, enough
 * for every lattice size; it is held until the process ends). Calls that
 * overlap on one GPU share that buffer and race: serialise them (one
 * stream, or events). Errors: QLA_EINVAL for bad parameters or null or
 * misaligned pointers, QLA_EDEVICE if a launch fails. */
qla_status qla_energy_noalloc(const qla_params *p, const float *d_n, const float *d_q, int64_t step,
                              qla_diag *d_out, void *hip_stream);

/* Copy the current state of every lattice to dst, lattices back to back in
 * batch order, 6*ny*nx FP32 each.
 *   what = 0: Q as stored;  what = 1: (E, B) with E_c = q_c / n_c (Eq. (15));
 *             (E, B) is staged in the idle state buffer
 *   dst_is_host = 1: dst is host memory; 0: device memory
 * Synchronises the stream. */
qla_status qla_fields(qla_ctx *ctx, float *dst, int32_t what, int32_t dst_is_host);

/* qla_fields for lattice index of the context only (6*ny*nx FP32). */
qla_status qla_fields_at(qla_ctx *ctx, int32_t index, float *dst, int32_t what, int32_t dst_is_host);

/* Overwrite the current state of lattice index with src (6*ny*nx FP32 Q,
 * host memory if src_is_host, else device memory); the step count is
 * unchanged. Synchronises the stream when src is host memory. */
qla_status qla_load_at(qla_ctx *ctx, int32_t index, const float *src, int32_t src_is_host);

/* The launch geometry in use (never 0 fields). */
qla_status qla_get_launch(qla_ctx *ctx, qla_launch *out);

/* Request a launch geometry for later qla_step calls (0 fields: default).
 * QLA_EINVAL if a field is out of range, in which case the previous geometry
 * stays. Results are bitwise identical for every geometry. */
qla_status qla_set_launch(qla_ctx *ctx, const qla_launch *req);

/* Device pointer of the buffer holding the current state (d_q or d_q_pong)
 * of lattice 0, or of lattice index. */
qla_status qla_state(qla_ctx *ctx, float **d_current);
qla_status qla_state_at(qla_ctx *ctx, int32_t index, float **d_current);

/* Release the context's host memory. Safe on NULL. Does not synchronise. */
void qla_free(qla_ctx *ctx);

/* Message describing the last failure on this thread ("" if none). */
const char *qla_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* QLA_H */
