/*
 * tpf.h -- C ABI of the MI355X batched fixed-point power-flow library (libtpf.so).
 *
 * Method: the tensor ("dense") fixed-point power flow of Giraldo, Salazar Duque
 * et al., "Tensor Power Flow Formulations for Multidimensional Analyses in
 * Distribution Systems" (arXiv 2403.04578):
 *   Sec. II Eq. (1)   nodal admittance Y of a network with one slack (substation)
 *                     node and b demand nodes, partitioned into Y_ss, Y_sd, Y_ds, Y_dd;
 *   Sec. II Eq. (2)   with constant-power loads the iteration
 *                     v <- F conj(v)^(-1) + w,  F = -Y_dd^-1 diag(s*),  w = -Y_dd^-1 Y_ds v_s,
 *                     i.e. V <- Z conj(S ./ V) + w with Z = -Y_dd^-1;
 *   Sec. IV-A Eq.(12) all power flows (time steps, scenarios, ...) reshaped into the
 *                     columns of one matrix and iterated together;
 *   Algorithm 1       flat start 1 + j0, iterate until the voltage step falls
 *                     below a tolerance or an iteration cap is reached.
 *
 * Conventions shared by every call
 *   - Per unit throughout.  S > 0 is consumption (Eq. (1) writes -i_d), so a PV
 *     injection is a negative S.
 *   - PQ order: column/bus index q of S and V is the q-th non-slack bus in
 *     ascending bus number.
 *   - Complex arrays are interleaved (re, im): dtype TPF_C128 = 2 x double,
 *     TPF_C64 = 2 x float.  S and V have the same dtype.
 *   - Arrays named "device" are device pointers on the current HIP device
 *     (16-byte aligned, contiguous, row-major: [tau][n] or [P][T][n]); arrays
 *     named "host" are host pointers.  The caller owns every array it passes.
 *   - Calls that take a stream are stream-ordered and asynchronous: the return
 *     code reports argument and launch errors only.  Non-convergence is data
 *     (status_out), never an error code.
 *   - On error a call returns a negative TPF_ERR_* code and tpf_last_error()
 *     (thread-local) describes it; outputs are then unspecified.
 */
#ifndef TPF_H_
#define TPF_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tpf_network_s *tpf_network; /* opaque; immutable after build */
typedef struct tpf_mlp_s *tpf_mlp;         /* opaque learned warm start (see below) */

enum {
    TPF_OK = 0,
    TPF_ERR_INVALID_ARG = -1, /* bad sizes, indices, pointers, tolerances */
    TPF_ERR_SINGULAR = -2,    /* Y_dd not invertible (e.g. a bus not connected to the slack) */
    TPF_ERR_DEVICE = -3,      /* HIP runtime error */
    TPF_ERR_OOM = -4,         /* host or device allocation failed */
    TPF_ERR_UNSUPPORTED = -5  /* valid request this build does not implement */
};

enum { TPF_C64 = 0, TPF_C128 = 1 };

/* Arithmetic of the sweeps.
 *   FP64        every sweep in FP64 (MFMA FP64), state in FP64;
 *   FP32        every sweep in FP32 (MFMA FP32), state kept as FP32 drop V - w;
 *   MIXED_BF16  sweeps on BF16 MFMA with FP32 accumulation until the low-precision
 *               iteration stalls, then FP32-accurate sweeps (one full FP32 sweep, then
 *               sweeps on the change of the injections) to the tolerance;
 *   MIXED_FP16  the same with FP16 operands under a per-column power-of-two scale; its
 *               FP32-accurate sweep splits Z and I into FP16 high and low parts.
 *   Convergence is only declared on an FP32-accurate iterate.  In FP32 and mixed
 *   modes tol must be >= 5e-7 pu (the FP32 state floor).
 * Network size: these four modes run any n.  FP64 beyond 320 PQ buses, and FP32 and
 * the mixed modes beyond 128, use a per-sweep kernel sequence (dense Z no longer fits
 * one workgroup's registers), queued up to max_iter sweeps without waiting for the
 * device (a sweep with no active column left exits at once); smaller networks run one
 * persistent kernel per solve. */
/* TREE_FP64   the FP64 iteration with Z I evaluated by two passes over the feeder's
 *             tree instead of the dense product: on a radial network without shunts,
 *             -Z is the path-impedance matrix, so Z I = -D with branch currents
 *             J_b = I_b + sum over b's children of J (leaves to slack) and drops
 *             D_b = D_parent + z_b J_b (slack to leaves).  Same iterates up to rounding,
 *             O(n) instead of 8 n^2 flops per column and sweep.  Needs a network with
 *             n_bus - 1 branches (a tree): single-phase with n <= 1024 PQ buses, or
 *             three-phase (3x3 blocks per branch) with at most 408 PQ buses in TREE_FP64
 *             (the LDS holds 400 bytes of state per bus) and 512 in TREE_FP32; returns
 *             TPF_ERR_UNSUPPORTED otherwise.  With a constant-impedance ZIP share
 *             (tpf_build_network_zip) each subtree is a Norton load G x + J seen from
 *             its parent: per column G'_b = G_b / (1 + z_b G_b), G_b = alpha_Z,b s_b* +
 *             sum of the children's G', formed once, then per sweep
 *             J'_b = k_b (I_b + sum of the children's J') with k_b = 1 - z_b G'_b
 *             and D_b = k_b D_parent + z_b (J'_b + G'_b v_s), V = v_s - D: the exact
 *             B^-1 solve of Eq. (2) for that column.  Single-phase only; the extra
 *             per-column state limits TREE_FP64 to about 800 PQ buses there. */
/* TREE_FP32   the tree operator in FP32 arithmetic with the state kept as the FP32 drop
 *             V - w (as in FP32 mode; tol >= 5e-7 pu); the same networks as TREE_FP64. */
enum {
    TPF_MODE_FP64 = 0,
    TPF_MODE_FP32 = 1,
    TPF_MODE_MIXED_BF16 = 2,
    TPF_MODE_MIXED_FP16 = 3,
    TPF_MODE_TREE_FP64 = 4,
    TPF_MODE_TREE_FP32 = 5
};

/* Per-column outcome written to status_out. */
enum { TPF_ST_CONVERGED = 0, TPF_ST_MAX_ITER = 1, TPF_ST_NONFINITE = 2 };

typedef struct {
    int32_t mode;          /* TPF_MODE_*; default TPF_MODE_FP64 */
    int32_t reserved0;
    const void *V0;        /* device [tau][n] start voltages (same dtype as S), or NULL for the
                              flat start 1 + j0 of Algorithm 1.  A column whose V0 holds a
                              non-finite value or a modulus outside [0.5, 1.5] pu starts flat. */
    double *mismatch_out;  /* device [tau] float64, or NULL: per-column max |S + V.*conj(Y_ds v_s +
                              Y_dd V)| of the returned V, computed in FP64 (Eq. (1) balance). */
    tpf_mlp warm_start;    /* learned warm start (tpf_mlp_create / tpf_mlp_load on this device) or
                              NULL.  The solve evaluates it on S (as tpf_mlp_predict, into the
                              workspace) and starts each column from its output, guarded like V0;
                              V0 must then be NULL.  Any mode. */
    const int64_t *t_index;  /* device int64 [tau]: minute index of each column for the warm
                              start's calendar features, or NULL (t = column index) */
    double reserved1[2];
} tpf_options;

/* Sec. II Eq. (1)-(2): build the network from its branch list.
 *   n_bus            number of buses including the slack (>= 2)
 *   n_branch         number of series branches (>= 1)
 *   from, to         host int32 [n_branch], bus numbers in [0, n_bus), from != to
 *   r, x             host float64 [n_branch], branch impedance r + jx pu, finite, not both 0
 *   slack_bus        the slack bus number
 *   vs_re, vs_im     slack voltage v_s
 *   out              receives the handle (library-owned; free with tpf_free_network)
 * Assembles Y (parallel branches add up; meshed networks allowed), partitions it,
 * factorises Y_dd in FP64 (LU, partial pivoting) and forms Z = -Y_dd^-1 and
 * w = -Y_dd^-1 Y_ds v_s.  Host work only; device copies are made on first use on
 * each device.  Errors: TPF_ERR_INVALID_ARG, TPF_ERR_SINGULAR (a bus unreachable
 * from the slack, or a numerically singular Y_dd), TPF_ERR_OOM. */
int tpf_build_network(int32_t n_bus, int32_t n_branch, const int32_t *from, const int32_t *to,
                      const double *r, const double *x, int32_t slack_bus, double vs_re,
                      double vs_im, tpf_network *out);

/* Sec. II Eq. (2) with a ZIP load model: the same network whose loads draw, at bus q,
 * the current alpha_Z[q] s* v + alpha_I[q] s* + alpha_P[q] s* / conj(v) (constant-impedance,
 * constant-current and constant-power shares of the nominal power s), i.e. the power
 * s (alpha_P + alpha_I v + alpha_Z |v|^2).  Eq. (2) then has A = diag(alpha_P s*),
 * B = diag(alpha_Z s*) + Y_dd, c = Y_ds v_s + alpha_I s*.
 *   alpha_z          host float64 [n] or NULL (all zero): constant-impedance shares
 *   alpha_i, alpha_p host float64 [n] per PQ bus (PQ order), finite; any values
 *                    (they need not sum to 1)
 * Without a constant-impedance share B = Y_dd for every column and the sweeps compute
 * V <- Z (alpha_P conj(S./V) + alpha_I conj(S)) + w in every mode.  With one (some
 * alpha_z[q] != 0) B differs per column.  The tree modes eliminate it per column along
 * the tree (no B^-1 is formed: the iterates of Eq. (2) with that B); the dense modes keep
 * the shared Z and carry the constant-impedance current in the injection,
 * V <- Z (alpha_P conj(S./V) + alpha_I conj(S) + alpha_Z conj(S) V) + w, which has the
 * same fixed point (other iterates; it converges while the load impedances are large
 * against the feeder's, as in any distribution feeder).  The FP16 form widens its
 * per-column scale by max_q |alpha_P[q]| + |alpha_I[q]| + |alpha_Z[q]| so that the larger
 * injections stay in range.  Other arguments and errors as
 * tpf_build_network; TPF_ERR_INVALID_ARG for a NULL or non-finite share.  The mismatch
 * (options.mismatch_out, tpf_mismatch) is the balance of these loads:
 * S (alpha_P + alpha_I V + alpha_Z |V|^2) + V conj(Y_ds v_s + Y_dd V). */
int tpf_build_network_zip(int32_t n_bus, int32_t n_branch, const int32_t *from, const int32_t *to,
                          const double *r, const double *x, int32_t slack_bus, double vs_re, double vs_im,
                          const double *alpha_z, const double *alpha_i, const double *alpha_p,
                          tpf_network *out);

/* Sec. II Eq. (1) for a three-phase (unbalanced) network: Eq. (1) is written per node,
 * and here every bus has three phase nodes, node 3 b + p for phase p in (a, b, c).
 *   zabc     host float64 [n_branch][3][3][2]: the series impedance matrix of each
 *            branch (self terms on the diagonal, mutual coupling off it), invertible
 *   vs_abc   host float64 [3][2]: slack phase voltages (a balanced source is
 *            1, e^{-j 2 pi/3}, e^{+j 2 pi/3})
 * Each branch stamps Y_b = zabc^-1 as a 3x3 block (Y_ff += Y_b, Y_tt += Y_b,
 * Y_ft -= Y_b, Y_tf -= Y_b); the three slack nodes form the slack block of the partition,
 * and the network has n = 3 (n_bus - 1) demand nodes: column q of S and V is phase
 * q % 3 of the (q / 3)-th non-slack bus.  Everything downstream (modes, solve calls,
 * mismatch) is the same as for a single-phase network with n demand nodes.  Other
 * arguments and errors as tpf_build_network; TPF_ERR_INVALID_ARG for a non-finite or
 * singular zabc block. */
int tpf_build_network_3ph(int32_t n_bus, int32_t n_branch, const int32_t *from, const int32_t *to,
                          const double *zabc, int32_t slack_bus, const double *vs_abc, tpf_network *out);

void tpf_free_network(tpf_network net);

/* Number of demand nodes n: n_bus - 1 (single phase), 3 (n_bus - 1) (three phase). */
int tpf_network_n_pq(tpf_network net);

/* Copies Z = -Y_dd^-1 (host float64 [n][n][2]) and w (host float64 [n][2]) out of the
 * handle.  Either pointer may be NULL. */
int tpf_network_get_zw(tpf_network net, double *Z_out, double *w_out);

/* Bytes of device workspace that tpf_solve_* needs for tau columns with these
 * options (opts may be NULL).  The solve calls allocate nothing themselves.  Small
 * networks need 256 B; the per-sweep path for large networks holds its state, operand
 * and active lists there (about tau * 2n * 16 B in FP64); a warm start adds its V0
 * (tau * n * 16 B) and inference scratch. */
size_t tpf_workspace_bytes(tpf_network net, int64_t tau, const tpf_options *opts);

/* Algorithm 1 over a [T][n] load matrix (Sec. IV-A: each time step is a column).
 *   S            device [T][n] complex loads, dtype TPF_C64 or TPF_C128
 *   T            number of power flows (>= 0)
 *   tol          stop a column once max_i |V'_i - V_i| < tol (pu); tol >= 0
 *   max_iter     sweep cap per column (>= 0); 0 returns the start voltages
 *   opts         may be NULL (FP64, flat start, no mismatch)
 *   V_out        device [T][n] complex, same dtype as S
 *   iters_out    device int32 [T]: sweeps done per column
 *   status_out   device int8  [T]: TPF_ST_*
 *   workspace    device, >= tpf_workspace_bytes(net, T, opts) bytes, 256-byte aligned
 *   stream       hipStream_t (NULL = default stream) */
int tpf_solve_timeseries(tpf_network net, const void *S, int32_t dtype, int64_t T, double tol,
                         int32_t max_iter, const tpf_options *opts, void *V_out,
                         int32_t *iters_out, int8_t *status_out, void *workspace,
                         size_t workspace_bytes, void *stream);

/* Same over a [P][T][n] tensor (Sec. IV-A Eq. (12): any leading dimensions collapse into
 * tau = P*T columns without changing any iterate).  Arrays are [P][T][n], [P][T]. */
int tpf_solve_tensor(tpf_network net, const void *S, int32_t dtype, int64_t n_scen, int64_t T,
                     double tol, int32_t max_iter, const tpf_options *opts, void *V_out,
                     int32_t *iters_out, int8_t *status_out, void *workspace,
                     size_t workspace_bytes, void *stream);

/* Allocation-free variant of tpf_solve_timeseries, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments and results as tpf_solve_timeseries without the workspace: the scratch its
 * kernels need (the atomic column queue of the persistent sweep kernels) lives in a static
 * device array of 4096 bytes that each GPU holds until the process ends.  It allocates
 * nothing: the network must already be resident on the current device (the first
 * tpf_solve_timeseries, tpf_solve_tensor or tpf_mismatch call with it there uploads it), else
 * TPF_ERR_UNSUPPORTED.  A request whose tpf_workspace_bytes exceeds 4096 -- the per-sweep path
 * of large networks, a learned warm start -- returns TPF_ERR_UNSUPPORTED.  Every call on a
 * GPU uses that GPU's one array (cleared by each call where it must start at zero), so calls
 * that overlap on one GPU (other streams or threads) race: the caller serialises them. */
int tpf_solve_timeseries_noalloc(tpf_network net, const void *S, int32_t dtype, int64_t T, double tol,
                                 int32_t max_iter, const tpf_options *opts, void *V_out, int32_t *iters_out,
                                 int8_t *status_out, void *stream);

/* FP64 power-balance mismatch of given voltages (Eq. (1)):
 * out[c] = max_i |S_ci + V_ci conj((Y_ds v_s)_i + (Y_dd V_c)_i)|
 * (for a ZIP network the load term S_ci is S_ci (alpha_P,i + alpha_I,i V_ci +
 * alpha_Z,i |V_ci|^2)).  NaN when a term is NaN; the maximum is taken over |.|^2, so a
 * mismatch above about 1e154 pu reads inf.
 *   S, V   device [tau][n], dtype TPF_C64 or TPF_C128;  out  device float64 [tau]. */
int tpf_mismatch(tpf_network net, const void *S, const void *V, int32_t dtype, int64_t tau,
                 double *out, void *stream);

/* ---------------------------------------------------------------------------------------
 * Learned warm start.  Not part of the paper's method: a multilayer perceptron that maps a
 * time step's loads to an estimate of its converged voltages, used as V0 so that Algorithm 1
 * starts closer to its fixed point (the flat start stays the fallback through the V0 guard
 * of tpf_solve_*).  Definitions:
 *   features  x = [50 Re S, 50 Im S, sin/cos(2 pi (t mod 1440)/1440),
 *                  sin/cos(2 pi (floor(t/1440) mod 365)/365)]  (2n + 4 values, t = minute index)
 *   layers    h_l = gelu(h_{l-1} W_l^T + b_l) for the hidden layers, y = h_L W^T + b (2n outputs);
 *             gelu(z) = z (1 + erf(z/sqrt 2))/2; products in BF16 on MFMA, FP32 accumulation
 *   output    V0 = v_s + (y_re + j y_im) / 20
 *   training  loss = mean (y - 20 [Re(V - v_s), Im(V - v_s)])^2 over rows and outputs;
 *             AdamW (beta1 0.9, beta2 0.999, eps 1e-8, decoupled weight decay) on FP32 master
 *             parameters, BF16 copies refreshed after each step.
 * Parameters are one flat float32 vector [W_1 (out x in, row-major), b_1, W_2, b_2, ...].
 * A handle is bound to the device that is current when it is created.
 * --------------------------------------------------------------------------------------- */
/* n_pq PQ buses, `layers` hidden layers of width `hidden`; params: host float32 [num_params]
 * initial values (NULL: zeros); vs: slack voltage.  Errors: INVALID_ARG, DEVICE, OOM. */
int tpf_mlp_create(int32_t n_pq, int32_t hidden, int32_t layers, const float *params, double vs_re,
                   double vs_im, tpf_mlp *out);
void tpf_mlp_free(tpf_mlp mlp);
int64_t tpf_mlp_num_params(tpf_mlp mlp);
/* Host float32 [num_params] copies of the FP32 master parameters (synchronous). */
int tpf_mlp_get_params(tpf_mlp mlp, float *params_out);
int tpf_mlp_set_params(tpf_mlp mlp, const float *params);

/* Device workspace for `rows` rows of training or prediction. */
size_t tpf_mlp_workspace_bytes(tpf_mlp mlp, int64_t rows);

/* Loss and FP32 gradient of a batch.
 *   S        device [rows][n] loads (TPF_C64 / TPF_C128);  t_index  device int64 [rows] minute index
 *   V        device [rows][n] target voltages, same dtype as S
 *   loss_out device float32 [1];  grad_out  device float32 [num_params] */
int tpf_mlp_loss_grad(tpf_mlp mlp, const void *S, int32_t dtype, const int64_t *t_index, const void *V,
                      int64_t rows, float *loss_out, float *grad_out, void *workspace, size_t workspace_bytes,
                      void *stream);

/* One AdamW step on a batch (same inputs); loss_out may be NULL. */
int tpf_mlp_train_step(tpf_mlp mlp, const void *S, int32_t dtype, const int64_t *t_index, const void *V,
                       int64_t rows, float lr, float weight_decay, float *loss_out, void *workspace,
                       size_t workspace_bytes, void *stream);

/* Mini-batch training over a set of solved power flows: epochs first_epoch ..
 * first_epoch + epochs - 1 of a run of total_epochs epochs.
 *   S, V       device [rows][n] loads and target voltages (same dtype);  t_index  device int64 [rows]
 *   batch      rows per AdamW step (batch > rows means one batch of all rows); an epoch takes
 *              rows / batch steps over a fresh permutation of the rows, computed on the device
 *              from (seed, epoch) (a 4-round Feistel network on 2h-bit integers, 4^h >= rows,
 *              restricted to [0, rows) by cycle walking), so a resumed run revisits the same
 *              batches; the rows past (rows / batch) * batch sit out that epoch
 *   lr, lr_min cosine schedule over the run's total_epochs * (rows / batch) steps:
 *              lr_k = lr_min + (lr - lr_min)(1 + cos(pi k / (total - 1)))/2 at global step k
 *   epoch_loss_out  device float32 [epochs] mean batch loss per epoch (before each step), or NULL
 *   workspace  >= tpf_mlp_workspace_bytes(mlp, min(batch, rows)) bytes
 * The AdamW state (moments and step count) lives in the handle, so splitting a run into
 * several calls, with tpf_mlp_save / tpf_mlp_load in between, gives the same parameters bit
 * for bit as one call.  Errors: INVALID_ARG (sizes, epoch range, negative rates), DEVICE. */
int tpf_mlp_train(tpf_mlp mlp, const void *S, int32_t dtype, const int64_t *t_index, const void *V, int64_t rows,
                  int32_t first_epoch, int32_t epochs, int32_t total_epochs, int32_t batch, float lr, float lr_min,
                  float weight_decay, uint64_t seed, float *epoch_loss_out, void *workspace, size_t workspace_bytes,
                  void *stream);

/* Warm start V0 (device [rows][n], same dtype as S) for the loads S at minute indices t_index.
 * When every padded layer width is <= 256 (the 99-bus network's 202 -> 256 x 3 -> 198), one
 * fused kernel per 128-row tile computes it with the activations in LDS and erf from
 * Abramowitz-Stegun 7.1.26 (|error| < 1.5e-7, below the BF16 rounding of the activations);
 * the workspace is then unused but still checked.  Wider networks run layer by layer. */
int tpf_mlp_predict(tpf_mlp mlp, const void *S, int32_t dtype, const int64_t *t_index, int64_t rows, void *V0_out,
                    void *workspace, size_t workspace_bytes, void *stream);

/* Binary file with sizes, slack voltage, AdamW step count, the FP32 parameters and the
 * AdamW moments (format TPFMLP02; tpf_mlp_load also reads the parameters-only TPFMLP01
 * format, whose optimiser restarts at step 0 with zero moments). */
int tpf_mlp_save(tpf_mlp mlp, const char *path);
int tpf_mlp_load(const char *path, tpf_mlp *out);

/* Description of the last error on this thread ("" if none). */
const char *tpf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TPF_H_ */
