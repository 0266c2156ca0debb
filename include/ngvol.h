/*
 * ngvol — querying and training a volumetric neural representation on
 * AMD Instinct MI355X (gfx950).
 *
 * The representation is the paper's Phi: R^3 -> R (Section 3): a
 * multi-resolution hash-grid encoding (Section 3.1, Fig. 1B) feeding a tiny
 * bias-free ReLU MLP.  This library evaluates it (forward, for batch queries
 * and for the sample-streaming ray marcher of Section 5.2.1), differentiates
 * it, and runs the training step of Section 4 (sampling step, loss, backward,
 * Adam) — all on the GPU, as hand-written HIP kernels.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Status: every call returns NGVOL_OK (0) or a negative NGVOL_E* code;
 *   ngvol_last_error() gives a message for the calling thread.  Arguments are
 *   validated on the host before anything is launched; a failing call has
 *   launched nothing.  No C++ exception crosses this interface.
 * Memory: every pointer named d_* or documented as "device" is device memory
 *   owned by the caller; the library allocates no device memory in any call
 *   (workspaces are passed in).  Parameter vectors, FP16 tables, feature
 *   inputs of ngvol_mlp_fwd, volumes, the transfer-function table, images,
 *   counters and workspaces must be 16-byte aligned; coordinate, target,
 *   output and gradient buffers 4-byte aligned.  The library owns only the
 *   host-side plan.
 * Streams: calls enqueue work on the given hipStream_t (NULL = the legacy
 *   default stream) and return without synchronising, unless stated.
 * Plans: a plan is immutable after creation and may be shared between
 *   threads; calls that write the same output buffers must not overlap.
 * n = 0 is a no-op that returns NGVOL_OK.
 * Coordinates are clamped to [0,1] before use; a NaN coordinate is treated
 *   as 0.
 *
 * Parameter vector (FP32 master, n_params floats)
 * ----------------------------------------------
 *   [ level 0 table | level 1 table | ... | W_0 | W_1 | ... | W_out ]
 * Level l has N_l vertices per axis spanning [0,1]; its table holds
 * T_l = min(2^log2T, N_l^3) entries of F features, entry-major ([T_l][F]).
 * A level with N_l^3 <= 2^log2T is dense (slot = vx + N_l (vy + N_l vz));
 * otherwise the slot is the spatial hash of the encoding the paper adopts
 * (vx*1 XOR vy*2654435761 XOR vz*805459861, mod 2^32, then mod 2^log2T).
 * The MLP matrices follow, row-major [out][in], without biases or padding:
 * W_0 [width][L*F], then (n_hidden-1) x [width][width], then W_out [1][width].
 * The optional FP16 table copy has the table part's order (n_table_params
 * halves).
 */
#ifndef NGVOL_H
#define NGVOL_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NGVOL_OK 0
#define NGVOL_EINVAL (-1)       /* bad argument (shape, pointer, alignment, size) */
#define NGVOL_ENOMEM (-2)       /* host allocation failed, or workspace too small */
#define NGVOL_EDEVICE (-3)      /* a HIP runtime call failed */
#define NGVOL_EUNSUPPORTED (-4) /* valid but unsupported combination (e.g. width 48) */

#define NGVOL_MAX_LEVELS 32
#define NGVOL_MAX_LAYERS 9

/* MLP arithmetic of a plan. */
#define NGVOL_FP32 0 /* FP32 operands on the matrix cores (v_mfma_f32_16x16x4_f32) */
#define NGVOL_BF16 1 /* BF16 operands on MFMA with FP32 accumulation */
#define NGVOL_FP16 2 /* FP16 operands on MFMA with FP32 accumulation */

/* Element types of volumes and feature buffers. */
/* Training loss (Section 3.1 names L1 as the default loss; the DNS
 * experiment of Section 7.1 uses L2). */
#define NGVOL_LOSS_L2 0 /* L = (1/B) sum (Phi(x)-y)^2 */
#define NGVOL_LOSS_L1 1 /* L = (1/B) sum |Phi(x)-y|; dL/dPhi = sign(Phi(x)-y)/B, sign(0) = 0 */

/* Activation of the output neuron.  Section 3.1 describes ReLU activations
 * for the MLP layers; the network listing of the appendix for time-varying
 * data ends in a ReLU.  The hidden layers always use ReLU. */
#define NGVOL_ACT_NONE 0 /* identity output */
#define NGVOL_ACT_RELU 1 /* Phi = max(0, w_out . h); its derivative at 0 is taken as 0 */

#define NGVOL_DT_F32 0
#define NGVOL_DT_F16 1
#define NGVOL_DT_BF16 2

typedef struct ngvol_plan ngvol_plan;

/*
 * Model configuration (Section 3.1; hyper-parameter names follow the
 * configuration listings of the paper's appendix).
 * Supported: 1 <= n_levels <= 32; n_features in {2,4,8};
 * n_levels * n_features <= 64; 1 <= log2_hashmap_size <= 28;
 * n_neurons in {32,64}; 1 <= n_hidden_layers <= 8; the weights of a
 * forward must fit in LDS and the backward (ngvol_mlp_bwd,
 * ngvol_train_step) needs W and W^T in LDS (else NGVOL_EUNSUPPORTED; dW
 * accumulates in LDS too when that leaves room for four waves, else in the
 * workspace's per-workgroup partial sums);
 * the tables hold at most 2^30 - 4 floats (4 GiB of FP32, else
 * NGVOL_EUNSUPPORTED).
 * Vertices per axis: resolutions[l] if given; else N_l = base * b^l, used as
 * is when it is an integer (within 1e-9 relative) and rounded up otherwise,
 * with b = per_level_scale, or b = exp((ln max_resolution - ln base)/(L-1))
 * when max_resolution > 0.  Every N_l must be in [2, 65536].
 */
typedef struct ngvol_config {
    int32_t n_levels;
    int32_t n_features;
    int32_t log2_hashmap_size;
    int32_t base_resolution;
    double per_level_scale;
    int32_t max_resolution;
    const int32_t* resolutions; /* host pointer, optional */
    int32_t n_neurons;
    int32_t n_hidden_layers;
    int32_t precision; /* NGVOL_FP32 | NGVOL_BF16 | NGVOL_FP16 */
    int32_t loss;      /* NGVOL_LOSS_L2 (0) | NGVOL_LOSS_L1; used by ngvol_train_step */
    int32_t output_activation; /* NGVOL_ACT_NONE (0) | NGVOL_ACT_RELU */
} ngvol_config;

/* Derived layout of a plan (host struct filled by ngvol_get_layout). */
typedef struct ngvol_layout {
    int32_t n_levels, n_features, n_input, n_neurons, n_hidden_layers, precision;
    int32_t resolution[NGVOL_MAX_LEVELS];
    int32_t dense[NGVOL_MAX_LEVELS];
    int64_t level_entries[NGVOL_MAX_LEVELS];
    int64_t level_offset[NGVOL_MAX_LEVELS + 1]; /* in entries; times F gives floats */
    int64_t n_table_params;
    int64_t n_mlp_params;
    int64_t n_params;
    int64_t layer_offset[NGVOL_MAX_LAYERS]; /* offset of each matrix in the parameter vector */
} ngvol_layout;

/* Weights used by forward calls.  table_f16 (optional) is an FP16 copy of
 * the table part; when non-NULL the encoding gathers it instead of the FP32
 * tables (the MLP always reads the FP32 matrices). */
typedef struct ngvol_weights {
    const float* params;       /* device [n_params] */
    const uint16_t* table_f16; /* device [n_table_params] or NULL */
} ngvol_weights;

/* Training state (all device memory).  grad must be all zero before the
 * first step; every step leaves it zero again.  m and v start at zero. */
typedef struct ngvol_train_state {
    float* params;       /* [n_params] FP32 master */
    uint16_t* table_f16; /* [n_table_params] FP16 shadow, or NULL */
    float* grad;         /* [n_params] */
    float* adam_m;       /* [n_params] */
    float* adam_v;       /* [n_params] */
    int64_t* step;       /* [1] number of applied (not skipped) Adam steps */
    int32_t* skipped;    /* [1] 1 if the last step was skipped (non-finite gradient) */
    double* loss;        /* [1] mean loss of the last step (unscaled) */
    void* workspace;     /* ngvol_train_workspace_bytes(plan, B) bytes */
    size_t workspace_bytes;
    int64_t* draws;      /* [1] or NULL: number of steps taken, applied or skipped (every step adds 1) */
} ngvol_train_state;

/* Macro-cells (Section 5.3): a grid of disjoint cells of `cell` voxels per
 * axis over a volume of dims = (Dx, Dy, Dz) voxels, M_a = ceil(D_a / cell)
 * cells per axis (the grid may extend past the volume), cell-major
 * [Mz][My][Mx].  A point p (clamped to [0,1], NaN as 0) lies in cell
 * c_a = min(floor(p_a * D_a) / cell, M_a - 1), p_a * D_a rounded to binary32.
 * range[2c], range[2c+1] hold the minimum and maximum value seen in cell c as
 * order-preserving keys of binary32 (k(v) = bits | 2^31 for sign 0, ~bits
 * for sign 1; an empty cell is (0xFFFFFFFF, 0)); the online construction of
 * Section 5.3 feeds them the training samples.  mu[c] is the largest opacity
 * the transfer function takes over the cell's range, 0 for an empty cell.
 * All arrays are device memory owned by the caller. */
typedef struct ngvol_macrocells {
    int32_t dims[3];  /* Dx, Dy, Dz, each in [1, 2^20] */
    int32_t cell;     /* voxels per cell per axis, >= 1; Mx*My*Mz <= 2^24 */
    uint32_t* range;  /* [Mz*My*Mx][2] */
    float* mu;        /* [Mz*My*Mx] */
} ngvol_macrocells;

/* One training batch (Section 4, the sampling step).  Either explicit
 * samples (xyz != NULL: coordinates and targets given), or generated on the
 * device: coordinate axis a of sample i is the binary32 uniform
 * (r >> 40) * 2^-24 of counter-based SplitMix64 output r for (seed, stream 3,
 * index = step_index*B*3 + 3*i + a), and its target is the cell-centred
 * trilinear, clamp-to-edge sample of the volume (voxel i centred at
 * (i+1/2)/D, x fastest). */
typedef struct ngvol_batch {
    int64_t batch_size;
    const float* xyz;    /* device [B][3] or NULL */
    const float* target; /* device [B] (when xyz != NULL) */
    const void* volume;  /* device [Dz][Dy][Dx] (when xyz == NULL) */
    int32_t dims[3];     /* Dx, Dy, Dz, each >= 2 */
    int32_t volume_dtype; /* NGVOL_DT_F32 | NGVOL_DT_F16 */
    uint64_t seed;       /* < 2^56 */
    int64_t step_index;  /* >= 0; or -1 (ngvol_train_step only): the batch index is read on the device from
                          * the state's draw counter (or, if the state has none, its step counter), so a
                          * captured graph draws a new batch on every replay (with the step counter, a
                          * skipped step would draw the same batch again) */
    const ngvol_macrocells* macrocells; /* optional (ngvol_train_step): the batch's (coordinate, target)
                                         * samples extend the cells' value ranges (NaN targets are ignored) */
} ngvol_batch;

/* Adam (Kingma and Ba) with bias correction and an exponentially decaying
 * learning rate; the paper trains with Adam under an exponential decay
 * (Section 3.1; decay start, interval and base and the L2 regularisation are
 * the parameters of the appendix's default optimiser configuration).
 * Gradients are divided by loss_scale before use; if any unscaled
 * contribution is non-finite the whole step is skipped.
 * Step k (0-based count of applied steps, the state's step counter) uses
 *   lr_k = learning_rate * decay_base^floor((k - decay_start) / decay_interval)
 * when decay_interval > 0 and k >= decay_start, else learning_rate.
 * l2_reg adds l2_reg * w to the gradient of every MLP weight w (not to the
 * tables).  Zero l2_reg and decay_interval give plain Adam. */
typedef struct ngvol_adam {
    double learning_rate, beta1, beta2, epsilon;
    double l2_reg;          /* >= 0 */
    int64_t decay_start;    /* >= 0 */
    int64_t decay_interval; /* >= 0; 0 = no decay */
    double decay_base;      /* in (0, 1] when decay_interval > 0 */
} ngvol_adam;

/* Pinhole camera: the unnormalised direction through pixel centre (px,py)
 * is (dir00 + (px+1/2) du) + (py+1/2) dv, evaluated in binary32. */
typedef struct ngvol_camera {
    float origin[3];
    float du[3];
    float dv[3];
    float dir00[3];
} ngvol_camera;

/* Counters a render call writes to device memory (optional). */
typedef struct ngvol_render_counters {
    unsigned long long samples_evaluated; /* network samples computed */
    unsigned long long samples_used;      /* samples composited before termination */
    unsigned long long rays;              /* rays with at least one sample */
    unsigned long long pad;
} ngvol_render_counters;

/* ----------------------------------------------------------------------- */
const char* ngvol_last_error(void);
const char* ngvol_version(void);

/* Debug mode (also switched on by NGVOL_DEBUG=1 in the environment): every
 * call then waits for the device after its launches (hipDeviceSynchronize)
 * and returns NGVOL_EDEVICE with the runtime's message if one of them
 * failed.  On a stream that is being captured into a graph it only checks
 * the launch status (hipGetLastError), which leaves the capture intact. */
int ngvol_set_debug(int32_t on);

/* Create / destroy a plan.  EINVAL for out-of-range fields, EUNSUPPORTED for
 * valid but unsupported widths or feature counts. */
int ngvol_plan_create(const ngvol_config* cfg, ngvol_plan** out);
int ngvol_plan_destroy(ngvol_plan* plan);
int ngvol_get_layout(const ngvol_plan* plan, ngvol_layout* out);

/* Encoding (Section 3.1): feat[n][L*F] (FP32, device) = concatenation over
 * levels of the trilinear interpolation of the 8 enclosing vertices'
 * features. */
int ngvol_encode(const ngvol_plan* plan, const ngvol_weights* w, const float* d_xyz, int64_t n, float* d_feat,
                 hipStream_t stream);

/* Corner slots and weights of the encoding: idx[n][L][8] (slot within the
 * level's table, no level offset) and w[n][L][8]; corner k has offset
 * (k&1, (k>>1)&1, (k>>2)&1).  Either output may be NULL. */
int ngvol_encode_debug(const ngvol_plan* plan, const float* d_xyz, int64_t n, uint32_t* d_idx, float* d_w,
                       hipStream_t stream);

/* MLP forward (Section 3.1) on given features: out[n] (FP32) from
 * feat[n][L*F] of type feat_dtype (NGVOL_DT_F32, NGVOL_DT_BF16 or
 * NGVOL_DT_F16), with the plan's precision. */
int ngvol_mlp_fwd(const ngvol_plan* plan, const float* d_params, const void* d_feat, int32_t feat_dtype, int64_t n,
                  float* d_out, hipStream_t stream);

/* Query (Sections 3.1 and 3.2): out[n] = Phi(xyz), encoding + MLP.  Without
 * a workspace (d_workspace == NULL) one fused kernel evaluates the queries
 * in the given order (best for coherent inputs such as already sorted or
 * ray-ordered coordinates).  With a workspace of
 * ngvol_infer_workspace_bytes(plan, n) bytes the queries are first grouped
 * by spatial cell (a counting sort on the device) so that neighbouring
 * queries share table cache lines; for large sets whose tables exceed one
 * XCD's L2 (FP16 tables given, n >= 2^20) the grouped queries are then
 * evaluated level group by level group, each XCD interpolating its own
 * levels for all queries into feature planes in the workspace, followed by
 * the MLP on those planes.  Every output lands in its own slot.  The fused
 * kernel gives the same values in either order; the level-split path sums
 * the first layer's products in another order, so its values agree with the
 * fused kernel to FP32 rounding (with 16-bit operands a hidden activation
 * may round differently).  The bytes query returns 0 when n is too small
 * for reordering to pay off.  n < 2^31. */
int ngvol_infer_workspace_bytes(const ngvol_plan* plan, int64_t n, size_t* bytes);
int ngvol_infer(const ngvol_plan* plan, const ngvol_weights* w, const float* d_xyz, int64_t n, float* d_out,
                void* d_workspace, size_t workspace_bytes, hipStream_t stream);

/* The two halves of a reordered ngvol_infer, for coordinates that are
 * queried more than once: ngvol_sort_queries groups xyz[n] by spatial cell
 * into the workspace (ngvol_infer_workspace_bytes; EINVAL if that is 0), and
 * ngvol_infer_sorted evaluates the grouped queries of that workspace, writing
 * each output to its original slot of out[n].  The plan and n must be those
 * of the sort; ngvol_infer_sorted also uses the rest of the workspace as
 * scratch (the grouped records are kept, so it may be called again). */
int ngvol_sort_queries(const ngvol_plan* plan, const float* d_xyz, int64_t n, void* d_workspace,
                       size_t workspace_bytes, hipStream_t stream);
int ngvol_infer_sorted(const ngvol_plan* plan, const ngvol_weights* w, void* d_workspace, int64_t n,
                       float* d_out, hipStream_t stream);

/* MLP backward: given d_out[n] = dL/dout, adds dL/dW into the MLP part of
 * d_grad (n_params floats, the table part is untouched) and, if
 * d_dfeat != NULL, writes dL/dfeat [n][L*F].  The forward is recomputed from
 * d_feat in the plan's precision (BF16 rounds the features first, as
 * ngvol_mlp_fwd does).  Needs ngvol_mlp_bwd_workspace_bytes(plan, n) bytes
 * of workspace. */
int ngvol_mlp_bwd_workspace_bytes(const ngvol_plan* plan, int64_t n, size_t* bytes);
int ngvol_mlp_bwd(const ngvol_plan* plan, const float* d_params, const float* d_feat, int64_t n, const float* d_dout,
                  float* d_dfeat, float* d_grad, void* d_workspace, size_t workspace_bytes, hipStream_t stream);

/* Allocation-free MLP backward, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same computation and outputs as ngvol_mlp_bwd
 * (dW added into the MLP part of d_grad; dL/dfeat into d_dfeat if non-NULL),
 * with no workspace argument.  Its per-workgroup dW partial sums live in a
 * static device array of ngvol_mlp_bwd_noalloc_scratch_bytes() bytes (8 MiB)
 * that the library holds on every GPU it runs on until the process ends; no
 * call allocates or frees memory.  One partial-sum row (4 * n_mlp bytes) per
 * workgroup: the call uses at most (8 MiB - 256) / (4 n_mlp) workgroups
 * (each takes more tiles when that is fewer than ngvol_mlp_bwd would use),
 * and returns NGVOL_EINVAL if not even one row fits.  Every row a call reads
 * is written by that call first, so nothing carries over from the previous
 * call; but all calls on one GPU share the array, so calls that overlap in
 * time on one GPU (different streams or threads) race and must be ordered by
 * the caller.  The address of the array is looked up on the first call on
 * each device (the calling thread's current device). */
size_t ngvol_mlp_bwd_noalloc_scratch_bytes(void);
int ngvol_mlp_bwd_noalloc(const ngvol_plan* plan, const float* d_params, const float* d_feat, int64_t n,
                          const float* d_dout, float* d_dfeat, float* d_grad, hipStream_t stream);

/* Encoding backward: accumulates grad_table[slot][f] += w_corner *
 * dfeat[l*F+f] over all samples, levels and corners into d_grad (atomic,
 * so the summation order is unspecified). */
int ngvol_encode_bwd(const ngvol_plan* plan, const float* d_xyz, int64_t n, const float* d_dfeat, float* d_grad,
                     hipStream_t stream);

/* Sampling step alone: fills xyz[B][3] and target[B] as a generated batch
 * would (batch->xyz must be NULL). */
int ngvol_sample_batch(const ngvol_plan* plan, const ngvol_batch* batch, float* d_xyz, float* d_target,
                       hipStream_t stream);

/* Workspace a training step of batch B needs.  A step scatters B * 8 * L
 * table-gradient records with 32-bit positions: B * 8 * L >= 2^32 is
 * NGVOL_EINVAL; tables of more than 40960 gradient buckets (2^12 entries per
 * bucket for F = 2, 2^11 for F = 4, 2^10 for F = 8), whose histogram would
 * not fit in LDS, are NGVOL_EUNSUPPORTED.  ngvol_train_step checks the same
 * before launching anything. */
int ngvol_train_workspace_bytes(const ngvol_plan* plan, int64_t batch_size, size_t* bytes);

/* One training step (Section 4): sampling, forward, the plan's loss
 * (NGVOL_LOSS_L2 or NGVOL_LOSS_L1, mean over the batch), backward through the MLP (activations
 * recomputed from the stored encoding) and the encoding, then Adam on all
 * parameters; the FP16 shadow (if any) is refreshed by round-to-nearest-even
 * from the master.  Gradients are formed at loss_scale times their value
 * and divided by it in the update. */
int ngvol_train_step(const ngvol_plan* plan, const ngvol_train_state* state, const ngvol_batch* batch,
                     const ngvol_adam* adam, float loss_scale, hipStream_t stream);

/* Adam update alone on state->grad (left zero afterwards). */
int ngvol_adam_step(const ngvol_plan* plan, const ngvol_train_state* state, const ngvol_adam* adam, float loss_scale,
                    hipStream_t stream);

/* FP16 copy of the tables from FP32 parameters. */
int ngvol_make_f16_tables(const ngvol_plan* plan, const float* d_params, uint16_t* d_table_f16, hipStream_t stream);

/* Sum over all voxel centres (i+1/2)/D of (Phi - volume)^2, added to
 * *d_sum_sq (device double).  MSE = sum / (Dx Dy Dz); PSNR = -10 log10 MSE
 * for values normalised to [0,1] (Section 6). */
int ngvol_sq_error_grid(const ngvol_plan* plan, const ngvol_weights* w, const void* d_volume, const int32_t dims[3],
                        int32_t volume_dtype, double* d_sum_sq, hipStream_t stream);

/* Decoding quality (Section 6): the network evaluated at every voxel centre
 * (i+1/2)/D of the volume, *d_mse (device double) = mean of (Phi - v)^2 over
 * all voxels, accumulated in FP64 on the device, and, if d_psnr is non-NULL,
 * *d_psnr (device double) = -10 log10(MSE), the PSNR of values normalised to
 * [0,1] (peak 1).  Both outputs are overwritten; nothing is synchronised. */
int ngvol_psnr(const ngvol_plan* plan, const ngvol_weights* w, const void* d_volume, const int32_t dims[3],
               int32_t volume_dtype, double* d_mse, double* d_psnr, hipStream_t stream);

/* Macro-cells (Section 5.3).  reset: every cell empty.  update: extend the
 * ranges with n explicit samples (xyz[n][3], values[n], device).  opacity:
 * mu of every cell for a transfer function d_lut[256][4] (RGBA, the alpha
 * of the shading below: piecewise linear in v over nodes i/255), the maximum
 * over the two range ends and every node strictly inside. */
int ngvol_mc_reset(const ngvol_macrocells* mc, hipStream_t stream);
int ngvol_mc_update(const ngvol_macrocells* mc, const float* d_xyz, const float* d_values, int64_t n,
                    hipStream_t stream);
int ngvol_mc_opacity(const ngvol_macrocells* mc, const float* d_lut, hipStream_t stream);

/* Workspace for ngvol_render (a few counters). */
size_t ngvol_render_workspace_bytes(void);

/*
 * Ray-marched emission-absorption rendering through Phi (Section 5.2.1),
 * sample streaming in one persistent launch: rays are taken from a device
 * queue; each round a ray streams K = 8 sample coordinates, the network is
 * evaluated on them, and the samples are shaded front to back; finished rays
 * are replaced from the queue.
 * Geometry in binary32 without FMA: d = dir/sqrt(dir.dir); slab test against
 * [0,1]^3; t_near = max(t_min,0); n = max(0, ceil((t_max-t_near)/dt - j)) if
 * t_near < t_max else 0; t_k = t_near + (k+j) dt; p_k = o + t_k d, with
 * jitter j the binary32 uniform of (frame_seed, stream 5, pixel py*W+px).
 * Shading: v = clamp(Phi,0,1); u = 255 v; i = min(floor(u),254);
 * c = lut[i](1-(u-i)) + lut[i+1](u-i); C += (1-A) c.a c.rgb; A += (1-A) c.a;
 * a ray stops after the sample at which A >= 0.99.
 * mc (nullable): empty-space skipping (Section 5.3): a sample whose
 * macro-cell has mu = 0 (mc->mu as left by ngvol_mc_opacity) is neither
 * evaluated nor composited; a ray scans its samples 64 at a time for them.
 * rgba[H][W][4] FP32 (premultiplied colour, alpha); n_geo[H][W] (nullable):
 * geometric sample counts n; n_used (nullable): samples composited;
 * counters (nullable, device): totals.  lut: device [256][4].
 */
/* dt must be in [2^-20, 1]; a ray whose span exceeds 2^24 steps (only a
 * degenerate camera can produce one) gets no samples. */
int ngvol_render(const ngvol_plan* plan, const ngvol_weights* w, const ngvol_camera* cam, const float* d_lut,
                 int32_t width, int32_t height, float dt, uint32_t frame_seed, const ngvol_macrocells* mc,
                 float* d_rgba, uint32_t* d_n_geo, uint32_t* d_n_used, ngvol_render_counters* d_counters,
                 void* d_workspace, size_t workspace_bytes, hipStream_t stream);

/* Rendering options of ngvol_render_ex. */
#define NGVOL_RENDER_RM 0        /* emission-absorption ray marching (Section 5.2.1) */
#define NGVOL_RENDER_RM_SHADOW 1 /* ray marching with a single-shot heuristic shadow (Section 5.2) */
#define NGVOL_RENDER_PT 2        /* volumetric path tracing (Section 5.2.2, Algorithm 1) */

typedef struct ngvol_render_opts {
    int32_t mode; /* NGVOL_RENDER_RM, NGVOL_RENDER_RM_SHADOW or NGVOL_RENDER_PT */
    /* RM: adaptive marching through the macro-cells (Section 5.3; needs mc
     * with mu set).  Samples stay on the ray's grid t_k; from sample k in
     * cell c of maximum opacity mu: mu = 0 bypasses the cell (k moves to the
     * first sample outside it, found by a DDA step along the ray and an exact
     * check of the neighbouring samples' cells); otherwise the sample is
     * evaluated and stands for m = min(n(mu), exit(c) - k, n - k) grid steps
     * with n(mu) = max(1, floor(max(1 + (step_max - 1) |min(mu,1) - 1|^p, 1)))
     * in binary32 (the power by repeated multiplication), its opacity is
     * corrected to 1 - (1 - alpha)^m (alpha itself for m = 1), and k moves
     * by m.  0: fixed steps, with mc only skipping samples in transparent
     * cells as ngvol_render does.  RM only. */
    int32_t adaptive;
    float step_max;   /* s2 in grid steps, >= 1 (the paper uses 64) */
    int32_t step_exp; /* p, 1..8 (the paper uses 2) */
    /* RM_SHADOW and PT: direction towards a directional light (normalised in
     * binary32 on the device; must not be zero).
     * RM_SHADOW: the primary ray is marched as in RM (mc: empty cells
     * skipped); its sample of largest contribution (1 - A_{k-1}) alpha_k,
     * the first on ties, is the shading point.  A shadow ray leaves that
     * sample's position along the light direction with the pixel's jitter
     * and the primary rays' sample rule, from its sample k = 1 on, and
     * multiplies the transmittance T by (1 - alpha) per sample, ending after
     * the sample at which T <= 0.01.  The pixel is (T C, A). */
    float light_dir[3];
    /* PT: medium of extinction density * alpha(phi) and albedo rgb(phi)
     * (the transfer function at the clamped network value phi), isotropic
     * scattering; majorant density * mu per macro-cell when mc is given (the
     * cells visited by a 3-D DDA, the optical thickness accumulated per
     * cell), else density * (largest alpha of the table) for the whole cube.
     * A scattering ray that meets a real collision spawns a shadow ray
     * towards the light, tracked the same way: leaving the cube it adds
     * throughput * light_radiance / (4 pi), meeting a real collision it adds
     * nothing; the path then scatters into a uniformly drawn direction.  A
     * scattering ray leaving the cube adds throughput * background and ends
     * the path.  From real scattering collision rr_depth + 1 on, Russian
     * roulette keeps the path with probability q = min(1, max throughput)
     * and divides the throughput by q; a path also ends after max_depth
     * scattering collisions and after 65536 tentative collisions.  Random
     * numbers come from stream 8 of the library's counter generator, keyed
     * by (frame_seed, (pixel * spp + path) * 2^24 + draw).  Output: rgba =
     * (mean radiance over spp paths, fraction of paths whose camera ray met
     * a real collision); n_geo counts the pixel's real collisions, n_used
     * its tentative collisions (network samples). */
    float light_radiance[3];
    float background[3];
    float density;     /* > 0 */
    int32_t spp;       /* paths per pixel, 1..256 */
    int32_t rr_depth;  /* >= 0 (the paper uses 4) */
    int32_t max_depth; /* 1..1024 */
    /* Per-pixel output [H][W].  RM_SHADOW (required): the index k of the
     * shading point on the primary ray, UINT32_MAX when there is none; the
     * camera rays are marched first, recording these, then the shadow rays
     * in a second pass (as the paper's listing runs them), which scales the
     * recorded colours by T.  Other modes: unused. */
    uint32_t* d_aux;
} ngvol_render_opts;

/* ngvol_render with options (opts NULL: the defaults of ngvol_render, i.e.
 * mode RM with fixed steps).  Counters and outputs as ngvol_render (RM and
 * RM_SHADOW: n_geo and n_used count the primary ray's samples; PT: see
 * ngvol_render_opts; counters = {network samples, PT: real collisions, else
 * composited primary samples, PT: paths, else rays, 0}).  RM_SHADOW with
 * adaptive marching is NGVOL_EUNSUPPORTED. */
int ngvol_render_ex(const ngvol_plan* plan, const ngvol_weights* w, const ngvol_camera* cam, const float* d_lut,
                    int32_t width, int32_t height, float dt, uint32_t frame_seed, const ngvol_macrocells* mc,
                    const ngvol_render_opts* opts, float* d_rgba, uint32_t* d_n_geo, uint32_t* d_n_used,
                    ngvol_render_counters* d_counters, void* d_workspace, size_t workspace_bytes, hipStream_t stream);

/* ----------------------------------------------------------------------- */
/* Out-of-core sampling (Section 4.1)                                      */
/* ----------------------------------------------------------------------- */
/* A volume larger than memory is sampled through a buffer of R blocks of
 * about 64 KB chosen at random, S of which are replaced before every
 * sampling step; samples pick a buffered block, a voxel of it, and jitter the
 * voxel centre by up to half a voxel (a one-voxel ghost layer around every
 * block holds the neighbours the trilinear interpolation needs).  Here the
 * buffer lives in device memory and the samples are drawn on the device; the
 * blocks come from a bricked file (one record per block) read by host threads.
 *
 * Schedule (both the block choice and the sample draws use the library's
 * counter generator): blocks are b^3 voxels, the last block of an axis
 * possibly partial, numbered x-fastest over the block grid
 * G_a = ceil(D_a / b).  Block load j takes block ((r_j >> 40) * n_blocks) >> 24
 * with r_j from stream 9 at index j; loads 0..R-1 fill slots 0..R-1 (step 0,
 * the warm-up), and step k >= 1 makes loads R + (k-1) S + i (i < S) into
 * slots ((k-1) S + i) mod R.  Sample i of step k draws the slot, a voxel of
 * the slot's block and the jitter u in [0,1)^3 from stream 10 at indices
 * (k B + i) 8 + 0..6 (as ((r >> 40) n) >> 24 and (r >> 40) 2^-24); its
 * coordinate is x_a = (v_a + u_a) / D_a in binary32 and its target the
 * volume's cell-centred trilinear sample at x (as ngvol_sample_batch). */
typedef struct ngvol_ooc ngvol_ooc;

typedef struct ngvol_ooc_info {
    int32_t dims[3], dtype, block, grid[3];
    int64_t n_blocks, record_bytes, R, S;
} ngvol_ooc_info;

/* Write the bricked copy of a raw volume ([Dz][Dy][Dx], x fastest, FP32 or
 * FP16 as dtype) that ngvol_ooc_open reads: a 4096-byte header, then one
 * record per block, in block order, of (block + 2)^3 values x-fastest (the
 * block and its ghost layer, indices clamped to the volume), padded to a
 * multiple of 4096 bytes.  block in [2, 254].  Host only; EINVAL on a short
 * or unreadable input or a failed write. */
int ngvol_ooc_brick_file(const char* raw_path, const int32_t dims[3], int32_t dtype, int32_t block,
                         const char* bricked_path);

/* Open a bricked file for sampling with R slots and S refreshes per step
 * (1 <= S <= R < 2^31), draws keyed by seed, n_threads host reader threads
 * (1..64).  Allocates pinned host staging for two chunks of S records and a
 * copy stream of its own (default priority) on the current device.  Host
 * objects only; the caller owns the device buffer (ngvol_ooc_device_bytes). */
int ngvol_ooc_open(const char* bricked_path, int64_t R, int64_t S, uint64_t seed, int32_t n_threads,
                   ngvol_ooc** out);
int ngvol_ooc_close(ngvol_ooc* ooc);
int ngvol_ooc_get_info(const ngvol_ooc* ooc, ngvol_ooc_info* out);
/* Bytes of the caller's device buffer: the R slots, a staging area for S
 * records, and the slot table. */
size_t ngvol_ooc_device_bytes(const ngvol_ooc* ooc);

/* Load the blocks of step `step` into their slots of d_buf (16-byte
 * aligned): all R at step 0, S from step 1 on; steps must follow each other
 * (0, 1, 2, ...; 0 restarts).  The records of a step are read by the host
 * threads into pinned staging: in the background right after the previous
 * refresh returns (the schedule is known in advance), else during the call.
 * The copies and a placement kernel run on the library's copy stream after
 * all work enqueued on `stream` before the call (so they may overlap
 * whatever the caller enqueues next, e.g. the training step of the previous
 * samples); the next ngvol_ooc_sample on `stream` waits for them.  One
 * ngvol_ooc is used by one host thread at a time. */
int ngvol_ooc_refresh(ngvol_ooc* ooc, int64_t step, void* d_buf, hipStream_t stream);

/* The B samples of step `step` (after its refresh): d_xyz [B][3] and
 * d_target [B] (FP32, 4-byte aligned), on `stream`.  B < 2^31. */
int ngvol_ooc_sample(ngvol_ooc* ooc, int64_t step, int64_t B, const void* d_buf, float* d_xyz, float* d_target,
                     hipStream_t stream);

/* Host copy of the block id held by each slot after the last refresh
 * (R int32). */
int ngvol_ooc_slots(const ngvol_ooc* ooc, int32_t* host_slot_block);

/* ----------------------------------------------------------------------- */
/* Batches of independent neural volumes                                   */
/* ----------------------------------------------------------------------- */
#define NGVOL_MULTI_MAX 16
typedef struct ngvol_multi ngvol_multi;

/* Device bytes of the descriptor table of a group of k models (the k
 * descriptors and the persistent query's work counter). */
size_t ngvol_multi_table_bytes(int32_t k);

/* Groups k plans (1 <= k <= 16) that share precision, n_features (2), the
 * padded input width (32 or 64 features), n_neurons and n_hidden_layers
 * (NGVOL_EUNSUPPORTED otherwise); the models may differ in levels,
 * resolutions and table sizes.  Their descriptors are copied into d_table
 * (caller-owned device memory of ngvol_multi_table_bytes(k) bytes, valid for
 * the group's lifetime); the call synchronises the stream once.  The plans
 * may be destroyed afterwards. */
int ngvol_multi_create(const ngvol_plan* const* plans, int32_t k, void* d_table, size_t table_bytes,
                       hipStream_t stream, ngvol_multi** out);
int ngvol_multi_destroy(ngvol_multi* group);

/* Queries of all k models in one call: model i writes Phi_i(xyz[i][j]) to
 * out[i][j] for j < n[i], with weights w[i] (host arrays of k entries; the
 * pointers they hold are device pointers, either all with or all without
 * FP16 tables).  By default one persistent launch: work is cut into chunks
 * of 16-sample tiles of one model, ordered model by model, taken in order
 * from a work counter in the group's table by the workgroups, which restage
 * the MLP weights in LDS when the model changes.  The counter is shared by
 * the group's calls: calls on one group must not overlap (issue them on one
 * stream).  After ngvol_multi_autotune it may instead issue one single-model
 * launch per model, back to back on the stream, when that was faster. */
int ngvol_multi_infer(const ngvol_multi* group, const ngvol_weights* w, const float* const* xyz, const int64_t* n,
                      float* const* out, hipStream_t stream);

/* Autotuner: times the candidate launch shapes (workgroups per compute unit
 * x tiles per chunk of the persistent launch, and one launch per model) on
 * these inputs (outputs are written), keeps the fastest for later
 * ngvol_multi_infer calls on the group and reports it (either pointer may be
 * NULL; 0 and 0 for one launch per model).  Synchronises the stream; not
 * thread-safe with other calls on the same group. */
int ngvol_multi_autotune(ngvol_multi* group, const ngvol_weights* w, const float* const* xyz, const int64_t* n,
                         float* const* out, hipStream_t stream, int32_t* blocks_per_cu, int32_t* chunk_tiles);

/* Training steps of all k models of the group in one call (Section 4 per
 * model; the batch of volumes of the multi-volume workload): model i takes
 * one ngvol_train_step with states[i] and batches[i] (host arrays of k
 * entries, distinct states) and the shared Adam settings and loss scale.
 * Every model's arguments are checked before anything is launched.  The steps
 * are spread over the group's own streams (up to 4), forked from `stream`
 * and joined back to it, so small steps of different models run
 * concurrently; captured on `stream`, the call becomes a graph with parallel
 * branches.  Results equal k separate ngvol_train_step calls. */
int ngvol_multi_train_step(const ngvol_multi* group, const ngvol_train_state* states, const ngvol_batch* batches,
                           const ngvol_adam* adam, float loss_scale, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* NGVOL_H */
