/*
 * lst.h - C ABI of the MI355X line-segment-tracking object builder.
 *
 * The library builds, from one event's (or a batch of events') outer-tracker
 * hits, the four LST track-segment collections of the paper's Table 1 steps
 * 1-4 (arXiv:2403.13166, Sec. 1):
 *   mini-doublets (MD): two hits on the two sensors of one pT-module;
 *   line segments (LS): two MDs on adjacent modules with consistent pT;
 *   triplets (T3):      two LSs sharing an MD;
 *   quintuplets (T5):   two T3s sharing an MD,
 * each passing geometric cuts, and scores every T5 with the T5-DNN of Sec. 2
 * (two hidden layers of 32 nodes, sigmoid output).
 *
 * Conventions (all entry points):
 *  - Every pointer named *_dev, and every pointer inside lst_hits and
 *    lst_objects, is a DEVICE pointer owned by the caller. Blobs and the
 *    lst_* structs themselves are host memory owned by the caller.
 *  - Work is ordered on the HIP stream passed as `stream` (NULL = default
 *    stream). The library allocates device memory only in lst_load_geometry
 *    and lst_load_model (its own tables, freed by lst_destroy); build and
 *    score calls never allocate: scratch is the caller's workspace.
 *  - Every function returns an lst_status; details of the last error are in
 *    lst_last_error(ctx). A context is not thread safe; calls that share a
 *    workspace must not overlap.
 */
#ifndef LST_H
#define LST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lst_status;
#define LST_OK 0
#define LST_E_INVAL (-1)     /* bad argument, bad blob, sensor id out of range, or a hit off its sensor */
#define LST_E_STATE (-2)     /* geometry / model not loaded */
#define LST_E_CAPACITY (-3)  /* an output or candidate capacity was too small */
#define LST_E_HIP (-4)       /* a HIP runtime call failed */
#define LST_E_NOMEM (-5)     /* device allocation failed (load calls only) */

/* lst_options.mode */
#define LST_MODE_DNN 0       /* T5-DNN scores every T5; no r-phi fit cut (Sec. 2) */
#define LST_MODE_PRE_DNN 1   /* r-phi circle-fit chi2 cut instead of the DNN (Sec. 2, Table 2) */
/* precision of the T5-DNN / lst_score */
#define LST_PREC_F32 0       /* FP32 vector ALU */
#define LST_PREC_BF16 1      /* BF16 inputs and weights on MFMA, FP32 accumulation */
/* lst_options.flags */
#define LST_ASYNC 1          /* do not synchronise; counts stay on the device */
/* lst_score x_dtype */
#define LST_DTYPE_F32 0
#define LST_DTYPE_BF16 1

/* counts_dev layout (int64 each) */
#define LST_COUNT_MD 0
#define LST_COUNT_LS 1
#define LST_COUNT_T3 2
#define LST_COUNT_T5 3
#define LST_COUNT_ERR 4      /* bit 0 bad sensor id, bit 1 candidate cap, bit 2 object cap,
                                bit 3 an MD anchor hit off its sensor */
#define LST_COUNT_MAXCAND 5  /* largest candidate count of any stage (required cand cap) */
#define LST_COUNT_T5PRE 6    /* T3 pairs passing the quintuplet's FP32 cuts (bounded by cand cap) */
#define LST_COUNT_LSCAND 7   /* MD pairs the line-segment stage evaluated (after its windows) */
#define LST_COUNTS_LEN 8

#define LST_N_FEATURES 42

typedef struct lst_ctx lst_ctx;

/* Hits, structure of arrays, device pointers, n entries each. Batched calls
 * concatenate events; x, y, z in cm; sensor = 2 * module + (0 anchor sensor,
 * 1 other sensor) in the numbering of the geometry blob. */
typedef struct {
    const float *x, *y, *z;
    const int32_t *sensor;
    int64_t n;
} lst_hits;

/* Capacities that size the workspace; the output arrays of lst_objects must
 * hold at least md / ls / t3 / t5 entries. cand bounds the candidate pairs
 * examined by any one stage (all events of a batch together). */
typedef struct {
    int64_t hits, events, md, ls, t3, t5, cand;
} lst_caps;

/* Output collections (device pointers, caller-owned). Objects are given by
 * index: MD by the input indices of its (anchor, other) hits, LS by its
 * (inner, outer) MD indices, T3 by its (inner, outer) LS indices, T5 by its
 * (inner, outer) T3 indices; for batches all indices are into the batch's
 * concatenated arrays. Order within a collection is deterministic (sorted by
 * event, then by the anchor MD or module) but not otherwise specified. */
typedef struct {
    int32_t *md_hits;            /* [caps.md][2] */
    int32_t *ls_md;              /* [caps.ls][2] */
    int32_t *t3_ls;              /* [caps.t3][2] */
    int32_t *t5_t3;              /* [caps.t5][2] */
    float *t5_score;             /* [caps.t5], NaN in PRE_DNN mode */
    float *t5_chi2_rphi;         /* [caps.t5] */
    float *t5_chi2_rz;           /* [caps.t5] */
    float *t5_feat;              /* optional [caps.t5][42] DNN inputs before standardisation, or NULL */
    int64_t *counts_dev;         /* [LST_COUNTS_LEN] required counts and error bits */
    int64_t n_md, n_ls, n_t3, n_t5;   /* host copies, filled unless LST_ASYNC */
} lst_objects;

typedef struct {
    int32_t mode;                /* LST_MODE_DNN or LST_MODE_PRE_DNN */
    int32_t precision;           /* LST_PREC_F32 or LST_PREC_BF16 (T5-DNN) */
    float score_min;             /* keep T5 with score >= score_min (DNN mode); NaN keeps all */
    int32_t flags;               /* LST_ASYNC */
} lst_options;

/* Create a context on HIP device `device` (the device is made current). */
lst_status lst_create(int device, lst_ctx **out);
void lst_destroy(lst_ctx *ctx);

/* Load the detector geometry and module map ("LSTG" blob v1, host memory,
 * copied): module records (barrel cylinder patches / endcap annulus sectors,
 * two sensors each, Sec. 1 pT-modules), the module map that defines which
 * module pairs are "adjacent" for line segments (Sec. 1), and the selection
 * parameters. Per-module FP32 thresholds are derived here from the FP64
 * parameters. LST_E_INVAL on a malformed blob or more than 524288 modules. */
lst_status lst_load_geometry(lst_ctx *ctx, const void *blob, size_t nbytes);

/* Load the T5-DNN ("LSTM" blob v1, host memory, copied): 42 -> 32 -> 32 -> 1
 * weights (Sec. 2) and the per-feature standardisation. */
lst_status lst_load_model(lst_ctx *ctx, const void *blob, size_t nbytes);

/* Bytes of device workspace a build call with these capacities needs
 * (256-byte aligned base required). */
lst_status lst_workspace_size(const lst_ctx *ctx, const lst_caps *caps, size_t *bytes);

/* Build MD, LS, T3, T5 and T5 scores for ONE event (Table 1 steps 1-4 and the
 * Sec. 2 T5-DNN). Returns LST_E_CAPACITY (after a sync) when any count
 * exceeds its capacity: out->n_* / counts_dev then hold the required counts
 * and the output contents are unspecified. Hits must lie on their sensor
 * (within 2e-3 cm of its surface and extent and 2e-5 rad of its phi range):
 * an MD whose anchor hit does not gives LST_E_INVAL (error bit 3). With
 * LST_ASYNC nothing is checked on the host; read counts_dev after the stream
 * completes. */
lst_status lst_build_objects(lst_ctx *ctx, const lst_hits *hits, const lst_options *opt,
                             const lst_caps *caps, lst_objects *out, void *workspace,
                             size_t ws_bytes, void *stream);

/* lst_build_objects without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc). Scratch is a static array of
 * LST_NOALLOC_SCRATCH_MIB MiB per GPU, allocated with the library's code
 * object and held until the process ends; the call itself allocates nothing.
 * Capacities whose workspace (lst_workspace_size) exceeds that size give
 * LST_E_INVAL with the required size in lst_last_error. All calls on one GPU
 * share its array: calls that overlap on one GPU (any contexts, any streams)
 * race and must be ordered by the caller. Results, errors and LST_ASYNC are
 * as for lst_build_objects. */
#define LST_NOALLOC_SCRATCH_MIB 128
lst_status lst_build_objects_noalloc(lst_ctx *ctx, const lst_hits *hits, const lst_options *opt,
                                     const lst_caps *caps, lst_objects *out, void *stream);

/* Same for a batch of n_events events whose hits are concatenated:
 * event e owns hits [event_offsets_dev[e], event_offsets_dev[e + 1]) (int64,
 * device, n_events + 1 entries, event_offsets_dev[0] = 0, last = hits->n).
 * Objects of all events go to one set of collections, grouped by event; on
 * return event_obj_offsets_dev (int64 device [4][n_events + 1], may be NULL)
 * holds for MD, LS, T3, T5 the first index of each event's objects. Grid
 * shapes depend only on caps, so the call can be captured in a HIP graph. */
lst_status lst_build_objects_batched(lst_ctx *ctx, const lst_hits *hits,
                                     const int64_t *event_offsets_dev, int32_t n_events,
                                     const lst_options *opt, const lst_caps *caps,
                                     lst_objects *out, int64_t *event_obj_offsets_dev,
                                     void *workspace, size_t ws_bytes, void *stream);

/* Score n feature rows with the loaded T5-DNN (Sec. 2): X_dev is [n][42]
 * row-major, FP32 or BF16 (x_dtype), features before standardisation (the
 * model's mu / sd are applied); scores_dev receives n FP32 sigmoid outputs.
 * precision LST_PREC_F32 runs on the vector ALU, LST_PREC_BF16 on MFMA. */
lst_status lst_score(lst_ctx *ctx, const void *X_dev, int32_t x_dtype, int64_t n,
                     float *scores_dev, int32_t precision, void *stream);

/* Track-candidate selection (Sec. 1 and Table 1 steps 5-8) with duplicate
 * removal (named in Sec. 2), on the objects of a completed build and a list of
 * pixel seeds (pLS, Table 1 step 0; inputs here, from an upstream iteration).
 * The paper gives the steps in words only; the library's rules:
 *  - every T5 and T3 gets helix parameters (kappa = signed half-curvature with
 *    the sign of A x E, phi0 = direction at the beam line, cot(theta), z0)
 *    from its first (A) and last (E) MD anchor hits on a circle through the
 *    beam line, in FP64;
 *  - seed p and object o match when chi2 = sum over the four parameters of
 *    (p_i - o_i)^2 / (sigma_p,i^2 + sigma_o,i^2) <= chi2_max (phi0 difference
 *    wrapped to (-pi, pi]; object widths from the options, sigma_kappa,o =
 *    sigma_kappa_rel |kappa_o| + sigma_kappa_abs);
 *  - kind 0 pT5: seed and T5 that are each other's best match (smallest chi2
 *    rounded to FP32, ties to the smaller index); kind 1 T5: the other T5s;
 *    kind 2 pT3: the same mutual best match between the seeds left and the T3s
 *    that are not one of the two T3s of a pT5's T5; kind 3 pLS: the seeds left;
 *  - duplicate removal: two TCs with outer-tracker MDs (pT5 / T5: the T5's 5,
 *    pT3: the T3's 3) are duplicates when they share more than half of the
 *    smaller one's MDs; a TC is removed when it has a duplicate of higher
 *    priority: kind (0 < 1 < 2), then quality (T5: higher score, or lower
 *    r-phi chi2 when the score is NaN; pT3: lower match chi2 as FP32), then
 *    the smaller object index. pLS TCs are never removed.
 * Seeds: params device [n][8] FP32 = kappa (1/cm), phi0 (rad), cot(theta),
 * z0 (cm), then their sigmas in the same order; event_off device int64
 * [n_events + 1] seed ranges per event (event_off[0] = 0, last = n). */
typedef struct {
    const float *params;
    const int64_t *event_off;
    int64_t n;
} lst_seeds;

typedef struct {
    float chi2_max;                       /* match threshold, > 0 */
    float sigma_kappa_abs, sigma_kappa_rel, sigma_phi0, sigma_cot, sigma_z0;   /* object widths, >= 0 */
} lst_tc_options;

/* Selected TCs (device arrays of cap entries, caller-owned), in order: pT5 by
 * T5 index, T5 by T5 index, pT3 by T3 index, pLS by seed index; object and
 * seed indices as in the objects / seeds given. counts_dev (device, 8
 * entries): kept TCs of kind 0..3, kept in total, TCs before duplicate
 * removal. n is filled on return. */
typedef struct {
    int32_t *kind;
    int32_t *seed;                        /* seed index, -1 for kind 1 */
    int32_t *obj;                         /* T5 (kinds 0, 1) or T3 (kind 2) index, -1 for kind 3 */
    int64_t *counts_dev;
    int64_t cap;
    int64_t n;
} lst_tcs;

/* Workspace bytes of lst_select_tcs for these object and seed counts
 * (256-byte aligned base required). */
lst_status lst_tc_workspace_size(const lst_ctx *ctx, const lst_objects *objects, int64_t n_seeds,
                                 int32_t n_events, size_t *bytes);

/* Select TCs. hits: the build's input hits (device); objects: its outputs with
 * the host counts n_md .. n_t5 filled (a synchronous build); event_obj_offsets:
 * the batched build's device [4][n_events + 1] offsets, or NULL when
 * n_events = 1. Synchronises the stream. LST_E_CAPACITY when more TCs are kept
 * than out->cap (out->n then holds the number needed); LST_E_INVAL on a bad
 * argument. */
lst_status lst_select_tcs(lst_ctx *ctx, const lst_hits *hits, const lst_objects *objects,
                          const int64_t *event_obj_offsets_dev, int32_t n_events, const lst_seeds *seeds,
                          const lst_tc_options *opt, lst_tcs *out, void *workspace, size_t ws_bytes,
                          void *stream);

/* Stage timing for measurement: while enabled, every build records HIP
 * events on its stream around the pipeline's stages (also when the build is
 * captured into a HIP graph). lst_stage_times then returns, for the most
 * recent completed build, n <= 10 durations in ms: 0 whole build, 1 hit
 * binning, 2 MD, 3 LS, 4 T3 (2-4: each stage's candidate-evaluation kernel
 * alone), 5 T5 compaction kernels, 6 T5 features + DNN scoring, 7 MD, 8 LS,
 * 9 T3 (7-9: the whole stage, through the CSR offsets the next stage
 * reads). The caller synchronises the stream first; LST_E_STATE if timing
 * was never enabled. */
lst_status lst_set_timing(lst_ctx *ctx, int32_t enable);

/* Failure injection, for testing how callers handle a failed build (no paper
 * passage: the paper describes no error handling). With stage k in 1..6
 * (1 hit binning, 2 MD, 3 LS, 4 T3, 5 T5, 6 T5-DNN scoring), every build call
 * on ctx enqueues only the stages before k, synchronises its stream and
 * returns LST_E_HIP with the stage in lst_last_error; outputs and counts are
 * then undefined, and the context stays usable. 0 turns it off. The
 * environment variable LST_FAIL_AT_STAGE=k sets it for every context created
 * afterwards. LST_E_INVAL for k outside [0, 6]. */
lst_status lst_set_fail_stage(lst_ctx *ctx, int32_t stage);
lst_status lst_stage_times(lst_ctx *ctx, float *ms, int32_t n);

/* Edge classifier on a graph of LST objects (the GNN proposed in Sec. 4:
 * nodes are lower-level objects, e.g. line segments, and edges the
 * higher-level objects joining two of them, e.g. triplets). The paper gives no
 * architecture; the library runs an interaction network: node encoder
 * 7 -> 64 -> 64, edge init 128 -> 64, two message-passing steps (residual edge
 * update 192 -> 64 -> 64 on [h_src, h_dst, e]; sum of the states of the edges
 * entering each node; residual node update 128 -> 64 -> 64 on [h, m]), and an
 * edge head 64 -> 32 -> 1 with a sigmoid; ReLU on every hidden layer. Dense
 * layers use BF16 MFMA with FP32 accumulation; states are FP32.
 * lst_load_gnn takes the "LSTE" blob v1 (host memory, copied): header
 * {"LSTE", 1, 7, 64, 32, 2} then, per layer in the order enc1, enc2, einit,
 * then per step edge_a, edge_b, node_a, node_b, then head1, head2, an FP32
 * weight [out][in] followed by its bias [out]. LST_E_INVAL on any other shape. */
lst_status lst_load_gnn(lst_ctx *ctx, const void *blob, size_t nbytes);

/* Device workspace bytes for a graph of this size (256-byte aligned base). */
lst_status lst_gnn_workspace_size(const lst_ctx *ctx, int64_t n_nodes, int64_t n_edges, size_t *bytes);

/* Score every edge: x_dev [n_nodes][7] FP32 node features, src_dev / dst_dev
 * int32 [n_edges] node ids with dst_dev sorted ascending (edges entering a
 * node are contiguous), scores_dev FP32 [n_edges] receives the sigmoid
 * outputs. All device pointers, caller-owned. Unless flags has LST_ASYNC the
 * call synchronises and returns LST_E_INVAL if an id is out of range or dst
 * is not sorted (scores are then unspecified; the kernels never access memory
 * outside the arrays). */
lst_status lst_gnn_score(lst_ctx *ctx, const float *x_dev, int64_t n_nodes, const int32_t *src_dev,
                         const int32_t *dst_dev, int64_t n_edges, float *scores_dev, void *workspace,
                         size_t ws_bytes, int32_t flags, void *stream);

/* The graph Sec. 4 proposes building with LST: MDs as nodes, LSs as edges.
 * From a completed build (host counts filled): features_dev [n_md][7] FP32
 * per MD, all local to it: r_A / 100, phi_A / pi, z_A / 100 (anchor hit A,
 * cm), 10 alpha (angle from the radial direction at the chord midpoint to the
 * chord towards the other hit, transverse plane), asinh(dz / dr) of the chord
 * clipped to [-5, 5], is_endcap, layer / 11; src_dev / dst_dev int32 [n_ls]:
 * LS (inner a, outer b) as the edge b -> a, so dst is sorted ascending as
 * lst_gnn_score requires. The paper fixes no features; these are the
 * library's. Asynchronous on `stream`; LST_E_STATE without a geometry. */
lst_status lst_md_graph(lst_ctx *ctx, const lst_hits *hits, const lst_objects *objects, float *features_dev,
                        int32_t *src_dev, int32_t *dst_dev, void *stream);

/* Track candidates read off the classified graph (Sec. 4: a GNN on the
 * LST-built graph "to produce TCs"; the paper gives no rule, the library's
 * is): the connected components of the edges with score >= threshold,
 * labels_dev [n_nodes] = the smallest node index of each node's component;
 * *n_tc_dev (device int64) = the number of components with at least min_mds
 * nodes. Synchronises; LST_E_INVAL when an edge's node id is out of range
 * (such edges are skipped, the rest is still labelled). */
lst_status lst_graph_components_workspace_size(const lst_ctx *ctx, int64_t n_nodes, size_t *bytes);
lst_status lst_graph_components(lst_ctx *ctx, int64_t n_nodes, const int32_t *src_dev, const int32_t *dst_dev,
                                const float *scores_dev, int64_t n_edges, float threshold, int32_t min_mds,
                                int32_t *labels_dev, int64_t *n_tc_dev, void *workspace, size_t ws_bytes,
                                void *stream);

/* Launch shapes of the build kernels. They never change results: every stage
 * writes its objects in candidate order whatever the tiling, so a tuning only
 * changes speed (the autotuner in the Python package times them).
 *   bin_split    sensor-id ranges per event in hit binning, each sorted by one
 *                block in LDS (1..256; raised at launch to the number of ranges
 *                of at most 512 sensor ids that cover the geometry);
 *   tile_per[s]  candidates per thread of a 256-thread compaction tile, for
 *                stage s = 0 MD {2,4,8}, 3 T5 FP32 pre-cuts {1,2,4}, 4 T5
 *                FP64 fits {1,2}; entries 1 ({2,4,8}) and 2 ({1,2,4}) are
 *                accepted and have no effect (the line-segment and T3 stages
 *                have no compaction tiles);
 *   eval_blocks  blocks of the compaction kernels (256..8192);
 *   t3_masks     pass masks of 64 candidates the T3 stage keeps per
 *                wavefront of 64 inner LSs (1..8); the T3 of a wavefront
 *                with more candidates are written by a second kernel that
 *                evaluates the candidates beyond them again.
 * Defaults: {4, {4, 8, 2, 2, 1}, 8192, 8}. lst_set_tuning(ctx, NULL) restores
 * them; an unsupported value gives LST_E_INVAL and leaves the tuning as it
 * was. The tuning in force when a build is enqueued (or captured) is used. */
typedef struct {
    int32_t bin_split;
    int32_t tile_per[5];
    int32_t eval_blocks;
    int32_t t3_masks;
} lst_tuning;

lst_status lst_get_tuning(const lst_ctx *ctx, lst_tuning *out);
lst_status lst_set_tuning(lst_ctx *ctx, const lst_tuning *tuning);

const char *lst_status_string(lst_status s);
const char *lst_last_error(const lst_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* LST_H */
