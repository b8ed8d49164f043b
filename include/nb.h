/*
 * nb.h - C ABI of libnbgpu, a gfx950 (MI355X) library for the data-parallel
 * hot path of group-wise Naive Bayes malware detection (Sahay & Chaudhari,
 * "An Efficient Detection of Malware by Naive Bayes Classifier Using GPGPU").
 *
 * Conventions shared by every entry point
 *   - Every function returns an int status: NB_OK (0) or a negative NB_E*
 *     code; nb_last_error() then holds a message for the calling thread.
 *     Nothing throws across this boundary.
 *   - Pointers named x, y, labels, log_post, scores, workspace and model->dev
 *     are DEVICE pointers on the current HIP device; the caller owns all of
 *     them.  Host pointers are named *_host.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Work is enqueued on it and the call returns; outputs are valid once the
 *     stream has completed it.  Argument errors are returned before anything
 *     is enqueued.
 *   - Feature matrices are row-major [n rows (files) x F features] with a row
 *     stride of `ld` ELEMENTS (ld >= F).  The buffer must hold
 *     (n - 1) * ld + F elements.  Features are non-negative occurrence counts
 *     (the paper's per-file opcode occurrences, section 3); scoring does not
 *     re-validate them.
 *   - Alignment of feature matrices (nb_train, nb_score, nb_score_groups,
 *     nb_serve): x must be 4-byte aligned and the row stride ld * element
 *     size a multiple of 4 bytes, since every row is read with dword-aligned
 *     vector loads.  A byte matrix whose F is not a multiple of 4 is passed
 *     with a padded stride (for example the [:, :F] view of an [n, F + 3 & ~3]
 *     buffer; the padding bytes are never read as features); a contiguous
 *     one fails with NB_EINVAL before anything is enqueued.  nb_gather_features
 *     and nb_quantize_fp8 take any stride.
 *   - Class labels: 0 = benign, 1 = malware for the two-class detector;
 *     exact ties are decided for the lowest class index (section 4: malware
 *     only if its posterior is higher, otherwise benign).
 */
#ifndef NB_H
#define NB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
#define NB_OK          0
#define NB_EINVAL     -1  /* bad argument (shape, type, NULL, alpha <= 0, ...)  */
#define NB_EOVERFLOW  -2  /* a count would not fit its exact integer type      */
#define NB_EMINFILES  -3  /* a class has fewer training files than required    */
#define NB_ENOMODEL   -4  /* no group has a trained model to fall back on      */
#define NB_EDATA      -5  /* label outside [0, C), negative feature value, or
                             feature index outside [0, F)                      */
#define NB_ENOMEM     -6  /* workspace or arena too small                       */
#define NB_EHIP       -7  /* a HIP runtime call failed                           */
#define NB_EREJECTED  -8  /* serving: request can never fit the arena           */

/* Naive Bayes variant.  The paper does not name one (section 4); both
 * classical forms over occurrence counts are provided. */
#define NB_MULTINOMIAL 0  /* P(x|c) = prod_f theta_cf^x_f (occurrences)        */
#define NB_BERNOULLI   1  /* P(x|c) = prod_f theta_cf^b_f (1-theta_cf)^(1-b_f), b = x > 0 */
#define NB_GAUSSIAN    2  /* P(x|c) = prod_f N(x_f; mean_cf, var_cf) over the counts */

/* Feature element types. */
#define NB_X_U8   0       /* uint8 counts (clipped at 255 by the producer)       */
#define NB_X_I32  1       /* int32 counts                                         */
#define NB_X_FP8  2       /* OCP FP8-e4m3 (e4m3fn) bytes of quantised counts      */

/* Scoring table precision (accumulation is always FP32). */
#define NB_W_F32  0       /* table rounded once from FP64 to FP32 (plain path)   */
#define NB_W_BF16 1       /* table rounded once from FP64 to BF16                */

/* nb_train flags */
#define NB_TRAIN_ASYNC 1  /* do not synchronise; read the outcome later with
                             nb_model_status() */

const char* nb_version(void);
/* Message for the last error on this thread ("" if none). */
const char* nb_last_error(void);

/* ------------------------------------------------------------------ model
 * A model is a position-independent byte buffer in device memory, owned by
 * the caller (any allocator), of nb_model_bytes(C, F) bytes, 256-byte
 * aligned.  It holds the exact training counts (the model's real state: the
 * tables are a pure function of them), the FP64 table and the FP32/BF16
 * scoring tables.  Offsets of each part are given by nb_model_layout(). */
typedef struct {
  int32_t kind;        /* NB_MULTINOMIAL or NB_BERNOULLI                       */
  int32_t n_classes;   /* C, 2 .. 256                                           */
  int32_t n_features;  /* F, 1 .. 1048576                                       */
  int32_t trained;     /* set to 1 by a successful synchronous nb_train         */
  void*   dev;         /* device buffer of nb_model_bytes(C, F) bytes           */
} nb_model;

typedef struct {
  size_t  total_bytes;
  int32_t padded_features;  /* Fp: F rounded up to a multiple of 1024          */
  int32_t form_rows;        /* P: 1 (two classes: log-odds row) or C            */
  size_t  off_status;       /* int32[4]: status, trained flag, reserved         */
  size_t  off_class_totals; /* int64[C]  N_c: training files per class          */
  size_t  off_class_sums;   /* int64[C]  S_c: sum_f T_cf (multinomial) or N_c   */
  size_t  off_counts;       /* int32[C*F] T_cf (occurrences) or D_cf (presence) */
  size_t  off_log_theta;    /* double[C*F] log theta_cf                          */
  size_t  off_log_1m_theta; /* double[C*F] log(1 - theta_cf) (Bernoulli)        */
  size_t  off_weight;       /* double[C*F] W: scorer weights, s = bias + g(x).W^T */
  size_t  off_bias;         /* double[C]   bias_c (log prior [+ sum log(1-theta)]) */
  size_t  off_form_f32;     /* float[(P+1)*Fp] scoring rows, FP32, zero padded  */
  size_t  off_form_bf16;    /* uint16[(P+1)*Fp] the same rows rounded to BF16   */
  size_t  off_form_bias;    /* float[P+1] biases of the scoring rows            */
  double  alpha;            /* unused by the layout; kept for ABI growth         */
  /* Gaussian models (present in every layout, used by NB_GAUSSIAN only) */
  size_t  off_sumsq;        /* int64[C*F]  Q_cf = sum_{i: y_i = c} x_if^2       */
  size_t  off_mean;         /* double[C*F] mean_cf = T_cf / N_c                  */
  size_t  off_var;          /* double[C*F] var_cf (population) + epsilon         */
  size_t  off_form2_f32;    /* float[(P+1)*Fp] Gaussian: rows c < C hold h_cf    */
  size_t  off_form2_bf16;   /* uint16[(P+1)*Fp] the same rows rounded to BF16    */
  size_t  off_epsilon;      /* double[1] the variance floor epsilon              */
} nb_layout;

/* Bytes of a model buffer; 0 if C or F is out of range. */
size_t nb_model_bytes(int32_t n_classes, int32_t n_features);
/* Fill *out with the model buffer layout for (C, F).
 * The scoring rows restate the weight form without changing posteriors:
 * for C = 2 row 0 is W_1 - W_0 (the log-odds) and the aux row is W_0; for
 * C > 2 row c is W_c - mean_c W and the aux row is the mean.  Every row is
 * computed in FP64 and rounded once. */
int nb_model_layout(int32_t n_classes, int32_t n_features, nb_layout* out);

/* ------------------------------------------------------------------ train
 * Section 4: fit one Naive Bayes model on labelled training files.
 *   N_c  = #{i : y_i = c}                                  (exact, int64)
 *   T_cf = sum_{i: y_i = c} x_if   (multinomial, Gaussian) (exact, int32)
 *   D_cf = #{i : y_i = c, x_if > 0} (Bernoulli)            (exact, int32)
 *   Q_cf = sum_{i: y_i = c} x_if^2  (Gaussian)             (exact, int64)
 *   log prior_c = log N_c - log N   (empirical)
 *   multinomial: log theta_cf = log(T_cf + a) - log(S_c + a F)
 *   Bernoulli:   log theta_cf = log(D_cf + a) - log(N_c + 2a),
 *                log(1-theta) = log(N_c - D_cf + a) - log(N_c + 2a)
 *   Gaussian:    mean = T / N_c, var = (N_c Q - T^2) / N_c^2 + epsilon,
 *                epsilon = 1e-9 x the largest variance of a feature over all
 *                training files (the variance numerators are exact
 *                integers); the density's own form s_c = bias_c +
 *                sum_f h_cf (x_f - mean_cf)^2 with weight h = -1 / (2 var)
 *                and bias = log prior - (1/2) sum_f log(2 pi var); its
 *                scoring rows are the per-class means (off_form_*) and h
 *                (off_form2_*), rounded once, the biases b_1 - b_0 and b_0
 *                for two classes; alpha is not used (any value > 0 is
 *                accepted)
 * in FP64 on the device, then the FP32/BF16 scoring rows (round once).
 * x: [n x F] features (NB_X_U8 or NB_X_I32), y: int32[n] labels.
 * alpha > 0 (Laplace smoothing when 1).  min_files_per_class >= 1: a class
 * with fewer files fails with NB_EMINFILES (the paper's rule uses 6).
 * workspace: device scratch of at least nb_train_workspace_bytes(...) bytes.
 * Errors: NB_EINVAL (arguments), NB_EOVERFLOW (n*255 > INT32_MAX for bytes,
 * or a count above INT32_MAX for int32 features; for a Gaussian model also
 * an int32 feature of 65536 or more, whose squares could overflow the
 * exact sums), NB_EDATA (label outside [0, C), negative feature, or a
 * Gaussian model whose training files are all identical: every variance
 * zero), NB_EMINFILES.  Device-detected errors are
 * reported after the stream is synchronised (the default), or by
 * nb_model_status() with NB_TRAIN_ASYNC. */
size_t nb_train_workspace_bytes(int32_t n_classes, int32_t n_features, int64_t n, int32_t xtype);
int nb_train(nb_model* model, const void* x, int32_t xtype, int64_t n, int64_t ld,
             const int32_t* y, double alpha, int32_t min_files_per_class,
             void* workspace, size_t workspace_bytes, int32_t flags, void* stream);
/* Synchronise `stream` and return the device-side outcome of the last
 * nb_train on this model (NB_OK, NB_EDATA, NB_EOVERFLOW, NB_EMINFILES);
 * sets model->trained accordingly. */
int nb_model_status(nb_model* model, void* stream);

/* ------------------------------------------------------------------ score
 * Section 4: per-file joint log-likelihoods s_c = bias_c + sum_f g(x_f) W_cf
 * (g = identity for multinomial, 1[x > 0] for Bernoulli; the class-constant
 * multinomial coefficient is omitted), the label (highest posterior, ties to
 * the lowest class index) and the log posteriors s_c - logsumexp_c s_c.
 * x: [n x F] features of type xtype; wtype selects the FP32 or BF16 table;
 * accumulation is FP32.  Outputs (device, any may be NULL but not all):
 *   labels int32[n], log_post float[n x C], scores float[n x C] (raw s_c).
 * n == 0 is a no-op.  The per-file summation order depends only on (F, C,
 * xtype, wtype), never on n or on other files.
 * Gaussian models: s_c = bias_c + sum_f h_cf (x_f - mean_cf)^2 (the density's
 * own form: no large terms cancel when a variance is tiny), two classes,
 * uint8 or int32 features, F up to 8192. */
int nb_score(const nb_model* model, const void* x, int32_t xtype, int64_t n, int64_t ld,
             int32_t wtype, int32_t* labels, float* log_post, float* scores, void* stream);

/* ------------------------------------------------------------- features
 * FP8-e4m3 encoding of byte counts: q = RNE_e4m3fn(min(x, 240)).
 * x: uint8 [n x F] (stride ld_x), out: uint8 [n x F] (stride ld_out). */
int nb_quantize_fp8(const uint8_t* x, int64_t n, int32_t n_features, int64_t ld_x,
                    uint8_t* out, int64_t ld_out, void* stream);

/* ------------------------------------------------------ feature selection
 * Section 3: each size group keeps the k opcodes that best separate its
 * malware from its benign files, ranked by the difference of the two
 * classes' normalised occurrences; section 4 trains and classifies each
 * group on those k features.  The normalisation is only cited by the paper;
 * the library's reading, for a trained two-class model with counts T and
 * class sums S (nb_layout: off_counts, off_class_sums, i.e. occurrences and
 * their class total for multinomial models, presence counts and N_c for
 * Bernoulli ones):
 *     d_f = | T_1f / S_1 - T_0f / S_0 |
 * The ranking is exact: d_f S_0 S_1 = |T_1f S_0 - T_0f S_1| is compared as
 * a 128-bit integer (when one class has S_c = 0, d_f is the other class's
 * share, ranked by its T_f).  An exact tie goes to the lower feature index.
 *
 * models: n_models trained two-class models (trained != 0), any kinds and
 * feature counts, 1 <= k <= F of every model.
 * idx: device int32 [n_models x ld_idx], ld_idx >= k: row m receives the k
 * selected feature indices of models[m] in ascending order.
 * Enqueues on `stream` and returns.  Errors: NB_EINVAL. */
int nb_select_features(const nb_model* models, int32_t n_models, int32_t k, int32_t* idx, int64_t ld_idx,
                       void* stream);

/* The model trained on a subset of features, built from a trained model's
 * counts without re-reading its training files: out's counts are the
 * columns idx[0..k) of full's counts (column sums, so equal to counting the
 * gathered training files), its class totals are full's, and its tables
 * follow from these counts exactly as in nb_train with smoothing alpha (so
 * a multinomial S_c is the sum over the k selected columns only).
 * full: trained.  out: its own buffer of nb_model_bytes(C, k), kind and
 * n_classes equal to full's, n_features = k.  idx: device int32[k] with
 * values in [0, F) of full (any order, repeats allowed); an index outside
 * that range is detected on the device and fails with NB_EDATA.
 * workspace: device scratch of nb_model_select_workspace_bytes(C, k) bytes,
 * 8-byte aligned.  Synchronises `stream` and returns the outcome, unless
 * flags holds NB_TRAIN_ASYNC (then nb_model_status() reports it).
 * Errors: NB_EINVAL, NB_ENOMEM, NB_EDATA. */
size_t nb_model_select_workspace_bytes(int32_t n_classes, int32_t k);
int nb_model_select(const nb_model* full, const int32_t* idx, int32_t k, double alpha, nb_model* out,
                    void* workspace, size_t workspace_bytes, int32_t flags, void* stream);

/* The k-feature model widened to the full feature vector: out scores a
 * file's full F-feature row with the same terms as km scores its k selected
 * features (the summation order follows the full width, so sums agree to
 * rounding, not bit for bit) (section 4: each group classifies with its own
 * top-k features), so the
 * scoring kernels read each full row once instead of a gather writing and
 * re-reading the k selected bytes.  out's weights, log tables, counts and
 * scoring rows are km's at the features idx[j] and zero elsewhere; its
 * class totals, class sums and biases are km's (a Bernoulli bias keeps the
 * sum of log(1 - theta) over the selected features only).
 * km: trained, multinomial or Bernoulli, k = km->n_features features.
 * idx: device int32[k], strictly ascending, in [0, n_features) (as
 * nb_select_features writes them); otherwise the call fails with NB_EDATA
 * (device check); read while the call's kernels run (keep it alive until
 * the stream has passed them).  out: kind and n_classes of km,
 * n_features >= k, its own buffer, not overlapping km's.  Synchronises `stream` and returns the outcome unless flags holds
 * NB_TRAIN_ASYNC (then nb_model_status() reports it).
 * Errors: NB_EINVAL, NB_EDATA. */
int nb_model_expand(const nb_model* km, const int32_t* idx, nb_model* out, int32_t flags, void* stream);

/* Gather each file's selected features: out[i][j] = x[i][idx[j]].
 * x: [n x F] elements of xtype (any of NB_X_*; stride ld >= F), idx: device
 * int32[k] (any order, repeats allowed), out: [n x k] of the same type
 * (stride ld_out >= k).  int32 data must be 4-byte aligned.  An index
 * outside [0, F) writes 0 and, when status is not NULL, sets bit 0 of the
 * device word *status (the library never clears it).  n == 0 is a no-op.
 * Errors: NB_EINVAL. */
int nb_gather_features(const void* x, int32_t xtype, int64_t n, int32_t n_features, int64_t ld,
                       const int32_t* idx, int32_t k, void* out, int64_t ld_out, int32_t* status,
                       void* stream);

/* ----------------------------------------------------------- size groups
 * Sections 3-4: group g has a model iff every class has >= min_files
 * training files; an untrained group's files are scored by the next trained
 * group (first trained index above), or, where none is above, the nearest
 * trained group below.  class_counts_host: int64[G x C]; route_host: int32[G]
 * receives the index of the group whose model scores group g.  Host only.
 * Errors: NB_EINVAL, NB_ENOMODEL (no group trained). */
int nb_route_groups(const int64_t* class_counts_host, int32_t n_groups, int32_t n_classes,
                    int32_t min_files, int32_t* route_host);

/* ------------------------------------------------- batched size groups
 * Sections 3-4: the files are split into size groups and each group is
 * classified by its own two-class model (benign / malware); a group without
 * a model is classified with the model of the next group that has one (the
 * first such group after it in `groups`, else the nearest one before it:
 * the rule of nb_route_groups).  Every group of a call is scored by ONE
 * persistent kernel launch over the concatenation of the groups' files;
 * each file's results are bit-identical to nb_score of its group alone
 * (same summation order), whatever the schedule, tile or grid.
 * Schedules: stream (the default when NS x Fp <= 2048 table floats: groups
 * cut into items of a few blocks, taken round-robin in memory order, each
 * wave's loads pipelined across items, the next item's table loaded with
 * them; for byte features of 1,792 to 2,032 per file (a multiple of 8),
 * 8-byte aligned inputs, row strides of at most 17/16 of a row and at most
 * 320 groups, a sweep instead: every wave takes
 * runs of four blocks of the concatenated groups in memory order, each
 * block fetched as one window of whole cache lines into LDS), static ranges
 * (each workgroup scores an equal contiguous run of files, staging a
 * group's table in LDS when its run enters that group), or dynamic items
 * (groups cut into tiles of tile_rows files, taken largest first from a
 * device counter).
 *
 * One group of files (device pointers as for nb_score): */
typedef struct {
  int32_t     model;     /* index into models[], or -1: no model of its own   */
  int32_t     reserved;  /* must be 0                                          */
  const void* x;         /* [n x F] features of the call's xtype, stride ld   */
  int64_t     n;         /* files of the group, >= 0 (0: skipped)             */
  int64_t     ld;        /* row stride in elements, >= F                       */
  int32_t*    labels;    /* int32[n]      or NULL                              */
  float*      log_post;  /* float[n x 2]  or NULL (8-byte aligned)             */
  float*      scores;    /* float[n x 2]  or NULL (8-byte aligned)             */
} nb_group;

/* Requirements: every model a group uses has two classes, and all of them
 * share the kind and the feature count F (the paper keeps k features per
 * group).  Each non-empty group needs at least one output.
 * tile_rows: 0 = the default schedule (stream, else static ranges); > 0 =
 * dynamic items of that many files (rounded up to whole blocks).
 * Errors: NB_EINVAL (arguments, per group), NB_ENOMODEL (every model is -1),
 * NB_ENOMEM (workspace too small), NB_EHIP. */

/* Device workspace for nb_score_groups with these arguments (0 on error). */
size_t nb_score_groups_workspace_bytes(const nb_model* models, int32_t n_models, const nb_group* groups,
                                       int32_t n_groups, int32_t xtype, int32_t wtype, int32_t tile_rows);
/* Build the work list, copy it into `workspace` (256-byte aligned, caller
 * owned) and launch: the list is staged through pinned host memory of the
 * library (allocated on first use, reused once its copy has run), so the
 * call returns once the copy and the launch are enqueued on `stream`.  The
 * workspace and the outputs must stay valid until the stream has passed
 * the launch; use a plan for repeated scoring. */
int nb_score_groups(const nb_model* models, int32_t n_models, const nb_group* groups, int32_t n_groups,
                    int32_t xtype, int32_t wtype, int32_t tile_rows, void* workspace, size_t workspace_bytes,
                    void* stream);

/* nb_score_groups for callers that cannot allocate device memory (code that
 * must not call hipMalloc or a caching allocator, tight serving loops,
 * harnesses that forbid allocation): no workspace argument; the work list
 * goes to a fixed array inside the library, NB_SCORE_GROUPS_STATIC_MAX_BYTES
 * bytes of device memory per device, held from the first call on that
 * device until the process ends.  Arguments, schedules and outputs are those
 * of nb_score_groups (the same kernels: bit-identical results).  A work list
 * larger than the array (nb_score_groups_workspace_bytes() above the
 * maximum) fails with NB_ENOMEM before anything is enqueued.  Allocates no
 * device memory (the work list is built in host memory reused by later
 * calls on the same thread).  Returns after `stream` has completed the
 * launch.  Every call on a device shares that device's array, which keeps
 * the last call's work list: calls that overlap on one device (from several
 * host threads) race and must be serialised by the caller; calls made one
 * after another never overlap.  Errors: those of nb_score_groups. */
#define NB_SCORE_GROUPS_STATIC_MAX_BYTES (4u << 20)
int nb_score_groups_static(const nb_model* models, int32_t n_models, const nb_group* groups, int32_t n_groups,
                           int32_t xtype, int32_t wtype, int32_t tile_rows, void* stream);

/* A plan fixes one grouped call (models, groups, buffers, types) and holds
 * its work list in device memory plus a HIP graph of the launch: each
 * nb_group_plan_launch replays the graph (one kernel node, no memset; the
 * kernel re-arms its own work counter), so new data written into the same
 * input buffers is scored with no host work.  Creation allocates device
 * memory (hipMalloc) and synchronises `stream`; launching allocates nothing.
 * Launches of one plan must not overlap (they share the work counter).
 * Schedule choice (tile_rows == 0): one recorded for the same shape (kept
 * in memory, and in the JSON file named by the NB_TUNE_CACHE environment
 * variable when set), else with NB_PLAN_TUNE the fastest of the stream at
 * several item sizes, static ranges and several dynamic tiles, timed on the
 * caller's data (this scores the groups, writing the outputs, a few
 * times), else the default schedule.
 * tile_rows > 0 fixes dynamic items of that size. */
typedef struct nb_group_plan nb_group_plan;
#define NB_PLAN_TUNE   1
#define NB_PLAN_STATIC 2  /* force static ranges (tile_rows ignored)           */
#define NB_PLAN_STREAM 4  /* force the stream, items of tile_rows files (0: the
                             default size); NB_EINVAL if the table is too big */

#define NB_SCHEDULE_STATIC  0
#define NB_SCHEDULE_DYNAMIC 1
#define NB_SCHEDULE_STREAM  2

typedef struct {
  int32_t tile_rows;       /* files per workgroup run (static) or full item    */
  int32_t n_items;         /* runs (static) or items (stream, dynamic)         */
  int32_t grid;            /* workgroups launched                              */
  int32_t tuned;           /* 0 default or caller's tile, 1 timed, 2 cached    */
  int64_t n_files;         /* files scored per launch                          */
  int32_t rows_per_block;  /* files per wave block of the kernel               */
  int32_t lds_bytes;       /* table bytes staged in LDS per workgroup          */
  int32_t schedule;        /* NB_SCHEDULE_STATIC, _DYNAMIC or _STREAM          */
  int32_t staged;          /* 1: the stream runs as the sweep whose blocks are
                              staged through LDS (two-chunk byte rows), 0 not */
} nb_group_plan_info;

int nb_group_plan_create(const nb_model* models, int32_t n_models, const nb_group* groups, int32_t n_groups,
                         int32_t xtype, int32_t wtype, int32_t tile_rows, int32_t flags, void* stream,
                         nb_group_plan** out);
/* A new step for an existing plan (sections 3-4: each step's files fall into
 * size groups of varying sizes): the same models' kind and feature count,
 * the same requested outputs, at most the plan's number of groups, any group
 * sizes, inputs and outputs.  The new work list (same schedule) is written
 * into the plan through pinned host memory and one copy enqueued on
 * `stream`; the captured graph is not touched (its kernel reads the counts
 * from the work list), so the next nb_group_plan_launch on `stream` scores
 * the new groups.  Returns without waiting for the device, except that a
 * third update waits until the first one's copy has run (two staging
 * buffers).  Launch and update a plan on one stream.  Room: work lists up
 * to four times the payload of the largest list the creation call could
 * make, and at least 1 MiB (65,536 items of the dynamic and stream
 * schedules; the sweep's and static ranges' lists do not grow with the
 * files).  Errors: NB_EINVAL (arguments, more groups than at creation, or
 * groups needing another kernel: another feature count or kind, other
 * outputs, rows that no longer qualify for the plan's row staging),
 * NB_ENOMEM (work list beyond the plan's room), NB_EHIP. */
int nb_group_plan_update(nb_group_plan* plan, const nb_model* models, int32_t n_models, const nb_group* groups,
                         int32_t n_groups, void* stream);
int nb_group_plan_launch(nb_group_plan* plan, void* stream);
int nb_group_plan_query(const nb_group_plan* plan, nb_group_plan_info* out);
/* Waits for the device, then frees the plan (NULL is a no-op). */
int nb_group_plan_destroy(nb_group_plan* plan);

/* ---------------------------------------------------------------- serving
 * Section 4's classifier behind a request queue: scan requests (a batch of
 * files for one resident two-class model) are served by continuous
 * batching.  nb_serve replays a request trace in real time: request i joins
 * the queue arrival_s seconds after the call starts.  Whenever fewer than
 * n_streams batches are in flight, the queue's head requests (arrival
 * order, no overtaking) are admitted while their device footprint fits the
 * arena (first fit; inputs when host resident, labels, log posteriors) and
 * up to max_batch_requests of them form a batch: host-to-device copies, one
 * persistent grouped launch per feature count present (the kernel of
 * nb_score_groups: each request is a group with its own model), device-to-
 * host copies of the outputs, all on one stream of the batch.  A finished
 * batch frees its arena space.  A request whose footprint exceeds the whole
 * arena is rejected (status NB_EREJECTED); the others proceed.  Outputs are
 * identical to nb_score of the request alone.
 * Requests: */
typedef struct {
  int32_t     model;          /* index into models[]                              */
  int32_t     status;         /* out: NB_OK or NB_EREJECTED (or NB_E* on failure) */
  const void* x;              /* [n x F] features of cfg.xtype, rows contiguous;
                                 host memory (pinned, for asynchronous copies),
                                 or device memory with NB_SERVE_DEVICE_INPUTS     */
  int64_t     n;              /* files, >= 1                                      */
  double      arrival_s;      /* seconds after the start of the call, >= 0        */
  int32_t*    labels_host;    /* out: int32[n] (host, pinned) or NULL             */
  float*      log_post_host;  /* out: float[n x 2] (host, pinned) or NULL         */
  double      done_s;         /* out: seconds after the start when the outputs were
                                 observed in host memory (or the rejection)       */
} nb_request;

#define NB_SERVE_DEVICE_INPUTS 1  /* request x pointers are device memory        */
#define NB_SERVE_SIMULATE      2  /* no device work: each batch completes after
                                     sim_batch_s + bytes / sim_bytes_per_s; for
                                     testing the scheduler and for capacity
                                     planning (models need no device buffers)     */

typedef struct {
  void*   arena;              /* device memory, 256-byte aligned, caller owned   */
  size_t  arena_bytes;
  int32_t max_batch_requests; /* >= 1                                             */
  int32_t n_streams;          /* batches in flight, 1 .. 16                       */
  int32_t xtype;              /* feature type of every request                    */
  int32_t wtype;              /* scoring table type                               */
  int32_t flags;              /* NB_SERVE_* flags                                 */
  int32_t reserved;           /* must be 0                                        */
  double  sim_batch_s;        /* NB_SERVE_SIMULATE: fixed time per batch          */
  double  sim_bytes_per_s;    /* NB_SERVE_SIMULATE: feature bytes per second      */
} nb_serve_cfg;

typedef struct {
  double  p50_s, p99_s;       /* latency arrival -> outputs in host memory,       */
  double  mean_s, max_s;      /*   over served requests                           */
  double  makespan_s;         /* first arrival -> last completion                 */
  double  files_per_s;        /* served files / makespan                          */
  double  bytes_per_s;        /* served feature bytes / makespan                  */
  int64_t served, rejected, batches;
  int64_t peak_arena_bytes;   /* largest arena footprint in use at once           */
  int32_t max_in_flight;      /* most batches in flight at once                   */
  int32_t reserved;
} nb_serve_stats;

/* Blocks until every request is served or rejected.  Models: two classes,
 * any mix of feature counts and kinds.  Errors: NB_EINVAL (arguments, checked
 * for every request before the trace starts), NB_EHIP. */
int nb_serve(const nb_model* models, int32_t n_models, nb_request* requests, int64_t n_requests,
             const nb_serve_cfg* cfg, nb_serve_stats* stats);

/* ---------------------------------------------------------------- probe
 * Read-only streaming kernel used to measure achievable HBM bandwidth:
 * reads `bytes` bytes (multiple of 16) at `src` and writes one uint32 per
 * workgroup to sink (>= nb_probe_sink_words() words).  Not part of the
 * method; measurement support. */
int32_t nb_probe_sink_words(void);
int nb_probe_read(const void* src, int64_t bytes, uint32_t* sink, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* NB_H */
