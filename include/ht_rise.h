/*
 * ht_rise.h - C ABI of the MI355X (gfx950) batch hierarchical Tucker library.
 *
 * The library computes, on one AMD GPU, the batch hierarchical Tucker (batch-HT)
 * representation of a stream of d-way tensors (Aksoy & Gorodetsky, "Incremental
 * Hierarchical Tucker Decomposition", arXiv 2412.16544):
 *
 *   - ht_init_batch   : BHT-l2r on the first batch (Sec. 3.1, Algorithm 1);
 *   - ht_rise_update  : HT-RISE on every later batch (Sec. 3.2, Algorithm 2);
 *   - ht_project      : Step 1 of HT-RISE alone - the latent code of a batch in
 *                       the current cores (Sec. 3.2, Step 1; Problem 1's encoder);
 *   - ht_reconstruct  : root-to-leaves contraction (Eq. htucker_reconstruction),
 *                       the decoder of Problem 1;
 *   - ht_query_ranks  : the HT rank vector R (Sec. 2.3) and accumulated count.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Tensors.  A batch Y is a DEVICE pointer to N samples stored C-order as
 *   [N][n_1]...[n_d]: each sample is contiguous, the batch index is slowest.  This
 *   is the paper's Y in R^{n_1 x ... x n_d x N} (Sec. 1) with the batch mode moved
 *   first, which the paper allows (Sec. 3.1 footnote on the batch position).
 *   Element type is cfg->in_dtype (float32 or float64).
 * Dimension tree.  Balanced binary tree, depth ceil(log2 d), the first half of a
 *   node's modes (ceil(q/2) of them) going to its first successor (Sec. 2.3), unless
 *   cfg->tree_parent gives another binary tree over runs of consecutive modes.
 *   Nodes are numbered layer by layer from the root, left to right; the HT rank
 *   vector R = [r_{1,1}, r_{1,2}, r_{2,1}, ...] (Sec. 2.3) lists the 2d-2 non-root
 *   nodes in that order.
 * Cores.  A leaf core is n_i x r; a transfer core is the (r_a r_b) x r matrix whose
 *   row index is i_a * r_b + i_b (the C-order fold to r_a x r_b x r of Eq.
 *   ht_tucker_core_reshape); the root core is r_{1,1} x r_{1,2} x N_acc (Sec. 3.1).
 * Streams.  hip_stream is a hipStream_t (NULL = the legacy default stream).  All
 *   device work of a call is enqueued on it.  The calls below synchronise that
 *   stream before returning (they need the rank decisions on the host to size
 *   the next launches), so on return every output is ready.
 * Memory.  The caller owns every buffer it passes (Y, ws, out, latent).  All
 *   device state of a handle lives in the caller's workspace ws; the library
 *   never allocates device memory.  The handle itself is a small host object.
 *   One handle is used by one host thread at a time.
 * Errors.  Every entry point returns an ht_status.  Argument errors are detected
 *   before any work is enqueued and leave the handle unchanged.  A device-side
 *   failure inside an update (rank capacity exceeded, a non-finite norm) rolls
 *   the handle back to its state before the call; so does a HIP runtime error
 *   met during an update (HT_EDEVICE), as far as the device still executes the
 *   restoring copies.  ht_last_error() returns a human-readable message for the
 *   calling thread's last failure.
 */
#ifndef HT_RISE_H
#define HT_RISE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ht_state* ht_handle;

typedef enum {
  HT_OK = 0,
  HT_EINVAL = 1,    /* invalid argument (null pointer, size out of range, ...)    */
  HT_ESHAPE = 2,    /* batch size above cfg->max_batch, or accumulation full      */
  HT_ENOMEM = 3,    /* workspace smaller than ht_workspace_bytes() reported       */
  HT_ERANKCAP = 4,  /* a rank decision exceeded cfg->rank_cap (handle rolled back) */
  HT_EDEVICE = 5,   /* no usable gfx950 device, or a HIP runtime error            */
  HT_ENUMERIC = 6   /* NaN or Inf met in a norm (handle rolled back)              */
} ht_status;

/* Precision of the contractions and Gram products.  Eigen solves, rank
 * decisions, re-orthogonalisation, the cores and the root are FP64 in every form.
 *   HT_FP64  every contraction and Gram product on FP64 matrix cores.
 *   HT_FP32  mixed form: in ht_rise_update, contractions of modes with at most 128
 *            rows and their residual Grams on FP32 matrix cores with FP64 partial
 *            sums, FP32 level tensors, and the skip test summed from the explicit
 *            residual energy of each contraction; the first batch (ht_init_batch)
 *            and ht_project run as HT_FP64.  Every decision taken from FP32 data is
 *            certified against an error bound of the FP32 steps (u = 2^-24: a residual
 *            formed in FP32 errs by 2 u sqrt(r+1) ||Y||, each FP32 contraction before
 *            it adds 0.75 u sqrt(r+1) ||Y|| in quadrature, and the rounding of a Gram
 *            product moves its tail sums by 4 u trace(G)): the skip test must hold with that margin
 *            around eps ||Y||, and each rank decision on both sides of eps_nw^2.  A
 *            rank decision that fails is taken again from an FP64 residual Gram; a
 *            skip test that fails, or a decision that fails again, runs the whole
 *            call in FP64.  When eps_rel / sqrt(2d-2) is below twice the residual
 *            error the model allows with every node at rank_cap in one chain (the
 *            precision gate, ht_update_precision), the updates run in FP64 from the
 *            start.  ht_update_info.prec_used and .recomputed report what ran.
 *   HT_BF16X3 is rejected (HT_EINVAL): a split-BF16 product carries ~2^-16
 *            relative error, which swamps eps_nw^2 when residuals are formed. */
typedef enum { HT_FP64 = 0, HT_FP32 = 1, HT_BF16X3 = 2 } ht_precision;

/* Element type of Y and of reconstructions. */
typedef enum { HT_F32 = 0, HT_F64 = 1 } ht_dtype;

typedef struct {
  int32_t d;              /* modes per sample, d >= 2                                    */
  const int64_t* n;       /* n[0..d-1] >= 1 mode sizes (copied at init)                  */
  double eps_rel;         /* relative tolerance, 0 < eps_rel < 1 (Alg. 1 and 2 input)    */
  int32_t rank_cap;       /* capacity: maximum rank of any node, >= 1                    */
  int64_t max_batch;      /* capacity: largest N of any single call, >= 1                */
  int64_t n_cap;          /* capacity: largest accumulated sample count N_acc, >= 1      */
  int32_t prec;           /* ht_precision                                                */
  int32_t in_dtype;       /* ht_dtype of Y                                               */
  uint64_t flags;         /* bitwise or of ht_flags (0: none)                            */
  const int32_t* tree_parent; /* NULL: the balanced tree below; else the dimension tree
                             (Sec. 2.3) as 2d-1 parent indices (copied at init):
                             tree_parent[0] = -1 is the root, every other node's parent
                             precedes it, every inner node has two successors (the
                             lower index first), and the nodes are numbered layer by
                             layer, left to right; the leaves, read left to right, are
                             modes 0..d-1, so every node holds a run of consecutive
                             modes.  Any other array is HT_EINVAL.  The rank vector
                             follows this numbering.                                   */
} ht_config;

/* Option bits of ht_config.flags.
 *   HT_ADAPTIVE_BUDGET  App. C's alternative error bound: after each layer (of BHT-l2r
 *                       and of every HT-RISE update) the nodewise tolerance of the
 *                       layers above becomes eps_nw = sqrt(eps_abs^2 - eps_l^2) /
 *                       sqrt(svd_rem), with eps_l^2 = ||Y||^2 - ||C_l||^2 the energy
 *                       the approximation has lost so far (HT_FP32: the energies the
 *                       contractions of the second projection discarded, summed, and
 *                       their error bound taken into the decision certificates),
 *                       eps_abs = eps_rel ||Y|| and svd_rem the non-root nodes of the
 *                       layers still to come.  One extra read-back per layer.
 *   HT_PLAIN_HT_BUDGET  the nodewise tolerance eps_rel ||Y|| / sqrt(2d-3) of the
 *                       leaves-to-root hierarchical Tucker algorithm (Sec. 2.3.1,
 *                       Thm. ht_nodewise_error) instead of sqrt(2d-2).  With N = 1 and
 *                       a batch mode among the modes (cfg->n = (N_samples, n_1..n_d)),
 *                       ht_init_batch then computes the plain HT decomposition with the
 *                       batch as a node of the tree: the two successors of the root
 *                       decide on the same matrix C_1 (one truncated SVD, Eq.
 *                       ht_last_svd), their cores are its left and right singular
 *                       vectors and the root is diag(Sigma_1) up to signs.
 *   HT_ST_HOSVD         the variant of the footnote of Sec. 2.3.1: the nodes of a layer
 *                       are truncated one after the other, left to right, each on the
 *                       level tensor its predecessors in the layer have already
 *                       contracted (sequentially truncated HOSVD), in BHT-l2r and in
 *                       each HT-RISE update; one eigen launch and read-back per node. */
typedef enum { HT_ADAPTIVE_BUDGET = 1, HT_PLAIN_HT_BUDGET = 2, HT_ST_HOSVD = 4 } ht_flags;

typedef struct {
  int32_t skipped;        /* 1 when the batch was represented well enough (Alg. 2 skip) */
  int32_t rank_growth;    /* sum over nodes of the ranks added by this call              */
  double norm_y;          /* ||Y||_F                                                     */
  double eps_proj;        /* sqrt(max(0, ||Y||^2 - ||C_1||^2)) before the update (HT_FP32:
                             sqrt of the summed residual energies of the projection)    */
  double eps_des;         /* eps_rel * ||Y||_F                                            */
  float device_ms;        /* device time of the call, from HIP events on hip_stream       */
  int32_t status;         /* ht_status of this handle's update (HT_OK, or why it was
                             rolled back; ht_rise_update_many reports one per handle)   */
  int32_t prec_used;      /* ht_precision of the contractions and Gram products that
                             produced the committed result (HT_FP64 when an HT_FP32
                             handle's call ran in FP64, see ht_precision)               */
  int32_t recomputed;     /* HT_FP32: decisions taken from FP64 residual Grams because
                             an FP32 result could not be certified or its kept vectors
                             would not be accurate enough (a node's Gram, taken in FP64
                             directly when the skip test's energies already show it, or
                             again; the whole call in FP64 counts one); 0 otherwise     */
} ht_update_info;

/* Bytes of device workspace a handle with this configuration needs.  Host only.
 * Returns HT_EINVAL for an invalid configuration. */
ht_status ht_workspace_bytes(const ht_config* cfg, size_t* bytes);

/* Precision in which the HT-RISE updates of a handle with this configuration run:
 * cfg->prec, except HT_FP64 for an HT_FP32 configuration whose eps_rel the precision
 * gate (see ht_precision) rules out for FP32.  Host only. */
ht_status ht_update_precision(const ht_config* cfg, int32_t* prec);

/* BHT-l2r (Sec. 3.1, Algorithm 1) on the first batch Y (N samples).
 * Creates *out, whose device state lives in ws (ws_bytes >= ht_workspace_bytes,
 * 256-byte aligned).  eps_nw = eps_rel ||Y|| / sqrt(2d-2); every node keeps the
 * minimal rank r >= 1 whose discarded energy is <= eps_nw^2.  ||Y|| = 0 is
 * HT_EINVAL.  info may be NULL. */
ht_status ht_init_batch(const ht_config* cfg, void* ws, size_t ws_bytes, const void* Y, int64_t N,
                        void* hip_stream, ht_handle* out, ht_update_info* info);

/* HT-RISE (Sec. 3.2, Algorithm 2) with batch Y of N samples: project (Step 1),
 * skip when sqrt(||Y||^2 - ||C_1||^2) <= eps_rel ||Y|| (Eq. relative_error_threshold),
 * else per layer from the leaves: residual (Eq. compute_residual), truncated
 * eigen-decomposition of its Gram (Eq. svd_on_residual), expansion of the bases
 * (Eq. concatenating_orthonormal_vectors), zero padding of the parents
 * (Eq. incremental_zero_padding1), projection onto the updated cores; finally the
 * root grows by the N new latent slices (Eq. incremental_root_concatenate).
 * info may be NULL. */
ht_status ht_rise_update(ht_handle h, const void* Y, int64_t N, void* hip_stream, ht_update_info* info);

/* HT-RISE on count independent handles at once (each with its own configuration,
 * tree and workspace), all on hip_stream: handle i takes batch Ys[i] of Ns[i]
 * samples, exactly as ht_rise_update would.  The handles advance in lock step:
 * every projection (Step 1) is launched before one read-back of all skip tests,
 * and then, layer by layer from the leaves (trees of different depths aligned at
 * their leaves), the Gram products of every updating handle precede one shared
 * eigen launch (one workgroup per node of every handle) and one read-back of the
 * decisions, so a call costs a few host round trips instead of a few per handle.
 * infos (may be NULL) receives one entry per handle; device_ms is the time of the
 * whole call.  Argument errors are returned before any work, leaving every handle
 * unchanged.  A handle whose update fails (HT_ERANKCAP, HT_ENUMERIC) is rolled
 * back alone, its infos[i].status says why, the others commit, and the call
 * returns the first failing handle's status.  A HIP runtime error during the call
 * rolls every handle back and returns HT_EDEVICE.  A handle may appear once. */
ht_status ht_rise_update_many(ht_handle* hs, const void* const* Ys, const int64_t* Ns, int32_t count,
                              void* hip_stream, ht_update_info* infos);

/* Latent codes of a batch in the current cores, without changing the handle:
 * latent is a device buffer of N * r_{1,1} * r_{1,2} float64, C-order [N][r11][r12]. */
ht_status ht_project(ht_handle h, const void* Y, int64_t N, void* latent, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops): ht_project without the handle's workspace buffers.  The
 * intermediate level tensors of the projection chain live in a static device array
 * of 256 MiB that the library holds on every GPU it runs on until the process ends;
 * the batch is projected in chunks of as many samples as fit.  No device memory is
 * allocated or freed.  Returns HT_ESHAPE, before any work, when one sample's chain
 * (its two largest alternating intermediates, FP64) needs more than 256 MiB.  Every
 * call on a GPU shares that GPU's array: calls that overlap on one GPU (different
 * streams or threads) race and must be serialised by the caller.  Same arguments,
 * layout and result as ht_project. */
ht_status ht_project_static(ht_handle h, const void* Y, int64_t N, void* latent, void* hip_stream);

/* Reconstruction of accumulated samples [first, first+count) into the device
 * buffer out (count * prod(n) elements of type dtype, C-order [count][n_1]...[n_d]). */
ht_status ht_reconstruct(ht_handle h, int64_t first, int64_t count, void* out, int32_t dtype,
                         void* hip_stream);

/* The decoder of Problem 1: the tensors of N latent codes (device, float64, C-order
 * [N][r_{1,1}][r_{1,2}], as ht_project writes them) contracted root-to-leaves with
 * the current cores (Eq. htucker_reconstruction) into the device buffer out
 * (N * prod(n) elements of type dtype, C-order [N][n_1]...[n_d]). */
ht_status ht_decode(ht_handle h, const double* latent, int64_t N, void* out, int32_t dtype, void* hip_stream);

/* Relative test error of N samples Y (device, cfg->in_dtype, not accumulated): for
 * each sample i, rel_err[i] (host) = ||Y_i - decode(encode(Y_i))||_F / ||Y_i||_F, the
 * summand of the relative test error (Sec. 4.1, Eq. generalization_performance; the
 * RTE is their mean).  The reconstruction is the orthogonal projection of Y_i onto
 * the span of the HT bases, so the error is taken as sqrt(||Y_i||^2 - ||C_i||^2)
 * from the FP64 per-sample norms of the sample and of its latent code C_i, without
 * materialising the reconstruction (the subtraction leaves an absolute error of
 * about 1e-15 / rel_err[i] in rel_err[i]).  Synchronises. */
ht_status ht_rte(ht_handle h, const void* Y, int64_t N, double* rel_err, void* hip_stream);

/* Copies the rank vector R (2d-2 entries, order as above) into ranks[0..cap-1],
 * the entry count into *n_ranks and N_acc into *n_accum (each pointer may be NULL).
 * Host memory; synchronises the handle's last stream.  cap < 2d-2 is HT_EINVAL
 * unless ranks is NULL. */
ht_status ht_query_ranks(ht_handle h, int32_t* ranks, int32_t cap, int32_t* n_ranks, int64_t* n_accum);

/* Test and inspection export of the whole representation as float64 into host
 * memory: for each non-root node in rank-vector order its core matrix
 * (rows x r, column-major), then the root as C-order [N_acc][r11][r12].
 * *needed receives the byte count; host_buf may be NULL to query it.  A buffer
 * shorter than *needed is HT_ENOMEM.  Synchronises. */
ht_status ht_export_cores(ht_handle h, double* host_buf, size_t bytes, size_t* needed);

/* Releases the host handle (the workspace stays the caller's).  NULL is a no-op. */
void ht_destroy(ht_handle h);

/* Static description of a status code. */
const char* ht_status_str(ht_status s);

/* Message of the calling thread's last failed call ("" if none). */
const char* ht_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HT_RISE_H */
