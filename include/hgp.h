/*
 * hgp.h -- C ABI of the MI355X (gfx950) constrained multilevel hypergraph
 * partitioner.
 *
 * The operation is the one of "Hypergraph Partitioning on GPU with Distinct
 * Incident Hyperedges and Size Constraints": given a directed weighted
 * hypergraph G(N, E, omega) (Sec. II-A), find a partitioning rho minimising
 * connectivity (Eq. connectivity) subject to every partition p having
 * size(p) <= Omega and at most Delta distinct inbound h-edges (Sec. II-B),
 * by multilevel coarsening (Sec. V) and refinement (Sec. VI).
 *
 * Conventions shared by every call
 *  - Every call returns hgp_status; HGP_OK is 0.  No call aborts or throws
 *    across this boundary.  After an error, hgp_last_error() returns a
 *    message describing it; the context stays usable (and destroyable).
 *  - Ids are zero-based int32.  Offsets are int64.  Weights are int32 >= 1.
 *  - Inputs are copied; callers keep ownership of every buffer they pass.
 *    Outputs are written into caller buffers of the stated capacity.
 *  - The library owns all device memory it uses.  It allocates through the
 *    allocator in hgp_options (default: hipMallocAsync/hipFreeAsync on the
 *    context's stream).  All work is enqueued on the context's stream; calls
 *    that return host data synchronise that stream before returning.
 *  - One context per stream.  A context is not thread-safe.
 *  - Results are deterministic: the same inputs and options give bit-identical
 *    cluster maps, partitions, pin-count rows and objective on every run.
 */
#ifndef HGP_H_
#define HGP_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum hgp_status {
    HGP_OK = 0,
    HGP_E_INVALID = 1,    /* malformed argument or hypergraph */
    HGP_E_INFEASIBLE = 2, /* a node alone breaks Omega or Delta, or k-way cannot seat a node */
    HGP_E_NOMEM = 3,      /* the allocator returned NULL */
    HGP_E_DEVICE = 4,     /* a HIP runtime call failed */
    HGP_E_STATE = 5,      /* call out of order (e.g. refine before coarsen) */
    HGP_E_UNSUPPORTED = 6 /* input outside a documented implementation limit */
} hgp_status;

typedef enum hgp_mem { HGP_MEM_HOST = 0, HGP_MEM_DEVICE = 1 } hgp_mem;

/* Device allocator: returns a pointer to at least `bytes` bytes of device
 * memory usable in stream order on `stream`, or NULL.  `user` is passed
 * through. */
typedef void* (*hgp_alloc_fn)(size_t bytes, void* stream, void* user);
typedef void (*hgp_free_fn)(void* ptr, size_t bytes, void* stream, void* user);

typedef struct hgp_options {
    int32_t device;        /* HIP device ordinal */
    void* stream;          /* hipStream_t; NULL = the library creates one */
    hgp_alloc_fn alloc;    /* NULL = hipMallocAsync on the stream */
    hgp_free_fn free;      /* NULL = hipFreeAsync on the stream */
    void* alloc_user;
    int32_t pi;            /* candidates per node = matching rounds (Sec. V-D); default 4, 1..8 */
    int32_t theta;         /* refinement repetitions per level (Sec. VI-A); default 16 */
    uint64_t seed;         /* seed of the symmetric histogram noise (Sec. V-C); default 0 */
    int32_t profile;       /* 1 = time every kernel launch with HIP events (see hgp_kernel_stats) */
    int32_t flags;         /* bit 0: use the sparse (hash-table) candidate proposal at every level;
                              by default it serves only levels whose ids need many dense id-range
                              passes while every neighbourhood fits a few hashed passes.
                              bit 1: use the dense (MFMA product) proposal wherever it fits;
                              bit 2: never use it; by default it is chosen per level by an
                              estimate of both proposals' time.
                              bit 3: compute the in-isolation moves of refinement as a dense
                              (MFMA) product wherever it fits; bit 4: never; by default per
                              level by an estimate.  Results are identical in every case.
                              bit 5: ablation without chain rounds (Sec. VII): every move is a
                              chain of its own, sequenced by gain alone (changes results).
                              bit 6: ablation with the prototype's greedy matching (Sec. VII-D)
                              instead of the exact one: every two-cycle of a round's proposal
                              graph is matched, and from the roots down each node left
                              unmatched takes the child proposing to it with the highest
                              score, ties to the larger id (changes results). */
    uint32_t profile_families; /* with profile = 1: bit i times only kernel family i (the order of
                                * hgp_kernel_stats' names); 0 = every family */
    int32_t delta_mode;    /* which h-edges Delta counts for a partition (constraint variants of
                            * Sec. II-B, whose reformulation the paper notes): HGP_DELTA_INBOUND
                            * (default: those with a destination pin in the part), _OUTBOUND (a
                            * source pin) or _INCIDENT (any pin; also undirected inputs).  The
                            * library applies it at load by relabelling pin roles: outbound
                            * swaps sources and destinations, incident makes every pin a
                            * destination.  Connectivity does not depend on roles. */
    int32_t tune[4];       /* tile and schedule choices (0 = default; results never depend on them):
                            * tune[0]: log2 of the hashed proposal's table slots, 10..13 (default 12);
                            * tune[1]: repetitions list the h-edges of their movers (instead of sweeping
                            *          all) while movers * tune[1] < nodes, 1..64 (default 4);
                            * tune[2], tune[3]: 0.  Written by the binding's autotuner (autotune.py). */
} hgp_options;

enum { HGP_DELTA_INBOUND = 0, HGP_DELTA_OUTBOUND = 1, HGP_DELTA_INCIDENT = 2 };

/* Fills `opt` with the defaults above. */
void hgp_default_options(hgp_options* opt);

typedef struct hgp_ctx hgp_ctx;

/* Creates a context on opt->device.  `opt` may be NULL (defaults). */
hgp_status hgp_create(hgp_ctx** out, const hgp_options* opt);

/* Destroys the context and frees its device memory.  NULL is a no-op. */
void hgp_destroy(hgp_ctx* ctx);

/*
 * Frees the device memory of the loaded job: the input hypergraph, the
 * coarsening hierarchy and the partition; with workspace_too != 0 also the
 * scratch buffers that the context otherwise keeps for its next job.  The
 * context stays valid and needs hgp_load_csr before any other call that
 * reads a job.  Returns HGP_E_INVALID for a NULL context.  For callers that
 * keep idle contexts (a pool of workers) and want the memory back between
 * jobs; a context that is loaded again frees the previous job anyway.
 */
hgp_status hgp_release(hgp_ctx* ctx, int32_t workspace_too);

/* Message describing the last error on this context ("" if none). */
const char* hgp_last_error(const hgp_ctx* ctx);

/*
 * Loads hypergraph G(N, E, omega) in the dual compressed layout of Sec. IV-B.
 *   he_off  [E+1] int64: h-edge e owns pins[he_off[e] .. he_off[e+1]); he_off[0] = 0
 *   he_nsrc [E]   int32: |src(e)|; the first he_nsrc[e] pins of e are its sources
 *   pins    [P]   int32: node ids; the source block and the destination block of
 *                        every h-edge are each strictly ascending
 *   hedge_w [E]   int32 >= 1, or NULL for all 1   (omega(e))
 *   node_w  [N]   int32 >= 1, or NULL for all 1   (size(n))
 *   where: whether the five arrays are host or device pointers.
 * Validation (on the device, before anything else runs): N >= 1; E >= 0;
 * every h-edge non-empty and at most 4,096 pins (HGP_E_UNSUPPORTED beyond);
 * 0 <= he_nsrc[e] <= |e|; pins in [0, N); blocks strictly ascending;
 * src(e) ∩ dst(e) = ∅ (Sec. II-A); weights >= 1; sum of h-edge weights and
 * sum of node weights each below 2^31.  Violations give HGP_E_INVALID.
 * Loading replaces any previous hypergraph and discards its hierarchy.
 */
hgp_status hgp_load_csr(hgp_ctx* ctx, int32_t n_nodes, int32_t n_hedges, const int64_t* he_off,
                        const int32_t* he_nsrc, const int32_t* pins, const int32_t* hedge_w,
                        const int32_t* node_w, hgp_mem where);

/*
 * Sets the constraints of Sec. II-B.  omega >= 1 caps the node-weight sum of
 * every partition; delta >= 0 caps its distinct inbound h-edges (pass
 * INT64_MAX for no cap).  k = 0 selects the constrained method: the coarsest
 * clusters are the initial partitions.  k > 0 selects the k-way adapter of
 * Sec. VII-A: coarsening also stops below 4,096 nodes and the coarsest nodes
 * are seated greedily into k parts (largest first, each into the lightest part
 * that keeps both caps); the caller sets omega = (1+eps)*W/k.
 * Returns HGP_E_INFEASIBLE if a single node already exceeds a cap.
 */
hgp_status hgp_set_limits(hgp_ctx* ctx, int64_t omega, int64_t delta, int32_t k);

/*
 * The k-way adapter of Sec. VII-A with the balance parameter eps =
 * eps_num / eps_den: Omega = floor((eps_den + eps_num) * ceil(W / k) /
 * eps_den), W the total node weight, then hgp_set_limits(ctx, Omega, delta,
 * k).  The paper leaves Delta uncapped in this mode; pass INT64_MAX for that,
 * or a cap to keep both constraints.  *omega_out (may be NULL) receives Omega.
 * Errors as hgp_set_limits; k >= 1, eps_num >= 0, eps_den >= 1.
 */
hgp_status hgp_set_kway_limits(hgp_ctx* ctx, int32_t k, int32_t eps_num, int32_t eps_den, int64_t delta,
                               int64_t* omega_out);

/*
 * Coarsening (Sec. III, Sec. V): repeats levels (candidate proposal, Pi
 * matching rounds, isolated pairing, contraction) until the node count reaches
 * ceil(W/Omega), a level merges nothing, or (k > 0) fewer than 4,096 nodes
 * remain.  *n_levels_out receives the number of hypergraphs in the hierarchy
 * (1 = no coarsening happened).
 */
hgp_status hgp_coarsen(hgp_ctx* ctx, int32_t* n_levels_out);

/*
 * Initial partitioning and uncoarsening (Sec. III, Sec. VI): partitions start
 * as the coarsest clusters (or the k-way seating), then every level from the
 * coarsest to the input is refined with theta repetitions after projecting
 * rho through the cluster map.  Requires hgp_coarsen.
 */
hgp_status hgp_refine(hgp_ctx* ctx);

/* Sizes of the hierarchy: out[4*l + {0,1,2,3}] = N, E, P and merged pairs of
 * level l, for l < n_levels (cap >= 4*n_levels). */
hgp_status hgp_get_levels(hgp_ctx* ctx, int64_t* out, int64_t cap);

/* Cluster map gamma of level `level` (Sec. III: each node of G_level to
 * the node of G_(level+1) that its cluster becomes; Sec. V-E), N_level
 * entries.  Coarse ids number the clusters by their smallest member.
 * 0 <= level < n_levels - 1; cap >= N_level. */
hgp_status hgp_get_cluster_map(hgp_ctx* ctx, int32_t level, int32_t* out, int64_t cap);

/* Candidate targets and scores computed while coarsening `level`
 * (N_level * pi entries each, -1 / 0 where fewer candidates exist), and the
 * final matching of that level (N_level entries, -1 = unmatched). */
hgp_status hgp_get_proposal(hgp_ctx* ctx, int32_t level, int32_t* cand, uint64_t* score, int32_t* match,
                            int64_t cap_nodes);

/* Copies level `level`'s hypergraph: he_off [E+1], he_nsrc [E], pins [P],
 * node_w [N]; any pointer may be NULL. */
hgp_status hgp_get_level_graph(hgp_ctx* ctx, int32_t level, int64_t* he_off, int32_t* he_nsrc, int32_t* pins,
                               int32_t* node_w);

/* Current partitioning rho of the input nodes (Sec. II-B: rho(n) is the
 * partition holding n, after uncoarsening and refinement, Sec. III and VI),
 * N entries in [0, *n_parts_out); partitions keep the coarsest level's ids, so
 * some may be empty.  Requires hgp_refine; cap >= N. */
hgp_status hgp_get_partition(hgp_ctx* ctx, int32_t* rho_out, int64_t cap, int32_t* n_parts_out);

/*
 * Rows of pins(p,e) and pins_in(p,e) (Sec. II-B) for the current partition
 * of the input hypergraph, only partitions with pins(p,e) > 0, ascending p.
 * row_off [E+1]; part/cnt/cnt_in [L].  *needed receives L; with part == NULL
 * or cap < L only *needed is written.
 */
hgp_status hgp_get_phi(hgp_ctx* ctx, int64_t* row_off, int32_t* part, int32_t* cnt, int32_t* cnt_in, int64_t cap,
                       int64_t* needed);

typedef struct hgp_eval {
    int64_t conn;        /* Eq. connectivity */
    int64_t cutnet;      /* Eq. cut-net */
    int64_t max_size;    /* max_p size(p) */
    int64_t max_inbound; /* max_p |{e : pins_in(p,e) > 0}| */
    int64_t violations;  /* partitions breaking Omega or Delta */
    int64_t n_parts;     /* non-empty partitions */
} hgp_eval;

/* Evaluates rho (N int32 in [0, n_parts), host memory; NULL = the current
 * partition) on the input hypergraph with the current limits. */
hgp_status hgp_evaluate(hgp_ctx* ctx, const int32_t* rho, int32_t n_parts, hgp_eval* out);

/*
 * hgp_evaluate for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc).
 * rho: N int32 in [0, n_parts) in DEVICE memory, read on the context's stream
 * (the caller orders its writes before the call); out: host struct.  Same
 * results as hgp_evaluate.  Calls no allocator: the pins(p,e) rows,
 * partition sizes, D(p) and the results live in one static device workspace
 * of 64 MiB per device (set up by hgp_create).  It holds 64 B of results,
 * sizes and D (8 * n_parts B each), lambda (4 * E B) and three row arrays
 * (4 * P B each), each rounded up to 256 B; an input needing more gives
 * HGP_E_UNSUPPORTED with the bytes needed (about 5.5 M pins fit).
 * Entries of rho out of range give HGP_E_INVALID.  Waits for the context's
 * stream twice (range check, results).  Every context on one device shares
 * that workspace and it keeps the last call's contents: calls that overlap on
 * one device (contexts on different streams or host threads) race and must
 * be serialised by the caller.
 */
hgp_status hgp_evaluate_noalloc(hgp_ctx* ctx, const int32_t* rho, int32_t n_parts, hgp_eval* out);

/* One refinement repetition on level 0 for a caller-supplied rho (host, N
 * entries, updated in place) with n_parts partitions; `rep` and theta select
 * the size-aware half (Sec. VI-B).  info[0..3] = moves proposed M, moves
 * applied (k*), applied connectivity gain, chain links.  Optional traces (host
 * buffers, NULL to skip): move_dst / move_gain [N] = every node's in-isolation
 * move (-1 / 0 for none) and gain (Eq. refinement_move_selection); seq /
 * seq_dst [N] = the movers in sequence order and their destinations (Sec.
 * VI-C); gseq [N] = in-sequence gains; prefix_gain [N+1] = C_k and prefix_viol
 * [N+1] = violated partitions V_k after the first k moves (Sec. VI-D).  Of the
 * sequence arrays the first M (M+1) entries are written.  Exposes a single step
 * of hgp_refine for step-level checks. */
hgp_status hgp_refine_rep(hgp_ctx* ctx, int32_t* rho, int32_t n_parts, int32_t rep, int64_t* info,
                          int32_t* move_dst, int64_t* move_gain, int32_t* seq, int32_t* seq_dst, int64_t* gseq,
                          int64_t* prefix_gain, int64_t* prefix_viol);

/*
 * Per-kernel timing when opt.profile = 1: for kernel family i (0 <= i <
 * *count), names[i] (static strings), launches[i] and total_ns[i] measured
 * with HIP events around each launch on the context's stream.  Pass NULL
 * arrays to query *count.  hgp_reset_kernel_stats clears the totals.
 */
hgp_status hgp_kernel_stats(hgp_ctx* ctx, const char** names, int64_t* launches, int64_t* total_ns, int32_t* count);
hgp_status hgp_reset_kernel_stats(hgp_ctx* ctx);

/*
 * Work units counted while a family is profiled, in the same family order as
 * hgp_kernel_stats (work[i] for 0 <= i < *count; NULL work queries *count):
 * "gains", the Phi row entries read by the 16-bit gains sweep (sum over nodes
 * n and e in I(n) of lambda(e), per pass; counted on the device);
 * "dense_gemm" and "gains_gemm", the int8 multiply-adds issued by the two
 * dense products (padded sizes); every other family reads 0.
 * hgp_reset_kernel_stats clears them.  Waits for the context's stream.
 */
hgp_status hgp_kernel_work(hgp_ctx* ctx, int64_t* work, int32_t* count);

/*
 * Per-level view of the profiled launches (opt.profile = 1): for level l <
 * *n_levels_out and family f (the order of hgp_kernel_stats),
 * out[3 * (l * count + f) + {0, 1, 2}] = launches, nanoseconds and algorithmic
 * bytes.  Launches belong to coarsening level l (building level l + 1 from
 * level l; loading counts as level 0) or to the refinement of level l.  The
 * bytes are counted by the streaming kernels themselves while profiled (the
 * compulsory reads and writes of what each launch processed: pins, offsets,
 * gathered partition or cluster ids, rows written) for the families phi,
 * part_stats, inseq, contract_edges and pack; other families read 0.  Pass
 * out = NULL to query *n_levels_out; cap >= 3 * levels * count.  Cleared by
 * hgp_reset_kernel_stats.
 */
hgp_status hgp_kernel_level_stats(hgp_ctx* ctx, int64_t* out, int64_t cap, int32_t* n_levels_out);

/* Per-level phase times of the last hgp_coarsen / hgp_refine (HIP events on
 * the context's stream): out[2*l] = coarsen ns of level l, out[2*l+1] =
 * refine ns of level l. */
hgp_status hgp_level_times(hgp_ctx* ctx, int64_t* out, int64_t cap);

/*
 * One partitioning job for hgp_run_jobs.  Inputs are host arrays laid out as
 * for hgp_load_csr (hedge_w / node_w may be NULL for unit weights); the
 * caller owns them and they must stay valid during the call.  Outputs are
 * written by the library.
 */
typedef struct hgp_job {
    int32_t n_nodes;
    int32_t n_hedges;
    const int64_t* he_off;
    const int32_t* he_nsrc;
    const int32_t* pins;
    const int32_t* hedge_w;
    const int32_t* node_w;
    int64_t omega, delta;
    int32_t k;
    double arrival_s;     /* seconds after the call starts at which the job may be admitted */
    int32_t* rho;         /* out (host, n_nodes entries, may be NULL): the partition */
    int32_t n_parts;      /* out: non-empty partitions */
    int32_t n_levels;     /* out: hierarchy levels */
    int64_t conn;         /* out: connectivity of the result (Eq. connectivity) */
    int64_t violations;   /* out: partitions breaking Omega or Delta */
    double start_s;       /* out: admission time, seconds after the call starts */
    double end_s;         /* out: completion time (partition on the host) */
    int64_t footprint;    /* out: the device-memory estimate used for admission, bytes */
    hgp_status status;    /* out: HGP_OK, or the error of the job's first failing call */
    int32_t reruns;       /* out: 1 if the job ran out of device memory beside other jobs and was run
                             again alone (start_s is then its first admission), else 0 */
} hgp_job;

/*
 * Runs n_jobs partitioning jobs (Sec. III: coarsening, initial partitioning,
 * refinement, each job alone) on one GPU with `workers` concurrent contexts,
 * each on a stream of its own (1 = one job at a time).  Jobs must be sorted by
 * arrival_s; they are admitted in that order, each when its arrival time has
 * passed, a worker is free and its footprint estimate fits into hbm_budget
 * bytes beside the jobs in flight (a job larger than the budget runs alone);
 * hbm_budget <= 0 uses 60% of the device's free memory.  opt gives the device,
 * pi, theta, seed and flags; its stream and allocator must be unset (workers
 * allocate stream-ordered from the device's pool).  Returns HGP_E_INVALID for
 * bad arguments and the first context-creation error if any; per-job failures
 * are reported in jobs[i].status.  Results equal those of separate runs.
 */
hgp_status hgp_run_jobs(const hgp_options* opt, hgp_job* jobs, int64_t n_jobs, int32_t workers,
                        int64_t hbm_budget);

#ifdef __cplusplus
}
#endif

#endif /* HGP_H_ */
