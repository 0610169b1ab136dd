/*
 * rcm.h -- Reverse Cuthill-McKee ordering of a symmetric sparsity pattern on
 * one AMD Instinct MI355X (gfx950), as a C ABI.
 *
 * The operation is the one stated in the paper "The Reverse Cuthill-McKee
 * Algorithm in Distributed-Memory" (Azad, Jacquelin, Buluc, Ng), Section I:
 * for a symmetric matrix A, find a permutation P such that P A P^T has a
 * small bandwidth.  The ordering is computed as in the paper:
 *
 *   - per connected component (Section III-B), taken in increasing order of
 *     the component's lowest vertex id, which is also the start vertex;
 *   - a pseudo-peripheral root found by repeated breadth-first searches
 *     (Algorithm 2; Algorithm 4 gives the same searches in matrix form);
 *   - a level-synchronous labelled BFS (Algorithm 3): each level is expanded
 *     by a sparse-matrix x sparse-vector product over the (select2nd, min)
 *     semiring so every new vertex takes its lowest-labelled parent, then the
 *     new level is ordered by (parent label, degree, vertex id) (SortPerm,
 *     Table I) and labelled consecutively;
 *   - the labels are reversed (last line of Algorithm 1).
 *
 * The search's BFSs of a large component run by default as a
 * label-correcting BFS without a barrier per level (the non-level-
 * synchronous BFS that Section VI leaves as future work; option
 * async_search): its distances, and so the search's result, equal those of
 * the level-synchronous BFS.  Option label_mode selects the other future
 * work of Section VI, labelling each level without the per-level sort.
 *
 * Every tie is broken deterministically, so the permutation is unique:
 * degree = number of off-diagonal entries in the row; "minimum degree"
 * ties go to the lower vertex id; the start vertex of a component is its
 * lowest id.  Bandwidth and envelope size (Section II-A) are reported for
 * the input order and for the result, with 0-based indices and the diagonal
 * treated as present: beta_k = k - min(k, lowest column in row k), bandwidth
 * = max beta_k, profile = sum beta_k (64-bit).
 *
 * Conventions shared by every entry point:
 *   - CSR arrays are DEVICE pointers owned by the caller (int32 rowptr[n+1],
 *     int32 colidx[nnz], nnz = rowptr[n] < 2^31).  Rows need not be sorted;
 *     self loops are allowed and ignored.  A pattern is a set of positions:
 *     a column repeated within a row is malformed and always rejected with
 *     RCM_ERR_BAD_CSR.  The library never frees caller memory and keeps no
 *     state between calls except the parsed tuning table (tuning_file).
 *   - perm_out[k] (device, int32[n]) receives the original vertex placed at
 *     position k (new -> old), so that B = A[perm][:, perm] = P A P^T.
 *   - iperm_out (device, int32[n], optional) receives old -> new.
 *   - stats (HOST pointer, optional) receives the statistics below.
 *   - stream is a hipStream_t passed as void* (NULL = the default stream).
 *     Work is enqueued on it; the call returns after that work completes
 *     (the component schedule and the statistics need small readbacks), so
 *     perm_out, iperm_out and stats are final on return.
 *   - Errors are returned as rcm_status; nothing is thrown across the ABI.
 *     On an error, output arrays may hold partial results.
 */
#ifndef RCM_H_
#define RCM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RCM_OK = 0,
  RCM_ERR_INVALID_ARGUMENT = 1,    /* n < 0, NULL pointer with n > 0, bad option */
  RCM_ERR_BAD_CSR = 2,             /* rowptr[0] != 0, decreasing rowptr, colidx out of
                                      range, or a column repeated within a row     */
  RCM_ERR_NOT_SYMMETRIC = 3,       /* (i,j) present without (j,i): always when a
                                      traversal leaves its component's label block,
                                      exhaustively with check_full                  */
  RCM_ERR_WORKSPACE_TOO_SMALL = 4, /* caller workspace below rcm_workspace_bytes()  */
  RCM_ERR_OUT_OF_MEMORY = 5,       /* internal device allocation failed             */
  RCM_ERR_ABORTED = 6,             /* the caller's abort flag was set, or a
                                      device-side wait exceeded its time limit     */
  RCM_ERR_HIP = 7                  /* a HIP runtime call failed                     */
} rcm_status;

/* Statistics of one ordering (one graph). */
typedef struct {
  int64_t bandwidth_before; /* Section II-A beta(A) of the input order        */
  int64_t profile_before;   /* |Env(A)| of the input order                     */
  int64_t bandwidth_after;  /* beta(P A P^T)                                   */
  int64_t profile_after;    /* |Env(P A P^T)|                                  */
  int64_t edges_traversed;  /* sum over components of (num_bfs + 1) * (directed
                               off-diagonal entries of the component): the
                               entries scanned by every level structure of the
                               pseudo-peripheral search plus the labelled BFS
                               (label_mode 1 and 2 with pp_variant 0: num_bfs
                               times, as no labelled BFS runs)                 */
  int32_t num_components;   /* connected components (isolated vertices count) */
  int32_t pseudo_diameter;  /* max over components of the root's eccentricity */
  int32_t num_bfs;          /* level structures computed by the pseudo-peripheral
                               search (Algorithm 2), summed over components;
                               an isolated vertex counts 2                     */
  int32_t num_levels;       /* levels of the labelled BFS (of the root's level
                               structure with label_mode 1 and 2), summed over
                               components                                    */
} rcm_stats;

/* Options.  Zero-initialised options select every default. */
typedef struct {
  int32_t pp_variant;    /* 0: root = start of the last BFS (Algorithm 2, default)
                            1: root = min-(degree, id) vertex of that BFS's last
                               level (Algorithm 4's return value)              */
  int32_t reverse_mode;  /* 0: reverse each component's label block (default)
                            1: reverse the whole label sequence (Algorithm 1)  */
  int32_t check_full;    /* 1: also check symmetry exhaustively and reject an
                            asymmetric pattern (NOT_SYMMETRIC) before any
                            ordering; costs O(sum over entries of the
                            partner row's length)                              */
  int32_t team_size;     /* work-groups cooperating on one large component;
                            0 = auto (256, one per compute unit, for graphs
                            of at least 2^18 vertices, else 64; 8 in batched
                            calls, 4 for a batch with more large components
                            than 8-wide teams start at once and no graph of
                            2^18 vertices or more); 1..256, capped at the
                            number of work-groups resident at once           */
  int32_t block_threads; /* threads per work-group of the large-component
                            team; 0 = auto (256); 256 or 512                   */
  int32_t small_cutoff;  /* components with at most this many vertices are
                            ordered by a single work-group each, many in
                            parallel, largest first; larger ones by teams of
                            team_size work-groups; 0 = auto (262144; 65536 in
                            batched calls)                                     */
  int32_t narrow_cutoff; /* levels narrower than this are expanded by one
                            work-group of the team without grid-wide barriers;
                            0 = auto (256), -1 = never                         */
  int32_t small_threads; /* threads per work-group of the single-work-group
                            teams; 0 = auto (256); 256 or 512                  */
  int32_t max_teams;     /* most large-component teams run at once; 0 = auto
                            (16; 32 in batched calls), at most 64.  With small
                            components too, half of the resident work-groups
                            are left to them, except in a batch that takes
                            teams of 4 by the auto rule above: there the
                            teams fill every resident work-group and take
                            the small components once the large ones are
                            gone                                              */
  int32_t rebalance_levels; /* wide levels of the level-synchronous passes keep
                            each work-group's share of the frontier in LDS
                            and redistribute it evenly every this many
                            levels; 0 = auto (8), 1 = every level             */
  int32_t label_mode;    /* how each level's vertices are ordered (the
                            alternatives to per-level sorting that Section VI
                            names as future work):
                            0: per-level SortPerm by (parent label, degree,
                               id), Algorithm 3 (default)
                            1: no sort: each level in increasing vertex id,
                               the order the frontier vector holds it in
                            2: one global sort at the end by (level, degree,
                               id), the parent key dropped
                            1 and 2 take the levels from the last level
                            structure of the root search (one more from the
                            returned vertex with pp_variant 1) and skip the
                            labelled BFS; the result is still reversed per
                            reverse_mode.                                      */
  int32_t async_search;  /* level structures of the pseudo-peripheral search
                            of a large component (a team's, at least n/8
                            vertices): 0 = auto (asynchronous), 1 =
                            asynchronous, -1 = level-synchronous.
                            Asynchronous is a label-correcting BFS whose
                            work-groups expand their own frontiers for
                            search_round steps between team barriers
                            instead of meeting once per level (the
                            non-level-synchronous BFS that Section VI leaves
                            as future work).  Same result; a pass whose
                            frontier outgrows its ring falls back to the
                            level-synchronous pass                         */
  int32_t label_team;    /* work-groups of a team that run the labelled BFS
                            (the others sleep meanwhile); 0 = auto (64), at
                            most team_size is used                         */
  int32_t search_round;  /* steps each work-group takes on its own between the
                            team barriers of an asynchronous search pass;
                            0 = auto (16)                                  */
  int32_t mode;          /* 0 = auto: a single graph whose CSR and per-vertex
                               state fit in one work-group's LDS (about 6,000
                               vertices of a 3D mesh, 7,000 of a 2D mesh) is
                               ordered by one work-group from LDS, in one
                               launch; others by the persistent team kernel;
                            1 = always the persistent team kernel;
                            2 = always the one-work-group LDS engine
                               (RCM_ERR_INVALID_ARGUMENT if the graph does
                               not fit, or with label_mode 1 or 2)          */
  int32_t shuffle_seed;  /* 0 = off.  Otherwise a seed that permutes, by seeded
                            bijections, which work-group of a launch plays
                            which team member, the order in which teams and
                            single work-groups take components (and the LDS
                            engine's work-groups their graphs), and delays
                            each work-group by a seeded few microseconds at
                            every team barrier.  The result must not change:
                            the knob exists to shake out order dependences
                            (a race shows up as a different permutation).
                            Slower; for tests                             */
  const char* tuning_file; /* NULL = the RCM_TUNING_FILE environment variable,
                              if set; else no table.  A table written by the
                              autotuner (paper_1610_08128_amd/tune.py) whose
                              entries, chosen by the graph's vertex and entry
                              counts, replace the auto value of every option
                              left at 0 here                               */
  const int32_t* abort_flag; /* NULL = none.  A flag from rcm_abort_flag_create
                              (coherent pinned host memory).  While it is
                              nonzero, a call returns RCM_ERR_ABORTED: before
                              its first launch when already set, else soon
                              after another host thread sets it: the kernels
                              poll it at component boundaries, every 64th
                              team barrier, every 64th level a work-group
                              walks alone, and between the passes of the
                              one-work-group engine (at least every 4096
                              levels), and then end normally.  Any other
                              pointer is RCM_ERR_INVALID_ARGUMENT          */
  int32_t relabel_levels; /* single graphs: when the first level structure of
                             vertex 0's component has at least this many
                             levels (a long mesh), that component is
                             renumbered in the structure's level order and
                             the rest of its ordering runs on the renumbered
                             copy, whose neighbouring levels sit together in
                             memory.  The result is the same (every tie is
                             broken by the caller's ids).  0 = auto (4096),
                             -1 = never.  Uses workspace that the component
                             search needs only later, so graphs with more
                             than 8 entries per vertex are not renumbered;
                             needs the asynchronous search and label_mode 0 */
  int32_t reserved;
} rcm_options;

/* Human-readable name of a status code (static string; any int32 value is
 * accepted).  Library infrastructure: no passage of the paper. */
const char* rcm_status_string(rcm_status s);

/* Fill *opts with the defaults (all zero).  Infrastructure. */
void rcm_default_options(rcm_options* opts);

/* Device workspace needed by rcm_order_ex for a graph with n vertices and
 * nnz entries (bytes, 256-byte aligned start expected; the same for any
 * nnz).  Pure host arithmetic; never fails (returns 0 for n <= 0).  Sizing
 * of this library's state (the per-vertex arrays of the level structures,
 * claims and the Cuthill-McKee order of Algorithms 2 and 3, and a 32-byte
 * copy of each row for graphs whose rows have at most 8 entries). */
size_t rcm_workspace_bytes(int32_t n, int64_t nnz, const rcm_options* opts);

/* Order one graph with default options; internal workspace; no iperm.
 * The operation of Section I (a permutation P so that P A P^T has a small
 * bandwidth), computed per Algorithm 2 (pseudo-peripheral vertex),
 * Algorithm 3 (labelled level-synchronous BFS with SortPerm) and the
 * reversal of Algorithm 1, one component after another (Section III-B);
 * the statistics are Section II-A's bandwidth and envelope.
 * perm_out: device int32[n].  stats: host, nullable. */
rcm_status rcm_order(int32_t n, const int32_t* rowptr, const int32_t* colidx,
                     int32_t* perm_out, rcm_stats* stats, void* stream);

/* Order one graph: rcm_order's operation (Section I; Algorithms 1-3) with
 * the options above (Algorithm 4's pick, the Section VI variants, launch
 * settings).  opts may be NULL (defaults).  workspace: device memory of
 * at least rcm_workspace_bytes(n, nnz, opts) bytes, or NULL to let the
 * library allocate (stream-ordered) and free it within the call. */
rcm_status rcm_order_ex(int32_t n, const int32_t* rowptr, const int32_t* colidx,
                        int32_t* perm_out, int32_t* iperm_out, rcm_stats* stats,
                        const rcm_options* opts, void* workspace, size_t workspace_bytes,
                        void* stream);

/* Size of the device array behind rcm_order_noalloc: graphs whose
 * rcm_workspace_bytes(n, nnz, opts) exceeds it are rejected. */
#define RCM_NOALLOC_SCRATCH_BYTES (256ull << 20)

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc, such as tight serving loops or harnesses that forbid it): the
 * ordering of rcm_order_ex, with a workspace that is a device array of
 * RCM_NOALLOC_SCRATCH_BYTES held by the library (one per device, from its
 * first use until the process ends) instead of caller memory.  Makes no
 * device allocation or free and creates no HIP events (RCM_TIMING is
 * ignored).  Arguments as for rcm_order_ex (opts nullable, iperm_out
 * nullable).  Errors: RCM_ERR_WORKSPACE_TOO_SMALL when the graph needs
 * more workspace than the array holds (about 1.2 million vertices at
 * 7 entries per row); RCM_ERR_HIP when the array's address cannot be
 * obtained.  The calls of one process on one device share the array and
 * are serialised by the library; every call initialises what it uses. */
rcm_status rcm_order_noalloc(int32_t n, const int32_t* rowptr, const int32_t* colidx,
                             int32_t* perm_out, int32_t* iperm_out, rcm_stats* stats,
                             const rcm_options* opts, void* stream);

/* Device workspace needed by rcm_order_batched (bytes): rcm_workspace_bytes
 * of the graphs' disjoint union plus its globalised CSR.  Infrastructure. */
size_t rcm_batched_workspace_bytes(int32_t num_graphs, int64_t total_vertices,
                                   int64_t total_nnz, const rcm_options* opts);

/* Order many independent graphs in one call (each exactly as rcm_order_ex
 * would, per graph): the graphs are ordered as the components of their
 * disjoint union, which Section III-B's one-RCM-per-component rule makes
 * equivalent.
 *   vtx_offsets, nnz_offsets: HOST int64[G+1], prefix sums of the graphs'
 *     vertex counts and entry counts (offsets[0] = 0).
 *   rowptr_cat: device int32, graph g's local rowptr (starting at 0, n_g+1
 *     entries) stored at rowptr_cat[vtx_offsets[g] + g].
 *   colidx_cat: device int32, graph g's local column indices at
 *     colidx_cat[nnz_offsets[g] ...].
 *   perm_cat: device int32[total_vertices]; graph g's permutation (local ids)
 *     at perm_cat[vtx_offsets[g] ...].
 *   stats: host rcm_stats[G], nullable.
 * Totals must stay below 2^31 vertices and entries.  The first invalid graph
 * decides the returned status; on error no graph's output is guaranteed. */
rcm_status rcm_order_batched(int32_t num_graphs, const int64_t* vtx_offsets,
                             const int64_t* nnz_offsets, const int32_t* rowptr_cat,
                             const int32_t* colidx_cat, int32_t* perm_cat, rcm_stats* stats,
                             const rcm_options* opts, void* workspace, size_t workspace_bytes,
                             void* stream);

/* The launch options a tuning table gives a call of num_graphs graphs (1 =
 * a single-graph call) with n vertices and nnz entries in total: every
 * field of *out still at 0 is set from the entry of the call's size class
 * (the exact class, else the nearest of the same kind); other fields are
 * left alone.  mode is taken only from the exact class, and a table's mode 2
 * is not passed on (it asks for what auto does: the one-work-group engine
 * where the graph fits).  This is what rcm_order_ex and rcm_order_batched apply when
 * rcm_options.tuning_file (or RCM_TUNING_FILE) names the table.  A table
 * file is parsed once per path and process.  Errors:
 * RCM_ERR_INVALID_ARGUMENT for a NULL path or out, negative sizes, or a
 * table that cannot be read or holds anything but launch options.
 * Format (text, one line per size class, written by tune.py):
 *   single:n2^<floor log2 n>:d<nnz/n rounded half to even> <option>=<int> ...
 * Launch options: team_size block_threads small_cutoff narrow_cutoff
 * small_threads max_teams rebalance_levels async_search label_team
 * search_round mode relabel_levels. */
rcm_status rcm_tuning_options(const char* path, int32_t num_graphs, int64_t n, int64_t nnz,
                              rcm_options* out);

/* Cancellation (for callers that must stop a long ordering: a serving
 * loop's deadline, an interactive tool).  rcm_abort_flag_create allocates one
 * int32 of coherent pinned host memory on the current device, zeroed, that
 * the GPU reads while a call runs; the caller passes it as
 * rcm_options.abort_flag and sets it (*flag = 1, from any host thread, also
 * while the call runs) to make the call return RCM_ERR_ABORTED, or back to 0
 * to let later calls run.  A call's outputs are unspecified after an abort;
 * its workspace can be reused at once.  Errors: RCM_ERR_INVALID_ARGUMENT for
 * a NULL out, RCM_ERR_HIP when the allocation fails.  rcm_abort_flag_destroy
 * frees it (NULL is ignored); no call may still use it. */
rcm_status rcm_abort_flag_create(int32_t** flag_out);
void rcm_abort_flag_destroy(int32_t* flag);

/* Wall-clock phase timings of the last call made by this host thread, in
 * milliseconds, measured with HIP events on the call's stream when the
 * environment variable RCM_TIMING=1 is set (zero otherwise), and the
 * launch settings that call used. */
typedef struct {
  float validate_ms;     /* CSR checks, degrees, bandwidth/profile before  */
  float components_ms;   /* connected components and the component schedule */
  float order_ms;        /* pseudo-peripheral searches + labelled BFS + reversal */
  float after_ms;        /* bandwidth/profile after and statistics          */
  float total_ms;
  float small_kernel_ms; /* the launch ordering small components, one work-group each */
  float team_kernel_ms;  /* the launch ordering large components with a team */
  float team_pp_ms;      /* device clock of that launch: pseudo-peripheral passes */
  float team_label_ms;   /* device clock of that launch: labelled BFS */
  int32_t team_pp_levels;    /* levels expanded by the pseudo-peripheral passes */
  int32_t team_label_levels; /* levels of the labelled BFS */
  /* The settings the call used (filled whatever RCM_TIMING says): the
     engine (1 persistent team kernel, 2 one-work-group LDS engine, 3 the
     team kernel, which renumbered the graph after its first level
     structure: see relabel_levels, 4 the same renumbering, after which one
     work-group walked the remaining level structures from an LDS window of
     the renumbered ids; RCM_WINDOW=0 keeps that engine out), the
     team size, threads per team work-group (with engine 2: 512 for its
     bounded-row variant, whose rows hold at most 8 off-diagonal entries,
     64 for the general one), labelling sub-team and
     asynchronous round length of the launch with teams (0 if none ran), and
     the small-component cutoff.  Shows what a tuning table changed.      */
  int32_t used_mode;
  int32_t used_team_size;
  int32_t used_block_threads;
  int32_t used_label_team;
  int32_t used_search_round;
  int32_t used_small_cutoff;
  int64_t phase_ticks[28];   /* diagnostics, 100 MHz device clock of work-group 0
                                of the team launch: [0..3] wide unlabelled levels
                                (expand, append, barrier ticks; level count);
                                [4, 5] unlabelled levels of the LDS engine (ticks,
                                count); [6, 7] one-work-group global unlabelled
                                levels; [8, 9] wide labelled levels; [10, 11]
                                labelled levels of the LDS engine; [12..15] wide
                                labelled levels: count phase, first barrier,
                                placement, claims and second barrier; [16..19]
                                unlabelled LDS engine levels: table clearing,
                                expansion, reduction and barrier, bookkeeping;
                                [20..25] asynchronous search passes: rounds,
                                steps, records expanded and records skipped as
                                superseded (work-group 0's), ticks in steps,
                                ticks in round barriers -- or, when the one-
                                work-group LDS engine ordered the graph
                                (mode), its ticks for loading the graph, the
                                row checks, the searches (with a labelled pass
                                that served as one), the labelled passes, the
                                reversal and the result statistics; [26, 27]
                                spare                                          */
} rcm_timings;
/* Copy the calling thread's last timings into *out (NULL is ignored).
 * Diagnostics of this library: no passage of the paper. */
void rcm_last_timings(rcm_timings* out);

#ifdef __cplusplus
}
#endif

#endif /* RCM_H_ */
