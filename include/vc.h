/*
 * vc.h -- C ABI of libvc: exact minimum / parameterized vertex cover on one
 * AMD Instinct MI355X (gfx950).
 *
 * Problem (Sec. II-A of "Faster Vertex Cover Algorithms on GPUs with
 * Component-Aware Parallel Branching"): for a simple undirected graph G,
 *   MVC(G)    = the smallest |C| such that every edge has an endpoint in C;
 *   PVC(G, k) = whether some vertex cover has |C| <= k.
 * Method: component-aware branch-and-reduce (Alg. 2) with the degree-one,
 * degree-two triangle and high-degree rules (Sec. II-B), clique / chordless
 * cycle component rules (Sec. III-D), a component branch registry whose
 * post-processing runs in the last descendant to finish (Sec. III-C),
 * early termination for PVC (Sec. III-E), and the root reduce-then-induce
 * step with narrow degree types (Sec. IV-B, IV-D).  Every step runs in HIP
 * kernels on the device; the host only validates, plans and launches.
 *
 * Conventions for every entry point:
 *   - Return value: VC_OK (0) or a negative vc_status.  On error no output
 *     is written.
 *   - Graphs are borrowed for the duration of the call and never modified.
 *   - Output arrays are owned by the caller and live in host memory.
 *   - A vc_ctx owns all device memory it allocates; it is not thread-safe
 *     (one host thread at a time per context).
 */
#ifndef VC_H
#define VC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    VC_OK = 0,
    VC_EINVAL = -1,      /* malformed graph or argument                      */
    VC_ENOMEM = -2,      /* device memory (or a capacity limit) exhausted    */
    VC_EDEVICE = -3,     /* a HIP call failed                                */
    VC_EAGAIN = -4,      /* a submitted request is still pending              */
    VC_ETIMEDOUT = -5,   /* the search-node limit in vc_opts was reached     */
    VC_ECANCELED = -6,   /* the request was cancelled                        */
    VC_ERANGE = -7       /* a size does not fit the library's limits         */
} vc_status;

/* vc_csr.flags */
#define VC_CSR_DEVICE 1u /* offsets and cols are device pointers (HBM)      */

/*
 * A simple undirected graph in symmetric CSR (Sec. II-A, IV-A):
 *   offsets[n+1] (uint32, offsets[0] = 0, non-decreasing, offsets[n] = nnz)
 *   cols[nnz]    (uint16 when col_bytes == 2, which needs n <= 65536, else
 *                 uint32), both directions of every edge present.
 * Rows need not be sorted.  Self-loops, repeated entries in a row, asymmetric
 * rows and cols >= n are rejected with VC_EINVAL.  nnz must be < 2^32.
 * With VC_CSR_DEVICE both arrays live in device memory of the context's
 * device; otherwise they are host memory.
 */
typedef struct {
    uint32_t n;
    uint64_t nnz;
    const uint32_t *offsets;
    const void *cols;
    uint32_t col_bytes;
    uint32_t flags;
} vc_csr;

/* vc_opts.flags: ablation switches (all off by default) */
#define VC_OPT_NO_COMPONENTS 1u /* never branch on components (Alg. 1)     */
#define VC_OPT_NO_LOAD_BALANCE 2u /* no worklist donation: every child stays
                                     on its worker's own stack              */
#define VC_OPT_VALIDATE_SKIP 4u /* trust the caller: skip the CSR checks     */
#define VC_OPT_NO_GRAPH 8u      /* batches: launch the kernels one by one
                                   instead of replaying a captured hipGraph */
#define VC_OPT_NO_SMALL 16u     /* no register-resident small-node solver   */
#define VC_OPT_NO_INDUCE 32u    /* single solves: no root reduction and no
                                   induced subgraph; the search starts from
                                   the input graph in its own ids (Sec. IV-B
                                   off, Table II)                           */
#define VC_OPT_NO_COMPACT 64u   /* rebuild the live list by a sweep of the
                                   whole degree array after every rule pass
                                   instead of filtering the previous list
                                   (bounding of non-zero entries off,
                                   Table II)                                */
#define VC_OPT_CROWN 128u       /* single solves: run the crown reduction at
                                   the root whatever the size (by default it
                                   runs when the degree rules leave at least
                                   4096 vertices)                           */
#define VC_OPT_NO_CROWN 256u    /* single solves: never run the crown
                                   reduction                                */
#define VC_OPT_STRONG_ORDER 512u /* add agent-scope release fences before
                                   every publication of a node, cover or
                                   registry update and acquire fences after
                                   every consumption, on top of the
                                   coherent accesses and completion waits
                                   the search always uses (all entry
                                   points)                                  */
#define VC_OPT_EAGER_INDUCE 2048u /* the worker that branches on components
                                   induces every component's subgraph at
                                   registration (by default only the one it
                                   continues with; each other component's
                                   subgraph is induced by the worker that
                                   starts it)                               */
#define VC_OPT_NO_ROOT_CACHE 4096u /* single solves: read the root's induced
                                   subgraph from HBM at every node instead
                                   of copying it into a worker's LDS graph
                                   cache when it fits                      */
#define VC_OPT_CHECK_REGISTRY 1024u /* after a search that ran to its end,
                                   read the component branch registry back
                                   and check its end state (Sec. III-C):
                                   every LiveNodes and LiveComps counter at
                                   0 and every entry completed exactly once;
                                   the result is in vc_stats (single solves) */
#define VC_OPT_POISON 8192u     /* testing: fill every device buffer the
                                   context allocates or carves with the byte
                                   0xA7 first (every low flag bit set, every
                                   index out of range), so that a read of
                                   memory no step of the call wrote shows up
                                   (slower; synchronises the device at each
                                   allocation)                              */

/*
 * Tuning knobs.  Zero in any field selects the library default.
 *   workers       persistent search workers (one 64-lane wave each); the
 *                 default is one per compute unit (two for batches), within
 *                 the LDS and HBM budgets.
 *   donate_slack  a worker donates a child to the shared worklist while
 *                 idle workers outnumber queued nodes by more than this.
 *   worklist_cap  worklist capacity in nodes.
 *   registry_cap  component branch registry capacity in entries; when full,
 *                 the search branches on a vertex instead (still exact).
 *   hbm_budget    bytes of device memory the search may use.
 *   node_limit    stop with VC_ETIMEDOUT after this many tree nodes (in a
 *                 batch: per instance, and only that instance stops).
 *   watchdog_ms   a worker that has waited this long for work while work
 *                 is still outstanding stops the search with VC_EDEVICE
 *                 (default 120000).
 *   donate_min    a node with fewer live vertices is never donated (its
 *                 subtree is too small to pay for the move).  A donating
 *                 worker gives away its oldest pending node, so the test
 *                 applies to that node (default 48).
 *   serve_n_max   serving: the largest induced subgraph (vertices after the
 *                 root reduction) a request may leave for the resident
 *                 search (default 4096); larger ones run alone between
 *                 resident launches.
 *   serve_slots   serving: instance slots of one resident launch (default
 *                 4096); when they or its graph arena run out, the resident
 *                 kernel drains and is launched again.
 *   small_max     nodes with at most this many live vertices are solved in
 *                 registers (bit masks, one wave; at most 128).  Default: 64
 *                 for vc_min / vc_param (one tree must split over the
 *                 workers), 128 for batches and served requests (many
 *                 instances keep the workers busy).  VC_OPT_NO_SMALL turns
 *                 it off.
 *   gcache_words  LDS graph cache per worker, in 32-bit words: components
 *                 whose induced subgraph fits are re-induced with local ids,
 *                 and the root's induced subgraph is held there when it fits
 *                 (default: what the LDS share of the workers per CU leaves,
 *                 at most 32K words).
 */
typedef struct {
    uint32_t workers;
    uint32_t donate_slack;
    uint32_t worklist_cap;
    uint32_t registry_cap;
    uint64_t hbm_budget;
    uint64_t node_limit;
    uint32_t flags;
    uint32_t watchdog_ms;
    uint32_t donate_min;
    uint32_t gcache_words;
    uint32_t serve_n_max;
    uint32_t serve_slots;
    uint32_t small_max;
} vc_opts;

/* Statistics of the last completed solve on a context. */
typedef struct {
    uint64_t tree_nodes;         /* search-tree nodes processed (Table III) */
    uint64_t component_branches; /* nodes that branched on components      */
    uint64_t components;         /* component children registered          */
    uint64_t donations;          /* nodes handed to the shared worklist    */
    uint64_t pushes;             /* node slots written to HBM (stacks and
                                    worklist); each is read back once       */
    uint64_t local_views;        /* components re-induced with local ids   */
    uint64_t bytes_nodes;        /* bytes written into node slots in HBM   */
    uint64_t bytes_registry;     /* bytes of registry entries, cover bitmaps
                                    and per-component graphs written        */
    uint64_t cycles[6];          /* shader cycles summed over workers:
                                    fetch, rules, components, vertex branch,
                                    registry completion, idle (Sec. V-D)    */
    uint32_t n_input;            /* vertices of the input graph             */
    uint32_t n_kernel;           /* vertices left after the root reduction  */
    uint64_t nnz_kernel;         /* CSR entries of the induced subgraph     */
    uint32_t forced_root;        /* vertices the root reduction put in C   */
    uint32_t greedy_size;        /* initial bound from the greedy cover     */
    uint32_t max_degree_kernel;  /* maximum degree of the induced subgraph  */
    uint32_t deg_bytes;          /* 1, 2 or 4: degree-array element size    */
    uint32_t workers;            /* search workers launched                 */
    uint32_t root_rounds;        /* rounds of the root reduction            */
    uint32_t slot_bytes;         /* bytes of one search-node slot           */
    uint32_t bitmap_bytes;       /* bytes of one registry cover bitmap      */
    double ms_root;              /* device time: degrees, greedy, reduce    */
    double ms_induce;            /* device time: induce + plan readback     */
    double ms_search;            /* device time: persistent search          */
    double ms_total;             /* wall time of the whole call             */
    uint32_t crown_cover;        /* vertices crowns put in the cover (|H|)  */
    uint32_t crown_removed;      /* vertices crowns removed (|I|)           */
    uint32_t crown_rounds;       /* crowns found at the root                */
    uint64_t stale_reads;        /* worklist reads that saw an older payload
                                    of the slot and read it again            */
    uint32_t reg_entries;        /* registry entries allocated by the search */
    uint32_t reg_checked;        /* 1: the registry end state was checked
                                    (VC_OPT_CHECK_REGISTRY, search complete) */
    uint32_t reg_open;           /* entries found not completed exactly once
                                    or with a counter not back at 0 (0 when
                                    the protocol held)                       */
    uint32_t reg_parents;        /* parent entries (branches on components) */
    uint32_t reg_depth;          /* deepest nesting of branches on components
                                    (1: none inside a component)             */
    uint32_t lists_in_hbm;       /* 1: the induced subgraph was too large for
                                    the workers' lists in LDS, which were
                                    kept in HBM (Sec. IV-A)                  */
    uint64_t bytes_rows;         /* CSR bytes (entries and offsets) read from
                                    HBM-resident views for the rows of the
                                    vertices the search removed             */
    uint32_t comp_hist[8];       /* branches on components by the number of
                                    components registered (Table III): 2,
                                    3-4, 5-8, 9-16, 17-32, 33-64, 65-128,
                                    more                                     */
    uint64_t bytes_views;        /* bytes of component subgraphs (and the
                                    root's) copied from HBM into the
                                    workers' LDS graph caches, each time a
                                    worker switched to another view          */
} vc_stats;

typedef struct vc_ctx vc_ctx;

/*
 * Create a context on HIP device `device`.
 *   stream       a hipStream_t to run on; the caller keeps ownership, and
 *                orders its writes to device inputs before each call on
 *                that stream.  NULL: the library creates its own
 *                non-blocking stream, which before reading device inputs
 *                waits for the legacy default stream (so inputs written on
 *                the default stream, PyTorch's default among them, are
 *                complete).
 *   arena        NULL with arena_bytes == 0: device buffers come from
 *                hipMalloc and grow on demand.  Otherwise caller-owned
 *                device memory of this device (for example a PyTorch uint8
 *                tensor), arena_bytes long, that must outlive the context:
 *                every device buffer of the context is carved from it and
 *                the library allocates no device memory.  The blocking calls
 *                reuse the arena from its start (nothing is kept between
 *                them); a call whose buffers do not fit returns VC_ENOMEM.
 *                Served requests carve from it too, until the next blocking
 *                call.  VC_EINVAL if only one of the two is given or the
 *                pointer is not device memory of `device`.
 *   opts         may be NULL (defaults).
 * Creating the first context on a device also looks up the device address
 * of the library's static scratch used by vc_min_static (no allocation).
 */
vc_status vc_ctx_create(int device, void *stream, void *arena, uint64_t arena_bytes,
                        const vc_opts *opts, vc_ctx **out);

/* Release every device buffer of the context; ctx may be NULL. */
vc_status vc_ctx_destroy(vc_ctx *ctx);

/*
 * Check a CSR graph against the rules stated at vc_csr.  Host arrays are
 * checked exactly on the host and ctx may be NULL; device arrays need a
 * context and are checked by kernels: offsets, ranges, self-loops and
 * repeated entries exactly; symmetry by a 64-bit signed hash sum over the
 * unordered pairs, which vanishes for every symmetric graph (an asymmetric
 * one is accepted only on a hash collision; host input is checked exactly).
 * The same checks run at the start of every solve of a device graph.
 * Returns VC_OK or VC_EINVAL (VC_ERANGE when nnz >= 2^32).
 */
vc_status vc_validate(vc_ctx *ctx, const vc_csr *g);

/*
 * Minimum vertex cover (Alg. 2).  Writes MVC(G) to *size and, if cover is
 * not NULL, one minimum cover (original vertex ids, ascending, capacity n)
 * to cover with its length (== *size) to *cover_len.
 */
vc_status vc_min(vc_ctx *ctx, const vc_csr *g, uint32_t *size,
                 uint32_t *cover, uint32_t *cover_len);

/*
 * vc_min without device memory allocation, for callers that cannot
 * allocate (code between graph captures, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, results and errors as vc_min;
 * every device buffer of the solve is carved from a static 256 MiB scratch
 * array in the library's device code (one per GPU, held until the process
 * ends), and the search plan is fitted to it (fewer workers than vc_min
 * where their stacks would not fit).  Limits: n <= 2^20 and nnz <= 2^24;
 * a larger graph, or one whose buffers or search do not fit the scratch,
 * returns VC_ERANGE.  Calls on one GPU share its scratch: calls that
 * overlap in time (two host threads, or two contexts on one device) race
 * and must not be made.  Everything the solve needs zeroed is cleared by
 * the call itself.  VC_EAGAIN while served requests are in flight.
 */
vc_status vc_min_static(vc_ctx *ctx, const vc_csr *g, uint32_t *size,
                        uint32_t *cover, uint32_t *cover_len);

/*
 * Parameterized vertex cover (Sec. II-B, III-E): *yes = 1 iff MVC(G) <= k.
 * On yes and a non-NULL cover, writes a cover of size <= k (ascending ids)
 * and its length; on no, *cover_len = 0.  The search stops as soon as a
 * cover within k is known.
 */
vc_status vc_param(vc_ctx *ctx, const vc_csr *g, uint32_t k, int *yes,
                   uint32_t *cover, uint32_t *cover_len);

/*
 * Enumeration variant of PVC (described in Sec. III-E, not built in the
 * paper): all minimal vertex covers of size <= k.  Every cover of size <= k
 * contains one of them (a cover is minimal when each of its vertices has a
 * neighbour outside it).  They are enumerated per connected component, each
 * within k minus a lower bound of the other components, and combined on the
 * device.
 *   *count       the number of minimal covers of size <= k (saturates at
 *                UINT64_MAX; exact below it)
 *   covers       (host, capacity max_covers * k) cover t at covers[t * k],
 *                its ids ascending, t < min(*count, max_covers); the order
 *                of the covers is unspecified.  May be NULL when k = 0.
 *   sizes        (host, capacity max_covers) the length of cover t.
 *                May be NULL when max_covers = 0 (count only).
 * A graph without edges has one minimal cover, the empty set.  Limits: every
 * connected component has at most 64 vertices, at most 2^26 covers are
 * listed over all components, and (components + 1) * (k + 1) <= 2^26
 * (VC_ERANGE otherwise); vc_opts.node_limit bounds each component's
 * enumeration (VC_ETIMEDOUT).  VC_EAGAIN while served requests are in
 * flight.
 */
vc_status vc_param_enum(vc_ctx *ctx, const vc_csr *g, uint32_t k, uint64_t max_covers,
                        uint32_t *covers, uint32_t *sizes, uint64_t *count);

/*
 * A batch of independent graphs packed into one offsets buffer and one cols
 * buffer.  Instance i is the CSR (as for vc_csr) with
 *   offsets[offs_base[i] .. offs_base[i] + n[i]]   (offsets[offs_base[i]] = 0,
 *                                                   the last one = nnz[i])
 *   cols[cols_base[i] .. cols_base[i] + nnz[i] - 1] (ids local to instance i)
 * The descriptor arrays (offs_base, cols_base, n, nnz) are host memory; with
 * VC_CSR_DEVICE the packed offsets and cols are device memory, else host.
 * Every instance is checked as vc_validate checks a graph.
 */
typedef struct {
    uint32_t count;
    const uint64_t *offs_base;
    const uint64_t *cols_base;
    const uint32_t *n;
    const uint64_t *nnz;
    const uint32_t *offsets;
    const void *cols;
    uint32_t col_bytes;
    uint32_t flags;
} vc_batch;

/*
 * Minimum vertex cover of every instance of a batch in one persistent
 * search launch (the batched use of Alg. 2): workers claim instances from a
 * device-side cursor and help on any instance through the shared worklist.
 * The launch sequence is captured once as a hipGraph and replayed while the
 * batch geometry and buffers stay the same (VC_OPT_NO_GRAPH: plain
 * launches).  Outputs (host memory):
 *   sizes[count]        MVC of each instance;
 *   inst_status[count]  (may be NULL) VC_OK, or VC_ETIMEDOUT when the
 *                       instance reached vc_opts.node_limit; its size and
 *                       cover are then the best found (an upper bound);
 *   covers, cover_offs  (both NULL, or capacity sum(n) and count+1): the
 *                       cover of instance i, ascending local ids, is
 *                       covers[cover_offs[i] .. cover_offs[i+1]).
 * Returns VC_ETIMEDOUT if an instance stopped at the limit and inst_status
 * is NULL; otherwise per-instance limits are reported only there.
 */
vc_status vc_min_batch(vc_ctx *ctx, const vc_batch *b, uint32_t *sizes,
                       int32_t *inst_status, uint32_t *covers,
                       uint64_t *cover_offs);

/*
 * Parameterized vertex cover of every instance with its own bound k[i]
 * (host array): yes[i] = 1 iff MVC <= k[i].  An instance stops as soon as it
 * has its answer; the others go on.  Covers as in vc_min_batch: a cover of
 * size <= k[i] for a yes, none for a no.  An instance at the node limit has
 * inst_status VC_ETIMEDOUT and yes = 0 (undecided).
 */
vc_status vc_param_batch(vc_ctx *ctx, const vc_batch *b, const uint32_t *k,
                         int *yes, int32_t *inst_status, uint32_t *covers,
                         uint64_t *cover_offs);

/* vc_submit kinds */
#define VC_MIN 0   /* minimum vertex cover                                 */
#define VC_PARAM 1 /* parameterized: is there a cover of size <= k         */

/* The outcome of a served request (vc_poll). */
typedef struct {
    int32_t status;        /* VC_OK, or the request's error status          */
    int32_t kind;          /* VC_MIN or VC_PARAM                            */
    uint32_t size;         /* VC_MIN: MVC; VC_PARAM yes: size of the cover  */
    int32_t yes;           /* VC_PARAM: 1 iff MVC <= k                      */
    uint32_t cover_len;    /* vertices written to the cover array           */
    uint32_t n;            /* vertices of the request's graph               */
    uint64_t tree_nodes;   /* search-tree nodes spent on the request        */
    double ms_queued;      /* submit -> admitted to the resident search     */
    double ms_latency;     /* submit -> result ready                        */
} vc_result;

/*
 * Serving (continuous batching).  vc_submit copies the graph (host or
 * device CSR; a device CSR is read after the work queued before on the
 * context's stream, or on the default stream when the context has its own)
 * and returns at once with a ticket: the caller may free the graph then.  A
 * device graph of more than 256 vertices is copied device to device into a
 * 64 MiB request ring that the server allocates with itself (contexts whose
 * buffers come from hipMalloc); when the ring is full, and for every other
 * graph, the copy goes to host memory.  A server thread of the context admits
 * requests, by HBM footprint (an instance slot and room in the graph arena),
 * into a persistent search launch that works on all admitted requests at
 * once (each request is an instance as in vc_min_batch): idle workers pick
 * new instances up while the others run.  A request of at most 256
 * vertices may be checked on the host (as vc_validate checks a host graph)
 * and admitted as it is, the worker that claims it taking its first bound
 * from the degree rules and a greedy dive: always while a launch runs, and
 * between launches unless the root steps have lately been removing most of
 * the vertices of such requests (then it takes them as a larger request
 * does).  A larger request first runs the root
 * reduction and induce steps on a side stream (checked on the device as
 * vc_validate checks a device graph), between search launches; requests
 * those steps decide never reach the search.  An invalid request is
 * answered with status VC_EINVAL.  Thread-safe: vc_submit, vc_poll and
 * vc_cancel may be called from any thread.  While requests are in flight no
 * other solve may run on the context (VC_EAGAIN).
 *   kind  VC_MIN or VC_PARAM (then k is the bound).
 */
vc_status vc_submit(vc_ctx *ctx, const vc_csr *g, int kind, uint32_t k,
                    uint64_t *ticket);

/*
 * VC_EAGAIN while the request is pending; otherwise fills *out and, if
 * cover is not NULL, the cover (ascending ids, capacity n), returns VC_OK
 * and forgets the ticket.  A cancelled request returns VC_ECANCELED (also
 * forgotten); an unknown ticket VC_EINVAL.
 */
vc_status vc_poll(vc_ctx *ctx, uint64_t ticket, vc_result *out,
                  uint32_t *cover);

/* Cancel a pending request: it is dropped before or during its search. */
vc_status vc_cancel(vc_ctx *ctx, uint64_t ticket);

/* Copy the statistics of the last completed solve. */
vc_status vc_last_stats(vc_ctx *ctx, vc_stats *out);

/* Human-readable name of a status code (static storage). */
const char *vc_status_str(vc_status s);

#ifdef __cplusplus
}
#endif

#endif /* VC_H */
