/*
 * psc.h -- C ABI of an MI355X (gfx950) executor for application DAGs of data-parallel kernels,
 * after PySchedCL (Ghose et al., "PySchedCL: Leveraging Concurrency in Heterogeneous
 * Data-Parallel Systems").
 *
 * Model (Sec. III): an application is a DAG G = <(K, B), (E_I, E_O, E)> of kernels K that read
 * input buffers and write output buffers; an edge of E makes a producer kernel's output buffer a
 * consumer kernel's input buffer.  An input buffer with no incoming edge is an *isolated write*
 * (copied host -> device, H2D) and an output buffer with no outgoing edge is an *isolated read*
 * (copied device -> host, D2H).  A schedule (Def. 5) maps every kernel with its copies onto
 * in-order queues -- here HIP streams -- so that kernels run in a topological order; the
 * command-queue structure (Def. 4) is the per-stream op lists plus cross-stream precedence pairs,
 * realised with HIP events.  Coarse-grained scheduling uses one stream; fine-grained scheduling
 * uses several, so independent kernels run concurrently and copies overlap compute (Sec. II-A).
 *
 * Calling sequence: psc_dag_create -> psc_add_buffer* -> psc_add_kernel* -> psc_add_edge* ->
 * psc_schedule(policy) -> psc_run* -> psc_sched_destroy -> psc_dag_destroy.
 *
 * Conventions for every function below:
 *  - Return value: PSC_OK (0) on success, a negative psc_status on failure.  No C++ exception
 *    crosses this boundary.  On failure psc_last_error() returns a message describing it.
 *  - Strings are NUL-terminated; the library copies every string it keeps.
 *  - Matrices are row-major.  A buffer has `rows` x `cols` elements of its dtype.  A *view* is a
 *    rows x cols window at (row_off, col_off) of a parent buffer and shares the parent's storage
 *    and leading dimension (the root buffer's `cols`).
 *  - Pointers named *_out / *out are written only on success.
 *  - The DAG and schedule objects are not thread safe: calls on one object must not overlap.
 *  - Only functions marked [GPU] touch the GPU; all others are host-only and work without one.
 */
#ifndef PSC_H
#define PSC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PSC_ABI_VERSION 1

typedef enum psc_status {
  PSC_OK = 0,
  PSC_ERR_ARG = -1,      /* NULL pointer, bad enum, negative size, out-of-range id */
  PSC_ERR_NAME = -2,     /* unknown or duplicate buffer / kernel name */
  PSC_ERR_SHAPE = -3,    /* operand shapes or dtypes do not fit the kernel, or an edge joins
                            buffers that share no storage, or an input is only partly produced */
  PSC_ERR_CYCLE = -4,    /* the edges form a cycle */
  PSC_ERR_RACE = -5,     /* two kernels touch overlapping storage, one writing, without an edge
                            path ordering them; or an input that a kernel produces has no edge */
  PSC_ERR_STATE = -6,    /* call not allowed in the object's current state */
  PSC_ERR_HIP = -7,      /* a HIP runtime call failed (message names it) */
  PSC_ERR_OOM = -8,      /* device or host allocation failed */
  PSC_ERR_UNSUPPORTED = -9,
  PSC_ERR_TIMEOUT = -10, /* a run did not finish within psc_sched_opts.timeout_ms */
  PSC_ERR_IO = -11       /* a file could not be read or written, or its contents are truncated,
                            altered (checksum), malformed or hold non-finite values */
} psc_status;

typedef enum psc_dtype { PSC_F32 = 0, PSC_BF16 = 1 } psc_dtype;

/* Kernel kinds (Sec. V builds each attention head from these; add is the vadd of Sec. II).
 *  PSC_GEMM      inputs {A (M x K), B (K x N)}, output {C (M x N)}: C = alpha * A * B.
 *                A and B share a dtype: F32 runs FP32 matrix-core arithmetic, BF16 runs BF16
 *                matrix-core products with FP32 accumulation.  C is F32 or BF16 (rounded to
 *                nearest even from the FP32 accumulator).
 *  PSC_TRANSPOSE inputs {A (R x C)}, output {B (C x R)}, same dtype: B[j][i] = A[i][j].
 *  PSC_SOFTMAX   inputs {X (R x C)}, output {Y (R x C)}: each row normalised exponential,
 *                max-subtracted, with the max and sum reductions in FP32.
 *  PSC_ADD       inputs {A, B}, output {C}, all of one shape: C = A + B in FP32. */
typedef enum psc_kind { PSC_GEMM = 0, PSC_TRANSPOSE = 1, PSC_SOFTMAX = 2, PSC_ADD = 3 } psc_kind;

/* Coarse: one stream, kernels in breadth-first topological order, each with its isolated
 * writes just before and isolated reads just after it (the enq rules of Sec. III).
 * Fine: n_streams streams, kernels mapped by the mapper below, with event precedences.
 * Device: the precedences are enforced on the GPU at tile granularity: one persistent kernel
 * runs the tiles of every kernel from per-workgroup task lists that the host plans ahead of the
 * run (list scheduling of tiles onto workgroups in one topological order), each workgroup waiting
 * on the completion counters of a task's predecessor kernels.  Uploads and read-backs of
 * page-locked host memory that the device maps at the same address are run by the executor too,
 * as copy tasks on W / 16 (at most 32) workgroups of their own -- the first-needed upload first
 * -- so later layers' inputs arrive while earlier layers compute, each kernel waiting on its
 * inputs' upload counters; other host memory is copied by DMA on one stream before (H2D) and
 * after (D2H) the executor, and device-resident runs use a plan without copy tasks.  Op times of
 * executor-run copies come from the device clock, DMA copies have none.  The grid is sized to the workgroups the GPU holds at once
 * (psc_sched_executor_info), and progress assumes they all become resident: a task may wait for
 * any other workgroup's earlier task.  If other work keeps CUs occupied for longer than a wait's
 * bound (5 s of device time), the waiting workgroups flag the error, every workgroup leaves its
 * list, and psc_run fails with PSC_ERR_HIP instead of hanging.  Its exported structure puts each kernel on its own queue with a wait on every
 * predecessor kernel and on the H2D copies of its inputs, which is what the device enforces.
 * Eager and HEFT: the dynamic coarse-grained baselines of Sec. V (Experiments 2 and 3, after
 * StarPU's policies), run through the scheduling loop of Algorithm 1 (schedule, select, cb):
 * every kernel is its own task component, and each of n_streams streams is one device with one
 * command queue.  At run time the host keeps a ready queue of kernels whose predecessors have all
 * finished, ordered by bottom-level rank (predicted durations from the cost model in the options,
 * else the heuristic), and the set of available streams.  It dispatches the top kernel with its
 * uploads and read-backs to a stream -- eager: the lowest-numbered available one; HEFT: the one
 * with the earliest predicted finish time, waiting if that one is still busy -- followed by a
 * host callback (hipLaunchHostFunc) that, when the stream reaches it, marks the kernel finished,
 * moves newly ready successors into the ready queue and returns the stream, under a lock; the
 * dispatching thread sleeps until a callback arrives.  No two kernels of one DAG edge are ever in
 * flight together, so no device-side precedence is needed (uploads shared between streams are
 * ordered by an event).  psc_sched_export reports the structure of the last run (PSC_ERR_STATE
 * before the first): each kernel waits for its predecessors on other streams, whose completion
 * the host saw before dispatching it.  Not with use_graph, fault_inject_op, timeout_ms,
 * mark_components or PSC_DISPATCH_AQL. */
typedef enum psc_policy {
  PSC_COARSE = 0, PSC_FINE = 1, PSC_DEVICE = 2, PSC_EAGER = 3, PSC_HEFT = 4
} psc_policy;

/* Stream choice of the fine policy.
 *  PSC_MAP_RR         round robin per kernel in breadth-first order from the DAG's roots
 *                     (sel_rr of Sec. IV-B, Algorithm 1) -- the plain heuristic.
 *  PSC_MAP_EFT        list scheduling under the cost model given in the options: kernels by
 *                     descending bottom-level rank (Sec. V, clustering) on predicted durations,
 *                     each on the stream where it can start first (ties: the earliest predicted
 *                     finish with the streams then busy, as HEFT's EFT rule; then the lower
 *                     stream); the stream stays busy for that predicted, contended duration.
 *  PSC_MAP_COMPONENT  every kernel of task component c on stream c mod n_streams. */
typedef enum psc_mapper { PSC_MAP_RR = 0, PSC_MAP_EFT = 1, PSC_MAP_COMPONENT = 2 } psc_mapper;

typedef enum psc_op_type { PSC_OP_H2D = 0, PSC_OP_KERNEL = 1, PSC_OP_D2H = 2 } psc_op_type;

/* How psc_run hands a coarse or fine schedule to the GPU (the command queues and events of
 * Sec. III, Def. 4, and the dispatch step of Algorithm 1).
 *  PSC_DISPATCH_HIP  every stream a HIP stream, every precedence a HIP event record and wait,
 *                    kernels by hipLaunchKernel, copies by hipMemcpyAsync.
 *  PSC_DISPATCH_AQL  every stream that holds a kernel an HSA user-mode queue of the GPU's
 *                    command processor: the host writes one AQL dispatch packet per kernel; every
 *                    op completes a signal, and a cross-stream precedence is a barrier-AND
 *                    packet on the waiting queue (five signals per packet); copies go to the DMA
 *                    engines (hsa_amd_memory_async_copy, with the same signals as dependencies),
 *                    in the order of their stream.  Host memory of psc_host_io must then be
 *                    page-locked (psc_host_alloc); strided copies need 4-byte aligned rows.
 *                    Not with use_graph or fault_inject_op.  The kernels are the same code
 *                    object the HIP path runs (libpsc_kernels.hsaco beside libpsc.so). */
typedef enum psc_dispatch { PSC_DISPATCH_HIP = 0, PSC_DISPATCH_AQL = 1 } psc_dispatch;

/* Kernel classes of a task component (Defs. 1-3 of Sec. III); a kernel may be in FRONT and END. */
typedef enum psc_kclass { PSC_FRONT = 1, PSC_END = 2, PSC_IN = 4 } psc_kclass;

typedef struct psc_dag psc_dag;
typedef struct psc_sched psc_sched;
typedef struct psc_mlp psc_mlp;

typedef struct psc_kernel_params {
  float alpha;          /* GEMM scale; ignored by the other kinds.  Zero-initialised params
                           (or params == NULL) mean alpha = 1. */
  int32_t alpha_set;    /* nonzero: use alpha as given (so alpha = 0 is expressible) */
  int32_t tile;         /* GEMM tile configuration index, -1 or 0 = automatic; for a transpose
                           the tile of the input a block moves: 1 = 64 x 64, 2 = 64 x 128,
                           3 = 128 x 64, 4 = 64 x 256 (rows x columns; 2 to 4 need 16-byte
                           aligned operands, else 1), 0 = automatic (4 for transposes of 256 MiB
                           and more, else 1) */
  int32_t reserved;
} psc_kernel_params;

typedef struct psc_sched_opts {
  int32_t n_streams;    /* number of streams (the paper's command queues per device), 1..64;
                           forced to 1 by PSC_COARSE */
  int32_t mapper;       /* psc_mapper; used by PSC_FINE */
  int32_t copy_stream;  /* 0: copies on their kernel's stream (paper's enq rules);
                           1: every H2D on one extra stream (index n_streams), enqueued before
                              any kernel, so uploads overlap compute; every D2H on a second extra
                              stream (index n_streams + 1, present when the DAG has isolated
                              reads) after an event wait on its producer, so read-backs overlap
                              the kernels that follow on the producer's stream */
  int32_t use_graph;    /* 1: psc_run builds the schedule as one hipGraph -- a node per op, an
                           edge per stream-order or wait precedence -- once (again when the host
                           pointers change) and launches it with hipGraphLaunch */
  int32_t record_ops;   /* 1: psc_run records start/end events around every op (timeline and
                           cost-model samples); incompatible with use_graph */
  int32_t device;       /* HIP device ordinal */
  const psc_mlp *cost;  /* learned cost model for PSC_MAP_EFT; NULL = heuristic model */
  int32_t host_threads; /* host threads that enqueue in psc_run (stream s is enqueued by thread
                           s mod host_threads); 0 = one per stream, 1 = the caller only */
  int32_t mark_components; /* 1: psc_run stamps the device clock before the first op and after
                              every END kernel of each task component (a one-thread marker
                              kernel, also inside the graph), so psc_sched_component_times can
                              report when each component finished -- per-instance latency of a
                              batch.  PSC_DEVICE always keeps per-kernel clocks instead. */
  int32_t fault_inject_op; /* failure-path testing: 0 = off; k > 0 = every psc_run of this schedule
                              treats op k-1 (psc_sched_export's op id = host order) as failed to
                              launch: the ops before it in host order are enqueued eagerly (one
                              host thread, also for a use_graph schedule), psc_run waits for them
                              and returns PSC_ERR_HIP naming op k-1; nothing from op k-1 on runs.
                              The schedule stays usable.  Not for PSC_DEVICE. */
  int32_t timeout_ms;   /* 0 = psc_run waits for the end of the run however long it takes;
                           t > 0 = it waits at most t milliseconds after enqueueing and returns
                           PSC_ERR_TIMEOUT when the run has not finished.  The work stays in
                           flight: the next psc_run of the schedule, and psc_sched_destroy, first
                           wait for it to finish.  Outputs of a timed-out run are unspecified. */
  int32_t dispatch;     /* psc_dispatch (PSC_FINE and PSC_COARSE) */
  int32_t out_of_order; /* 0: every stream is an in-order queue (Def. 4): an op starts after the
                           previous op of its stream has completed.
                           1 (PSC_FINE with PSC_DISPATCH_AQL only): out-of-order queues, as in
                           OpenCL's out-of-order execution mode -- a kernel may start while
                           earlier kernels of its queue still run (AQL dispatch packets without
                           the barrier bit), so one queue runs independent kernels concurrently
                           without more hardware queues.  Every precedence, within a queue too,
                           is then an explicit wait (a barrier-AND packet on the producer's
                           completion signal); each queue's kernels are issued by DAG level
                           (longest path from a root), earlier ops of the mapper's order first
                           within a level, so a wait holds back only kernels of later levels.
                           psc_sched_export lists every direct precedence of each op, and
                           psc_sched_queue_order reports the mode: stream position then orders
                           nothing.  Copies stay in order on their stream. */
  int32_t copy_roots;   /* 0: one upload per isolated write, a window of a larger buffer copied
                           as a strided rectangle (Sec. III: each isolated write its own command);
                           1: isolated writes that are windows of a root buffer no kernel writes
                           are uploaded together as one dense copy of the whole root, before the
                           first kernel that reads any of them (e.g. one copy of a d x d weight
                           matrix instead of one 128-byte-row rectangle per attention head).  The
                           host then gives the root's array (psc_host_io names the root). */
  int32_t exec_per_cu;  /* PSC_DEVICE only: at most this many executor workgroups per CU (>= 0).
                           0: the covering executor instance with the most resident workgroups
                           (two per CU for the attention DAGs); 1: one per CU.  Which is faster
                           depends on the DAG: measured, one per CU on the one-layer 512
                           attention DAG (0.119 against 0.155 ms), two on the 12-layer 1024
                           one (3.93 against 4.38 ms), so the benchmark times both. */
} psc_sched_opts;

/* One op of an exported schedule.  Its cross-stream precedences are waits[wait_off ..
 * wait_off + n_waits) in the array filled by psc_sched_export (ids of ops it waits for). */
typedef struct psc_op {
  int32_t id;
  int32_t type;         /* psc_op_type */
  int32_t kernel;       /* kernel id for PSC_OP_KERNEL, else -1 */
  int32_t buffer;       /* buffer id for copies (a root buffer for H2D), else -1 */
  int32_t stream;       /* stream index */
  int32_t pos;          /* position in its stream */
  int32_t host_order;   /* position in the host's enqueue sequence */
  int32_t n_waits;
  int32_t wait_off;
} psc_op;

/* Host memory for one isolated write (read from) or isolated read (written to).  `bytes` must
 * equal the buffer's rows*cols*element size; data is dense row-major.  For overlap the memory
 * should be pinned (hipHostMalloc, torch pin_memory).  A buffer with no entry is not copied:
 * its device storage is used as it stands (device-resident inputs and outputs). */
typedef struct psc_host_io {
  const char *name;
  void *host_ptr;
  size_t bytes;
} psc_host_io;

typedef struct psc_run_stats {
  double makespan_ms;      /* GPU time from the start event (recorded before the first op) to
                              the end event (after every stream joined); with PSC_DISPATCH_AQL
                              the device clock of a start mark, which every stream waits for,
                              to that of an end mark, after every stream joined */
  double host_enqueue_ms;  /* host wall time spent enqueueing (graph launch only, in graph mode) */
  int32_t n_ops, n_kernels, n_h2d, n_d2h, n_waits, n_streams, graph;
  int32_t aql_packets;     /* AQL packets written (PSC_DISPATCH_AQL), else 0 */
} psc_run_stats;

/* Per-op timing of the last psc_run with record_ops = 1, relative to the start event. */
typedef struct psc_op_time {
  int32_t op;
  int32_t stream;
  float start_us;
  float end_us;
} psc_op_time;

/* ---------------------------------------------------------------------------------------------
 * DAG construction (host-only)
 * ------------------------------------------------------------------------------------------- */

/* A new empty DAG, owned by the caller until psc_dag_destroy. */
psc_status psc_dag_create(psc_dag **out);

/* Frees the DAG.  Every schedule made from it must be destroyed first (PSC_ERR_STATE otherwise).
 * NULL is accepted and ignored. */
psc_status psc_dag_destroy(psc_dag *dag);

/* Declares buffer `name` (B of Sec. III; the <type, size> of a buffer tuple in Sec. IV-A) of
 * dtype x rows x cols.  With view_of != NULL it is a window of that buffer at (row_off, col_off),
 * which must lie inside it.  Zero rows or cols are allowed (empty buffer).
 * Errors: PSC_ERR_NAME (duplicate name, unknown parent), PSC_ERR_SHAPE (window outside the
 * parent, dtype differs from the parent's), PSC_ERR_STATE (DAG already scheduled). */
psc_status psc_add_buffer(psc_dag *dag, const char *name, int32_t dtype, int64_t rows,
                          int64_t cols, const char *view_of, int64_t row_off, int64_t col_off);

/* Adds kernel `name` of kind `kind` reading buffers inputs[0..n_in) and writing
 * outputs[0..n_out) (E_I and E_O of Sec. III).  Shapes are checked when the DAG is scheduled.
 * *kernel_id (may be NULL) receives the kernel's id: ids count up from 0 in call order.
 * Errors: PSC_ERR_NAME, PSC_ERR_ARG (wrong operand count for the kind), PSC_ERR_STATE. */
psc_status psc_add_kernel(psc_dag *dag, const char *name, int32_t kind,
                          const char *const *inputs, int32_t n_in, const char *const *outputs,
                          int32_t n_out, const psc_kernel_params *params, int32_t *kernel_id);

/* Edge k_i,b_r -> k_j,b_s of the specification file (Sec. IV-A): output buffer `src_output` of
 * kernel src_kernel feeds input buffer `dst_input` of kernel dst_kernel.  On one device the two
 * must share storage (the same buffer, or overlapping windows of one root buffer): the consumer
 * reads what the producer wrote, with no copy.  Errors: PSC_ERR_ARG (bad ids), PSC_ERR_NAME
 * (buffer is not an output / input of that kernel), PSC_ERR_SHAPE (no shared storage),
 * PSC_ERR_STATE. */
psc_status psc_add_edge(psc_dag *dag, int32_t src_kernel, const char *src_output,
                        int32_t dst_kernel, const char *dst_input);

/* What psc_dag_from_json built (any field may be ignored). */
typedef struct psc_spec_info {
  int32_t n_kernels, n_buffers, n_edges;
  int32_t n_components;  /* task components: one per tc sub-list, then one per kernel in none */
  int32_t gpu_queues;    /* the file's cq entry for the GPU (0 if it gives none): the paper's
                            command-queue count, to pass as psc_sched_opts.n_streams */
  int32_t reserved[3];
} psc_spec_info;

/* The specification file of Sec. IV-A (the dag.json of PySchedCL, in JSON text) lowered onto the
 * calls above: a new DAG in *out, owned by the caller (psc_dag_destroy).
 *   json       NUL-terminated UTF-8 text of one object with the members
 *     "kernels"  list of {"id": 0..n-1, "name": "gemm"|"matmul"|"transpose"|"softmax"|"add"|"vadd",
 *                "dev": "gpu" (optional; any other device is PSC_ERR_UNSUPPORTED: one GPU),
 *                "inputBuffers" / "outputBuffers": buffer tuples {"type": "float"|"bfloat16",
 *                "size": elements, "pos": argument position} (and optionally "name": buffers of
 *                one name in several kernels share storage, e.g. an input read by many kernels;
 *                "view_of" + "row_off"/"col_off": a window of a "buffers" entry),
 *                "varArguments": tuples {"type": "int"|"float", "pos", "value"}: in position
 *                order the integers are M, N, K for a GEMM (C = alpha A B, A M x K, B K x N, C
 *                M x N; an optional float is alpha) and rows, cols for the others (transpose of
 *                rows x cols gives cols x rows), "globalWorkSize": evaluated, otherwise unused --
 *                each kernel chooses its own grid; "ioBuffers" must be absent or empty}.
 *                Buffer arguments are the inputs then the output in position order; each "size"
 *                must equal the element count the kernel's dimensions give (PSC_ERR_SHAPE).
 *     "edges"    list of "k_i,b_r -> k_j,b_s" strings (or [k_i, b_r, k_j, b_s]): the output at
 *                argument position b_r of kernel k_i is the input at position b_s of k_j.
 *     "tc"       optional list of lists of kernel ids: the task components, in order.
 *     "cq"       optional {"gpu": n} or ["gpu:n"]: command queues per device.
 *     "buffers"  optional list of {"name", "type", "rows", "cols"}: storage that arguments window.
 *     "symbols"  optional object of default symbol values.
 *   Numbers anywhere may be expressions over symbols: + - * / % ( ), integers where an integer
 *   is meant.  sym_names[0..n_sym) / sym_values bind symbols at load time, over the defaults.
 * Buffers are named by "name", else "k<i>_a<pos>" after the producing kernel's argument (or the
 * first reader's); kernels "<name>_<id>", ids as in the file.  Every error destroys what was
 * built and leaves *out untouched: PSC_ERR_ARG (malformed JSON, with line and column; unbound
 * symbol; wrong argument counts), PSC_ERR_NAME (edge argument that is not an output / input,
 * name clashes), PSC_ERR_SHAPE, PSC_ERR_UNSUPPORTED (CPU device, ioBuffers, unknown kernel);
 * cycles and races are found by psc_schedule as for any DAG. */
psc_status psc_dag_from_json(const char *json, const char *const *sym_names, const int64_t *sym_values,
                             int32_t n_sym, psc_dag **out, psc_spec_info *info);

/* Description of buffer `id` (ids as psc_buffer_id): its name (NUL-terminated, truncated to
 * name_cap - 1 bytes; name may be NULL), dtype, shape and, for a view, its parent's id and offset
 * (parent -1 for a root).  Output pointers may be NULL.  PSC_ERR_ARG for a bad id. */
psc_status psc_buffer_desc(const psc_dag *dag, int32_t id, char *name, int32_t name_cap, int32_t *dtype,
                           int64_t *rows, int64_t *cols, int32_t *parent, int64_t *row_off, int64_t *col_off);

/* Description of kernel `id`: name, kind, input buffer ids (inputs[0..*n_in), capacity 2),
 * output buffer id, GEMM alpha and task component.  Output pointers may be NULL. */
psc_status psc_kernel_desc(const psc_dag *dag, int32_t id, char *name, int32_t name_cap, int32_t *kind,
                           int32_t *inputs, int32_t *n_in, int32_t *output, float *alpha, int32_t *component);

/* Edge `e` (in psc_add_edge order): producer kernel and buffer, consumer kernel and buffer. */
psc_status psc_edge_desc(const psc_dag *dag, int32_t e, int32_t *src_kernel, int32_t *src_buffer,
                         int32_t *dst_kernel, int32_t *dst_buffer);

/* Puts a kernel in task component `component` (>= 0; all kernels start in component 0).
 * Components drive the classification below and PSC_MAP_COMPONENT. */
psc_status psc_set_component(psc_dag *dag, int32_t kernel, int32_t component);

/* Uses caller-owned device memory at `dptr` (>= the buffer's rows*cols*element bytes, dense
 * row-major) as the storage of root buffer `name` instead of library-allocated memory.  The
 * memory must stay valid while schedules of this DAG run.  Errors: PSC_ERR_NAME (unknown, or a
 * view), PSC_ERR_ARG (NULL or too small), PSC_ERR_STATE. */
psc_status psc_bind_device(psc_dag *dag, const char *name, void *dptr, size_t bytes);

/* Counts of kernels, buffers and edges (any pointer may be NULL). */
psc_status psc_dag_info(const psc_dag *dag, int32_t *n_kernels, int32_t *n_buffers,
                        int32_t *n_edges);

/* Id of buffer `name` (ids count up from 0 in psc_add_buffer order). */
psc_status psc_buffer_id(const psc_dag *dag, const char *name, int32_t *id);

/* Classification of task component `component` (Sec. III): kclass[k] (n_kernels entries) gets
 * PSC_FRONT | PSC_END | PSC_IN bits for kernels of the component, 0 for others: FRONT = no
 * producer inside the component, END = no consumer inside it, IN = neither.  edge_inter[e]
 * (n_edges entries, edge ids in psc_add_edge order) gets 1 for an inter edge (the two kernels
 * lie in different components), 0 for an intra edge.  Either array may be NULL.
 * Validates the DAG like psc_schedule does. */
psc_status psc_dag_classify(psc_dag *dag, int32_t component, int32_t *kclass,
                            int32_t *edge_inter);

/* ---------------------------------------------------------------------------------------------
 * Scheduling (host-only) and execution
 * ------------------------------------------------------------------------------------------- */

/* Validates and freezes the DAG (no further psc_add_* calls), then builds the command-queue
 * structure for `policy` (setup_cq of Sec. IV-B): per-stream op lists and the event waits that
 * realise rules (i)-(iii) of Sec. III.  Waits already implied by stream order or by earlier waits
 * are omitted.  opts == NULL means: 4 streams, PSC_MAP_RR, no copy stream, no graph, device 0.
 * The schedule references the DAG, which must outlive it.  No GPU call is made here (except that
 * a PSC_MAP_EFT with an MLP cost model evaluates the model on the GPU).
 * Errors: PSC_ERR_SHAPE, PSC_ERR_CYCLE, PSC_ERR_RACE (see psc_status), PSC_ERR_ARG. */
psc_status psc_schedule(psc_dag *dag, int32_t policy, const psc_sched_opts *opts,
                        psc_sched **out);

/* Schedules the DAGs dags[0..n) as one batch (n >= 1): the schedule holds its own copy of their
 * disjoint union, planned with `policy` and `opts` as psc_schedule plans one DAG, run by one
 * psc_run (one hipGraph with use_graph).  In the union, buffer and kernel names are "<i>/<name>"
 * with i the DAG's position in `dags` (psc_host_io names them so); ids follow DAG order (DAG i's
 * buffers, kernels and edges after DAG i-1's, each in its own order); task component c of DAG i
 * becomes component c + (sum of the component counts of DAGs 0..i-1), so DAGs whose kernels all
 * lie in component 0 become components 0..n-1 (per-instance completion times with
 * mark_components).  Buffers bound with psc_bind_device keep their caller memory (DAGs may share
 * device-resident weights that way).  The source DAGs are not modified, not frozen and may be
 * destroyed right after this call.  Errors: as psc_schedule (validation errors name the buffer or
 * kernel with its "<i>/" prefix); PSC_ERR_ARG for n < 1 or a NULL DAG. */
psc_status psc_schedule_batch(psc_dag *const *dags, int32_t n, int32_t policy, const psc_sched_opts *opts,
                              psc_sched **out);

/* The command-queue structure of Def. 4 (Sec. III): per-queue op lists (stream, pos) and the
 * cross-queue precedences (waits), for the schedule validator.
 * Copies the schedule's ops (ordered by id) into ops[0..cap) and their waits into
 * waits[0..waits_cap); *n_ops / *n_waits receive the totals.  With ops == NULL or waits == NULL
 * only the totals are returned.  PSC_ERR_ARG if a capacity is too small. */
psc_status psc_sched_export(const psc_sched *sched, psc_op *ops, int32_t cap, int32_t *n_ops,
                            int32_t *waits, int32_t waits_cap, int32_t *n_waits);

/* Number of streams the schedule uses (n_streams, plus the upload and read-back streams of
 * copy_stream). */
psc_status psc_sched_streams(const psc_sched *sched, int32_t *n_streams);

/* [GPU] Allocates device storage for every unbound root buffer (one arena), creates streams
 * and events, and prepares kernel launches.  Called by the first psc_run if not called before.
 * Errors: PSC_ERR_HIP, PSC_ERR_OOM. */
psc_status psc_sched_prepare(psc_sched *sched);

/* [GPU] The dispatch step of Algorithm 1 (Sec. IV-B): after setup_cq has built the queues, flush
 * them to the device with their precedences and wait for completion.
 * Runs the schedule once and waits for it: records a start event, enqueues every op in
 * host order (each wait as hipStreamWaitEvent on the producing op's event), joins all streams
 * and waits for the end event.  io[0..n_io) gives host memory for isolated writes / reads by
 * buffer name (see psc_host_io); buffers not listed are not copied.  stats may be NULL.
 * Errors: PSC_ERR_NAME (io names no isolated write or read), PSC_ERR_ARG (byte count), PSC_ERR_HIP. */
psc_status psc_run(psc_sched *sched, const psc_host_io *io, int32_t n_io, psc_run_stats *stats);

/* Per-op timeline of the last psc_run made with record_ops = 1: out[0..cap), *n = op count. */
psc_status psc_sched_op_times(const psc_sched *sched, psc_op_time *out, int32_t cap, int32_t *n);

/* Host-only check for PSC_DISPATCH_AQL: builds every kernel launch of the schedule on stand-in
 * addresses and looks each kernel up in the code object's argument table (libpsc_kernels.kargs:
 * named by its host handle, explicit record within the launch record, only implicit arguments
 * of the kinds the dispatcher fills).  *n_kernels (may be NULL) = distinct kernels, or -1 if one
 * is not dispatchable, with the reason in why[0..why_cap) (may be NULL).  Returns PSC_OK either
 * way (errors only for bad arguments). */
psc_status psc_sched_aql_check(const psc_sched *sched, int32_t *n_kernels, char *why, int32_t why_cap);

/* [GPU] Completion of each task component in the last psc_run: done_us[c] = microseconds from
 * the run's start mark to the end of component c's last END kernel (a kernel with no successor
 * in its component, Def. 2), or -1 for a component with no kernel.  *n = number of components
 * (largest component id + 1).  Needs mark_components (or PSC_DEVICE).  PSC_ERR_STATE without
 * such a run; PSC_ERR_ARG if cap < *n (done_us may be NULL to query *n). */
psc_status psc_sched_component_times(const psc_sched *sched, float *done_us, int32_t cap, int32_t *n);

/* 1 if the schedule's queues are out of order (psc_sched_opts.out_of_order), else 0: in an
 * exported out-of-order schedule the precedences are the waits alone. */
psc_status psc_sched_queue_order(const psc_sched *sched, int32_t *out_of_order);

/* [GPU after prepare] Device address of buffer `name` (a view's address is inside its root's
 * storage) and its leading dimension in elements.  PSC_ERR_STATE before psc_sched_prepare. */
psc_status psc_sched_device_ptr(const psc_sched *sched, const char *name, void **dptr,
                                int64_t *ld);

/* [GPU after prepare] Copies the current device contents of buffer `name` (any buffer or view,
 * also intermediates that no isolated read brings back) into host memory, rows x cols elements of
 * its dtype packed row-major (BF16 as bfloat16 bits); bytes must equal that size (PSC_ERR_SHAPE
 * otherwise).  Waits for all work on the device first.  For inspection and tests: a DAG's
 * intermediate results live on the device between the kernels of Sec. III's dependent edges.
 * PSC_ERR_STATE before psc_sched_prepare, PSC_ERR_NAME for an unknown name. */
psc_status psc_sched_read(const psc_sched *sched, const char *name, void *host, size_t bytes);

/* [GPU] Launches kernel `kernel` of a prepared schedule `iters` times back to back on its own
 * stream, on the storage the schedule uses, and returns the mean duration per launch measured
 * with HIP events on that stream.  For kernel-level timing. */
psc_status psc_kernel_time(psc_sched *sched, int32_t kernel, int32_t iters, float *avg_us);

/* [GPU] Page-locked host memory (hipHostMalloc) of `bytes` bytes for psc_host_io buffers, so
 * copies run asynchronously and overlap compute.  Freed with psc_host_free.  Errors: PSC_ERR_ARG
 * (NULL out), PSC_ERR_OOM. */
psc_status psc_host_alloc(size_t bytes, void **out);

/* [GPU] Frees memory from psc_host_alloc.  NULL is ignored. */
psc_status psc_host_free(void *ptr);

/* [GPU] Properties of `device` for reports: its name and architecture (NUL-terminated, truncated
 * to cap bytes each; either may be NULL), compute units, peak engine clock in MHz and device
 * memory in bytes (any output may be NULL). */
psc_status psc_device_info(int32_t device, char *name, int32_t name_cap, char *arch, int32_t arch_cap,
                           int32_t *compute_units, int32_t *clock_mhz, int64_t *memory_bytes);

/* [GPU] Waits until all work the library enqueued on `device` has finished (hipDeviceSynchronize). */
psc_status psc_device_sync(int32_t device);

/* Host-only check of the multi-threaded enqueue: runs psc_run's dispatch threads (host_threads
 * as in psc_sched_opts) against a recording backend instead of HIP, with a random sleep of up
 * to jitter_us microseconds before every recorded call (seeded by `seed`).  out[0 .. 3*n) gets
 * one (kind, op, arg) triple per call in the order the calls happened: kind 0 = wait (arg = the
 * awaited op), 1 = the op itself, 2 = event record of the op, 3 = stream finished (op = -1,
 * arg = stream).  *n = number of triples; PSC_ERR_ARG if cap < 3 * n. */
psc_status psc_sched_dispatch_trace(const psc_sched *sched, int32_t host_threads, int32_t jitter_us,
                                    uint32_t seed, int32_t *out, int32_t cap, int32_t *n);

/* ---------------------------------------------------------------------------------------------
 * Learned cost model (machine-learning assisted scheduling, future work of Sec. VII).
 *
 * Every op is described by PSC_FEATURES float32 features:
 *   [0..5]  one-hot kind: GEMM, transpose, softmax, add, H2D, D2H
 *   [6]     log2 M (output rows; for a copy, the buffer's rows)   [7] log2 N (output columns)
 *   [8]     log2 K (GEMM inner dimension, else 0)                 [9] log2 of the algorithmic bytes
 *   [10]    1 if the first operand (or the copied buffer) is BF16  [11] other streams with an op
 *                                                                      in flight when it starts
 * The model is a perceptron PSC_FEATURES -> 64 -> 64 -> 1 with ReLU that predicts ln(duration in
 * microseconds) from z-scored features; parameters are PSC_MLP_PARAMS float32 values laid out as
 * W1 (64 x 12, row-major), b1 (64), W2 (64 x 64), b2 (64), W3 (64), b3 (1).  It is trained on the
 * GPU (forward, back-propagation and Adam kernels) from the samples psc_sched_samples returns and
 * is used by PSC_MAP_EFT through psc_sched_opts.cost.  A model belongs to one device; calls on one
 * model are serialised internally.
 * ------------------------------------------------------------------------------------------- */
#define PSC_FEATURES 12
#define PSC_MLP_PARAMS 5057

typedef struct psc_mlp_train_opts {
  int32_t epochs;         /* passes over the samples (>= 1) */
  int32_t batch;          /* samples per Adam step (>= 1); the last step of a pass may be smaller */
  float lr, beta1, beta2, eps;  /* Adam (Kingma and Ba, 2015); e.g. 1e-3, 0.9, 0.999, 1e-8 */
  uint64_t shuffle_seed;  /* 0: samples in their given order every pass; else a seeded shuffle */
  int32_t reserved[4];
} psc_mlp_train_opts;

/* [GPU] A model on `device` with all parameters zero and identity feature scaling. */
psc_status psc_mlp_create(int32_t device, psc_mlp **out);
psc_status psc_mlp_destroy(psc_mlp *m);

/* [GPU] Sets / reads the PSC_MLP_PARAMS parameters (n must equal it).  Setting them also clears
 * the Adam moments and step count.  PSC_ERR_ARG on a wrong n or NULL. */
psc_status psc_mlp_set_params(psc_mlp *m, const float *params, int64_t n);
psc_status psc_mlp_get_params(psc_mlp *m, float *params, int64_t n);

/* [GPU] Feature scaling: the network sees (x[f] - mean[f]) / std[f].  std must be > 0. */
psc_status psc_mlp_set_norm(psc_mlp *m, const float *mean, const float *std_dev);

/* [GPU] Predictions (ln microseconds) y[0..n) for feature rows x[n][PSC_FEATURES] (host memory). */
psc_status psc_mlp_predict(psc_mlp *m, const float *x, int64_t n, float *y);

/* [GPU] Gradient of the mean squared error mean((y - t)^2) over the n rows with respect to every
 * parameter (grads: PSC_MLP_PARAMS floats, may be NULL) and the loss itself (*loss, may be NULL),
 * without changing the parameters.  For gradient checks. */
psc_status psc_mlp_grad(psc_mlp *m, const float *x, const float *t, int64_t n, float *grads, double *loss);

/* [GPU] psc_mlp_grad without any device allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, results and errors as psc_mlp_grad (the gradient is bit-identical to it; the
 * loss is reduced on the device in float64, so it may differ from psc_mlp_grad's in the last
 * bits), but the samples, activations, errors and gradient of the pass live in one fixed array
 * of ~4.4 MB per GPU, held from the first call on that GPU until the process ends, so n is
 * limited to PSC_MLP_STATIC_MAX rows: larger n gives PSC_ERR_ARG.  No hipMalloc or hipFree is
 * made (the model's parameters were allocated by psc_mlp_create).  Every call on one GPU uses
 * that GPU's array and leaves its last contents there; calls on one GPU are serialised by a lock
 * in the library, so overlapping calls from several threads wait for each other rather than
 * race.  x and t are host memory (n x PSC_FEATURES and n floats); grads (PSC_MLP_PARAMS floats)
 * and loss may be NULL. */
#define PSC_MLP_STATIC_MAX 4096
psc_status psc_mlp_grad_static(psc_mlp *m, const float *x, const float *t, int64_t n, float *grads, double *loss);

/* [GPU] Saves the model's full training state to `path`: parameters, Adam first and second
 * moments and step count, and the feature scaling, with a 64-bit FNV-1a checksum of the contents
 * (a binary file of fixed size; written to path.tmp and renamed, so a reader never sees half a
 * file).  psc_mlp_load restores all of it, so psc_mlp_train continues exactly where it stopped
 * (training 2 passes equals 1 pass, save, load into a new model, 1 pass, bit for bit, with
 * shuffle_seed 0).  Errors: PSC_ERR_IO (cannot write), PSC_ERR_HIP.
 * The paper's future work (Sec. VII) names machine-learning assisted scheduling; keeping the
 * trained model lets a scheduler start from it. */
psc_status psc_mlp_save(psc_mlp *m, const char *path);
/* [GPU] Loads a file written by psc_mlp_save into m.  The file is checked whole first -- size,
 * magic, network shape, checksum, every value finite, scales positive, second moments >= 0 --
 * and on any failure m is left unchanged and PSC_ERR_IO names the reason.  A caller that cannot
 * load its model schedules with the heuristic (psc_sched_opts.cost = NULL). */
psc_status psc_mlp_load(psc_mlp *m, const char *path);
/* Host-only: the checks of psc_mlp_load without a model; *step (may be NULL) = the saved Adam
 * step count.  PSC_OK if the file would load. */
psc_status psc_mlp_file_check(const char *path, int64_t *step);

/* [GPU] Trains on n samples (features x, targets t = ln microseconds): opts->epochs passes of
 * mini-batch Adam steps.  epoch_loss[e] (may be NULL) receives the mean squared error over all n
 * samples after pass e.  Errors: PSC_ERR_ARG (sizes, hyper-parameters), PSC_ERR_HIP. */
psc_status psc_mlp_train(psc_mlp *m, const float *x, const float *t, int64_t n, const psc_mlp_train_opts *opts,
                         float *epoch_loss);

/* Predicted microseconds of each feature row under the cost model `m`, or under the roofline
 * heuristic when m == NULL (host only in that case). */
psc_status psc_cost_predict(psc_mlp *m, const float *x, int64_t n, float *us);

/* Feature row (PSC_FEATURES floats into f) of kernel `kernel` of a validated DAG (one that has
 * been scheduled) with `in_flight` other streams busy.  Host only.  Errors: PSC_ERR_ARG,
 * PSC_ERR_STATE (DAG not validated yet). */
psc_status psc_kernel_features(const psc_dag *dag, int32_t kernel, int32_t in_flight, float *f);

/* Training samples from the last psc_run made with record_ops = 1: one per op that did work (a
 * launched kernel, a copy that was given host memory), in op order.  features[i][PSC_FEATURES]
 * and log_us[i] = ln(measured duration in microseconds); feature 11 counts the other streams
 * with an op whose recorded interval contains this op's start.  Either array may be NULL;
 * *n = number of samples; PSC_ERR_ARG if cap < *n; PSC_ERR_STATE without a recorded run. */
psc_status psc_sched_samples(const psc_sched *sched, float *features, float *log_us, int32_t cap, int32_t *n);

/* Host-only view of the PSC_DEVICE executor's plan for `workers` workgroups (the run uses one per
 * resident slot of the GPU): every kernel is cut into tasks (output tiles or row groups), and
 * the tasks are list-scheduled onto the workgroups.  Tasks are sized here for `workers`
 * workgroups; a run holding more than one workgroup per CU sizes them for one per CU.  tasks[3*i .. 3*i+2] = (kernel, tile,
 * signal) of the i-th task, where the lists of workgroups 0, 1, ... follow each other and
 * workgroup w's list is tasks [work_off[w], work_off[w+1]); signal > 0 means that after this
 * task the workgroup publishes that many completed tiles of the kernel (the run of its tiles
 * ending here).  *n_tasks = total; with tasks and work_off NULL only the total is returned;
 * work_off holds workers + 1 entries.  The plan shown is the one with the host copies:
 * node ids below the kernel count are kernels, the following ones the device plan's uploads and
 * read-backs in op order (psc_sched_export of a PSC_DEVICE schedule), their tasks on the last
 * workers / 16 (at most 32) workgroups.  Any schedule of the DAG may be passed (its policy is not
 * used; copy_roots is).  PSC_ERR_ARG if cap < *n_tasks. */
psc_status psc_sched_device_tasks(const psc_sched *sched, int32_t workers, int32_t *tasks, int32_t cap,
                                  int32_t *n_tasks, int32_t *work_off);

/* ---------------------------------------------------------------------------------------------
 * GEMM tile autotuner.  Tile configurations are numbered 1 .. n-1 (psc_gemm_tile_count gives n):
 * 1..5 large-tile kernels (128x128, 64x64, 32x32, 128x64, 64x128), 6..12 K-split small-tile
 * kernels staging operands through LDS (64x64, 32x64, 64x32, 32x32, 16x32, 32x16, 16x16), 13..15
 * K-split 16-row kernels reading operands directly into matrix-core registers (16x16, 16x32,
 * 16x64), 16 a 256x256 BF16 tile of eight wavefronts, 17..19 BF16 K-split kernels that load each
 * wavefront's whole share of K at once (16x16, 16x32, 32x32; for FP32 operands they mean 12, 10
 * and 9), 20 and 21 256x256 BF16 tiles whose operands go straight from global memory into LDS,
 * of four wavefronts with 128x128 each and of eight with 128x64 each (32x32 matrix-core blocks).
 * Tiles 16, 20 and 21 need M and N multiples of 256, K of 64, 16-byte aligned A and B and
 * leading dimensions that are multiples of 8, else they run as tile 4; with FP32 operands they
 * run as tile 1.  A GEMM whose params leave tile at
 * 0 takes the process-wide cache entry for its (M, N, K, operand dtype, output dtype) when there
 * is one, and a size heuristic otherwise; the choice is made when a schedule is prepared.  The
 * cache is thread safe.  (The paper leaves autotuning to future work, Sec. VII.)
 * ------------------------------------------------------------------------------------------- */

/* Number of tile configuration indices (valid configurations are 1 .. *n - 1). */
psc_status psc_gemm_tile_count(int32_t *n);

/* Sets (tile > 0) or removes (tile = 0) the cache entry for one GEMM shape and dtype pair. */
psc_status psc_tile_cache_set(int32_t M, int32_t N, int32_t K, int32_t ab_dtype, int32_t c_dtype,
                              int32_t tile);

/* Cache entry for a shape, 0 if none. */
psc_status psc_tile_cache_get(int32_t M, int32_t N, int32_t K, int32_t ab_dtype, int32_t c_dtype,
                              int32_t *tile);

/* Empties the cache; *n_removed (may be NULL) receives the number of entries it held. */
psc_status psc_tile_cache_clear(int32_t *n_removed);
/* [GPU] The key a saved tile cache is valid for on `device`: its architecture name (gcnArchName),
 * compute-unit count, the HIP runtime version, this library's ABI version and tile count, as one
 * word (e.g. "gfx950:sramecc+:xnack-/cu256/hip70226015/abi1/tiles17").  key gets at most cap
 * bytes including the NUL; PSC_ERR_ARG if it does not fit. */
psc_status psc_tile_cache_key(int32_t device, char *key, int32_t cap);
/* Host-only: writes every cached tile choice to `path` (text: a header, the key, one line per
 * (M, N, K, operand dtype, output dtype, tile), a checksum line; written to path.tmp and renamed)
 * under `key` (a word without blanks, normally psc_tile_cache_key's).  PSC_ERR_IO if it cannot
 * be written. */
psc_status psc_tile_cache_save(const char *path, const char *key);
/* Host-only: merges the choices saved in `path` into the cache (a loaded entry replaces the
 * cached one for its shape).  The file is checked whole before anything is merged: PSC_ERR_IO
 * if it is missing, malformed, altered (checksum) or names a tile outside 1 .. count-1;
 * PSC_ERR_STATE if it was saved under another key (another architecture, runtime or library
 * version: its timings do not apply).  *n_loaded (may be NULL) = entries merged. */
psc_status psc_tile_cache_load(const char *path, const char *key, int32_t *n_loaded);

/* [GPU] Times every tile configuration for C (M x N) = A (M x K) * B (K x N) on zero-filled
 * device buffers (iters back-to-back launches between HIP events, after 3 warm-up launches),
 * stores the fastest in the cache and returns it in *best_tile and its mean microseconds in
 * *best_us.  us_per_tile[t] for t < cap receives every configuration's time (index 0 unused);
 * a configuration that resolves to another for this shape and dtype (16-21 with FP32 operands,
 * 16, 20 and 21 on shapes that are not whole 256 x 256 tiles) is not timed and its entry is left
 * unchanged, so the cache always names the tile a launch uses.
 * Any output pointer may be NULL.  Errors: PSC_ERR_ARG, PSC_ERR_HIP, PSC_ERR_OOM. */
psc_status psc_autotune_gemm(int32_t device, int32_t M, int32_t N, int32_t K, int32_t ab_dtype,
                             int32_t c_dtype, int32_t iters, int32_t *best_tile, float *best_us,
                             float *us_per_tile, int32_t cap);

/* [GPU] psc_autotune_gemm for every distinct GEMM shape of the DAG whose tile is automatic;
 * *n_tuned (may be NULL) receives the number of shapes tuned.  Schedules prepared afterwards
 * use the tuned tiles. */
psc_status psc_autotune_dag(psc_dag *dag, int32_t device, int32_t iters, int32_t *n_tuned);

/* [GPU] Tile choice by the schedule itself: isolated kernel times do not predict a GEMM's time
 * beside the concurrent kernels of a fine schedule (a tile that wins alone can lose in the DAG
 * by holding more LDS and registers).  For every GEMM shape class of the DAG (operand and output
 * dtype included; kernels with a fixed tile are left alone) this first runs psc_autotune_gemm,
 * then, for the max_classes heaviest classes (isolated time x kernels), heaviest first, schedules
 * the DAG with `policy` and `opts` once per candidate among the class's top_k isolated tiles --
 * the other classes at their current choice -- and times `iters` device-resident runs on seeded
 * inputs; the tile with the lowest median makespan goes into the tile cache (lighter classes keep
 * the isolated winner).  *n_changed (may be NULL) = classes whose choice differs from the
 * isolated winner.  The DAG must be schedulable with these options. */
psc_status psc_autotune_dag_in_schedule(psc_dag *dag, int32_t policy, const psc_sched_opts *opts, int32_t top_k,
                                        int32_t max_classes, int32_t iters, int32_t *n_changed);

/* [GPU] Schedule autotuner: builds a `policy` schedule of the DAG for each of the n candidate
 * option sets, runs each `iters` times on device-resident data (after 2 warm-up runs) and returns
 * the index of the one with the smallest mean wall time per run in *best; ms_per_run[i] (may be
 * NULL) receives candidate i's mean milliseconds.  Candidates that fail to schedule get a time
 * of -1 and are skipped.  Paired with psc_autotune_dag it chooses tiles, stream count, mapper
 * and enqueue threads by measurement.  Errors: PSC_ERR_ARG (no candidate ran), PSC_ERR_HIP. */
psc_status psc_autotune_schedule(psc_dag *dag, int32_t policy, const psc_sched_opts *candidates,
                                 int32_t n, int32_t iters, int32_t *best, float *ms_per_run);

/* [GPU after prepare] Tile configuration a prepared schedule uses for GEMM kernel `kernel`. */
psc_status psc_sched_kernel_tile(const psc_sched *sched, int32_t kernel, int32_t *tile);

/* [GPU after prepare] The device executor a prepared PSC_DEVICE schedule launches: its workgroup
 * count, workgroups resident per CU, and the tile-function groups of the compiled instance it
 * uses (bit i = group i; groups 0-5 FP32 GEMM tiles, 6-12 BF16 GEMM tiles, 13 softmax, transpose
 * and add, 14 the BF16 64 x 64 K-split tile for K >= 256, held only by instances of one workgroup
 * per CU).  The library holds several instances of the executor, each with a subset of the tile
 * functions: registers are the union of what an instance holds, so a smaller instance keeps more
 * workgroups per CU; prepare takes, among the instances that cover every tile function the DAG
 * needs, the one with the most resident workgroups.  Any pointer may be NULL.
 * PSC_ERR_STATE if the schedule is not prepared or not a PSC_DEVICE schedule. */
psc_status psc_sched_executor_info(const psc_sched *sched, int32_t *workers, int32_t *per_cu,
                                   uint32_t *groups);

/* Frees device storage, streams, events and graphs of the schedule.  NULL is ignored. */
psc_status psc_sched_destroy(psc_sched *sched);

/* Message of the most recent call on this thread if it failed, "" if it succeeded.  Valid until
 * the next call on this thread. */
const char *psc_last_error(void);

/* PSC_ABI_VERSION of the loaded library. */
int32_t psc_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PSC_H */
