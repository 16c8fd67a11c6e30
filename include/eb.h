/*
 * eb.h — edge-based grid metrics on one MI355X (gfx950), C ABI.
 *
 * Computes, for a triangle (dim = 2), tetrahedral (dim = 3) or pentatope
 * (dim = 4) grid, the metrics of the node-centred edge-based discretization
 * (Nishikawa,
 * "An Efficient Implementation of Edge-Based Discretization without Forming
 * Dual Control Volumes", Section 2, eq. threed_fv_semidiscrete_system_00)
 * directly from element geometry, never forming a median dual:
 *
 *   n_e  lumped directed-area vector of every edge e = {j,k}, j < k, pointing
 *        from j to k (Section 2: edges run from the smaller node number);
 *          n_jk = 2/(D(D+1)) * sum_{E contains jk} n_j^E        (eq.
 *                 efficient_njk_formula_general_D, Section 3.2.3)
 *               + 1/(D(D+1)) * sum_{boundary elements B containing jk} n_B
 *        where n_j^E is the outward area vector of the face of E opposite j;
 *   b_j  dual-face area vector at boundary node j: (1/D) sum_{B contains j}
 *        n_B (the boundary term of the closure check, Section 3.2.3);
 *   V_j  median-dual volume: sum_{E contains j} |E|/(D+1) (Section 4.2), or
 *        by the edge loop (1/(2D)) sum_k (x_k - x_j).n_jk (Section 4.1).
 *
 * and the topology those loops need (unique edges, element -> edge map with
 * orientation signs, boundary elements, incidence lists), plus the adjoint of
 * n, b and V with respect to the node coordinates.
 *
 * Conventions
 *   - Every array argument is a DEVICE pointer on the current HIP device
 *     unless its name ends in _host.  Pointers must be 16-byte aligned
 *     (hipMalloc and torch allocations are); lengths are element counts.
 *   - coords is structure-of-arrays FP64 [dim][n_nodes]; elem is int32
 *     [n_elems][dim+1] with any local vertex order (either orientation).
 *   - All outputs are overwritten, never accumulated into; inputs are const.
 *   - A grid needs at least one node; it may have no elements.  Such a grid
 *     has no edges, boundary faces or boundary nodes, so every per-node sum
 *     (V, the residual, the gradient) is zero and the per-edge and
 *     per-boundary-node outputs, having no entries, may be null.
 *   - ne = dim(dim+1)/2 local edges per element (3, 6 or 10), in lexicographic
 *     local pair order: 2D (0,1)(0,2)(1,2); 3D (0,1)(0,2)(0,3)(1,2)(1,3)(2,3);
 *     4D (0,1)(0,2)(0,3)(0,4)(1,2)(1,3)(1,4)(2,3)(2,4)(3,4).
 *   - dim 4 (the general-D formula of Section 3.2.3 with D = 4, which the
 *     paper leaves to future work) is supported by eb_build_edges,
 *     eb_build_edges_emit, eb_directed_areas and eb_dual_volumes; the other
 *     calls return EB_EINVAL for it.
 *   - Calls enqueue work on `stream` and return at once, except
 *     eb_build_edges and eb_check_errors, which synchronize `stream`.
 *   - The caller owns every buffer.  The library allocates no device memory
 *     and keeps no state between calls except a thread-local error detail
 *     string, the events armed by eb_time_next_launch (thread-local) and the
 *     gather launch shape (eb_set_gather_shape); scratch
 *     lives in the caller's workspace `ws`.
 *   - Returns EB_OK (0) or a negative eb_status.  Errors found on the host
 *     (bad arguments, sizes beyond int32 indexing, workspace too small) return
 *     at once and enqueue nothing.  Errors found by kernels (node id out of
 *     range, zero-measure element, a face shared by more than two elements,
 *     a node beyond the plan's per-node limits) set a sticky status word in `ws`;
 *     eb_build_edges reports it, other calls leave it for eb_check_errors.
 *     Outputs are undefined after any error.  HIP failures return EB_EHIP
 *     with hipGetErrorString text in eb_last_error_detail().
 *   - Calls that share one `ws` must not run concurrently on different
 *     streams.
 */
#ifndef EB_H
#define EB_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  EB_OK = 0,
  EB_EINVAL = -1,       /* null pointer, bad dim/mode, misaligned, negative size */
  EB_ERANGE = -2,       /* element references a node id outside [0, n_nodes) */
  EB_EDEGENERATE = -3,  /* element of zero measure */
  EB_ENONMANIFOLD = -4, /* face (3D) or edge (2D) shared by more than two elements */
  EB_EWORKSPACE = -5,   /* ws_bytes below eb_workspace_bytes() */
  EB_EOVERFLOW = -6,    /* counts that would overflow int32 indexing */
  EB_EHIP = -7,         /* HIP runtime error */
  EB_ECAPACITY = -8,    /* a node beyond the kernel plan's per-node limits:
                           more than EB_MAX_NODE_ELEMS elements, or more than
                           EB_MAX_OUT_EDGES edges with it as tail (neighbours
                           with a larger id) */
  EB_ETIMEOUT = -9      /* the fused persistent kernel gave up waiting for an
                           earlier phase (its waits are bounded; outputs are
                           then undefined) */
} eb_status;

/* Per-node limits of the kernel plan (eb_topology.plan).  Neither the number
 * of distinct neighbours nor the number of faces around a node is otherwise
 * bounded. */
#define EB_MAX_NODE_ELEMS 65535
#define EB_MAX_OUT_EDGES 1023

typedef enum { EB_REDUCE_ATOMIC = 0, EB_REDUCE_GATHER = 1 } eb_reduce;
typedef enum { EB_VOL_ELEMENT = 0, EB_VOL_EDGE = 1 } eb_vol_mode;
typedef enum { EB_BFLUX_NODE = 0, EB_BFLUX_LINEAR = 1 } eb_bflux;

/* Sizes of one grid; filled by eb_build_edges.  plan_bytes is the size of
 * the kernel plan (eb_topology.plan); plan_param records the plan's layout
 * for the library: callers copy eb_sizes whole and never set or interpret
 * it. */
typedef struct {
  int32_t dim;
  int64_t n_nodes, n_elems, n_edges, n_bfaces, n_bnodes;
  int64_t plan_bytes;
  int64_t plan_param[2];
} eb_sizes;

/* Topology arrays (device).  Every integer output is uniquely defined, so two
 * builds of the same grid give identical bits.
 *   edge           [2][n_edges]   row 0 tails, row 1 heads (tail < head), in
 *                                 ascending (tail, head) order (the paper's
 *                                 edge(e,1), edge(e,2), Section 2)
 *   node_edge_off  [n_nodes+1]    edges with tail j are [off[j], off[j+1])
 *   elem_edge      [n_elems][ne]  edge id of each local edge
 *   elem_edge_sign [n_elems][ne]  +1 iff elem[p] < elem[q] (local p -> q is
 *                                 the edge direction), else -1
 *   edge_inc_off   [n_edges+1]    optional (NULL skips): elements of each edge
 *   edge_inc       [ne*n_elems]     as elem*ne + local, ascending per edge
 *   node_inc_off   [n_nodes+1]    elements of each node as elem*(dim+1) +
 *   node_inc       [(dim+1)*n_elems]  local vertex, ascending per node
 *   node_in_off    [n_nodes+1]    ids of edges whose head is the node,
 *   node_in_edge   [n_edges]        ascending per node
 *   bface          [n_bfaces][dim] boundary elements (faces of exactly one
 *                                 element), ascending by sorted vertex ids;
 *                                 vertices ordered so that the area vector
 *                                 2D (dy,-dx) of v0->v1, 3D (1/2)(v1-v0)x(v2-v0)
 *                                 points out of the domain; 3D rotated so the
 *                                 smallest id comes first; 4D ascending, the
 *                                 last two swapped when the area vector
 *                                 (1/6) N(v1-v0, v2-v0, v3-v0) of that order
 *                                 points into the domain (N(u,v,w).x =
 *                                 det[x; u; v; w])
 *   bface_owner    [n_bfaces]     elem*(dim+1) + local index of the owner's
 *                                 vertex opposite the face
 *   bface_edge     [n_bfaces][dim*(dim-1)/2]  edge ids of the face's vertex
 *                                 pairs (vp,vq), p < q, in lexicographic order
 *   bnode          [n_bnodes]     ascending ids of nodes on boundary faces
 *   node_bnode     [n_nodes]      index into bnode, or -1 for interior nodes
 *   bnode_face_off [n_bnodes+1]   boundary faces of each boundary node,
 *   bnode_face     [dim*n_bfaces]   ascending per node
 *   plan           [plan_bytes]   the kernel plan: the library's own
 *                                 per-node view of the incidences (each
 *                                 node's elements with their other vertices
 *                                 and out-edge positions, laid out for the
 *                                 node-centred kernels), written by
 *                                 eb_build_edges_emit and read by the
 *                                 EB_REDUCE_GATHER paths.  Opaque: its
 *                                 format is private to the library and may
 *                                 change between versions; 256-byte aligned.
 *                                 (dim 4 makes no plan: one placeholder line.)
 */
typedef struct {
  int32_t *edge;
  int32_t *node_edge_off;
  int32_t *elem_edge;
  int8_t *elem_edge_sign;
  int32_t *edge_inc_off, *edge_inc;
  int32_t *node_inc_off, *node_inc;
  int32_t *node_in_off, *node_in_edge;
  int32_t *bface;
  int32_t *bface_owner;
  int32_t *bface_edge;
  int32_t *bnode;
  int32_t *node_bnode;
  int32_t *bnode_face_off, *bnode_face;
  void *plan;
} eb_topology;

/* Bytes of workspace every call below needs for a grid of this size. */
size_t eb_workspace_bytes(int dim, int64_t n_nodes, int64_t n_elems);

/* Bytes of workspace eb_directed_areas_backward needs with EB_REDUCE_GATHER:
 * the above grown to hold one gradient piece (dim doubles) per incidence
 * slot of the kernel plan.  A workspace this large serves every call; the
 * sticky status word sits at its start in either case, so the same
 * workspace is passed to every call on one grid. */
size_t eb_backward_workspace_bytes(const eb_sizes *sizes);

/* Edge extraction, phase 1 (Section 2: the edge array; Section 3.2: boundary
 * elements).  Validates the grid, builds the node -> element lists into the
 * caller's node_inc_off [n_nodes+1] and node_inc [(dim+1)*n_elems] (their
 * sizes are known in advance; ws keeps a richer copy for phase 2), counts
 * unique edges, boundary faces and boundary nodes into ws, and fills
 * *sizes_host.  Synchronizes `stream` once and returns the sticky device
 * status.  coords [dim][n_nodes] are needed to orient boundary faces outward
 * and to reject zero-measure elements. */
int eb_build_edges(int dim, int64_t n_nodes, int64_t n_elems, const int32_t *elem,
                   const double *coords, int32_t *node_inc_off, int32_t *node_inc,
                   void *ws, size_t ws_bytes, eb_sizes *sizes_host, hipStream_t stream);

/* Edge extraction, phase 2: writes every other eb_topology array (sized from
 * *sizes) from what eb_build_edges left in ws (the same ws, untouched in
 * between).  topo->node_inc_off and topo->node_inc must be the arrays phase 1
 * filled.  edge_inc_off/edge_inc may be NULL; topo->plan must hold
 * sizes->plan_bytes bytes, 256-byte aligned. */
int eb_build_edges_emit(const eb_sizes *sizes, const int32_t *elem, const double *coords,
                        const eb_topology *topo, void *ws, size_t ws_bytes,
                        hipStream_t stream);

/* Lumped directed-area vectors n_edge [dim][n_edges] (eq.
 * efficient_njk_formula_general_D plus the boundary correction, Section
 * 3.2.3), boundary dual-face normals b_node [dim][n_bnodes] (NULL to skip)
 * and element-based dual volumes vol [n_nodes] (Section 4.2; NULL to skip),
 * in one pass over the grid.
 *   EB_REDUCE_ATOMIC: one thread per element, then one per boundary face;
 *     each block sums its contributions per edge and per node in LDS, then
 *     adds each sum to the zeroed outputs with one FP64 atomic (summation
 *     order varies from run to run).
 *   EB_REDUCE_GATHER: one thread per node gathers over its elements in
 *     node_inc order and owns the edges it is the tail of; every output is
 *     written once, bitwise reproducible.  Needs node_inc, node_edge_off,
 *     edge, node_bnode, bnode_face_off/bnode_face, bface.  Boundary nodes
 *     follow in a second pass, a group of lanes each.  dim 4: one thread per
 *     node walks its node_inc row (no plan).
 *   dim 4, both reductions (and eb_dual_volumes, both modes): the points
 *     are first copied as 32-byte rows into ws, in space the build uses only
 *     until eb_build_edges_emit, when 32 n_nodes bytes fit there (80 per
 *     element, less the edge loop's 8 per edge); otherwise the kernels read
 *     coords directly. */
int eb_directed_areas(const eb_sizes *sizes, const eb_topology *topo, const int32_t *elem,
                      const double *coords, int reduce, double *n_edge, double *b_node,
                      double *vol, void *ws, size_t ws_bytes, hipStream_t stream);

/* Forward-pass variants, for measuring what the paper's operation counts
 * cost on this hardware (Table 3; the remark that one area vector n_j^E
 * serves every edge with tail j).  Same outputs and requirements as
 * eb_directed_areas with EB_REDUCE_GATHER; results agree with it to rounding:
 *   EB_VARIANT_NODE_NORMALS  exactly eb_directed_areas (one n_j^E per node
 *                            and element);
 *   EB_VARIANT_EDGE_NORMALS  n_j^E formed again for every edge with tail j
 *                            (one normal per local edge, 6 per tet);
 *   EB_VARIANT_DUAL_FACES    the traditional construction (Section 3.1): each
 *                            edge's median-dual face in each element from the
 *                            edge midpoint, face and element centroids, and
 *                            b from the boundary faces' median-dual pieces. */
typedef enum {
  EB_VARIANT_NODE_NORMALS = 0,
  EB_VARIANT_EDGE_NORMALS = 1,
  EB_VARIANT_DUAL_FACES = 2
} eb_variant;
int eb_directed_areas_variant(const eb_sizes *sizes, const eb_topology *topo,
                              const int32_t *elem, const double *coords, int variant,
                              double *n_edge, double *b_node, double *vol, void *ws,
                              size_t ws_bytes, hipStream_t stream);

/* Dual volumes vol [n_nodes].
 *   EB_VOL_ELEMENT: sum of |E|/(D+1) over the elements of each node
 *     (Section 4.2); n_edge unused.
 *   EB_VOL_EDGE: the edge loop V_j = (1/(2D)) sum_k (x_k - x_j).n_jk over the
 *     edges of j (Section 4.1), from the boundary-corrected n_edge
 *     [dim][n_edges] of eb_directed_areas.  ATOMIC: thread per edge, FP64
 *     atomics to both ends; GATHER: each edge's term once into ws, then one
 *     thread per node sums its out-edges (node_edge_off) and in-edges
 *     (node_in rows) in that order. */
int eb_dual_volumes(const eb_sizes *sizes, const eb_topology *topo, const int32_t *elem,
                    const double *coords, int mode, const double *n_edge, int reduce,
                    double *vol, void *ws, size_t ws_bytes, hipStream_t stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the edge loop of
 * eb_dual_volumes (EB_VOL_EDGE, same results, same kernels) without a
 * workspace.  EB_REDUCE_GATHER keeps its per-edge terms in a fixed device
 * array of the library, EB_NOALLOC_SCRATCH_BYTES on every GPU the library
 * runs on, held until the process ends; grids with more than
 * EB_NOALLOC_SCRATCH_BYTES / 8 edges get EB_EWORKSPACE.  Every term is
 * written before it is read, so nothing is cleared.  No device memory is
 * allocated or freed.  All calls on one GPU share its array: calls that
 * overlap on one GPU (different streams or threads) race.  The first call on
 * a device looks the array's address up (hipGetSymbolAddress) with that
 * device current.  No kernel of the edge loop detects errors, so there is
 * no status word either. */
#define EB_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int eb_dual_volumes_noalloc(const eb_sizes *sizes, const eb_topology *topo,
                            const double *coords, const double *n_edge, int reduce,
                            double *vol, hipStream_t stream);

/* Edge-loop residual, the consumer of the metrics (the edge-based
 * discretization of Section 2): given nodal flux values flux [dim][n_nodes]
 * (F_j), res [n_nodes] (overwritten) = sum over the edges (j,k) of node j of
 * +-(F_j + F_k)/2 . n_jk (+ at the tail, - at the head) plus the boundary
 * flux of j:
 *   EB_BFLUX_NODE    F_j . b_j (b_node [dim][n_bnodes] required);
 *   EB_BFLUX_LINEAR  per boundary face B of j, n_B/dim . (weighted F of B's
 *                    nodes: 2D 5/6 own + 1/6 other, 3D 6/8 own + 1/8 each
 *                    other), computed from coords; with the lumped n of
 *                    eb_directed_areas this makes res_j = (div F) V_j exactly
 *                    for every linear F, at every node.
 * Constant F gives res = 0 (closure).  Two passes like the edge loop (edge
 * terms into ws, ordered node sums), then the boundary nodes; bitwise
 * reproducible.  Needs edge, node_edge_off, node_in_off/node_in_edge, bnode
 * (and bnode_face, bface for LINEAR). */
int eb_edge_residual(const eb_sizes *sizes, const eb_topology *topo, const int32_t *elem,
                     const double *coords, const double *n_edge, const double *b_node,
                     const double *flux, int bflux, double *res, void *ws, size_t ws_bytes,
                     hipStream_t stream);

/* Adjoint: given grad_n = dL/dn [dim][n_edges], grad_b = dL/db [dim][n_bnodes]
 * and grad_vol = dL/dV [n_nodes] (any may be NULL = zero), writes
 * grad_coords = dL/dx [dim][n_nodes] for the metrics eb_directed_areas
 * computes (element-based V).  Derivative of the element and boundary
 * formulas above; the orientation sign of each element is held fixed.
 * ATOMIC: thread per element, then per boundary face (each block's per-node
 * sums first gathered in LDS, one FP64 atomic per node and component).  GATHER: an
 * element pass writes each element's gradient with respect to each of its
 * vertices into the workspace at that incidence's slot of the plan, then
 * one thread per node sums its slots in node_inc order and adds its boundary
 * faces in bnode_face order: no atomics, bitwise reproducible.  GATHER needs
 * topo->plan and ws_bytes >= eb_backward_workspace_bytes(sizes) (else
 * EB_EINVAL / EB_EWORKSPACE). */
int eb_directed_areas_backward(const eb_sizes *sizes, const eb_topology *topo,
                               const int32_t *elem, const double *coords,
                               const double *grad_n, const double *grad_b,
                               const double *grad_vol, int reduce, double *grad_coords,
                               void *ws, size_t ws_bytes, hipStream_t stream);

/* Profiling aid.  Arms two events (created by the caller, e.g. with
 * hipEventCreate) for the principal kernel of the next eb_directed_areas,
 * eb_dual_volumes or eb_directed_areas_backward call made on this thread:
 * the element- or node-pass kernel that carries the call's main traffic
 * (gather forward: the node pass; gather adjoint: the element pass; atomic
 * paths: the element pass; volumes: the one kernel).  That launch records
 * `start` just before the kernel and `stop` just after it on the call's
 * stream (hipExtLaunchKernelGGL), so hipEventElapsedTime gives the kernel's
 * own duration.  The next such call consumes the events whether or not it
 * launches; NULL, NULL disarms.  Returns EB_EINVAL if only one is NULL. */
int eb_time_next_launch(hipEvent_t start, hipEvent_t stop);

/* Profiling aid.  Arms two events that bracket the kernels of the next
 * eb_directed_areas call made on this thread: `start` is recorded just
 * before its first kernel (gather: the node pass; atomic: the element pass)
 * and `stop` just after its last (the boundary pass), on the call's stream
 * (hipExtLaunchKernelGGL), so hipEventElapsedTime gives the call's kernel
 * time, the zero fills of the atomic path excluded.  Consumed like
 * eb_time_next_launch's events by the next call that takes those (another
 * call brackets only its principal kernel with them), and taking
 * precedence over them; NULL, NULL disarms.  Returns EB_EINVAL if only one
 * is NULL. */
int eb_time_next_call(hipEvent_t start, hipEvent_t stop);

/* Launch shape of the node-centred (EB_REDUCE_GATHER) kernels: nodes per
 * block (64, 128 or 256; default 64), incidences per chunk (1, 2 or 4,
 * default 2: a chunk's points load while the chunk before is formed), and
 * whether consecutive node tiles are kept on one XCD (0/1, default 1).  Process-wide setting (the one piece of state the library keeps,
 * besides the error detail), meant to be set once from a tuning run; it
 * changes speed only, never results.  Returns EB_EINVAL for other values. */
int eb_set_gather_shape(int tile, int unroll, int xcd_remap);
void eb_get_gather_shape(int *tile, int *unroll, int *xcd_remap);

/* ------------------------------------------------------------------------
 * Batches of grids, the fused forward + adjoint, graphs, tuning.
 *
 * A batch of meshes is passed as ONE grid: node ids of mesh m are offset by
 * node_off[m] and its elements follow those of mesh m-1 (elem_off[m]).  The
 * meshes are disconnected, so eb_build_edges / _emit and every call above
 * treat the whole batch in one launch each, and each mesh's edges, boundary
 * nodes and boundary faces form contiguous ranges of the outputs.  Results
 * per mesh equal those of the mesh on its own (same ids up to the offsets). */

/* Per-mesh output ranges of a batch (host arrays of n_mesh+1 entries):
 * edge_off (n_edge, grad_n rows), bnode_off (b_node, bnode), bface_off
 * (bface), from node_off / elem_off (host, n_mesh+1 entries each, starting
 * at 0, node_off strictly increasing to n_nodes, elem_off non-decreasing to
 * n_elems).  Checks on the device that every element of mesh m references
 * only mesh m's nodes (EB_EINVAL with the element in the detail otherwise).
 * Uses the gather-adjoint part of ws as scratch (needs ws_bytes >=
 * eb_workspace_bytes + 40 (n_mesh+1) rounded; eb_backward_workspace_bytes
 * is always enough for n_mesh <= n_nodes / 4).  Synchronizes `stream` and
 * returns (and clears) the sticky device status, like eb_check_errors. */
int eb_batch_offsets(const eb_sizes *sizes, const eb_topology *topo, const int32_t *elem,
                     int n_mesh, const int64_t *node_off_host, const int64_t *elem_off_host,
                     int64_t *edge_off_host, int64_t *bnode_off_host, int64_t *bface_off_host,
                     void *ws, size_t ws_bytes, hipStream_t stream);

/* Forward and adjoint together: n_edge, b_node, vol as eb_directed_areas
 * with EB_REDUCE_GATHER, and grad_coords as eb_directed_areas_backward with
 * EB_REDUCE_GATHER, for the loss weights grad_n / grad_b / grad_vol (any may
 * be NULL = zero; the loss is linear, so its adjoint needs no forward
 * output).  One persistent kernel, no larger than the grid that is resident
 * at once, runs three phases (forward node tiles and adjoint element tiles,
 * then forward boundary and adjoint node tiles, then adjoint boundary
 * tiles), block b taking items b, b + grid, ... of each; a block with work
 * in a later phase waits (bounded, EB_ETIMEOUT) until every block has
 * finished the earlier one (counters in ws).  A small reset kernel runs
 * first, so the enqueue is two kernels and no memset (safe to capture in a
 * graph).  Same bits as the two separate gather calls up to
 * floating-point contraction; bitwise reproducible for any launch shape.
 * Needs everything both gather calls need, including ws_bytes >=
 * eb_backward_workspace_bytes(sizes).  Calls on one ws must not overlap. */
int eb_batch_forward_backward(const eb_sizes *sizes, const eb_topology *topo,
                              const int32_t *elem, const double *coords, const double *grad_n,
                              const double *grad_b, const double *grad_vol, double *n_edge,
                              double *b_node, double *vol, double *grad_coords, void *ws,
                              size_t ws_bytes, hipStream_t stream);

/* A HIP graph of eb_batch_forward_backward with these exact pointers,
 * captured on a private stream (so the caller's stream may be the null
 * stream).  Launching it recomputes every output from the current contents
 * of the inputs (e.g. coordinates updated in place on a deforming grid).
 * The shape in force at creation is baked in.  Destroy with
 * eb_graph_destroy; launches on one graph or ws must not overlap. */
typedef struct eb_graph_s *eb_graph;
int eb_batch_graph_create(const eb_sizes *sizes, const eb_topology *topo, const int32_t *elem,
                          const double *coords, const double *grad_n, const double *grad_b,
                          const double *grad_vol, double *n_edge, double *b_node, double *vol,
                          double *grad_coords, void *ws, size_t ws_bytes, eb_graph *graph);
int eb_graph_launch(eb_graph graph, hipStream_t stream);
int eb_graph_destroy(eb_graph graph);

/* Launch shape of the fused kernel: threads per block (64/128/256; = nodes
 * per node tile), loads in flight per thread (1/2/4) and resident blocks per
 * compute unit (1..32, capped by occupancy; 0 = as many as fit).
 * Process-wide, speed only. */
int eb_set_fused_shape(int tile, int unroll, int blocks_per_cu);
void eb_get_fused_shape(int *tile, int *unroll, int *blocks_per_cu);

/* How eb_batch_forward_backward runs: EB_FUSED_PERSISTENT (default) the one
 * persistent kernel described there; EB_FUSED_SEPARATE the gather forward
 * and the gather adjoint kernels one after the other (same results up to
 * rounding, also capturable; faster where the persistent kernel's shared
 * occupancy limit costs more than the launches it saves);
 * EB_FUSED_PERSISTENT_ATOMIC one persistent kernel whose adjoint sums with
 * FP64 atomics after per-block sums in LDS, as eb_directed_areas_backward's
 * EB_REDUCE_ATOMIC (two phases: forward node tiles with the adjoint's
 * element and boundary blocks, then forward boundary tiles; a fill kernel
 * zeroes grad_coords first); EB_FUSED_SEPARATE_ATOMIC the gather forward and
 * that atomic adjoint's kernels one after the other.  With either atomic
 * mode n, b and V are as in the others and grad_coords equal to rounding but
 * not bitwise reproducible.  Process-wide; eb_autotune keeps the reduction
 * in force (gather or atomic) and picks the persistent kernel's best shape
 * or the separate kernels, whichever is faster. */
typedef enum {
  EB_FUSED_PERSISTENT = 0,
  EB_FUSED_SEPARATE = 1,
  EB_FUSED_PERSISTENT_ATOMIC = 2,
  EB_FUSED_SEPARATE_ATOMIC = 3
} eb_fused_mode;
int eb_set_fused_mode(int mode);
int eb_get_fused_mode(void);

/* Bound of the fused kernel's phase waits, in polls of about a microsecond
 * (0 restores the default of 2^22).  A wait that runs out records
 * EB_ETIMEOUT and its block exits; every wave still ends. */
int eb_set_fused_wait_limit(int64_t spins);

/* Launch-shape tuner.  Times (reps runs each, after one warm-up, hipEvents
 * on `stream`) every gather shape of eb_directed_areas (tile x unroll x
 * xcd_remap) and every fused shape of eb_batch_forward_backward (tile x
 * unroll x blocks_per_cu in {1,2,4,8,0}) and the separate kernels on the
 * caller's grid and buffers, sets the fastest of each (eb_set_gather_shape,
 * eb_set_fused_shape, eb_set_fused_mode) and reports them.  With an atomic
 * mode in force it times the atomic persistent kernel's shapes and
 * EB_FUSED_SEPARATE_ATOMIC instead.  Outputs hold valid results afterwards
 * (all shapes give the same bits, but for the atomic modes' grad_coords).
 * Synchronizes `stream`. */
typedef struct {
  int32_t gather_tile, gather_unroll, gather_xcd_remap;
  float gather_ms;
  int32_t fused_tile, fused_unroll, fused_blocks_per_cu;
  float fused_ms;
  int32_t n_tried;
  int32_t fused_separate;  /* 1 if the separate kernels were faster and are set */
  float separate_ms;
} eb_tuning;
int eb_autotune(const eb_sizes *sizes, const eb_topology *topo, const int32_t *elem,
                const double *coords, const double *grad_n, const double *grad_b,
                const double *grad_vol, double *n_edge, double *b_node, double *vol,
                double *grad_coords, void *ws, size_t ws_bytes, int reps, hipStream_t stream,
                eb_tuning *out);

/* Diagnostic view of a kernel plan, for tests and tools that check the
 * plan against the topology it was built from.  Fills *view with device
 * pointers into `plan` and the plan's counts; no device access.  The
 * encoding of these arrays is private to the library (it is stated in the
 * library source, csrc/eb_plan.h) and may change between versions; no
 * computation needs them. */
typedef struct {
  const int32_t *slice_off;  /* [ceil(n_nodes/64)+1] */
  const uint64_t *entry;     /* [n_slots * words] */
  const uint32_t *step;      /* [n_slots], or NULL (some wide plans) */
  const int32_t *inc_slot;   /* [(dim+1)*n_elems] */
  int64_t n_slots;
  int32_t words;             /* 64-bit words per entry: 1 or 2 */
} eb_plan_view;
int eb_plan_describe(const eb_sizes *sizes, const void *plan, eb_plan_view *view);

/* Synchronizes `stream`, returns the sticky device status in ws and resets it
 * to EB_OK. */
int eb_check_errors(void *ws, hipStream_t stream);

/* Static text for a status code. */
const char *eb_status_string(int status);

/* Thread-local detail of the last error returned on this thread ("" if none). */
const char *eb_last_error_detail(void);

/* Library version string. */
const char *eb_version(void);

#ifdef __cplusplus
}
#endif

#endif /* EB_H */
