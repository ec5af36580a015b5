/*
 * rsi.h -- C ABI of the MI355X (gfx950) segment / triangle-mesh intersection
 * library (librsi.so).
 *
 * The problem (paper, Section 1): N_r line segments l_i = (r_start_i, r_end_i)
 * in R^3 are tested against a surface of N_t triangles, each an index triplet
 * into N_v vertices.  The default answer is one crossing flag per segment;
 * the paper's extended usage (Section 2.4) returns the crossing point and
 * triangle (`barycentric`) or the number of crossings (`intercept_count`).
 * Inputs use the layouts of the paper's input files (Section 2.5): vertices
 * FP32 x,y,z interleaved, triangles int32 triplets, segment starts and ends
 * FP32 x,y,z interleaved.
 *
 * The library builds a linear BVH over the triangles (Section 2: centroids,
 * quantisation to 2^21 levels per axis, 64-bit Morton codes, sort, binary
 * radix tree with bottom-up bounds and a per-node arrival counter, Section
 * 3.1) and answers queries by stack traversal with a Moller-Trumbore test at
 * the leaves (Section 2, Section 3.2, Section 3.3).
 *
 * Conventions for every call
 *   - Pointers named as device pointers must be device memory on the current
 *     HIP device (for example torch CUDA tensors); host structs are read
 *     before the call returns and may be freed afterwards.
 *   - `stream` is a hipStream_t (NULL = the default stream).  All device work
 *     is enqueued on it; calls return without waiting unless stated.
 *   - No exception crosses the ABI; every call returns an rsi_status and
 *     rsi_last_error() describes the last failure on the calling thread.
 *   - A handle serves one call at a time.
 */
#ifndef RSI_H
#define RSI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rsi_bvh *rsi_handle;

typedef enum {
    RSI_OK = 0,
    RSI_E_INVALID = 1,   /* bad argument: negative size, null pointer, out-of-range index, bad mode */
    RSI_E_NOMEM = 2,     /* a device allocation failed */
    RSI_E_HIP = 3,       /* a HIP runtime call or kernel launch failed */
    RSI_E_OVERFLOW = 4   /* a caller-sized buffer is too small; counts stay exact */
} rsi_status;

/* Query modes (bit mask).  RSI_FIRST_HIT may be combined with RSI_ALL_HITS
 * or RSI_COUNT; RSI_BOOL may be added to any of them and is then derived
 * from the same pass.  RSI_COUNT with RSI_ALL_HITS is the same as
 * RSI_ALL_HITS alone (which always writes the exact count). */
enum {
    RSI_BOOL = 1u,       /* crossing flag per segment (paper Section 1, default output) */
    RSI_FIRST_HIT = 2u,  /* crossing with the smallest t; exact ties go to the smaller
                            triangle id (our reading of `barycentric`, Section 2.4) */
    RSI_ALL_HITS = 4u,   /* exact count plus every crossing, ordered by (t, id)
                            (Section 2.4 and 2.6) */
    RSI_COUNT = 8u       /* exact number of crossings only, into out->count, no list
                            (`intercept_count`, Section 2.4; by Section 2.6 its odd
                            parity tells whether the start point lies inside a closed
                            surface) */
};

/* Build / query options; a zero field selects the default. */
typedef struct {
    int32_t leaf_size;    /* max triangles per BVH leaf, 1..16 (default 1) */
    int32_t block_size;   /* traversal workgroup size: 64, 128, 192 or 256 (default 128) */
    int32_t defer_lanes;  /* a wave tests its lanes' pending triangles once fewer than this many
                             of its lanes can still visit a node, 1..64 (default 32) */
    int32_t refill_lanes; /* a wave writes finished segments and takes new ones once this many
                             of its lanes are done, 1..64 (default 32) */
    int32_t chunk;        /* segments a wave claims per global atomic, 64..2^20
                             (default: about eight chunks per resident wave, 64..4096) */
    int32_t stack_depth;  /* traversal-stack entries per lane of the main pass, kept in LDS
                             (default 20 on the four-way walk, 17 for its boolean and counting
                             walks, 32 on the binary walk); a walk that needs more is finished
                             by the deep pass, whose stack continues in device memory.  A smaller
                             value raises occupancy. 1..255 */
    int32_t branching;    /* 4 (default): traverse the four-way view of the binary tree of
                             Section 3.1 (every node with its grandchildren as children, child
                             boxes quantised outward to 8 bits per plane, one 64-byte record
                             per node, laid out after each build, rebuild and refit); 2:
                             traverse the binary tree itself.  Both cull conservatively and
                             decide with the same FP32 triangle test, so their answers agree
                             except where that test is within rounding of its decision (the
                             looser quantised boxes let a few more triangles reach it). */
    int32_t reserved;
} rsi_opts;

/* Output buffers of rsi_query (host struct of device pointers, each [n_r...]).
 * Pointers for modes not requested are ignored and may be NULL. */
typedef struct {
    uint8_t *hit;      /* RSI_BOOL      [n_r]    1 if the segment crosses the mesh, else 0 */
    int32_t *tri;      /* RSI_FIRST_HIT [n_r]    triangle id (row of T) of the first hit; -1 on a miss */
    float *t;          /*               [n_r]    fraction along the segment, P = S + t (E - S); +inf on a miss */
    float *uv;         /*               [n_r*2]  weights of the triangle's 2nd and 3rd vertex; 0 on a miss */
    float *point;      /*               [n_r*3]  hit point P; 0 on a miss */
    int32_t *count;    /* RSI_ALL_HITS  [n_r]    exact number of crossings */
    int32_t *ids;      /*               [n_r*capacity] first min(count, capacity) crossings by (t, id); -1 padding */
    float *ts;         /*               [n_r*capacity] their t; +inf padding */
    int32_t capacity;  /* K >= 1 slots per segment for RSI_ALL_HITS */
    int32_t reserved;
    /* RSI_ALL_HITS, optional.  Segments with more than `capacity` crossings
     * keep their full lists, ordered by (t, id), in a spill pool: the
     * caller's (spill_ids / spill_ts, spill_cap entries each) when given,
     * else the library's (read it with rsi_spill_info / rsi_spill_read).
     * spill_off, when given, gets per segment the offset of its list in the
     * pool, or -1 (count <= capacity, or no room left in the pool). */
    int64_t *spill_off;  /*             [n_r] */
    int32_t *spill_ids;  /*             [spill_cap] */
    float *spill_ts;     /*             [spill_cap] */
    int64_t spill_cap;
} rsi_outputs;

/* Build a BVH over the mesh (paper Section 2: Morton-ordered binary radix
 * tree; Section 3.1 node definitions; Table 2 lists the build steps).
 *   V  device, float32 [n_v*3] vertex coordinates x,y,z (Section 2.5 layout)
 *   T  device, int32   [n_t*3] vertex indices per triangle, each in [0, n_v)
 *   opts host, may be NULL.
 * The handle keeps its own packed copy of the geometry; V and T are read
 * by the enqueued build and may be freed once it has run.  Asynchronous on
 * `stream`: nothing is read back (queries need no tree height on the host).
 * Errors: RSI_E_INVALID for n_v < 0, n_t < 0, n_t >= 2^27 or a NULL pointer
 * with a nonzero size; RSI_E_NOMEM; RSI_E_HIP.  A triangle index outside
 * [0, n_v) is found by the device and reported by rsi_query_stats
 * (RSI_E_INVALID) at the next synchronising call; the build then reads
 * vertex 0 in its place, so nothing outside V is touched.
 * n_t == 0 gives a handle whose queries report no crossing. */
rsi_status rsi_build(const float *V, int64_t n_v, const int32_t *T, int64_t n_t,
                     const rsi_opts *opts, void *stream, rsi_handle *out);

/* Rebuild the tree of an existing handle for new geometry with the same
 * triangle count n_t (all build steps of rsi_build, reusing the handle's
 * device memory, so nothing is allocated).  V, T, n_v as for rsi_build;
 * asynchronous on `stream`.  Errors as for rsi_build. */
rsi_status rsi_rebuild(rsi_handle h, const float *V, int64_t n_v, const int32_t *T, void *stream);

/* Recompute every bound and the packed geometry from new vertex positions
 * with the same triangles and the same tree topology (the bottom-up pass of
 * Section 3.1 with its arrival counters).  V: device float32 [n_v*3], n_v
 * the vertex count of the last build or rebuild (RSI_E_INVALID otherwise:
 * the triangles index that many vertices).  Asynchronous on `stream`. */
rsi_status rsi_refit(rsi_handle h, const float *V, int64_t n_v, void *stream);

/* Test n_r segments (paper Section 1; traversal of Section 3.2, kernel of
 * Section 3.3).
 *   S, E  device, float32 [n_r*3] segment starts and ends
 *   mode  bit mask of RSI_BOOL / RSI_FIRST_HIT / RSI_ALL_HITS (nonzero)
 *   out   host struct of device output pointers (see rsi_outputs)
 * RSI_BOOL alone stops each segment at its first crossing.  RSI_ALL_HITS keeps
 * the first `capacity` crossings by (t, id) of each segment in `ids`/`ts`
 * and the exact count; a segment with more keeps its full list in the
 * spill pool (see rsi_outputs), collected during the same walk (the
 * collision buffer of Section 3.2: atomic append, overflow detection).  The
 * library pool starts at max(2^20, n_r / 4) entries; when a query needs
 * more, rsi_query_stats returns RSI_E_OVERFLOW (counts and every list that
 * fitted stay exact), the pool grows to fit, and the caller queries again.
 * Always asynchronous on `stream`.  Reported t, u, v and P are re-solved in
 * FP64 from the FP32 inputs; the crossing decisions are the FP32 test.
 * Memory kept with the handle, allocated on first use and grown with n_r:
 * a retry queue (4 bytes per segment) and the deep pass's stack (a fixed
 * grid); for RSI_ALL_HITS also 16 bytes per segment of overflow table, the
 * arena and the library pool.
 * n_r == 0 is a no-op (output pointers are then not inspected).
 * Errors: RSI_E_INVALID (n_r < 0 or >= 2^30, mode 0 or unknown bits, missing output
 * pointer, capacity < 1, an incomplete caller pool), RSI_E_NOMEM, RSI_E_HIP. */
rsi_status rsi_query(rsi_handle h, const float *S, const float *E, int64_t n_r,
                     uint32_t mode, const rsi_outputs *out, void *stream);

/* rsi_query for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * handle, inputs and outputs are the caller's, as for rsi_query; the
 * library's own scratch (the deep pass's queue and stack) comes from one
 * fixed 32 MiB device array per GPU, held from the first call on that GPU
 * until the process ends.  No allocation of any kind is made, and nothing
 * is waited for.
 *   mode  nonzero mask of RSI_BOOL, RSI_FIRST_HIT, RSI_COUNT (RSI_ALL_HITS
 *         needs memory that grows with the crossings and is rejected)
 *   S, E, n_r, out as for rsi_query (only the arrays of `mode` are used)
 * The array holds the deep pass's stack (its size depends on block_size and
 * the stack options; about 16 MB at the defaults on 256 CUs) and a queue
 * of one entry per segment; a query with more segments than the queue
 * holds (about 4.3 million at the defaults) runs as consecutive parts of
 * that many segments each, with the same kernels and results as rsi_query.
 * rsi_query_stats then reports the last part's deep-pass count and the
 * flags of every part.
 * Every call on a GPU shares that GPU's array: calls that overlap in time on
 * one GPU (other streams, other handles, other threads) race and must be
 * ordered by the caller.  Its contents need no clearing between calls.
 * Errors: as rsi_query, plus RSI_E_INVALID when the current device is not
 * the handle's, for a batch handle, or when the options' deep-pass stack
 * leaves no room in the array (a block_size of 256 with the deepest stack
 * bound comes close; use a smaller block_size or rsi_query). */
rsi_status rsi_query_noalloc(rsi_handle h, const float *S, const float *E, int64_t n_r, uint32_t mode,
                             const rsi_outputs *out, void *stream);

/* Gradient of the first hit (t, u, v, P of RSI_FIRST_HIT) with respect to
 * the vertices and both segment ends, by the adjoint of the crossing system
 * S + t (E - S) = v0 + u (v1 - v0) + v (v2 - v0): the differentiable form of
 * the paper's `barycentric` output (Section 2.4).
 *   V        device float32 [n_v*3]: the vertices the handle was built or
 *            refit with (read-only); n_v must be the vertex count of the
 *            last build or rebuild (RSI_E_INVALID otherwise), since dV has
 *            that many rows and every triangle index is below it
 *   S, E     device float32 [n_r*3]: the segments of the forward query
 *   tri      device int32 [n_r]: first-hit triangle ids from the forward
 *            query (-1 = miss, contributes nothing)
 *   g_t      device float32 [n_r]   upstream dL/dt      (NULL = zero)
 *   g_uv     device float32 [n_r*2] upstream dL/d(u, v) (NULL = zero)
 *   g_point  device float32 [n_r*3] upstream dL/dP      (NULL = zero)
 *   dV       device float32 [n_v*3]: ACCUMULATED (dV += the gradient;
 *            the caller zeroes it for a plain gradient)
 *   dS, dE   device float32 [n_r*3]: written (zero for misses); NULL skips
 * (t, u, v) and the 3x3 transposed solve are evaluated in FP64 per segment.
 * The vertex gradient is summed without atomic operations in a fixed order
 * (per triangle in FP64, then per vertex), so repeated calls give the same
 * bits.  Memory kept with the handle and released by rsi_destroy (allocated
 * on first use, grown for a larger batch): about 64 bytes per segment
 * (records, sort pairs and the sort's scratch), 72 bytes per triangle and a
 * vertex incidence table of 36 bytes per triangle (rebuilt after
 * rsi_build / rsi_rebuild, kept across rsi_refit).
 * Asynchronous on `stream`.  Errors: RSI_E_INVALID (NULL pointers, n_r out
 * of range), RSI_E_NOMEM, RSI_E_HIP. */
rsi_status rsi_first_hit_backward(rsi_handle h, const float *V, int64_t n_v, const float *S, const float *E,
                                  int64_t n_r, const int32_t *tri, const float *g_t, const float *g_uv,
                                  const float *g_point, float *dV, float *dS, float *dE, void *stream);

/* After an RSI_ALL_HITS query (waits for it): entries of the overflow
 * table and pool entries in use (host out-parameters). */
rsi_status rsi_spill_info(rsi_handle h, int64_t *n_segments, int64_t *n_crossings);

/* Copy the overflow table and the pool of the last RSI_ALL_HITS query into
 * caller device buffers (waits for the query, then copies asynchronously on
 * `stream`):
 *   seg    int32 [n_segments]  segment index (batches: work item, i.e. the
 *                              segment's position in the concatenation of
 *                              the meshes' segment lists)
 *   offset int64 [n_segments]  first crossing of that segment in ids/ts
 *   count  int32 [n_segments]  its number of crossings; -1 marks a void
 *                              entry (a walk handed to the deep pass,
 *                              which made a new entry), to be skipped
 *   ids    int32 [n_crossings] triangle ids, per segment ordered by (t, id)
 *   ts     float [n_crossings] their t
 * Entries are grouped per segment; the order of the segments themselves is
 * unspecified. */
rsi_status rsi_spill_read(rsi_handle h, int32_t *seg, int64_t *offset, int32_t *count,
                          int32_t *ids, float *ts, void *stream);

/* State of the last call on the handle, after waiting for it (the
 * synchronising call that reports what the device found):
 *   bad_index           the last build met a triangle index outside [0, n_v)
 *                       (batches: outside its mesh's vertices)
 *   build_inconsistent  the build's own consistency checks failed
 *   walk_cut            a walk of the last query stopped at the node-visit
 *                       bound (only a damaged tree does that)
 *   stack_dropped       the deep pass dropped a stack entry (damaged tree)
 *   overflow_full       the last all-hits query's pool or arena was too small
 *   deep_segments       segments of the last query whose stack outgrew its
 *                       LDS part and were walked by the deep pass
 *   overflow_segments   all hits: segments with more crossings than slots
 *   overflow_crossings  all hits: pool entries they needed (their crossings)
 *   arena_records       all hits: crossings past the slots
 *   pool_capacity       all hits: pool entries available to the last query
 * Returns RSI_E_INVALID for bad_index / build_inconsistent, RSI_E_OVERFLOW
 * for overflow_full (the library pool has then grown to fit: query again),
 * else RSI_OK; `out` is filled in every case. */
typedef struct {
    int32_t bad_index;
    int32_t build_inconsistent;
    int32_t walk_cut;
    int32_t stack_dropped;
    int32_t overflow_full;
    int32_t reserved;
    int64_t deep_segments;
    int64_t overflow_segments;
    int64_t overflow_crossings;
    int64_t arena_records;
    int64_t pool_capacity;
} rsi_stats;
rsi_status rsi_query_stats(rsi_handle h, rsi_stats *out);

/* Segment order (the paper's v2.2 step, Section 4.1: rays sorted so that
 * neighbouring threads take similar paths).  order (device int32[n_r]) gets
 * the segment indices sorted by a key whose 3 most significant bits are the
 * octant of E - S and whose low 30 bits are the Morton code of the midpoint
 * quantised to 2^10 levels per axis inside the midpoints' bounding box;
 * stable (equal keys keep index order).  S, E: device float[3 n_r].  Uses
 * scratch kept with the handle (12 bytes per segment plus sort buffers).
 * Asynchronous on `stream`.  The order does not depend on the mesh: compute
 * it once, gather the segments into it, and query any number of meshes
 * (outputs then follow the gathered order). */
rsi_status rsi_segment_order(rsi_handle h, const float *S, const float *E, int64_t n_r, int32_t *order,
                             void *stream);

/* S_out[k] = S[order[k]], E_out[k] = E[order[k]] (device float[3 n_r] each;
 * must not alias S or E).  An order entry outside [0, n_r) reads segment 0
 * (no fault; an order from rsi_segment_order is always a permutation).
 * Asynchronous on `stream`. */
rsi_status rsi_gather_segments(rsi_handle h, const float *S, const float *E, const int32_t *order, int64_t n_r,
                               float *S_out, float *E_out, void *stream);

/* Compact outputs (paper Section 2.4, extended usage): the ids of the
 * segments that cross the mesh, in increasing order, and for `barycentric`
 * their distances, triangles and points.  Selection: hit[i] != 0 when `hit`
 * (an RSI_BOOL output) is given, else tri[i] >= 0 (an RSI_FIRST_HIT output).
 * With `tri`: dist[k] = t[i] * |E_i - S_i| (the distance from the start,
 * needs t, S, E), tri_out[k] = tri[i], point_out[3k..3k+2] = point[3i..];
 * any of dist, tri_out, point_out may be NULL.  All arrays are device
 * arrays; outputs need room for n_r entries (3 n_r floats for point_out).
 * *n_out (host) receives the number written; the call waits for it.
 * RSI_E_INVALID for NULL ids or n_out, n_r outside [0, 2^31), or a
 * combination not listed. */
rsi_status rsi_compact(rsi_handle h, const uint8_t *hit, const int32_t *tri, const float *t, const float *point,
                       const float *S, const float *E, int64_t n_r, int32_t *ids, float *dist, int32_t *tri_out,
                       float *point_out, int64_t *n_out, void *stream);

/* Odd-parity inside test (paper Section 2.4 gives the intercept count of a
 * segment, Section 2.6 notes that an odd count puts the segment's start point
 * inside a closed surface).  For every point P_i (device, float[3 n_p], AoS) the library
 * forms the segment from P_i to E_i = P_i + L_i u, u = (0.6, 0.41, 0.91)
 * normalised (FP32 0.515216053, 0.352064312, 0.781410992), L_i = |P_i - c| +
 * 2 R + 1 with c and R the centre and half diagonal of the mesh's bounding
 * box, so E_i lies outside the box; then counts the crossings exactly
 * (RSI_COUNT) and writes inside[i] = count & 1 (device, uint8[n_p]).
 * count (device int32[n_p]) and E (device float[3 n_p]) are optional
 * outputs: the counts and the far ends used; when NULL the library uses its
 * own scratch (kept with the handle).  The answer is meaningful for closed
 * (watertight) meshes; a segment through an edge or vertex is degenerate and
 * may be miscounted.  Asynchronous on `stream`; RSI_E_INVALID for a batch
 * handle, NULL pointers with n_p > 0, or n_p outside [0, 2^30). */
rsi_status rsi_inside(rsi_handle h, const float *P, int64_t n_p, uint8_t *inside, int32_t *count, float *E,
                      void *stream);

/* Work counters of the last query when it ran with counting enabled
 * (rsi_set_counting(h, 1)): node visits (internal nodes whose two child boxes
 * were tested), child box tests and triangle tests, summed over segments;
 * then wave-level counts of the persistent query loop (each wave of 64 lanes
 * adds one per iteration): all iterations, iterations that ran a node step,
 * a leaf phase, a refill.  node_visits / (64 * wave_node_steps) is the share
 * of lanes busy in node steps; of the others, summed over node steps,
 * lanes_blocked had a node but waited for pending leaf tests and
 * lanes_waiting had no node (walk over, or no segment).  wave_leaf_rounds
 * counts the rounds of the leaf phases (one triangle-leaf test per lane and
 * round) and leaf_lanes the lanes that tested a leaf in them, so
 * leaf_lanes / (64 * wave_leaf_rounds) is the share of lanes busy there. */
typedef struct {
    uint64_t node_visits;
    uint64_t box_tests;
    uint64_t tri_tests;
    uint64_t segments;
    uint64_t wave_loops;
    uint64_t wave_node_steps;
    uint64_t wave_leaf_phases;
    uint64_t wave_refills;
    uint64_t lanes_blocked;
    uint64_t lanes_waiting;
    uint64_t wave_leaf_rounds;
    uint64_t leaf_lanes;
} rsi_counters;
rsi_status rsi_set_counting(rsi_handle h, int enable);
rsi_status rsi_get_counters(rsi_handle h, rsi_counters *out);

/* Tree description for validation (host out-parameters / host buffers;
 * waits for the handle's last work to read the heights).
 *   n_nodes: number of node records (n_t, the last one being the entry node
 *   whose left child is the root, as in the paper's Section 2), height: levels
 *   of internal nodes below the entry node, leaf_size: as built. */
typedef struct {
    int64_t n_t;       /* triangles over all meshes */
    int64_t n_nodes;   /* node records (= n_t) */
    int32_t height;    /* largest tree height over the meshes */
    int32_t leaf_size;
    int32_t entry;     /* entry node of the first mesh */
    int32_t n_meshes;
} rsi_tree_info;
rsi_status rsi_get_tree_info(rsi_handle h, rsi_tree_info *out);

/* Per-mesh layout of a handle: mesh `mesh` owns triangles, sorted leaves and
 * node records [tri_offset, tri_offset + n_t); its entry node is the last of
 * them.  Any out-pointer may be NULL.  Reading the height waits for the
 * handle's last work. */
rsi_status rsi_get_mesh_info(rsi_handle h, int32_t mesh, int64_t *tri_offset, int64_t *n_t, int32_t *height);

/* Copy the tree to host buffers (blocking):
 *   boxes  float  [n_nodes*12] per node: left child lo xyz, hi xyz, right child lo xyz, hi xyz
 *   refs   int32  [n_nodes*2]  left and right child references: >= 0 internal
 *                              node index; < 0 leaf, with first sorted triangle
 *                              (ref & 0x07FFFFFF) and count ((ref >> 27) & 15) + 1
 *   order  int32  [n_t]        original triangle id at each sorted position
 *   keys   uint64 [n_t]        sorted Morton codes
 * Any pointer may be NULL to skip it. */
rsi_status rsi_export_tree(rsi_handle h, float *boxes, int32_t *refs, int32_t *order, uint64_t *keys);

/* ------------------------------------------------------------- batches --
 * Many meshes in one handle, built by the same launches (one launch per
 * build stage covers every mesh) and queried by ONE persistent launch over
 * all (mesh, segment) work items; the build + query sequence can be captured
 * once into a HIP graph and replayed with a single launch.  This extends the
 * paper's single-surface program (Section 2.3) to batches; callers are those
 * with many small meshes whose separate launches would be latency bound.
 *
 * rsi_batch_create: n_meshes in 1..65535; V, T host arrays of n_meshes
 * device pointers (vertex and triangle arrays as for rsi_build), n_v, n_t
 * host arrays of sizes.  The device pointers are kept: rsi_batch_rebuild and
 * captured rebuilds re-read the same buffers.  Triangle ids in outputs are
 * per mesh.  Asynchronous on `stream`.  Errors as for rsi_build. */
rsi_status rsi_batch_create(int32_t n_meshes, const float *const *V, const int64_t *n_v, const int32_t *const *T,
                            const int64_t *n_t, const rsi_opts *opts, void *stream, rsi_handle *out);

/* Rebuild every mesh of a batch from its (possibly updated) vertex and
 * triangle buffers; asynchronous on `stream`. */
rsi_status rsi_batch_rebuild(rsi_handle h, void *stream);

/* Query every mesh with its own segments in one launch.  S, E: host arrays of
 * n_meshes device pointers; n_r: host array of counts; outs: host array of
 * n_meshes rsi_outputs (hit / tri / t / uv / point / count / ids / ts /
 * spill_off as for rsi_query; one capacity for every mesh).  mode: a mask of
 * RSI_BOOL, RSI_FIRST_HIT, RSI_ALL_HITS.  All hits use the library's spill
 * pool (rsi_spill_*; its `seg` is then the work item).  Copies the tables
 * (waits for that copy), then runs asynchronously on `stream`. */
rsi_status rsi_batch_query(rsi_handle h, const float *const *S, const float *const *E, const int64_t *n_r,
                           uint32_t mode, const rsi_outputs *outs, void *stream);

/* Capture [rebuild of every mesh if `rebuild`] + the batched query with
 * these tables into a HIP graph held by the handle (replacing any previous
 * one).  All buffers named here must stay valid while the graph is used.
 * A replay may follow any change of the vertex values: the traversal is
 * sized from a bound on the tree height, not from the captured trees. */
rsi_status rsi_batch_capture(rsi_handle h, const float *const *S, const float *const *E, const int64_t *n_r,
                             uint32_t mode, const rsi_outputs *outs, int rebuild, void *stream);

/* Launch the captured graph on `stream`. */
rsi_status rsi_batch_replay(rsi_handle h, void *stream);

/* Change the options of a handle (all rsi_opts fields; zero keeps the
 * current value).  Query options apply to the next query; a new leaf_size
 * takes effect at the next rsi_rebuild / rsi_batch_rebuild.  A captured
 * graph of the handle is released (after waiting for the device); capture
 * again to replay with the new options.  rsi_tune does the same. */
rsi_status rsi_set_opts(rsi_handle h, const rsi_opts *opts);
rsi_status rsi_get_opts(rsi_handle h, rsi_opts *out);

/* Autotuner: time candidate option sets on a real query and keep the fastest.
 * For a single-mesh handle set V, n_v, T (used to rebuild when a candidate's
 * leaf size differs), S, E, n_r and out; for a batch handle set bS, bE, b_nr
 * and b_outs (per-mesh host arrays as for rsi_batch_query).  Each candidate
 * is applied, warmed up once, then timed `reps` times with HIP events on
 * `stream` (median written to ms[i]); the fastest is applied to the handle
 * (rebuilding if its leaf size differs) and its index written to *best.
 * The block size, leaf size, LDS stack depth, defer / refill lanes and chunk
 * are tunable.  Blocks until done. */
typedef struct {
    const float *V;
    int64_t n_v;
    const int32_t *T;
    const float *S;
    const float *E;
    int64_t n_r;
    const rsi_outputs *out;
    const float *const *bS;
    const float *const *bE;
    const int64_t *b_nr;
    const rsi_outputs *b_outs;
    uint32_t mode;
    int32_t reserved;
} rsi_tune_job;
rsi_status rsi_tune(rsi_handle h, const rsi_tune_job *job, const rsi_opts *candidates, int32_t n_candidates,
                    int32_t reps, float *ms, int32_t *best, void *stream);

/* Release the handle and its device memory (waits for its pending work). */
void rsi_destroy(rsi_handle h);

const char *rsi_status_str(rsi_status s);

/* Message of the last failure on the calling thread ("" if none). */
const char *rsi_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RSI_H */
