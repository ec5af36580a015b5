// query.hip -- segment queries against the linear BVH (paper Section 3.2,
// the traversal and candidate testing, and Section 3.3, the query kernel).
//
// Persistent wave64 kernel.  The grid holds as many workgroups as the GPU
// keeps resident; every lane owns one segment at a time and, when it is done,
// takes the next unprocessed segment from its wave's chunk; a wave claims a
// new chunk of segments with one atomic on the counter of its XCD's range of
// the segments (the other ranges once its own is used up).  The paper's
// kernel strides each thread over the rays instead (Section 3.3); with
// segments whose traversal lengths vary by an order of magnitude, a wave that
// waits for its slowest lane leaves most of its lanes idle, which the refill
// avoids.
//
// A lane walks the tree from the entry node with a stack laid out
// [depth][lane] in LDS so a wave's pushes and pops hit distinct banks.  The
// main pass keeps the whole stack in LDS (20 entries per lane on the
// four-way walk, 17 when it holds the top copy below; 32 on the binary
// walk); a walk that would push past it stops, queues its segment, and a
// deep pass (a small grid whose stacks continue in device memory up to a
// bound on the tree height) walks those segments again from the root.  No
// tree height is needed on the host, so builds, rebuilds and queries are
// enqueued without waiting for the device.
// Each node step loads one 64-byte record; the boolean and counting walks of
// a single mesh read the records of the top three four-way levels from a
// per-workgroup copy in LDS instead.
// The default four-way walk (Node4) tests the segment against the four
// quantised boxes of the node's grandchildren, keeps the touched leaf
// children as pending, descends into the nearest touched internal child and
// pushes the others; the binary walk (Node, branching 2) tests the two exact
// child boxes, keeps walking past one pending leaf and descends into the
// nearer touched child.  Pending leaves are tested once few lanes can still
// take a node step, so the triangle test runs with most lanes active.  The
// paper's bounded candidate list with resume (Section 3.2) is therefore not
// needed: candidates are tested soon after they are found.
//
// Modes
//   bool only   stop at the first crossing (any-hit, Section 3.2)
//   first hit   keep the crossing with the smallest (t, id); boxes that start
//               beyond it are pruned
//   all hits    count every crossing and keep the first K found (K slots per
//               segment); every crossing after the K-th goes to an arena as
//               an (overflow entry, rank, triangle) record, by one atomic
//               bump of the arena's counter.  When its walk ends, a segment
//               with more than K crossings reserves a range of the pool of
//               full lists (a second atomic bump) and stores its first K
//               there; two short passes then move the arena records into
//               the ranges and re-solve, order and copy each list (its
//               first K into the slots).  Nothing is walked twice and the
//               host never waits; a pool or arena that is too small sets a
//               flag (counts stay exact) that rsi_query_stats reports.
//   count       count every crossing, no list
// Segment ends are read, and results written, with nontemporal accesses:
// they stream through once, and must not push the tree out of the L2.
#include <hip/hip_runtime.h>
#include <float.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "../../include/rsi.h"
#include "rsi_host.h"

namespace rsi {
namespace {

enum : uint32_t { M_BOOL = RSI_BOOL, M_FIRST = RSI_FIRST_HIT, M_ALL = RSI_ALL_HITS, M_COUNT = RSI_COUNT };
// modes that must see every crossing (no early exit, no shrinking t limit)
constexpr uint32_t M_FULL = M_ALL | M_COUNT;

// Direction of the inside-test segments: (0.6, 0.41, 0.91) normalised, a
// direction not parallel to any axis or coordinate plane.
__constant__ float kInsideDir[3] = {0.515216053f, 0.352064312f, 0.781410992f};

struct QArgs {
    const Node *nodes;
    const Node4 *nodes4;  // four-way view (branching 4), else null
    const Tri *tris;
    int32_t n_tris;      // packed triangles (positions are checked against it before a re-solve)
    int32_t entry;
    const float *S;
    const float *E;
    int64_t n_items;     // work items of the main pass (segments, or (mesh, segment) pairs)
    QueryOut o;
    // all hits: overflow table, arena, pool (QueryOut) and their capacities
    int32_t *ovf_seg;
    int32_t *ovf_cnt;
    int64_t *ovf_off;
    int32_t *ovf_list;  // all hits: entries that are not void, in table order (kOvfValid of them)
    int64_t ovf_cap;
    int4 *arena;
    int64_t arena_cap;
    unsigned long long *ovf_part;  // all hits: per-part count sums of the pool-offset scan
    int32_t *scalars;
    Counters *counters;
    int32_t depth;       // stack entries per lane: the LDS part (main pass) or the height bound (deep pass)
    int32_t lds_depth;   // of which the first lds_depth live in LDS, the rest in gstack (deep pass)
    int32_t *gstack;     // deep pass: [(depth - lds_depth) x threads of the grid], laid out [entry][thread]
    int64_t gstack_cap;  // entries in gstack
    int32_t *retry_q;    // work items whose stack outgrew the main pass's LDS part
    int64_t retry_cap;
    int32_t max_steps;   // node records: a walk of a valid tree visits each at most once
    int32_t defer;       // test pending leaves once fewer lanes than this can step
    int32_t refill;      // fetch new segments once this many lanes are idle
    int32_t chunk;       // work items a wave claims per atomic on a range counter
    // batched queries: work item k belongs to mesh m with bt.seg_off[m] <= k < bt.seg_off[m+1]
    int32_t M;
    const int32_t *mesh_entry;
    BatchTables bt;
};

// Streaming accesses (segment ends in, results out).
template <typename T>
__device__ inline T ld_nt(const T *p) { return __builtin_nontemporal_load(p); }
template <typename T>
__device__ inline void st_nt(T *p, T v) { __builtin_nontemporal_store(v, p); }
typedef int32_t nt_i4 __attribute__((ext_vector_type(4)));
typedef float nt_f4 __attribute__((ext_vector_type(4)));
__device__ inline void st_nt4(int32_t *p, int32_t a, int32_t b, int32_t c, int32_t d)
{
    nt_i4 v = {a, b, c, d};
    __builtin_nontemporal_store(v, reinterpret_cast<nt_i4 *>(p));
}
__device__ inline void st_nt4(float *p, float a, float b, float c, float d)
{
    nt_f4 v = {a, b, c, d};
    __builtin_nontemporal_store(v, reinterpret_cast<nt_f4 *>(p));
}

__device__ inline void wave_add_u64(unsigned long long *dst, unsigned long long v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (__lane_id() == 0) atomicAdd(dst, v);
}

// Mask of the wave's active lanes whose predicate holds (the predicate
// stays a lane mask, never materialised as an integer per lane).
__device__ inline uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ inline uint32_t lanes_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// The four-way walk of a single mesh (boolean and counting modes) reads
// the records of the top three levels (the entry record, its internal
// children and theirs: at most 21) from a copy in LDS.  Every walk starts
// there, so these are the most visited records; served by LDS they leave
// the vector-memory path, which the walk keeps busy.  References at or above kTopRef name a record of the
// copy (internal references stay below 2^27).
constexpr int kTopNodes = 21;
constexpr int32_t kTopRef = 0x40000000;

// Modes that walk with the top copy: the boolean and counting walks.  The
// first-hit and all-hits walks go deeper on large meshes, and there the
// LDS entries the copy takes from the stack cost more than it saves.
constexpr bool top_copy(uint32_t mode) { return !(mode & (M_ALL | M_FIRST)); }

__device__ inline bool inner_ref(int32_t r) { return r >= 0 && r != kEmptySlot; }
__device__ inline int32_t ref_at(const int4 &c, int k) { return k == 0 ? c.x : (k == 1 ? c.y : (k == 2 ? c.z : c.w)); }

// Lane l < kTopNodes of the block's first wave fills slot l of the copy:
// slot 0 the entry record, slots 1..4 its children, slot 5 + 4k + j child j
// of slot 1 + k.  A slot whose record does not exist stays unused: no
// reference names it.  References between copied records are rewritten to
// kTopRef + slot.
__device__ inline void load_top(const Node4 *__restrict__ nodes4, int32_t entry, uint4 *top, int l)
{
    if (l >= kTopNodes || entry < 0) return;
    const int4 *rec = reinterpret_cast<const int4 *>(nodes4);
    const int4 c0 = rec[4 * (int64_t)entry + 3];
    int32_t id = -1;
    if (l == 0) {
        id = entry;
    } else if (l < 5) {
        const int32_t r = ref_at(c0, l - 1);
        id = inner_ref(r) ? r : -1;
    } else {
        const int32_t p = ref_at(c0, (l - 5) >> 2);
        if (inner_ref(p)) {
            const int32_t r = ref_at(rec[4 * (int64_t)p + 3], (l - 5) & 3);
            id = inner_ref(r) ? r : -1;
        }
    }
    if (id < 0) return;
    const uint4 *q = reinterpret_cast<const uint4 *>(nodes4 + id);
    int4 c = rec[4 * (int64_t)id + 3];
    if (l < 5) {
        const int32_t base = kTopRef + (l == 0 ? 1 : 5 + 4 * (l - 1));
        c.x = inner_ref(c.x) ? base : c.x;
        c.y = inner_ref(c.y) ? base + 1 : c.y;
        c.z = inner_ref(c.z) ? base + 2 : c.z;
        c.w = inner_ref(c.w) ? base + 3 : c.w;
    }
    top[4 * l] = q[0];
    top[4 * l + 1] = q[1];
    top[4 * l + 2] = q[2];
    top[4 * l + 3] = make_uint4((uint32_t)c.x, (uint32_t)c.y, (uint32_t)c.z, (uint32_t)c.w);
}

// All hits: overflow-table entries and arena records are handed out in
// blocks held by a wave (its next and end index in LDS), so the two counters
// that the whole GPU shares see one atomic per block rather than one per
// entry or crossing: atomics on one address are serialised device-wide, and
// at a few thousand per launch they already cost more than the walk's tests.
constexpr int32_t kEntBlock = 64;
constexpr int32_t kArenaBlock = 64;
constexpr int kXcds = 8;            // MI355X: 8 XCDs of 32 CUs, each with its own L2
constexpr int kWavesPerBlock = 4;   // the kernels' launch bound: 256 threads

// The XCD the calling wave runs on: hardware register XCC_ID, bits 3:0
// (s_getreg encoding: size - 1 in bits 15:11, offset in 10:6, register 20).
__device__ inline int xcd_id()
{
    return (int)(__builtin_amdgcn_s_getreg(((4 - 1) << 11) | (0 << 6) | 20) & (kXcds - 1));
}

// Per-lane query state for the segment it currently owns.
// All-hits capacities up to this many keep the hit list in registers.
constexpr int kRegSlots = 4;

struct Lane {
    Seg seg;
    float tlim;        // limit on t for boxes and triangles: 1, or just above the best t
    float best_t;
    int32_t best_id;
    int32_t best_pos;
    int32_t count;     // crossings found (all hits, count)
    int32_t e;         // all hits: overflow-table entry, -1 while count <= K
    int32_t item;      // work item (a segment, or a (mesh, segment) pair of a batch)
    int32_t seg_i;     // segment index (within its mesh for batched queries; below 2^30)
    const float *sp;   // this segment's start and end (3 floats each)
    const float *ep;
    int32_t mesh;      // batched queries: the segment's mesh
    int32_t hp0, hp1, hp2, hp3;  // all hits, capacity <= 4: the hit positions found so far
    bool found;
    bool retry;        // the stack outgrew the pass's stack: the deep pass walks this segment again
};

template <bool BATCH>
__device__ inline int32_t *slot_ids(const QArgs &a, const Lane &L) { return BATCH ? a.bt.ids[L.mesh] : a.o.ids; }
template <bool BATCH>
__device__ inline float *slot_ts(const QArgs &a, const Lane &L) { return BATCH ? a.bt.ts[L.mesh] : a.o.ts; }

// Void slot j of an overflow-table block (KIND 0: a negative count) or of
// an arena block (KIND 1: a record without entry).
template <int KIND>
__device__ inline void void_slot(const QArgs &a, int32_t j)
{
    if (KIND == 0) {
        if (j >= 0 && j < a.ovf_cap) a.ovf_cnt[j] = -1;
    } else {
        if (j >= 0 && j < a.arena_cap) a.arena[j] = make_int4(-1, 0, 0, 0);
    }
}

// Hand each active lane with `need` one slot of the block its wave holds
// (KIND 0: overflow-table entries, KIND 1: arena records); returns the slot,
// or -1 for a lane without `need`.  wst: the wave's (next, end) pairs in LDS,
// read by every active lane and written by one (LDS operations of a wave
// execute in order).  When the block cannot serve every requesting lane,
// the active lanes void its rest and the first claims a new block of
// kEntBlock / kArenaBlock slots (at least 64: one always suffices).
template <int KIND>
__device__ inline int32_t wave_take(const QArgs &a, volatile int32_t *wst, bool need)
{
    const uint64_t m = ballot(need);
    if (m == 0) return -1;
    const int32_t n = (int32_t)__popcll(m);
    const uint64_t act = ballot(true);
    const int leader = __builtin_ctzll(act);
    int32_t nxt = __builtin_amdgcn_readfirstlane(wst[2 * KIND]);
    int32_t end = __builtin_amdgcn_readfirstlane(wst[2 * KIND + 1]);
    if (nxt + n > end) {
        const int32_t na = (int32_t)__popcll(act);
        for (int32_t j = nxt + (int32_t)lanes_below(act); j < end; j += na) void_slot<KIND>(a, j);
        int32_t base = 0;
        if ((int)__lane_id() == leader)
            base = atomicAdd(&a.scalars[KIND == 0 ? kOvfSegs : kArenaLo], KIND == 0 ? kEntBlock : kArenaBlock);
        nxt = __builtin_amdgcn_readfirstlane(__shfl(base, leader, 64));
        end = nxt + (KIND == 0 ? kEntBlock : kArenaBlock);
    }
    if ((int)__lane_id() == leader) {
        wst[2 * KIND] = nxt + n;
        wst[2 * KIND + 1] = end;
    }
    return need ? nxt + (int32_t)lanes_below(m) : -1;
}

// A crossing of the lane's segment with the triangle at sorted position pos
// (original id `id`, parameter t): the first-hit candidate.
template <uint32_t MODE>
__device__ inline void take_first(Lane &L, float t, int32_t id, int32_t pos)
{
    if (t < L.best_t || (t == L.best_t && id < L.best_id)) {
        L.best_t = t;
        L.best_id = id;
        L.best_pos = pos;
        if (!(MODE & M_FULL)) L.tlim = fminf(1.0f, t * (1.0f + 0x1p-20f));
    }
}

// A crossing at sorted position pos, counted and (all hits) recorded: the
// first K positions in the lane's slots, the rest as arena records.
template <uint32_t MODE, bool BATCH>
__device__ inline void take_crossing(const QArgs &a, Lane &L, int32_t pos, volatile int32_t *wst)
{
    if ((MODE & M_COUNT) && !(MODE & M_ALL)) ++L.count;
    if (MODE & M_ALL) {
        const int32_t c = L.count++;
        const int32_t K = a.o.cap;
        if (c < K) {
            if (K <= kRegSlots) {
                // kept in registers until the segment is finished
                L.hp3 = L.hp2;
                L.hp2 = L.hp1;
                L.hp1 = L.hp0;
                L.hp0 = pos;
            } else {
                slot_ids<BATCH>(a, L)[(int64_t)L.seg_i * K + c] = pos;
            }
        } else {
            // past the slots: an arena record (entry, rank, position);
            // the segment's overflow-table entry is taken at its first
            const int32_t e = wave_take<0>(a, wst, c == K);
            if (c == K) L.e = e;
            const int32_t r = wave_take<1>(a, wst, true);
            if (L.e < a.ovf_cap && r >= 0 && r < a.arena_cap)
                a.arena[r] = make_int4(L.e, c, pos, 0);
            else
                atomicOr(&a.scalars[kOvfFull], 1);
        }
    }
}

// Test the triangles of one leaf; returns true when the lane may stop.
// wst: the wave's block state for all-hits overflow (see wave_take).
template <uint32_t MODE, bool BATCH, bool COUNT>
__device__ inline bool visit_leaf(const QArgs &a, Lane &L, int32_t ref, uint32_t &tests, volatile int32_t *wst)
{
    const int32_t first = leaf_first(ref);
    const int32_t cnt = leaf_count(ref);
    for (int32_t k = 0; k < cnt; ++k) {
        const int32_t pos = first + k;
        float v[9];
        int32_t id;
        tri_load(a.tris, pos, v, id);
        if (COUNT) ++tests;
        const float lim = (MODE & M_FULL) ? 1.0f : L.tlim;
        const MTHit h = mt_test(L.seg, v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7], v[8], lim);
        if (!h.hit) continue;
        L.found = true;
        if (MODE == M_BOOL) return true;
        if (MODE & M_FIRST) take_first<MODE>(L, h.tn / h.det, id, pos);
        take_crossing<MODE, BATCH>(a, L, pos, wst);
    }
    return false;
}

// Order the wave's LDS accesses on either side (its lanes exchange data
// through LDS).
__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Leaf phase of the four-way walk.  A lane holds up to four pending leaves
// (one per child slot of its last node); tested by their owners, a phase
// would take as many rounds as the busiest lane has leaves, with few lanes
// busy in each.  Instead the wave's pending (lane, leaf) pairs are gathered,
// slot by slot, into a queue of 64 in LDS and each lane tests one pair per
// round against the owner's segment (read from the owner's registers); the
// owners then take the outcomes back.  Pairs past the 64th wait for the next
// round.  The outcome of a leaf is the set of its triangles crossed (a bit
// mask) and, for the first hit, its best crossing in (t, id) order: the
// owner's results are the same as from testing its leaves itself, in any
// order.  The plain boolean query needs one bit per leaf and takes it from
// a ballot; the other modes get the outcome back through the queue entry.
template <uint32_t MODE>
using LeafEnt = typename std::conditional<MODE == M_BOOL, int2, int4>::type;

template <uint32_t MODE, bool BATCH, bool COUNT>
__device__ inline void leaf_phase4(const QArgs &a, Lane &L, int32_t &leaf0, int32_t &leaf1, int32_t &leaf2,
                                   int32_t &leaf3, int32_t &node, uint32_t &tests, volatile int32_t *wst,
                                   LeafEnt<MODE> *q, uint32_t &w_rounds, unsigned long long &w_lanes)
{
    const int32_t lane = (int32_t)__lane_id();
    for (;;) {
        const uint64_t b0 = ballot(leaf0 != 0), b1 = ballot(leaf1 != 0);
        const uint64_t b2 = ballot(leaf2 != 0), b3 = ballot(leaf3 != 0);
        const int32_t c0 = (int32_t)__popcll(b0), c1 = (int32_t)__popcll(b1);
        const int32_t c2 = (int32_t)__popcll(b2), c3 = (int32_t)__popcll(b3);
        const int32_t total = c0 + c1 + c2 + c3;
        if (total == 0) break;
        const int32_t p0 = (int32_t)lanes_below(b0);
        const int32_t p1 = c0 + (int32_t)lanes_below(b1);
        const int32_t p2 = c0 + c1 + (int32_t)lanes_below(b2);
        const int32_t p3 = c0 + c1 + c2 + (int32_t)lanes_below(b3);
        const bool in0 = leaf0 != 0 && p0 < 64, in1 = leaf1 != 0 && p1 < 64;
        const bool in2 = leaf2 != 0 && p2 < 64, in3 = leaf3 != 0 && p3 < 64;
        auto put = [&](bool in, int32_t p, int32_t ref) {
            if (!in) return;
            LeafEnt<MODE> e;
            e.x = ref;
            e.y = lane;
            q[p] = e;
        };
        put(in0, p0, leaf0);
        put(in1, p1, leaf1);
        put(in2, p2, leaf2);
        put(in3, p3, leaf3);
        wave_lds_sync();
        const int32_t n = total < 64 ? total : 64;
        const bool mine = lane < n;
        int2 ent = make_int2(0, lane);
        if (mine) {
            const LeafEnt<MODE> e = q[lane];
            ent = make_int2(e.x, e.y);
        }
        wave_lds_sync();
        if (COUNT) {
            ++w_rounds;
            w_lanes += (unsigned long long)n;
        }
        // the owner's segment and t limit
        const int32_t own = ent.y;
        Seg s;
        s.ox = __shfl(L.seg.ox, own, 64);
        s.oy = __shfl(L.seg.oy, own, 64);
        s.oz = __shfl(L.seg.oz, own, 64);
        s.dx = __shfl(L.seg.dx, own, 64);
        s.dy = __shfl(L.seg.dy, own, 64);
        s.dz = __shfl(L.seg.dz, own, 64);
        s.ix = s.iy = s.iz = 0.0f;
        float lim = (MODE & M_FULL) || MODE == M_BOOL ? 1.0f : __shfl(L.tlim, own, 64);
        uint32_t mask = 0;
        float bt = INFINITY;
        int32_t bid = 0x7FFFFFFF, bpos = -1;
        if (mine) {
            const int32_t first = leaf_first(ent.x);
            const int32_t cnt = leaf_count(ent.x);
            for (int32_t k = 0; k < cnt; ++k) {
                const int32_t pos = first + k;
                float v[9];
                int32_t id;
                tri_load(a.tris, pos, v, id);
                if (COUNT) ++tests;
                const MTHit h = mt_test(s, v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7], v[8], lim);
                if (!h.hit) continue;
                mask |= 1u << k;
                if (MODE == M_BOOL) break;
                if (MODE & M_FIRST) {
                    const float t = h.tn / h.det;
                    if (t < bt || (t == bt && id < bid)) {
                        bt = t;
                        bid = id;
                        bpos = pos;
                        if (!(MODE & M_FULL)) lim = fminf(1.0f, t * (1.0f + 0x1p-20f));
                    }
                }
            }
        }
        // outcomes back to the owners
        if constexpr (MODE == M_BOOL) {
            const uint64_t H = ballot(mask != 0);
            const bool hit = (in0 && ((H >> p0) & 1)) || (in1 && ((H >> p1) & 1)) || (in2 && ((H >> p2) & 1)) ||
                             (in3 && ((H >> p3) & 1));
            if (hit) {
                L.found = true;
                leaf0 = leaf1 = leaf2 = leaf3 = 0;
                node = -1;
            }
        } else {
            // each lane's outcome replaces the entry it tested
            q[lane] = make_int4((int32_t)mask, __float_as_int(bt), bid, bpos);
            wave_lds_sync();
            // the owner's outcomes; all hits: then its crossings, one per
            // iteration (the recording code appears once)
            uint32_t m0 = 0, m1 = 0, m2 = 0, m3 = 0;
            auto back = [&](bool in, int32_t p, uint32_t &m) {
                if (!in) return;
                const int4 r = q[p];
                m = (uint32_t)r.x;
                if (m == 0) return;
                L.found = true;
                if (MODE & M_FIRST) take_first<MODE>(L, __int_as_float(r.y), r.z, r.w);
                if ((MODE & M_COUNT) && !(MODE & M_ALL)) L.count += (int32_t)__popc(m);
            };
            back(in0, p0, m0);
            back(in1, p1, m1);
            back(in2, p2, m2);
            back(in3, p3, m3);
            wave_lds_sync();
            if constexpr ((MODE & M_ALL) != 0) {
                while ((m0 | m1 | m2 | m3) != 0) {
                    int32_t pos;
                    if (m0) {
                        pos = leaf_first(leaf0) + (int32_t)__builtin_ctz(m0);
                        m0 &= m0 - 1;
                    } else if (m1) {
                        pos = leaf_first(leaf1) + (int32_t)__builtin_ctz(m1);
                        m1 &= m1 - 1;
                    } else if (m2) {
                        pos = leaf_first(leaf2) + (int32_t)__builtin_ctz(m2);
                        m2 &= m2 - 1;
                    } else {
                        pos = leaf_first(leaf3) + (int32_t)__builtin_ctz(m3);
                        m3 &= m3 - 1;
                    }
                    take_crossing<MODE, BATCH>(a, L, pos, wst);
                }
            }
        }
        if (in0) leaf0 = 0;
        if (in1) leaf1 = 0;
        if (in2) leaf2 = 0;
        if (in3) leaf3 = 0;
    }
}

// Write the results of a finished segment (or queue it for the deep pass).
template <uint32_t MODE, bool RETRY, bool BATCH>
__device__ inline void finish(const QArgs &a, const Lane &L)
{
    if (!RETRY && L.retry) {
        const int32_t r = atomicAdd(&a.scalars[kRetryN], 1);
        if (r < a.retry_cap) a.retry_q[r] = L.item;
        else atomicOr(&a.scalars[kRetryLost], 1);
        // the records this walk left in the arena are void: the deep pass
        // takes a new overflow entry
        if ((MODE & M_ALL) && L.e >= 0 && L.e < a.ovf_cap) a.ovf_cnt[L.e] = -1;
        return;
    }
    const int64_t i = L.seg_i;
    if (MODE & M_BOOL) {
        uint8_t *hit = BATCH ? a.bt.hit[L.mesh] : a.o.hit;
        st_nt(hit + i, (uint8_t)(L.found ? 1 : 0));
    }
    if (MODE & M_FIRST) {
        int32_t *tri = BATCH ? a.bt.tri[L.mesh] : a.o.tri;
        float *tt = BATCH ? a.bt.t[L.mesh] : a.o.t;
        float *uv = BATCH ? a.bt.uv[L.mesh] : a.o.uv;
        float *pt = BATCH ? a.bt.point[L.mesh] : a.o.point;
        // the hit's sorted position, or -1: k_refine_first (in segment
        // order, so its stores fill whole lines) re-solves a hit and writes
        // the id, t, (u, v) and the point, or writes the miss values
        (void)tt;
        (void)uv;
        (void)pt;
        tri[i] = L.best_pos >= 0 ? L.best_pos : -1;
    }
    if ((MODE & M_COUNT) && !(MODE & M_ALL)) st_nt(a.o.count + i, L.count);
    if (MODE & M_ALL) {
        const int K = a.o.cap;
        int32_t *cnt_out = BATCH ? a.bt.count[L.mesh] : a.o.count;
        int64_t *soff = BATCH ? a.bt.spill_off[L.mesh] : a.o.spill_off;
        st_nt(cnt_out + i, L.count);
        int32_t *ids = slot_ids<BATCH>(a, L) + i * K;
        float *ts = slot_ts<BATCH>(a, L) + i * K;
        // The walk writes only the hits' sorted positions (the first K,
        // kept in registers up to four, else already in the slots):
        // k_refine_slots, running in segment order, re-solves them, orders
        // them by (t, id), pads the slots and writes the spill offset, with
        // stores that fill whole lines (stores from here land wherever the
        // finishing lanes' segments lie, each a partial line).  A segment
        // with more than K crossings also fills in its overflow-table entry;
        // the pool offsets are taken by a scan after the walk.
        if (L.count >= 1 && K <= kRegSlots) {
            const int32_t hp[kRegSlots] = {L.hp0, L.hp1, L.hp2, L.hp3};
            const bool vec = K == kRegSlots && (reinterpret_cast<uintptr_t>(ids) & 15) == 0;
            if (vec) {
                st_nt4(ids, hp[0], L.count > 1 ? hp[1] : -1, L.count > 2 ? hp[2] : -1, L.count > 3 ? hp[3] : -1);
            } else {
#pragma unroll
                for (int c = 0; c < kRegSlots; ++c)
                    if (c < L.count && c < K) ids[c] = hp[c];
            }
        }
        if (L.count > K) {
            if (L.e >= 0 && L.e < a.ovf_cap) {
                a.ovf_seg[L.e] = L.item;
                a.ovf_cnt[L.e] = L.count;
            } else {
                // no entry (a full table, reported): the slots say so (the count stays exact)
                atomicOr(&a.scalars[kOvfFull], 1);
                for (int c = 0; c < K; ++c) {
                    ids[c] = -1;
                    ts[c] = INFINITY;
                }
                if (soff) st_nt(soff + i, (int64_t)-1);
            }
        }
    }
}

// RETRY: the deep pass.  Work items come from the retry queue (its length
// is read on the device), and the stack continues past its LDS part into
// device memory up to a bound on the tree height, so it never outgrows it
// in a valid tree.  WIDE: walk the four-way view (Node4 records) instead of
// the binary nodes; leaves and triangles are the same, so are the results.
// The all-hits variants are held to six waves per SIMD (80 VGPRs): without
// the bound the compiler gives them 94 and five waves.
template <uint32_t MODE, bool RETRY, bool COUNT, bool BATCH, bool WIDE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu((MODE & M_ALL) ? 6 : 1))) void k_query(QArgs a)
{
    constexpr bool HYB = RETRY;
    // the deep pass is launched after every main pass; with nothing queued
    // (the usual case) every workgroup leaves before touching memory
    if (RETRY && a.scalars[kRetryN] == 0) return;
    extern __shared__ int32_t lds_dyn[];
    int32_t *const lds_stack = lds_dyn;
    constexpr bool TOP = WIDE && !BATCH && top_copy(MODE);
    __shared__ uint4 top4[TOP ? 4 * kTopNodes : 4];
    if constexpr (TOP) {
        if (threadIdx.x < 64) load_top(a.nodes4, a.entry, top4, threadIdx.x);
        __syncthreads();
    }
    int32_t *const stk = lds_stack + threadIdx.x;
    const int stride = blockDim.x;
    // work claiming: the main pass's items are cut into eight contiguous
    // ranges, one per XCD, each with its own counter on its own 128-byte
    // line; a wave takes chunks from its XCD's range first, then from the
    // others in turn.  A single counter line shared by all XCDs serialises
    // the claims in the memory fabric (measured: 0.83 against 0.69 ms for
    // the 10M-segment boolean query); with the ranges each XCD also walks
    // its own part of spatially ordered items.  The deep pass has one range.
    constexpr int kRanges = RETRY ? 1 : kXcds;
    int32_t *const work = &a.scalars[RETRY ? kWorkRetry : kWorkXcd];
    int range = RETRY ? 0 : xcd_id();  // wave-uniform
    int ranges_left = kRanges;
    // stack entry k >= lds_depth lives at gstack[(k - lds_depth) * gstride + gtid]
    const int64_t gstride = (int64_t)gridDim.x * blockDim.x;
    const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;

    // a lane's state starts defined: the leaf phase reads any lane's segment
    // and t limit with shuffles, including lanes that never take an item
    Lane L = {};
    L.tlim = 1.0f;
    L.retry = false;
    L.e = -1;
    // all hits: the wave's blocks of overflow-table entries and arena
    // records, (next, end) each, none held at first
    __shared__ int32_t wave_blocks[(MODE & M_ALL) ? 4 * kWavesPerBlock : 1];
    // four-way walk: the wave's leaf queue, past the stack's LDS part
    LeafEnt<MODE> *const leafq =
        reinterpret_cast<LeafEnt<MODE> *>(lds_dyn + (size_t)a.lds_depth * blockDim.x) + 64 * (threadIdx.x >> 6);
    volatile int32_t *const wst = wave_blocks + ((MODE & M_ALL) ? 4 * (threadIdx.x >> 6) : 0);
    if ((MODE & M_ALL) && __lane_id() == 0) {
        wst[0] = wst[1] = 0;
        wst[2] = wst[3] = 0;
    }
    // work items number below 2^30 (checked at the boundary), so item and
    // chunk arithmetic is 32-bit; the chunk bounds are wave-uniform
    int32_t item = -1;   // >= 0 owned work item; -1 idle; -2 no work left
    int32_t node = -1;   // next node to visit; < 0: none
    // stack pointer kept as an element offset into the [depth][lane] LDS
    // array (entries x stride), so a push or pop needs no multiply
    int32_t sp = 0;
    // without a global part the stack pointer is the LDS address of the
    // next free entry (a push or pop is one add)
    int32_t *sptr = stk;
    int32_t *const stk_end = stk + a.depth * stride;
    const int32_t depth_off = a.depth * stride;
    const int32_t lds_off = a.lds_depth * stride;
    // pending leaf references (leaf refs are negative; 0 = none): filled in
    // order in the binary walk, by child slot in the four-way walk
    int32_t leaf0 = 0, leaf1 = 0, leaf2 = 0, leaf3 = 0;
    // bound on a walk (a damaged tree can give wrong answers, never a hang):
    // each lane counts the node records it visits for its current segment; a
    // walk of a valid tree visits every record at most once, so a count past
    // the number of records can only come from a damaged tree.  Lanes check
    // their count every 64 node-step rounds of the wave (behind a
    // wave-uniform branch); a lane past the bound stops its walk and flags it.
    int32_t wround = 0;      // wave-uniform
    int32_t vis = 0;
    uint32_t visits = 0, boxes = 0, tests = 0, segs = 0;
    uint32_t w_loops = 0, w_steps = 0, w_leaf = 0, w_refill = 0;  // wave-uniform
    unsigned long long w_blocked = 0, w_waiting = 0;               // wave-uniform
    uint32_t w_lrounds = 0;                                        // wave-uniform
    unsigned long long w_llanes = 0;                               // wave-uniform
    int32_t chunk_next = 0, chunk_end = 0;  // the wave's claimed, not yet handed out items
    int32_t n_items = (int32_t)a.n_items;
    if (RETRY) {
        const int32_t q = a.scalars[kRetryN];
        n_items = q < (int32_t)a.retry_cap ? q : (int32_t)a.retry_cap;
    }
    bool exhausted = false;                 // every range's counter has passed its last item

    for (;;) {
        // ---- lanes whose walk is over write their results and take a new
        // work item, batched: only once `refill` lanes are waiting (or no
        // lane can make progress), so the epilogue and the segment set-up run
        // with many lanes at once.  Items come from the wave's chunk; a new
        // chunk is claimed from a range counter with one atomic.
        if (COUNT) ++w_loops;
        const bool done = item >= 0 && node < 0 && (WIDE ? (leaf0 | leaf1 | leaf2 | leaf3) == 0 : leaf0 == 0);
        const uint64_t waiting = ballot(done || item == -1);
        if (waiting != 0 &&
            ((int)__popcll(waiting) >= a.refill || ballot(item >= 0 && !done) == 0)) {
            if (COUNT) ++w_refill;
            if (done) {
                finish<MODE, RETRY, BATCH>(a, L);
                item = -1;
            }
            const uint64_t idle = ballot(item == -1);
            const int32_t n_idle = (int32_t)__popcll(idle);
            const int32_t rank = (int32_t)lanes_below(idle);
            int32_t k = -1;
            const int32_t avail = chunk_end - chunk_next;
            const int32_t used = avail < n_idle ? avail : n_idle;
            if (rank < used) k = chunk_next + rank;
            chunk_next += used;
            if (used < n_idle && !exhausted) {
                const int leader = __builtin_ctzll(idle);
                for (;;) {
                    const int32_t lo = (int32_t)((int64_t)n_items * range / kRanges);
                    const int32_t hi = (int32_t)((int64_t)n_items * (range + 1) / kRanges);
                    int32_t base = 0;
                    if ((int)__lane_id() == leader) base = atomicAdd(work + kWorkStride * range, a.chunk);
                    base = __builtin_amdgcn_readfirstlane(__shfl(base, leader, 64));
                    if (base < hi - lo) {
                        chunk_next = lo + base;
                        chunk_end = hi - chunk_next > a.chunk ? chunk_next + a.chunk : hi;
                        const int32_t room = chunk_end - chunk_next;
                        const int32_t more = n_idle - used < room ? n_idle - used : room;
                        if (rank >= used && rank - used < more) k = chunk_next + (rank - used);
                        chunk_next += more;
                        break;
                    }
                    // this range is used up: the next one
                    if (--ranges_left == 0) {
                        exhausted = true;
                        break;
                    }
                    range = range + 1 == kRanges ? 0 : range + 1;
                }
            }
            if (item == -1) {
                if (k >= 0) {
                    item = k;
                    const int32_t it = RETRY ? a.retry_q[k] : k;
                    int32_t i = it;
                    int32_t entry = (TOP && a.entry >= 0) ? kTopRef : a.entry;
                    if (BATCH) {
                        const int32_t m = mesh_of(a.bt.seg_off, a.M, it);
                        i = (int32_t)(it - a.bt.seg_off[m]);
                        L.mesh = m;
                        L.sp = a.bt.S[m] + 3 * (int64_t)i;
                        L.ep = a.bt.E[m] + 3 * (int64_t)i;
                        entry = a.mesh_entry[m];
                    } else {
                        L.mesh = 0;
                        L.sp = a.S + 3 * (int64_t)i;
                        L.ep = a.E + 3 * (int64_t)i;
                    }
                    L.item = it;
                    L.seg_i = i;
                    L.seg = make_seg(ld_nt(L.sp), ld_nt(L.sp + 1), ld_nt(L.sp + 2), ld_nt(L.ep), ld_nt(L.ep + 1),
                                     ld_nt(L.ep + 2));
                    L.tlim = 1.0f;
                    L.best_t = INFINITY;
                    L.best_id = 0x7FFFFFFF;
                    L.best_pos = -1;
                    L.count = 0;
                    L.e = -1;
                    L.found = false;
                    L.retry = false;
                    node = entry;  // < 0 for an empty mesh: the segment misses
                    sp = 0;
                    sptr = stk;
                    vis = 0;
                    if (COUNT && !RETRY) ++segs;
                } else if (exhausted) {
                    item = -2;
                }
            }
        }
        if (ballot(item >= 0) == 0) break;

        // a push that does not fit: in the main pass the walk stops and its
        // segment goes to the deep pass; in the deep pass (a damaged tree
        // only) the entry is dropped and flagged
        auto overflow = [&]() {
            if constexpr (RETRY) {
                atomicOr(&a.scalars[kStackDropped], 1);
            } else {
                L.retry = true;
            }
        };
        auto push = [&](bool cond, int32_t child) {
            if constexpr (!HYB) {
                if (cond) {
                    if (sptr < stk_end) {
                        *sptr = child;
                        sptr += stride;
                    } else {
                        overflow();
                    }
                }
            } else if (cond) {
                if (sp < depth_off) {
                    if (sp < lds_off) stk[sp] = child;
                    else a.gstack[(int64_t)((sp - lds_off) / stride) * gstride + gtid] = child;
                    sp += stride;
                } else {
                    overflow();
                }
            }
        };
        auto pop = [&]() -> int32_t {
            if constexpr (!HYB) {
                if (sptr <= stk) return -1;
                sptr -= stride;
                return *sptr;
            } else {
                if (sp <= 0) return -1;
                sp -= stride;
                if (sp < lds_off) return stk[sp];
                return a.gstack[(int64_t)((sp - lds_off) / stride) * gstride + gtid];
            }
        };
        // ---- node steps for every lane that has a node and at most one
        // pending leaf: a lane keeps walking past the first leaf it finds
        // (speculatively, the leaf may end the walk) so that leaf tests are
        // batched over more lanes and fewer lanes sit idle in node steps.
        // Steps repeat without the refill and leaf-phase checks while at
        // least `defer` lanes step; pending leaves are tested after the first
        // step made by fewer lanes.
        auto can_step = [&]() {
            return node >= 0 && (WIDE ? (leaf0 | leaf1 | leaf2 | leaf3) == 0 : leaf1 == 0);
        };
        uint64_t w;
        do {
            const bool want = can_step();
            // the two conditions' masks, each straight from its compare
            w = ballot(node >= 0) & ballot(WIDE ? (leaf0 | leaf1 | leaf2 | leaf3) == 0 : leaf1 == 0);
            if (w == 0) break;
            if (COUNT) {
                ++w_steps;
                const uint64_t has_node = ballot(node >= 0);
                w_blocked += (unsigned long long)__popcll(has_node & ~w);
                w_waiting += (unsigned long long)(64 - __popcll(has_node));
            }
            if constexpr (WIDE) {
              if (want) {
                ++vis;
                uint4 P, Q, R;
                int4 C;
                if (TOP && node >= kTopRef) {
                    const uint4 *t = top4 + 4 * (node - kTopRef);
                    P = t[0];
                    Q = t[1];
                    R = t[2];
                    const uint4 c = t[3];
                    C = make_int4((int32_t)c.x, (int32_t)c.y, (int32_t)c.z, (int32_t)c.w);
                } else {
                    const uint4 *q = reinterpret_cast<const uint4 *>(a.nodes4 + node);
                    P = q[0];
                    Q = q[1];
                    R = q[2];
                    C = reinterpret_cast<const int4 *>(a.nodes4 + node)[3];
                }
                const float lim = ((MODE & M_FIRST) && !(MODE & M_FULL) ? L.tlim : 1.0f) * (1.0f + 0x1p-20f);
                // grid steps, the corner's offset from the segment origin and
                // the margin that makes the plane evaluation conservative
                const float sx = __uint_as_float(R.z), sy = __uint_as_float(R.w), sz = __uint_as_float(P.w);
                const float Dx = __uint_as_float(P.x) - L.seg.ox;
                const float Dy = __uint_as_float(P.y) - L.seg.oy;
                const float Dz = __uint_as_float(P.z) - L.seg.oz;
                // per axis the plane met first: the lower one for a
                // non-negative direction component; the margin moves it
                // toward the segment origin and the other plane away
                const bool px = L.seg.ix >= 0.0f, py = L.seg.iy >= 0.0f, pz = L.seg.iz >= 0.0f;
                const float mx = fmaf(255.0f, sx, fabsf(Dx)) * (px ? 0x1p-19f : -0x1p-19f);
                const float my = fmaf(255.0f, sy, fabsf(Dy)) * (py ? 0x1p-19f : -0x1p-19f);
                const float mz = fmaf(255.0f, sz, fabsf(Dz)) * (pz ? 0x1p-19f : -0x1p-19f);
                // plane q of an axis lies at parameter fma(q, a, b)
                const float ax = sx * L.seg.ix, ay = sy * L.seg.iy, az = sz * L.seg.iz;
                const float bnx = (Dx - mx) * L.seg.ix, bny = (Dy - my) * L.seg.iy, bnz = (Dz - mz) * L.seg.iz;
                const float bfx = (Dx + mx) * L.seg.ix, bfy = (Dy + my) * L.seg.iy, bfz = (Dz + mz) * L.seg.iz;
                // child c: lower planes in byte c of Q.x, Q.y, Q.z, upper
                // planes in byte c of Q.w, R.x, R.y
                const uint32_t nqx = px ? Q.x : Q.w, fqx = px ? Q.w : Q.x;
                const uint32_t nqy = py ? Q.y : R.x, fqy = py ? R.x : Q.y;
                const uint32_t nqz = pz ? Q.z : R.y, fqz = pz ? R.y : Q.z;
                auto qb = [](uint32_t v, int c) { return (float)((v >> (8 * c)) & 0xFFu); };
                auto test = [&](int c, float &t) {
                    return qslab_hit(ax, ay, az, bnx, bny, bnz, bfx, bfy, bfz, qb(nqx, c), qb(nqy, c), qb(nqz, c),
                                     qb(fqx, c), qb(fqy, c), qb(fqz, c), lim, t);
                };
                float t0, t1, t2, t3;
                const bool h0 = test(0, t0) && C.x != kEmptySlot;
                const bool h1 = test(1, t1) && C.y != kEmptySlot;
                const bool h2 = test(2, t2) && C.z != kEmptySlot;
                const bool h3 = test(3, t3) && C.w != kEmptySlot;
                if (COUNT) {
                    ++visits;
                    boxes += (C.x != kEmptySlot) + (C.y != kEmptySlot) + (C.z != kEmptySlot) + (C.w != kEmptySlot);
                }
                leaf0 = (h0 && C.x < 0) ? C.x : 0;
                leaf1 = (h1 && C.y < 0) ? C.y : 0;
                leaf2 = (h2 && C.z < 0) ? C.z : 0;
                leaf3 = (h3 && C.w < 0) ? C.w : 0;
                const bool g0 = h0 && C.x >= 0, g1 = h1 && C.y >= 0, g2 = h2 && C.z >= 0, g3 = h3 && C.w >= 0;
                // descend into the nearest internal child that was hit; push the others
                float bt = INFINITY;
                int32_t near = -1;
                if (g0) { bt = t0; near = C.x; }
                if (g1 && t1 < bt) { bt = t1; near = C.y; }
                if (g2 && t2 < bt) { bt = t2; near = C.z; }
                if (g3 && t3 < bt) { bt = t3; near = C.w; }
                const bool p0 = g0 && C.x != near, p1 = g1 && C.y != near;
                const bool p2 = g2 && C.z != near, p3 = g3 && C.w != near;
                // at most three pushes (the nearest child is taken, not
                // pushed): with room for three more entries in LDS every
                // child is written at the top and the top advances past the
                // pushed ones only (a write past them lands in a free slot)
                bool room;
                if constexpr (HYB) room = sp + 3 * stride < lds_off;
                else room = sptr + 3 * stride < stk_end;
                if (room && HYB) {
                    stk[sp] = C.x;
                    sp += p0 ? stride : 0;
                    stk[sp] = C.y;
                    sp += p1 ? stride : 0;
                    stk[sp] = C.z;
                    sp += p2 ? stride : 0;
                    stk[sp] = C.w;
                    sp += p3 ? stride : 0;
                } else if (room) {
                    *sptr = C.x;
                    sptr += p0 ? stride : 0;
                    *sptr = C.y;
                    sptr += p1 ? stride : 0;
                    *sptr = C.z;
                    sptr += p2 ? stride : 0;
                    *sptr = C.w;
                    sptr += p3 ? stride : 0;
                } else {
                    push(p0, C.x);
                    push(p1, C.y);
                    push(p2, C.z);
                    push(p3, C.w);
                }
                node = near >= 0 ? near : pop();
                if (!RETRY && L.retry) {
                    // the stack is full: stop here, the deep pass takes over
                    node = -1;
                    leaf0 = leaf1 = leaf2 = leaf3 = 0;
                }
              }
            } else if (want) {
                ++vis;
                const float4 *q = reinterpret_cast<const float4 *>(a.nodes + node);
                const float4 q0 = q[0], q1 = q[1], q2 = q[2];
                const int4 q3 = reinterpret_cast<const int4 *>(a.nodes + node)[3];
                const float lim = (MODE & M_FIRST) && !(MODE & M_FULL) ? L.tlim : 1.0f;
                float tl, tr;
                const bool hl = slab_hit(L.seg, q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, lim, tl);
                const bool hr = slab_hit(L.seg, q1.z, q1.w, q2.x, q2.y, q2.z, q2.w, lim, tr);
                if (COUNT) {
                    ++visits;
                    boxes += 2;
                }
                const int32_t cl = q3.x, cr = q3.y;
                // add the hit leaf children to the pending list, kept in
                // ascending order: references are negative and 0 marks a free
                // slot, so the pending entries come first (at most one is
                // pending here, so three slots suffice); the order in which a
                // lane tests its leaves changes no result
                const int32_t n0 = (hl && cl < 0) ? cl : 0;
                const int32_t n1 = (hr && cr < 0) ? cr : 0;
                const int32_t lo01 = min(n0, n1), hi01 = max(n0, n1);
                leaf2 = max(leaf0, hi01);
                leaf1 = max(min(leaf0, hi01), lo01);
                leaf0 = min(leaf0, lo01);
                const bool gl = hl && cl >= 0;
                const bool gr = hr && cr >= 0;
                // descend into the nearer internal child that was hit; push the
                // other one when both were
                const bool take_l = gl && (!gr || tl <= tr);
                push(gl && gr, take_l ? cr : cl);
                node = (gl || gr) ? (take_l ? cl : cr) : pop();
                if (!RETRY && L.retry) {
                    node = -1;
                    leaf0 = leaf1 = leaf2 = 0;
                }
            }
            if (__builtin_expect((++wround & 63) == 0, 0)) {
                if (vis > a.max_steps) {
                    node = -1;
                    atomicOr(&a.scalars[kWalkCut], 1);
                }
            }
        } while ((int)__popcll(w) >= a.defer);

        // ---- test pending leaves once few lanes can still step
        const uint64_t pend = ballot(WIDE ? (leaf0 | leaf1 | leaf2 | leaf3) != 0 : leaf0 != 0);
        if (pend != 0) {
            if (COUNT) ++w_leaf;
            if constexpr (WIDE && !(MODE & M_ALL)) {
                leaf_phase4<MODE, BATCH, COUNT>(a, L, leaf0, leaf1, leaf2, leaf3, node, tests, wst, leafq,
                                                w_lrounds, w_llanes);
            } else if constexpr (WIDE) {
                // all hits: one pending leaf per lane and round, the first
                // occupied slot (the gathered phase needs more registers
                // than these variants have)
                do {
                    const int32_t cur = leaf0 ? leaf0 : (leaf1 ? leaf1 : (leaf2 ? leaf2 : leaf3));
                    if (COUNT) {
                        ++w_lrounds;
                        w_llanes += (unsigned long long)__popcll(ballot(cur != 0));
                    }
                    if (cur != 0) {
                        visit_leaf<MODE, BATCH, COUNT>(a, L, cur, tests, wst);
                        if (leaf0 == cur) {
                            leaf0 = 0;
                        } else if (leaf1 == cur) {
                            leaf1 = 0;
                        } else if (leaf2 == cur) {
                            leaf2 = 0;
                        } else {
                            leaf3 = 0;
                        }
                    }
                } while (ballot((leaf0 | leaf1 | leaf2 | leaf3) != 0) != 0);
            } else do {
                if (COUNT) {
                    ++w_lrounds;
                    w_llanes += (unsigned long long)__popcll(ballot(leaf0 != 0));
                }
                if (leaf0 != 0) {
                    const bool stop = visit_leaf<MODE, BATCH, COUNT>(a, L, leaf0, tests, wst);
                    leaf0 = stop ? 0 : leaf1;
                    leaf1 = stop ? 0 : leaf2;
                    leaf2 = 0;
                    if (stop) node = -1;
                }
            } while (ballot(leaf0 != 0) != 0);
        }

    }
    if constexpr ((MODE & M_ALL) != 0) {
        // every lane of the wave is here: void the unused rest of the wave's
        // blocks (the offset scan and k_spill_finish skip an entry whose
        // count is negative, k_spill_place a record without entry)
        const int32_t lane = (int32_t)__lane_id();
        for (int32_t j = wst[0] + lane; j < wst[1]; j += 64) void_slot<0>(a, j);
        for (int32_t j = wst[2] + lane; j < wst[3]; j += 64) void_slot<1>(a, j);
    }
    if (COUNT) {
        wave_add_u64(&a.counters->node_visits, visits);
        wave_add_u64(&a.counters->box_tests, boxes);
        wave_add_u64(&a.counters->tri_tests, tests);
        wave_add_u64(&a.counters->segments, segs);
        if (__lane_id() == 0) {
            atomicAdd(&a.counters->wave_loops, (unsigned long long)w_loops);
            atomicAdd(&a.counters->wave_node_steps, (unsigned long long)w_steps);
            atomicAdd(&a.counters->wave_leaf_phases, (unsigned long long)w_leaf);
            atomicAdd(&a.counters->wave_refills, (unsigned long long)w_refill);
            atomicAdd(&a.counters->lanes_blocked, w_blocked);
            atomicAdd(&a.counters->lanes_waiting, w_waiting);
            atomicAdd(&a.counters->wave_leaf_rounds, (unsigned long long)w_lrounds);
            atomicAdd(&a.counters->leaf_lanes, w_llanes);
        }
    }
}

// Segment and output arrays of work item `it` (a segment of a single mesh,
// or a (mesh, segment) pair of a batch).
template <bool BATCH>
struct ItemView {
    int64_t i;
    const float *S, *E;
    int32_t *ids;
    float *ts;
};
template <bool BATCH>
__device__ inline ItemView<BATCH> item_view(const QArgs &a, int64_t it)
{
    ItemView<BATCH> v;
    if (BATCH) {
        const int32_t m = mesh_of(a.bt.seg_off, a.M, it);
        v.i = it - a.bt.seg_off[m];
        v.S = a.bt.S[m];
        v.E = a.bt.E[m];
        v.ids = a.bt.ids[m];
        v.ts = a.bt.ts[m];
    } else {
        v.i = it;
        v.S = a.S;
        v.E = a.E;
        v.ids = a.o.ids;
        v.ts = a.o.ts;
    }
    return v;
}

// All hits, after the walk: pool offsets of the overflowed segments' full
// lists, the exclusive prefix sums of their counts in table order (a void
// entry counts 0), so the lists fill the pool contiguously, in exactly the
// entries they need.  The table [0, n) is cut into kOvfParts contiguous
// parts (n is read on the device): k_ovf_sums adds up each part's counts,
// k_ovf_scan_parts scans the part sums in one workgroup, and
// k_ovf_offsets scans each part again from its base.
constexpr int kOvfParts = 1024;

__device__ inline int64_t ovf_entries(const QArgs &a)
{
    const int32_t ne = a.scalars[kOvfSegs];
    return ne < a.ovf_cap ? ne : a.ovf_cap;
}

// Sum over the 256 threads of a workgroup (every thread gets it).
__device__ inline unsigned long long block_sum256(unsigned long long v, unsigned long long *sh)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (__lane_id() == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    const unsigned long long t = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
    return t;
}

// The scans run over one 64-bit value per entry: the entry's crossings in
// the low 40 bits (the pool is far smaller) and 1 above them for an entry
// that is not void, so one pass yields pool offsets and list positions.
constexpr int kOvfCrossBits = 40;
constexpr unsigned long long kOvfCrossMask = (1ull << kOvfCrossBits) - 1;
__device__ inline unsigned long long ovf_packed(int32_t c)
{
    return c > 0 ? (1ull << kOvfCrossBits) + (unsigned long long)c : 0ull;
}

__global__ __launch_bounds__(256) void k_ovf_sums(QArgs a)
{
    __shared__ unsigned long long sh[4];
    const int64_t n = ovf_entries(a);
    const int64_t chunk = (n + kOvfParts - 1) / kOvfParts;
    const int64_t lo = (int64_t)blockIdx.x * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    unsigned long long v = 0;
    for (int64_t e = lo + threadIdx.x; e < hi; e += 256) v += ovf_packed(a.ovf_cnt[e]);
    v = block_sum256(v, sh);
    if (threadIdx.x == 0) a.ovf_part[blockIdx.x] = v;
}

__global__ __launch_bounds__(kOvfParts) void k_ovf_scan_parts(QArgs a)
{
    __shared__ unsigned long long sh[kOvfParts / 64];
    const int tid = threadIdx.x;
    const unsigned long long mine = a.ovf_part[tid];
    unsigned long long incl = mine;
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned long long u = __shfl_up(incl, off, 64);
        if ((int)__lane_id() >= off) incl += u;
    }
    if (__lane_id() == 63) sh[tid >> 6] = incl;
    __syncthreads();
    unsigned long long before = 0;
    for (int w = 0; w < (tid >> 6); ++w) before += sh[w];
    a.ovf_part[tid] = before + incl - mine;
    if (tid == kOvfParts - 1) {
        const unsigned long long tot = (before + incl) & kOvfCrossMask;
        a.scalars[kOvfTotalLo] = (int32_t)(uint32_t)tot;
        a.scalars[kOvfTotalHi] = (int32_t)(uint32_t)(tot >> 32);
        a.scalars[kOvfValid] = (int32_t)((before + incl) >> kOvfCrossBits);
    }
}

// Per entry: its pool offset; its first min(K, count) positions (in its
// segment's slots) go to the head of its range, and its spill offset is
// written.  A list the pool cannot hold is reported (the count stays exact)
// and its slots say so.
template <bool BATCH>
__global__ __launch_bounds__(256) void k_ovf_offsets(QArgs a)
{
    __shared__ unsigned long long sh[4];
    const int64_t n = ovf_entries(a);
    const int64_t chunk = (n + kOvfParts - 1) / kOvfParts;
    const int64_t lo = (int64_t)blockIdx.x * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    const int K = a.o.cap;
    unsigned long long base = a.ovf_part[blockIdx.x];
    for (int64_t t0 = lo; t0 < hi; t0 += 256) {
        const int64_t e = t0 + threadIdx.x;
        const int32_t c = e < hi ? a.ovf_cnt[e] : -1;
        const unsigned long long mine = ovf_packed(c);
        // exclusive scan of the tile's counts
        unsigned long long incl = mine;
        for (int off = 1; off < 64; off <<= 1) {
            const unsigned long long u = __shfl_up(incl, off, 64);
            if ((int)__lane_id() >= off) incl += u;
        }
        if (__lane_id() == 63) sh[threadIdx.x >> 6] = incl;
        __syncthreads();
        unsigned long long before = 0;
        for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) before += sh[w];
        const unsigned long long tile = sh[0] + sh[1] + sh[2] + sh[3];
        __syncthreads();
        if (c > 0) {
            const ItemView<BATCH> v = item_view<BATCH>(a, a.ovf_seg[e]);
            int64_t *soff = BATCH ? a.bt.spill_off[mesh_of(a.bt.seg_off, a.M, a.ovf_seg[e])] : a.o.spill_off;
            int32_t *ids = v.ids + v.i * K;
            const unsigned long long at = base + before + incl - mine;
            const int64_t off = (int64_t)(at & kOvfCrossMask);
            a.ovf_list[at >> kOvfCrossBits] = (int32_t)e;
            if (off + c <= a.o.pool_cap) {
                a.ovf_off[e] = off;
                for (int k = 0; k < K; ++k) a.o.pool_ids[off + k] = ids[k];
                // the rest of the range is filled from the arena (an entry
                // no record reaches, after a full arena, stays a miss)
                for (int k = K; k < c; ++k) {
                    a.o.pool_ids[off + k] = -1;
                    a.o.pool_ts[off + k] = INFINITY;
                }
                if (soff) soff[v.i] = off;
            } else {
                a.ovf_off[e] = -1;
                atomicOr(&a.scalars[kOvfFull], 1);
                float *ts = v.ts + v.i * K;
                for (int k = 0; k < K; ++k) {
                    ids[k] = -1;
                    ts[k] = INFINITY;
                }
                if (soff) soff[v.i] = -1;
            }
        }
        base += tile;
    }
}

// Add a workgroup's per-thread counts to a device counter with one atomic.
__device__ inline void block_count(int32_t v, int32_t *sh, int32_t *counter)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (__lane_id() == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t t = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
        if (t) atomicAdd(counter, t);
    }
    __syncthreads();
}

// All hits, after the walk: every crossing of an overflowed segment is
// re-solved in FP64 into its place in the segment's pool range, one thread
// per crossing: items [0, n_arena) are the arena records (entry e, rank c,
// sorted position), the next n_valid * K items the first K crossings of
// each listed entry (their positions were copied to the head of its range).
// Records of a void entry (a walk handed to the deep pass) are skipped.
template <bool BATCH>
__global__ __launch_bounds__(256) void k_spill_place(QArgs a)
{
    __shared__ int32_t sh[4];
    const unsigned long long na = (uint32_t)a.scalars[kArenaLo] | ((unsigned long long)(uint32_t)a.scalars[kArenaHi] << 32);
    const int64_t n_arena = (int64_t)(na < (unsigned long long)a.arena_cap ? na : (unsigned long long)a.arena_cap);
    const int32_t K = a.o.cap;
    const int64_t n_valid = a.scalars[kOvfValid];
    const int64_t n = n_arena + n_valid * K;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t first = (int64_t)blockIdx.x * blockDim.x;
    for (int64_t r0 = first; r0 < n; r0 += stride) {
        const int64_t r = r0 + threadIdx.x;
        int32_t placed = 0;
        if (r < n) {
            int32_t e, c, pos = -1;
            if (r < n_arena) {
                const int4 rec = a.arena[r];
                e = rec.x;
                c = rec.y;
                pos = rec.z;
            } else {
                const int64_t j = (r - n_arena) / K;
                e = a.ovf_list[j];
                c = (int32_t)((r - n_arena) - j * K);
            }
            const int32_t cnt = (e >= 0 && e < a.ovf_cap) ? a.ovf_cnt[e] : -1;
            const int64_t off = cnt >= 0 ? a.ovf_off[e] : -1;
            if (cnt >= 0 && c < cnt && off >= 0 && off + cnt <= a.o.pool_cap) {
                if (r >= n_arena) pos = a.o.pool_ids[off + c];
                else placed = 1;
                int32_t id = 0x7FFFFFFF;
                float t = INFINITY;
                if (pos >= 0 && pos < a.n_tris) {
                    const ItemView<BATCH> v = item_view<BATCH>(a, a.ovf_seg[e]);
                    float w[9];
                    tri_load(a.tris, pos, w, id);
                    double td, u, vv;
                    mt_refine64(v.S[3 * v.i], v.S[3 * v.i + 1], v.S[3 * v.i + 2], v.E[3 * v.i], v.E[3 * v.i + 1],
                                v.E[3 * v.i + 2], w, td, u, vv);
                    t = (float)td;
                }
                a.o.pool_ids[off + c] = id;
                a.o.pool_ts[off + c] = t;
            }
        }
        block_count(placed, sh, &a.scalars[kArenaUsed]);
    }
}

// Order a list of n <= N crossings by (t, id) in registers: loaded at
// once, odd-even transposition rounds over fixed indices (entries past n
// are (inf, max) and stay behind the list), written back.
template <int N>
__device__ inline void sort_in_registers(int32_t *ids, float *ts, int32_t n)
{
    float t[N];
    int32_t id[N];
#pragma unroll
    for (int c = 0; c < N; ++c) {
        t[c] = c < n ? ts[c] : INFINITY;
        id[c] = c < n ? ids[c] : 0x7FFFFFFF;
    }
#pragma unroll
    for (int r = 0; r < N; ++r) {
#pragma unroll
        for (int c = r & 1; c + 1 < N; c += 2) {
            if (t[c + 1] < t[c] || (t[c + 1] == t[c] && id[c + 1] < id[c])) {
                const float tf = t[c];
                t[c] = t[c + 1];
                t[c + 1] = tf;
                const int32_t tk = id[c];
                id[c] = id[c + 1];
                id[c + 1] = tk;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < N; ++c) {
        if (c < n) {
            ts[c] = t[c];
            ids[c] = id[c];
        }
    }
}

// Order a longer list in place (shell sort, gaps 13, 4, 1).
__device__ inline void shell_sort(int32_t *ids, float *ts, int32_t n)
{
    const int gaps[3] = {13, 4, 1};
    for (int g = 0; g < 3; ++g) {
        const int gap = gaps[g];
        for (int x = gap; x < n; ++x) {
            const float kt = ts[x];
            const int32_t ki = ids[x];
            int y = x - gap;
            while (y >= 0 && (ts[y] > kt || (ts[y] == kt && ids[y] > ki))) {
                ts[y + gap] = ts[y];
                ids[y + gap] = ids[y];
                y -= gap;
            }
            ts[y + gap] = kt;
            ids[y + gap] = ki;
        }
    }
}

// All hits: every overflowed segment's re-solved crossings are ordered by
// (t, id) in the pool and the first K copied into the segment's slots.  A
// list of up to 16 is sorted by its own thread in registers; a longer one
// by the whole wave: staged in LDS, each lane ranks entries against the
// whole list (ties by position, so ranks are distinct) and writes them to
// their places.  Lists longer than the LDS stage fall back to one thread.
constexpr int kLongListStage = 1024;

template <bool BATCH>
__global__ __launch_bounds__(256) void k_spill_finish(QArgs a)
{
    __shared__ int32_t sh[4];
    __shared__ float st_t[4][kLongListStage];
    __shared__ int32_t st_id[4][kLongListStage];
    const int64_t n = a.scalars[kOvfValid];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int K = a.o.cap;
    const int lane = (int)__lane_id(), wave = (int)(threadIdx.x >> 6);
    for (int64_t j0 = (int64_t)blockIdx.x * blockDim.x; j0 < n; j0 += stride) {
        const int64_t j = j0 + threadIdx.x;
        const int32_t e = j < n ? a.ovf_list[j] : -1;
        int32_t cnt = e >= 0 ? a.ovf_cnt[e] : -1;
        block_count(cnt >= 0 ? 1 : 0, sh, &a.scalars[kOvfUsed]);
        int64_t off = -1;
        int32_t *sid = nullptr;
        float *sts = nullptr;
        if (cnt >= 0) {
            off = a.ovf_off[e];
            if (off < 0 || off + cnt > a.o.pool_cap) {
                cnt = -1;
            } else {
                const ItemView<BATCH> v = item_view<BATCH>(a, a.ovf_seg[e]);
                sid = v.ids + v.i * (int64_t)K;
                sts = v.ts + v.i * (int64_t)K;
            }
        }
        if (cnt >= 0 && (cnt <= 16 || cnt > kLongListStage)) {
            int32_t *ids = a.o.pool_ids + off;
            float *ts = a.o.pool_ts + off;
            if (cnt <= 8) sort_in_registers<8>(ids, ts, cnt);
            else if (cnt <= 16) sort_in_registers<16>(ids, ts, cnt);
            else shell_sort(ids, ts, cnt);
            for (int c = 0; c < K; ++c) {
                sid[c] = ids[c];
                sts[c] = ts[c];
            }
        }
        // the wave's long lists, one at a time
        uint64_t longm = ballot(cnt > 16 && cnt <= kLongListStage);
        while (longm != 0) {
            const int src = __builtin_ctzll(longm);
            longm &= longm - 1;
            const int32_t es = __shfl(e, src, 64);
            const int32_t m = __shfl(cnt, src, 64);
            const int64_t o = a.ovf_off[es];
            const ItemView<BATCH> v = item_view<BATCH>(a, a.ovf_seg[es]);
            int32_t *s_id = v.ids + v.i * (int64_t)K;
            float *s_t = v.ts + v.i * (int64_t)K;
            int32_t *ids = a.o.pool_ids + o;
            float *ts = a.o.pool_ts + o;
            for (int j = lane; j < m; j += 64) {
                st_t[wave][j] = ts[j];
                st_id[wave][j] = ids[j];
            }
            wave_lds_sync();
            for (int j = lane; j < m; j += 64) {
                const float tj = st_t[wave][j];
                const int32_t ij = st_id[wave][j];
                int32_t rank = 0;
                for (int i = 0; i < m; ++i) {
                    const float ti = st_t[wave][i];
                    const int32_t ii = st_id[wave][i];
                    rank += (ti < tj || (ti == tj && (ii < ij || (ii == ij && i < j)))) ? 1 : 0;
                }
                ts[rank] = tj;
                ids[rank] = ij;
                if (rank < K) {
                    s_t[rank] = tj;
                    s_id[rank] = ij;
                }
            }
            wave_lds_sync();
        }
    }
}

// Exclusive prefix over the 256 threads of a workgroup of one count per
// thread; *total gets the sum.  sh: 4 ints of LDS.  Every thread must call it.
__device__ inline int32_t block_prefix256(int32_t v, int32_t *sh, int32_t &total)
{
    const int lane = (int)__lane_id(), wave = (int)(threadIdx.x >> 6);
    int32_t incl = v;
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t u = __shfl_up(incl, off, 64);
        if (lane >= off) incl += u;
    }
    if (lane == 63) sh[wave] = incl;
    __syncthreads();
    int32_t before = 0;
    for (int w = 0; w < wave; ++w) before += sh[w];
    total = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
    return before + incl - v;
}

// Segment ends of work item k (a segment, or a (mesh, segment) pair).
template <bool BATCH>
__device__ inline void item_ends(const QArgs &a, int64_t k, float &sx, float &sy, float &sz, float &ex, float &ey,
                                 float &ez)
{
    const ItemView<BATCH> v = item_view<BATCH>(a, k);
    sx = ld_nt(v.S + 3 * v.i);
    sy = ld_nt(v.S + 3 * v.i + 1);
    sz = ld_nt(v.S + 3 * v.i + 2);
    ex = ld_nt(v.E + 3 * v.i);
    ey = ld_nt(v.E + 3 * v.i + 1);
    ez = ld_nt(v.E + 3 * v.i + 2);
}

// All hits, after the walk: every segment with 1..K crossings has their
// sorted positions in its first slots.  Re-solve them in FP64 (positions
// become triangle ids), order by (t, id), pad the slots (-1, +inf) and write
// ids and t; also the padding of segments without crossing and their spill
// offsets (-1).  Segments with more than K crossings are completed by
// k_spill_finish.  Kept out of the walk, whose register count (hence waves
// per SIMD) the FP64 solves would otherwise set.  A workgroup takes tiles
// of 256 segments in order; for K <= 4 the tile's (segment, slot) pairs are
// packed so that the FP64 solves run on full waves, their results pass
// through LDS, and every lane then writes its own segment's slots (the
// lanes' rows are contiguous, so the stores fill whole lines).  A tile's
// counts are loaded while the previous tile is packed, its positions and
// segment ends while the previous tile's pairs are solved.
template <bool BATCH>
__global__ __launch_bounds__(256) void k_refine_slots(QArgs a)
{
    const int K = a.o.cap;
    const int tid = threadIdx.x;
    __shared__ int32_t sh[4];
    __shared__ int32_t q_pair[256 * kRegSlots];  // (lane << 2) | slot
    __shared__ int32_t r_id[256 * kRegSlots];    // a pair's position, then its triangle id
    __shared__ float r_t[256 * kRegSlots];
    __shared__ float s_end[6][256];              // ends of the tile's segments with crossings
    // A thread's loads for its segment of a tile, in two steps so that they
    // overlap the previous tile's work: first the crossing count, then (with
    // the count known) the slot positions and the segment ends.
    struct Pre {
        int32_t n;  // crossings; -2: no segment
        int32_t pos[kRegSlots];
        float e[6];
    };
    auto fetch_count = [&](int64_t base, Pre &f) {
        const int64_t k = base + tid;
        f.n = -2;
        if (k < a.n_items) {
            const ItemView<BATCH> v = item_view<BATCH>(a, k);
            const int32_t *cnt = BATCH ? a.bt.count[mesh_of(a.bt.seg_off, a.M, k)] : a.o.count;
            f.n = cnt[v.i];
        }
    };
    auto fetch_rest = [&](int64_t base, Pre &f) {
        const int64_t k = base + tid;
        if (f.n > 0 && f.n <= K) {
            const ItemView<BATCH> v = item_view<BATCH>(a, k);
            const int32_t *ids = v.ids + v.i * (int64_t)K;
#pragma unroll
            for (int c = 0; c < kRegSlots; ++c) f.pos[c] = c < f.n ? ids[c] : -1;
            item_ends<BATCH>(a, k, f.e[0], f.e[1], f.e[2], f.e[3], f.e[4], f.e[5]);
        }
    };
    const int64_t gstride = (int64_t)gridDim.x * 256;
    Pre cur;
    fetch_count((int64_t)blockIdx.x * 256, cur);
    fetch_rest((int64_t)blockIdx.x * 256, cur);
    for (int64_t base = (int64_t)blockIdx.x * 256; base < a.n_items; base += gstride) {
        Pre nxt;
        fetch_count(base + gstride, nxt);
        // overflowed segments (more than K crossings) are k_spill_finish's
        const int32_t n = cur.n <= K ? cur.n : -1;
        // pack the tile's (segment, slot) pairs
        int32_t total;
        const int32_t q = block_prefix256(n > 0 ? n : 0, sh, total);
#pragma unroll
        for (int c = 0; c < kRegSlots; ++c) {
            if (c < n) {
                q_pair[q + c] = (tid << 2) | c;
                r_id[tid * kRegSlots + c] = cur.pos[c];
            }
        }
        if (n > 0) {
#pragma unroll
            for (int d = 0; d < 6; ++d) s_end[d][tid] = cur.e[d];
        }
        __syncthreads();
        fetch_rest(base + gstride, nxt);
#pragma unroll 1
        for (int j = tid; j < total; j += 256) {
            const int lt = q_pair[j] >> 2, c = q_pair[j] & 3;
            const int32_t pos = r_id[lt * kRegSlots + c];
            int32_t id = 0x7FFFFFFF;
            float t = INFINITY;
            if (pos >= 0 && pos < a.n_tris) {  // an entry no walk wrote is never read through
                float w[9];
                tri_load(a.tris, pos, w, id);
                double tt, u, ww;
                mt_refine64(s_end[0][lt], s_end[1][lt], s_end[2][lt], s_end[3][lt], s_end[4][lt], s_end[5][lt], w,
                            tt, u, ww);
                t = (float)tt;
            }
            r_id[lt * kRegSlots + c] = id;
            r_t[lt * kRegSlots + c] = t;
        }
        __syncthreads();
        if (n >= 0) {
            const int64_t k = base + tid;
            const ItemView<BATCH> v = item_view<BATCH>(a, k);
            int64_t *soff = BATCH ? a.bt.spill_off[mesh_of(a.bt.seg_off, a.M, k)] : a.o.spill_off;
            if (soff) st_nt(soff + v.i, (int64_t)-1);
            int32_t *ids = v.ids + v.i * (int64_t)K;
            float *ts = v.ts + v.i * (int64_t)K;
            int32_t id[kRegSlots];
            float t[kRegSlots];
#pragma unroll
            for (int c = 0; c < kRegSlots; ++c) {
                id[c] = c < n ? r_id[tid * kRegSlots + c] : 0x7FFFFFFF;
                t[c] = c < n ? r_t[tid * kRegSlots + c] : INFINITY;
            }
            // five-comparator network (unused entries sort last)
            auto cs = [&](int x, int y) {
                if (t[y] < t[x] || (t[y] == t[x] && id[y] < id[x])) {
                    const float tf = t[x];
                    t[x] = t[y];
                    t[y] = tf;
                    const int32_t tk = id[x];
                    id[x] = id[y];
                    id[y] = tk;
                }
            };
            cs(0, 1);
            cs(2, 3);
            cs(0, 2);
            cs(1, 3);
            cs(1, 2);
#pragma unroll
            for (int c = 0; c < kRegSlots; ++c)
                if (c >= n) id[c] = -1;
            const bool vec = K == kRegSlots &&
                             ((reinterpret_cast<uintptr_t>(ids) | reinterpret_cast<uintptr_t>(ts)) & 15) == 0;
            if (vec) {
                st_nt4(ids, id[0], id[1], id[2], id[3]);
                st_nt4(ts, t[0], t[1], t[2], t[3]);
            } else {
                for (int c = 0; c < K; ++c) {
                    st_nt(ids + c, id[c]);
                    st_nt(ts + c, t[c]);
                }
            }
        }
        __syncthreads();
        cur = nxt;
    }
}

// The same for K > 4: a segment per lane, its slots in order.
template <bool BATCH>
__global__ __launch_bounds__(256) void k_refine_slots_long(QArgs a)
{
    const int K = a.o.cap;
    const int tid = threadIdx.x;
    // a segment per lane, its slots in order
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + tid; k < a.n_items; k += stride) {
        const ItemView<BATCH> v = item_view<BATCH>(a, k);
        const int32_t *cnt = BATCH ? a.bt.count[mesh_of(a.bt.seg_off, a.M, k)] : a.o.count;
        int64_t *soff = BATCH ? a.bt.spill_off[mesh_of(a.bt.seg_off, a.M, k)] : a.o.spill_off;
        const int32_t n = cnt[v.i];
        if (n > K) continue;
        if (soff) st_nt(soff + v.i, (int64_t)-1);
        int32_t *ids = v.ids + v.i * (int64_t)K;
        float *ts = v.ts + v.i * (int64_t)K;
        if (n > 0) {
            float sx, sy, sz, ex, ey, ez;
            item_ends<BATCH>(a, k, sx, sy, sz, ex, ey, ez);
            for (int c = 0; c < n; ++c) {
                const int32_t pos = ids[c];
                if (pos < 0 || pos >= a.n_tris) {
                    ids[c] = 0x7FFFFFFF;
                    ts[c] = INFINITY;
                    continue;
                }
                float w[9];
                int32_t tid3;
                tri_load(a.tris, pos, w, tid3);
                double tt, u, ww;
                mt_refine64(sx, sy, sz, ex, ey, ez, w, tt, u, ww);
                ids[c] = tid3;
                ts[c] = (float)tt;
            }
            for (int x = 1; x < n; ++x) {  // insertion sort by (t, id): lists are short
                const float kt = ts[x];
                const int32_t ki = ids[x];
                int y = x - 1;
                while (y >= 0 && (ts[y] > kt || (ts[y] == kt && ids[y] > ki))) {
                    ts[y + 1] = ts[y];
                    ids[y + 1] = ids[y];
                    --y;
                }
                ts[y + 1] = kt;
                ids[y + 1] = ki;
            }
        }
        for (int c = n; c < K; ++c) {
            ids[c] = -1;
            ts[c] = INFINITY;
        }
    }
}

__global__ void k_fill_miss(int64_t n_r, uint32_t mode, QueryOut o)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_r) return;
    if (mode & M_BOOL) o.hit[i] = 0;
    if (mode & M_FIRST) {
        o.tri[i] = -1;
        o.t[i] = INFINITY;
        o.uv[2 * i] = o.uv[2 * i + 1] = 0.0f;
        o.point[3 * i] = o.point[3 * i + 1] = o.point[3 * i + 2] = 0.0f;
    }
    if (mode & (M_ALL | M_COUNT)) o.count[i] = 0;
    if (mode & M_ALL) {
        for (int c = 0; c < o.cap; ++c) {
            o.ids[i * (int64_t)o.cap + c] = -1;
            o.ts[i * (int64_t)o.cap + c] = INFINITY;
        }
        if (o.spill_off) o.spill_off[i] = -1;
    }
}

// Far end of the inside-test segment of every point: P + L u with the fixed
// direction u and L = |P - c| + 2R + 1 (c, R: centre and half diagonal of
// the mesh's bounding box, the entry node's first child box), so the end lies
// outside the box and every crossing of the surface is counted.
__global__ void k_inside_ends(const float *__restrict__ P, int64_t n, const Node *__restrict__ entry,
                              float *__restrict__ E)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float *b = entry->f;
    const float cx = 0.5f * (b[0] + b[3]), cy = 0.5f * (b[1] + b[4]), cz = 0.5f * (b[2] + b[5]);
    const float hx = 0.5f * (b[3] - b[0]), hy = 0.5f * (b[4] - b[1]), hz = 0.5f * (b[5] - b[2]);
    const float R = sqrtf(hx * hx + hy * hy + hz * hz);
    const float px = P[3 * i], py = P[3 * i + 1], pz = P[3 * i + 2];
    const float qx = px - cx, qy = py - cy, qz = pz - cz;
    const float L = sqrtf(qx * qx + qy * qy + qz * qz) + 2.0f * R + 1.0f;
    E[3 * i] = px + L * kInsideDir[0];
    E[3 * i + 1] = py + L * kInsideDir[1];
    E[3 * i + 2] = pz + L * kInsideDir[2];
}

__global__ void k_parity(const int32_t *__restrict__ count, int64_t n, uint8_t *__restrict__ inside)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) inside[i] = (uint8_t)(count[i] & 1);
}

// Reset the per-query device scalars with a kernel rather than a memset, so
// the sequence can be captured.
// Zero the per-query scalars.  keep != 0 (a later part of a query split
// into parts) keeps the flags of damaged-tree walks and the work counters,
// so they describe every part.
__global__ void k_reset(int32_t *scalars, Counters *c, int keep)
{
    const int32_t zero[] = {kWorkRetry, kRetryN,  kOvfSegs, kOvfTotalLo, kOvfTotalHi,   kArenaLo, kArenaHi,
                            kOvfFull,   kOvfUsed, kArenaUsed, kRetryLost, kStackDropped, kWalkCut};
    for (int r = 0; r < kXcds; ++r) scalars[kWorkXcd + kWorkStride * r] = 0;
    const int n = (int)(sizeof(zero) / sizeof(zero[0])) - (keep ? 3 : 0);
    for (int k = 0; k < n; ++k) scalars[zero[k]] = 0;
    if (c && !keep) {
        c->node_visits = c->box_tests = c->tri_tests = c->segments = 0;
        c->wave_loops = c->wave_node_steps = c->wave_leaf_phases = c->wave_refills = 0;
        c->lanes_blocked = c->lanes_waiting = 0;
        c->wave_leaf_rounds = c->leaf_lanes = 0;
    }
}

// FP64 re-solve of every first hit, after the walk: the walk leaves the
// sorted position of the hit triangle in tri, or -1 for a miss, and this
// pass writes the triangle's id, t, (u, v) and the point, or the miss values.
// Kept out of the walk, whose registers (hence waves per SIMD) it would
// otherwise raise for the whole traversal.  A workgroup takes tiles of 256
// segments in order; the tile's hits are packed so that the FP64 solves run
// on full waves, their results pass through LDS, and every lane then writes
// its own segment's outputs (consecutive lanes, consecutive segments: the
// stores fill whole lines).
template <bool BATCH>
__global__ __launch_bounds__(256) void k_refine_first(QArgs a)
{
    __shared__ int32_t sh[4];
    __shared__ int32_t q_lane[256];
    __shared__ int32_t q_pos[256];
    __shared__ int32_t r_id[256];
    __shared__ float r_f[6 * 256];  // t, u, v, Px, Py, Pz
    const int tid = threadIdx.x;
    for (int64_t base = (int64_t)blockIdx.x * 256; base < a.n_items; base += (int64_t)gridDim.x * 256) {
        const int64_t k = base + tid;
        int64_t i = k;
        int32_t *tri = a.o.tri;
        float *tt = a.o.t, *uv = a.o.uv, *pt = a.o.point;
        int32_t pos = -1;
        if (k < a.n_items) {
            if (BATCH) {
                const int32_t m = mesh_of(a.bt.seg_off, a.M, k);
                i = k - a.bt.seg_off[m];
                tri = a.bt.tri[m];
                tt = a.bt.t[m];
                uv = a.bt.uv[m];
                pt = a.bt.point[m];
            }
            pos = tri[i];
        }
        // a position past the triangles cannot come from a walk and is never read through
        const bool hit = pos >= 0 && pos < a.n_tris;
        int32_t nq;
        const int32_t q = block_prefix256(hit ? 1 : 0, sh, nq);
        if (hit) {
            q_lane[q] = tid;
            q_pos[q] = pos;
        }
        __syncthreads();
        if (tid < nq) {
            const int lt = q_lane[tid];
            float sx, sy, sz, ex, ey, ez;
            item_ends<BATCH>(a, base + lt, sx, sy, sz, ex, ey, ez);
            float v[9];
            int32_t id;
            tri_load(a.tris, q_pos[tid], v, id);
            double t, u, w;
            mt_refine64(sx, sy, sz, ex, ey, ez, v, t, u, w);
            r_id[lt] = id;
            r_f[lt] = (float)t;
            r_f[256 + lt] = (float)u;
            r_f[512 + lt] = (float)w;
            r_f[768 + lt] = (float)((double)sx + t * ((double)ex - (double)sx));
            r_f[1024 + lt] = (float)((double)sy + t * ((double)ey - (double)sy));
            r_f[1280 + lt] = (float)((double)sz + t * ((double)ez - (double)sz));
        }
        __syncthreads();
        if (k < a.n_items) {
            st_nt(tri + i, hit ? r_id[tid] : -1);
            st_nt(tt + i, hit ? r_f[tid] : INFINITY);
            st_nt(uv + 2 * i, hit ? r_f[256 + tid] : 0.0f);
            st_nt(uv + 2 * i + 1, hit ? r_f[512 + tid] : 0.0f);
            st_nt(pt + 3 * i, hit ? r_f[768 + tid] : 0.0f);
            st_nt(pt + 3 * i + 1, hit ? r_f[1024 + tid] : 0.0f);
            st_nt(pt + 3 * i + 2, hit ? r_f[1280 + tid] : 0.0f);
        }
        __syncthreads();
    }
}

template <bool BATCH>
hipError_t launch_refine_first(const QArgs &a, hipStream_t s)
{
    const int64_t blocks = (a.n_items + 255) / 256;
    hipLaunchKernelGGL(k_refine_first<BATCH>, dim3((unsigned)(blocks < 8192 ? blocks : 8192)), dim3(256), 0, s, a);
    return hipGetLastError();
}

// Grid of the deep pass: a few workgroups per CU (the queue is short); its
// device-memory stack holds one column per thread of this grid.
constexpr int kRetryBlocksPerCU = 1;

int device_cus()
{
    int dev = 0, n_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1;
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 1;
    return n_cu > 0 ? n_cu : 1;
}

template <uint32_t MODE, bool RETRY, bool COUNT, bool BATCH, bool WIDE>
hipError_t launch_kernel(const QArgs &a, int block, size_t lds, hipStream_t s)
{
    auto kern = k_query<MODE, RETRY, COUNT, BATCH, WIDE>;
    int64_t grid;
    QArgs b = a;
    if (RETRY) {
        grid = (int64_t)kRetryBlocksPerCU * device_cus();
        if (a.lds_depth < a.depth && (a.gstack == nullptr || grid * block * (int64_t)(a.depth - a.lds_depth) >
                                                                 a.gstack_cap))
            return hipErrorInvalidValue;
        b.chunk = 64;
    } else {
        int per_cu = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, block, lds);
        if (e != hipSuccess) return e;
        if (per_cu < 1) per_cu = 1;
        grid = (int64_t)per_cu * device_cus();
        const int64_t need = (a.n_items + block - 1) / block;
        if (grid > need) grid = need;
        if (grid < 1) grid = 1;
        if (b.chunk <= 0) {
            // about eight chunks per resident wave keeps the tail short while the
            // range counters see one atomic per chunk
            const int64_t waves = grid * (block / 64);
            int64_t c = (a.n_items + 8 * waves - 1) / (8 * waves);
            c = (c + 63) / 64 * 64;
            b.chunk = (int32_t)(c < 64 ? 64 : (c > 4096 ? 4096 : c));
        }
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(block), lds, s, b);
    return hipGetLastError();
}

template <uint32_t MODE, bool RETRY, bool COUNT, bool BATCH = false>
hipError_t launch_mode(const QArgs &a, int block, size_t lds, hipStream_t s)
{
    if (a.nodes4) return launch_kernel<MODE, RETRY, COUNT, BATCH, true>(a, block, lds, s);
    return launch_kernel<MODE, RETRY, COUNT, BATCH, false>(a, block, lds, s);
}

// The main pass, then the deep pass over the segments it queued.
template <uint32_t MODE, bool COUNT, bool BATCH = false>
hipError_t launch_passes(const QArgs &main, const QArgs &deep, int block, size_t lds, hipStream_t s)
{
    hipError_t e = launch_mode<MODE, false, COUNT, BATCH>(main, block, lds, s);
    if (e == hipSuccess) e = launch_mode<MODE, true, COUNT, BATCH>(deep, block, lds, s);
    return e;
}

template <bool COUNT>
hipError_t dispatch(uint32_t mode, const QArgs &a, const QArgs &d, int block, size_t lds, hipStream_t s)
{
    // RSI_BOOL is derived for free whenever a full pass runs
    switch (mode) {
    case M_BOOL: return launch_passes<M_BOOL, COUNT>(a, d, block, lds, s);
    case M_FIRST: return launch_passes<M_FIRST, COUNT>(a, d, block, lds, s);
    case M_FIRST | M_BOOL: return launch_passes<M_FIRST | M_BOOL, COUNT>(a, d, block, lds, s);
    case M_ALL: return launch_passes<M_ALL, COUNT>(a, d, block, lds, s);
    case M_ALL | M_BOOL: return launch_passes<M_ALL | M_BOOL, COUNT>(a, d, block, lds, s);
    case M_ALL | M_FIRST: return launch_passes<M_ALL | M_FIRST, COUNT>(a, d, block, lds, s);
    case M_ALL | M_FIRST | M_BOOL: return launch_passes<M_ALL | M_FIRST | M_BOOL, COUNT>(a, d, block, lds, s);
    case M_COUNT: return launch_passes<M_COUNT, COUNT>(a, d, block, lds, s);
    case M_COUNT | M_BOOL: return launch_passes<M_COUNT | M_BOOL, COUNT>(a, d, block, lds, s);
    case M_COUNT | M_FIRST: return launch_passes<M_COUNT | M_FIRST, COUNT>(a, d, block, lds, s);
    case M_COUNT | M_FIRST | M_BOOL: return launch_passes<M_COUNT | M_FIRST | M_BOOL, COUNT>(a, d, block, lds, s);
    default: return hipErrorInvalidValue;
    }
}

// Dynamic LDS of a query launch: the stack's LDS part, then in the
// four-way walk (all-hits modes aside) each wave's leaf queue (64 entries).
size_t query_lds(int block, int depth, int width, uint32_t mode)
{
    const size_t ent = mode == M_BOOL ? sizeof(int2) : sizeof(int4);
    const bool queue = width == 4 && !(mode & M_ALL);
    return (size_t)block * depth * sizeof(int32_t) + (queue ? (size_t)(block / 64) * 64 * ent : 0);
}

// Largest multiple of 64 not above `want` (and at most 256, the kernels'
// launch bound) whose LDS part fits in 64 KiB.
int fit_block(int want, int depth, int width, uint32_t mode)
{
    int b = want < 256 ? want : 256;
    while (b > 64 && query_lds(b, depth, width, mode) > 65536) b -= 64;
    return b;
}

// Traversal-stack entries a lane can need for a tree of the given height:
// one pushed sibling per binary level (height + 1); in the four-way walk up
// to three per four-way level, of which there are at most (height + 2) / 2 + 1.
int stack_need(int height, int width)
{
    if (width == 4) return 3 * ((height + 2) / 2 + 1) + 1;
    return height + 1;
}

// LDS stack entries per lane of the main pass: the `stack_depth` option, or
// 20 on the four-way walk (17 when the walk also holds the 1,344-byte copy
// of the top records), 32 on the binary walk; never more than the bound.
int lds_part(const rsi_bvh *h, bool top)
{
    const int width = h->width_built;
    const int bound = stack_need(h->height_bound, width);
    int cap = h->stack_cap;
    if (cap <= 0) cap = width == 4 ? (top ? 17 : 20) : 32;
    return cap < bound ? cap : bound;
}

QArgs make_args(rsi_bvh *h, const float *S, const float *E, int64_t n_items, const QueryOut &o)
{
    QArgs a;
    a.nodes = h->nodes;
    a.nodes4 = h->width_built == 4 ? h->nodes4 : nullptr;
    a.tris = h->tris;
    a.n_tris = (int32_t)h->n_t;
    a.entry = h->n_t > 0 ? (int32_t)(h->h_tri_off[1] - 1) : -1;
    a.S = S;
    a.E = E;
    a.n_items = n_items;
    a.o = o;
    a.ovf_seg = h->ovf_seg;
    a.ovf_cnt = h->ovf_cnt;
    a.ovf_off = h->ovf_off;
    a.ovf_cap = h->ovf_cap;
    a.arena = h->arena;
    a.arena_cap = h->arena_cap;
    a.ovf_part = h->ovf_part;
    a.ovf_list = h->ovf_list;
    a.scalars = h->scalars;
    a.counters = h->counters;
    a.depth = 0;
    a.lds_depth = 0;
    a.gstack = h->retry_stack;
    a.gstack_cap = h->retry_stack_cap;
    a.retry_q = h->retry_q;
    a.retry_cap = h->retry_cap;
    a.max_steps = (int32_t)(h->n_t > 0 ? h->n_t : 1);
    a.defer = h->defer_lanes;
    a.refill = h->refill_lanes;
    a.chunk = h->chunk;
    a.M = h->M;
    a.mesh_entry = h->mesh_entry;
    a.bt = h->bt;
    return a;
}

// Arguments of the two passes: the main pass keeps its whole stack (ld
// entries) in LDS; the deep pass has the same LDS part and continues in
// device memory up to the height bound.
void pass_args(const rsi_bvh *h, QArgs &main, QArgs &deep, int ld)
{
    main.depth = main.lds_depth = ld;
    deep = main;
    deep.depth = stack_need(h->height_bound, h->width_built);
    deep.lds_depth = ld;
    if (deep.depth < ld) deep.depth = ld;
}

hipError_t launch_all_hits_tail(const QArgs &a, bool batch, hipStream_t s)
{
    const int64_t blocks = (a.n_items + 255) / 256;
    const unsigned rgrid = (unsigned)(blocks < 8192 ? blocks : 8192);
    if (a.o.cap > kRegSlots) {
        if (batch) hipLaunchKernelGGL(k_refine_slots_long<true>, dim3(rgrid), dim3(256), 0, s, a);
        else hipLaunchKernelGGL(k_refine_slots_long<false>, dim3(rgrid), dim3(256), 0, s, a);
    } else if (batch) {
        hipLaunchKernelGGL(k_refine_slots<true>, dim3(rgrid), dim3(256), 0, s, a);
    } else {
        hipLaunchKernelGGL(k_refine_slots<false>, dim3(rgrid), dim3(256), 0, s, a);
    }
    hipLaunchKernelGGL(k_ovf_sums, dim3(kOvfParts), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_ovf_scan_parts, dim3(1), dim3(kOvfParts), 0, s, a);
    if (batch) hipLaunchKernelGGL(k_ovf_offsets<true>, dim3(kOvfParts), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_ovf_offsets<false>, dim3(kOvfParts), dim3(256), 0, s, a);
    const unsigned grid = (unsigned)(2 * device_cus());
    // one crossing per thread: enough workgroups that the usual few hundred
    // thousand take one round
    const unsigned pgrid = (unsigned)(8 * device_cus());
    if (batch) hipLaunchKernelGGL(k_spill_place<true>, dim3(pgrid), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_spill_place<false>, dim3(pgrid), dim3(256), 0, s, a);
    if (batch) hipLaunchKernelGGL(k_spill_finish<true>, dim3(grid), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_spill_finish<false>, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace

int64_t deep_stack_entries(const rsi_bvh *h, uint32_t mode)
{
    const int ld = lds_part(h, h->width_built == 4 && top_copy(mode));
    const int block = fit_block(h->block_size, ld, h->width_built, mode);
    const int need = stack_need(h->height_bound, h->width_built);
    return need > ld ? (int64_t)kRetryBlocksPerCU * device_cus() * block * (need - ld) : 0;
}

hipError_t launch_query(rsi_bvh *h, const float *S, const float *E, int64_t n_r, uint32_t mode,
                        const QueryOut &o, hipStream_t s)
{
    const QueryScratch sc = {h->retry_q, h->retry_cap, h->retry_stack, h->retry_stack_cap};
    return launch_query_scratch(h, S, E, n_r, mode, o, sc, false, s);
}

hipError_t launch_query_scratch(rsi_bvh *h, const float *S, const float *E, int64_t n_r, uint32_t mode,
                                const QueryOut &o, const QueryScratch &sc, bool keep_flags, hipStream_t s)
{
    if (n_r == 0) return hipSuccess;
    const int ld = lds_part(h, h->width_built == 4 && top_copy(mode));
    const int block = fit_block(h->block_size, ld, h->width_built, mode);
    const size_t lds = query_lds(block, ld, h->width_built, mode);
    QArgs a = make_args(h, S, E, n_r, o), d;
    a.retry_q = sc.retry_q;
    a.retry_cap = sc.retry_cap;
    a.gstack = sc.gstack;
    a.gstack_cap = sc.gstack_cap;
    if (a.retry_cap < n_r) return hipErrorInvalidValue;
    pass_args(h, a, d, ld);
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(1), 0, s, h->scalars, h->counting ? h->counters : nullptr,
                       keep_flags ? 1 : 0);
    hipError_t e = h->counting ? dispatch<true>(mode, a, d, block, lds, s) : dispatch<false>(mode, a, d, block, lds, s);
    if (e == hipSuccess && (mode & M_FIRST)) e = launch_refine_first<false>(a, s);
    if (e == hipSuccess && (mode & M_ALL)) e = launch_all_hits_tail(a, false, s);
    return e;
}

hipError_t launch_batch_query(rsi_bvh *h, const BatchTables &bt, int64_t n_total, uint32_t mode, int32_t cap,
                              hipStream_t s)
{
    if (n_total == 0) return hipSuccess;
    const int ld = lds_part(h, false);
    const int block = fit_block(h->block_size, ld, h->width_built, mode);
    const size_t lds = query_lds(block, ld, h->width_built, mode);
    QueryOut o = {};
    o.cap = cap;
    o.pool_ids = h->pool_ids;
    o.pool_ts = h->pool_ts;
    o.pool_cap = h->pool_cap;
    QArgs a = make_args(h, nullptr, nullptr, n_total, o), d;
    a.bt = bt;
    pass_args(h, a, d, ld);
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(1), 0, s, h->scalars, nullptr, 0);
    hipError_t e;
    switch (mode) {
    case M_BOOL: e = launch_passes<M_BOOL, false, true>(a, d, block, lds, s); break;
    case M_FIRST: e = launch_passes<M_FIRST, false, true>(a, d, block, lds, s); break;
    case M_FIRST | M_BOOL: e = launch_passes<M_FIRST | M_BOOL, false, true>(a, d, block, lds, s); break;
    case M_ALL: e = launch_passes<M_ALL, false, true>(a, d, block, lds, s); break;
    case M_ALL | M_BOOL: e = launch_passes<M_ALL | M_BOOL, false, true>(a, d, block, lds, s); break;
    case M_ALL | M_FIRST: e = launch_passes<M_ALL | M_FIRST, false, true>(a, d, block, lds, s); break;
    case M_ALL | M_FIRST | M_BOOL: e = launch_passes<M_ALL | M_FIRST | M_BOOL, false, true>(a, d, block, lds, s); break;
    default: return hipErrorInvalidValue;
    }
    if (e == hipSuccess && (mode & M_FIRST)) e = launch_refine_first<true>(a, s);
    if (e == hipSuccess && (mode & M_ALL)) e = launch_all_hits_tail(a, true, s);
    return e;
}

// A captured graph holds the addresses of the handle's scratch: before any
// of it is reallocated, wait for the device and release the graph (a replay
// then reports that nothing is captured).
static hipError_t release_graph(rsi_bvh *h)
{
    if (!h->graph) return hipSuccess;
    hipError_t e = hipDeviceSynchronize();
    (void)hipGraphExecDestroy(h->graph);
    h->graph = nullptr;
    return e;
}

hipError_t ensure_query_memory(rsi_bvh *h, int64_t n, bool all_hits)
{
    hipError_t e = hipSuccess;
    auto grow = [&](auto **p, int64_t &cap, int64_t want, size_t elem) {
        if (e != hipSuccess || cap >= want) return;
        if ((e = release_graph(h)) != hipSuccess) return;
        if (*p) (void)hipFree(*p);
        *p = nullptr;
        cap = 0;
        e = hipMalloc(reinterpret_cast<void **>(p), elem * (size_t)(want > 0 ? want : 1));
        if (e == hipSuccess) cap = want;
    };
    grow(&h->retry_q, h->retry_cap, n, sizeof(int32_t));
    // deep-pass stack: every thread of its grid, entries past the LDS part
    {
        const int width = h->width_built;
        const int ld_min = lds_part(h, width == 4);  // the smaller LDS part: the longer tail
        const int need = stack_need(h->height_bound, width);
        const int64_t want =
            need > ld_min ? (int64_t)kRetryBlocksPerCU * device_cus() * h->block_size * (need - ld_min) : 1;
        grow(&h->retry_stack, h->retry_stack_cap, want, sizeof(int32_t));
    }
    if (all_hits) {
        // waves that can hold a block of entries and one of records at
        // once: every resident wave of the main pass (at most 32 per CU,
        // and no more than the segments fill) and of the deep pass (one
        // workgroup of at most 4 waves per CU); each may leave its blocks'
        // unused rest void
        const int64_t cus = device_cus();
        const int64_t waves = ((n + 63) / 64 < 32 * cus ? (n + 63) / 64 : 32 * cus) + 4 * cus;
        // one entry per segment, plus room for the entries that walks handed
        // to the deep pass leave void, plus the void block tails
        const int64_t want = n + n / 8 + (int64_t)(kEntBlock - 1) * waves + 1024;
        if (h->ovf_cap < want) {
            // the four arrays share one capacity: it holds only once all grew
            int64_t c0 = 0, c1 = 0, c2 = 0, c3 = 0;
            h->ovf_cap = 0;
            grow(&h->ovf_seg, c0, want, sizeof(int32_t));
            grow(&h->ovf_cnt, c1, want, sizeof(int32_t));
            grow(&h->ovf_off, c2, want, sizeof(int64_t));
            grow(&h->ovf_list, c3, want, sizeof(int32_t));
            if (e == hipSuccess) h->ovf_cap = want;
        }
        const int64_t arena_want = (h->pool_want > (n / 4 > (1 << 20) ? n / 4 : (1 << 20)) ? h->pool_want
                                    : (n / 4 > (1 << 20) ? n / 4 : (1 << 20))) + (int64_t)(kArenaBlock - 1) * waves;
        grow(&h->arena, h->arena_cap, arena_want, sizeof(int4));
        grow(&h->ovf_part, h->ovf_part_cap, kOvfParts, sizeof(unsigned long long));
    }
    return e;
}

hipError_t ensure_pool(rsi_bvh *h, int64_t n)
{
    if (h->pool_cap >= n) return hipSuccess;
    hipError_t g = release_graph(h);
    if (g != hipSuccess) return g;
    if (h->pool_ids) (void)hipFree(h->pool_ids);
    if (h->pool_ts) (void)hipFree(h->pool_ts);
    h->pool_ids = nullptr;
    h->pool_ts = nullptr;
    h->pool_cap = 0;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(&h->pool_ids), sizeof(int32_t) * (size_t)n);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&h->pool_ts), sizeof(float) * (size_t)n);
    if (e == hipSuccess) h->pool_cap = n;
    return e;
}

hipError_t launch_inside_ends(const rsi_bvh *h, const float *P, int64_t n, float *E, hipStream_t s)
{
    if (n == 0 || h->n_t == 0) return hipSuccess;
    const Node *entry = h->nodes + (h->h_tri_off[1] - 1);
    hipLaunchKernelGGL(k_inside_ends, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, P, n, entry, E);
    return hipGetLastError();
}

hipError_t launch_parity(const int32_t *count, int64_t n, uint8_t *inside, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_parity, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, count, n, inside);
    return hipGetLastError();
}

hipError_t launch_clear_query(rsi_bvh *h, hipStream_t s)
{
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(1), 0, s, h->scalars, nullptr, 0);
    return hipGetLastError();
}

hipError_t launch_fill_miss(int64_t n_r, uint32_t mode, const QueryOut &o, hipStream_t s)
{
    if (n_r == 0) return hipSuccess;
    const int blk = 256;
    hipLaunchKernelGGL(k_fill_miss, dim3((unsigned)((n_r + blk - 1) / blk)), dim3(blk), 0, s, n_r, mode, o);
    return hipGetLastError();
}

}  // namespace rsi
