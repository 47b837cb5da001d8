// Step 4 of the paper (Section 2.2.1), hysteresis, as connected-component
// labelling on the GPU.  An edge pixel is a candidate (class >= 1) that is
// 8-connected through candidates to a strong pixel (class 2); equivalently,
// a candidate whose 8-connected component contains a strong pixel.  The
// paper keeps this step serial; here it is union-find, whose cost does not
// grow with the length of a propagation chain.
//
// The image is cut into 64-column x T-row tiles.  Three launches:
//   1. local:  each workgroup labels its tile in LDS.  Candidates in a row
//              form runs; a run is 8-connected to the runs of the row above
//              that meet columns c0 - 1 .. c1 + 1.  Each run start first
//              points at one of them (a plain store), pointer jumping
//              flattens the resulting trees, and union-find (atomicMin, roots
//              = smallest pixel index) joins the remaining pairs, which only
//              occur where two branches meet; every run start then finds its
//              root.  A component that is decided here -- it holds a
//              strong pixel, or it does not touch the tile border -- gets 255
//              or 0.  A component that touches the border is named globally
//              by tile * 256 + b, b (0..251) the largest index of its border
//              pixels.  Its union-find key is that name, plus 2^30 if the
//              component holds no strong pixel in the tile.  The pass
//              writes, per tile-border pixel, that key (or -1), initialises
//              the name's parent entry (a dense array of 256 entries per
//              tile, indexed by name) with it, and gives the pixels of a weak
//              border component the pending code 1 + b.  Non-candidates
//              get 0.
//   2. merge:  one thread per tile-border pixel on the right and bottom tile
//              edges unions its component with the 8-connected candidates
//              across the edge (global union-find over keys, atomicMin
//              linking: a root always links under a smaller key).  A set's
//              root therefore holds its smallest key, which is below 2^30
//              exactly when some component of the set holds a strong pixel:
//              the roots carry the global strong flags without a pass of
//              their own.
//   3. resolve: each workgroup with pending pixels walks the keys of its
//              weak border components towards their roots, stopping at the
//              first strong key (keys fall along a path, so the root is then
//              strong as well), and rewrites the pending pixels to 255 / 0.
// Border slots of a tile (clipped to the image): top row x -> x, bottom row
// x -> 64 + x, left column y -> 128 + y, right column y -> 128 + T + y.
// Border pixel index b (each border pixel once, for the pending code): top
// row x -> x, bottom row x -> 64 + x, left column y (not top or bottom) ->
// 127 + y, right column y -> 189 + y.
#include "canny_internal.h"

namespace canny {
namespace {

template <int T>
struct Tile {
    static constexpr int kPx = kHystCols * T;
    static constexpr int kPerim = 2 * kHystCols + 2 * T;
    static constexpr int kPPT = kPx / kWGThreads;      // pixels per thread (one row segment)
    static constexpr int kTPR = kHystCols / kPPT;      // threads per tile row
};

// find with path halving (each visited pointer is replaced by its grandparent,
// an ancestor); used only while unions are running, before the root walks
// that follow them, so a halving store can never overwrite a finished root
// pointer
// Volatile views of LDS arrays keep the LDS address space: a volatile access
// through a generic pointer compiles to a flat instruction (slower than an
// LDS one, and it waits on the vector-memory counter as well).
typedef __attribute__((address_space(3))) int lds_i32;
__device__ __forceinline__ volatile lds_i32* lds_volatile(int* p) { return (volatile lds_i32*)p; }

__device__ __forceinline__ int lds_find_halve(volatile lds_i32* L, int x) {
    for (int steps = x; steps >= 0; --steps) {  // pointers decrease: at most x + 1 hops
        const int p = L[x];
        if (p == x) return x;
        const int gp = L[p];
        if (gp == p) return p;
        L[x] = gp;
        x = gp;
    }
    return x;
}

__device__ __forceinline__ void lds_union(int* L, int a, int b) {
    volatile lds_i32* V = lds_volatile(L);
    // each retry follows a link that strictly lowers a, so a + 1 rounds suffice
    for (int round = a > b ? a : b; round >= 0; --round) {
        a = lds_find_halve(V, a);
        b = lds_find_halve(V, b);
        if (a == b) return;
        if (a < b) { const int t = a; a = b; b = t; }
        const int old = atomicMin(&L[a], b);
        if (old == a) return;
        a = old;
    }
}

// Union-find keys of border components: the global name, plus kWeakKey for a
// component without a strong pixel.  Names stay below 2^27 (at most 2^19
// tiles of 256 names), so a key fits 31 bits and -1 stays free for "none".
constexpr int kWeakKey = 1 << 30;
constexpr int kNameMask = kWeakKey - 1;

__device__ __forceinline__ int g_load(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// parent[name] holds a key: the entry's own key at a root, else a smaller
// one.  Keys strictly fall along a walk, so a walk from key k ends within
// k + 1 steps; the bound makes that explicit.
__device__ __forceinline__ int g_find(int* parent, int k) {
    int p = g_load(parent + (k & kNameMask));
    for (int steps = k; p != k && steps >= 0; --steps) {
        k = p;
        p = g_load(parent + (k & kNameMask));
    }
    return k;
}

__device__ __forceinline__ void g_union(int* parent, int a, int b) {
    for (int round = a > b ? a : b; round >= 0; --round) {  // a strictly decreases per retry
        a = g_find(parent, a);
        b = g_find(parent, b);
        if (a == b) return;
        if (a < b) { const int t = a; a = b; b = t; }
        const int old = atomicMin(parent + (a & kNameMask), b);
        if (old == a) return;
        a = old;
    }
}

struct TileGeom {
    int tile, ty, tx, X0, Y0, th, tw;
    int t;  // this thread's index in the workgroup
};

template <int T>
__device__ __forceinline__ TileGeom tile_geom(int tile, int tiles_x, int H, int W) {
    TileGeom g;
    g.tile = tile;
    g.ty = tile / tiles_x;
    g.tx = tile - g.ty * tiles_x;
    g.X0 = g.tx * kHystCols;
    g.Y0 = g.ty * T;
    g.th = min(T, H - g.Y0);
    g.tw = min(kHystCols, W - g.X0);
    g.t = threadIdx.x;
    return g;
}

// Candidate and strong bits of a thread's class codes, compressed to one bit
// per pixel (bit k = pixel k of the segment).
__device__ __forceinline__ uint32_t compress2(uint32_t x) {  // keeps bits 0, 2, 4, ...
    x &= 0x55555555u;
    x = (x | (x >> 1)) & 0x33333333u;
    x = (x | (x >> 2)) & 0x0F0F0F0Fu;
    x = (x | (x >> 4)) & 0x00FF00FFu;
    x = (x | (x >> 8)) & 0x0000FFFFu;
    return x;
}

// column of the first pixel of the run that covers column c, given the row's
// run-start bits S (bit c of S is set where a run begins)
__device__ __forceinline__ int run_start(uint64_t S, int c) {
    const uint64_t m = c >= 63 ? S : (S & ((2ull << c) - 1ull));
    return 63 - __clzll((long long)m);
}

// Per-tile labelling state shared by the local pass.
template <int T>
struct TileLabel {
    uint32_t cand, strong;  // this thread's segment, bit k = pixel k
    uint64_t m, S;          // candidate and run-start bits of this thread's row
};

// L[i] for a run start i: the pixel index of its root (bits 0..11) once the
// labels are final.  A root's own entry then also carries 1 + b in bits
// 17..24, b the largest border pixel index of its component (0: the
// component does not touch the tile border); whether the component holds a
// strong pixel is a separate bitmap, one bit per root.
constexpr int kRootMask = 0xFFFF;
constexpr int kBrepShift = 17;

// largest border pixel index (see border_index) of the run of row r covering
// columns c0..c1 in a tile clipped to th x tw, or -1 if it has none; a
// one-column tile's pixels count as the left column, as in border_index
__device__ __forceinline__ int run_border_max(int r, int c0, int c1, int th, int tw) {
    if (r == 0) return c1;
    if (r == th - 1) return kHystCols + c1;
    if (c1 == tw - 1 && c1 != 0) return 3 * kHystCols - 3 + r;
    if (c0 == 0) return 2 * kHystCols - 1 + r;
    return -1;
}

// A thread's 16 pixels as loaded, before classification: four quads of the
// signed strength map (float path) or one dword of the class map.  The
// loads are unconditional inside the row (quads past nq re-read the last one
// and are masked later), so all are in flight together; a tile's loads can
// be issued before the previous tile is labelled.
struct RawSeg {
    float4 q[4];
    uint32_t cls;
    int nq;  // float path: whole quads of the row from this segment on
};

template <int T>
__device__ __forceinline__ RawSeg load_raw(const HystArgs& a, const TileGeom& g) {
    using TL = Tile<T>;
    const int t = g.t;
    const int r = t / TL::kTPR;
    const int cb = (t % TL::kTPR) * TL::kPPT;
    RawSeg raw;
    raw.cls = 0;
    raw.nq = 0;
    if (r >= g.th) return raw;
    if (a.smag) {
        raw.nq = (int)min((int64_t)4, max((int64_t)0, (a.spitch - (g.X0 + cb)) >> 2));
        if (raw.nq > 0) {
            const float* row = a.smag + (int64_t)(g.Y0 + r) * a.spitch + g.X0 + cb;
#pragma unroll
            for (int q = 0; q < 4; ++q) raw.q[q] = reinterpret_cast<const float4*>(row)[min(q, raw.nq - 1)];
        }
    } else {
        const uint8_t* row = a.cls + (int64_t)(g.Y0 + r) * a.cpitch + ((g.X0 + cb) >> 2);
        const int avail = (int)(a.cpitch - ((g.X0 + cb) >> 2));  // bytes left in the row
        if (avail >= 4) {
            raw.cls = *reinterpret_cast<const uint32_t*>(row);
        } else {
            for (int k = 0; k < avail; ++k) raw.cls |= (uint32_t)row[k] << (8 * k);
        }
    }
    return raw;
}

// Candidate and strong masks of the thread's 16 pixels (bit k: pixel k).
// From the class map: code >= 1 and code 2.  From the signed strength map:
// kept (value > 0) and >= lo, kept and > hi.  There the floats' bit patterns
// are compared as int32: non-negative floats order like their bits and every
// negative float (a suppressed pixel, -0 included) lies below them, so
// "e > 0 and e >= lo" is bits(e) >= max(bits(lo), 1) and "e > hi" is
// bits(e) > max(bits(hi), 0) (which also reads a threshold of -0 as 0) --
// two compares per pixel and no branches.  Pixels past the image edge are 0.
struct SegMasks {
    uint32_t cand, strong;
};

template <int T>
__device__ __forceinline__ SegMasks raw_masks(const HystArgs& a, const TileGeom& g, const RawSeg& raw, float mx) {
    using TL = Tile<T>;
    const int t = g.t;
    const int r = t / TL::kTPR;
    const int cb = (t % TL::kTPR) * TL::kPPT;
    SegMasks m = {0u, 0u};
    if (r >= g.th) return m;
    if (a.smag) {
        const float lo = a.relative ? a.low * mx : a.low;
        const float hi = a.relative ? a.high * mx : a.high;
        const int lob = max(__float_as_int(lo), 1);
        const int hib = max(__float_as_int(hi), 0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float e[4] = {raw.q[q].x, raw.q[q].y, raw.q[q].z, raw.q[q].w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int b = __float_as_int(e[k]);
                m.cand |= (b >= lob ? 1u : 0u) << (4 * q + k);
                m.strong |= (b > hib ? 1u : 0u) << (4 * q + k);
            }
        }
        const uint32_t qm = raw.nq >= 4 ? 0xFFFFu : (1u << (4 * raw.nq)) - 1u;  // whole quads read
        m.cand &= qm;
        m.strong &= qm;
    } else {
        m.cand = compress2(raw.cls | (raw.cls >> 1));
        m.strong = compress2((raw.cls >> 1) & ~raw.cls);  // code 2
    }
    const int valid = min(max(a.W - (g.X0 + cb), 0), TL::kPPT);
    const uint32_t vm = valid >= 16 ? 0xFFFFu : (1u << valid) - 1u;
    m.cand &= vm;
    m.strong &= vm;
    return m;
}

// Inclusive prefix sum over the 64 lanes of a wave: DPP row shifts within
// each 16-lane row, then lane 15's and lane 31's sums broadcast into the rows
// after them.
__device__ __forceinline__ int wave_incl_sum(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, false);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, false);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, false);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, false);  // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);  // row_bcast:15 -> rows 1, 3
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false);  // row_bcast:31 -> rows 2, 3
    return v;
}

// Largest value over the 64 lanes of a wave, in every lane.
__device__ __forceinline__ uint32_t wave_umax(uint32_t v) {
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false));  // row_shr:1
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false));  // row_shr:2
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false));  // row_shr:4
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false));  // row_shr:8
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false));  // row_bcast:15
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false));  // row_bcast:31
    return (uint32_t)__builtin_amdgcn_readlane((int)v, kWave - 1);
}

// Orders a wave's LDS writes before its later LDS reads (a wave's LDS
// instructions execute in order; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Runs the items of a wave's lanes (lane l's items: the set bits of its w,
// item(bit) encoding each) spread over all 64 lanes.  In rounds of up to 64
// items the owners write their items to the wave's list in LDS and lane j
// runs item j of the round, so a wave takes (its item count / 64) rounds
// instead of the largest count of one lane.
template <typename Item, typename Work>
__device__ __forceinline__ void wave_spread(int lane, uint64_t w, uint32_t* list, Item item, Work work) {
    const int cnt = __popcll(w);
    const int incl = wave_incl_sum(cnt);
    const int total = __builtin_amdgcn_readlane(incl, kWave - 1);
    int idx = incl - cnt;  // this lane's first item
    for (int base = 0; base < total; base += kWave) {
        for (; w && idx < base + kWave; w &= w - 1, ++idx) list[idx - base] = item(__ffsll((long long)w) - 1);
        wave_lds_sync();
        if (lane < total - base) work(list[lane]);
        wave_lds_sync();
    }
}

// Columns 8-adjacent to the run of row mask m that starts at column c0:
// c0 - 1 .. c1 + 1, clipped to the row (c1 the run's last column).
__device__ __forceinline__ uint64_t adj_window(uint64_t m, int c0) {
    const uint64_t rest = ~m >> c0;
    const int c1 = c0 + (rest ? __ffsll((long long)rest) - 1 : 64 - c0) - 1;
    const uint64_t lo = c0 == 0 ? ~0ull : ~0ull << (c0 - 1);
    const uint64_t hi = c1 >= 62 ? ~0ull : (2ull << (c1 + 1)) - 1ull;
    return lo & hi;
}

__device__ __forceinline__ int ctz64(uint64_t v) { return __ffsll((long long)v) - 1; }

// Label the tile's candidates in LDS from this thread's candidate and strong
// masks.
// Afterwards L[r*64 + s] holds the root (smallest index) of the component
// of the run that starts at column s of row r (only run starts' entries are
// used), every root's entry carries its component's largest border index
// and `strong` its strong bit.  cm and smk hold the 64-bit candidate and
// strong masks of every tile row.
//   phase 1: row masks
//   phase 2: each run start with a run of the row above among its
//            8-neighbours points at one of them (the one holding the lowest
//            such column), any other run start at itself: a plain store, one
//            writer per entry (entries of other pixels are never read).  The runs
//            now form trees that follow the image upwards, as deep as the
//            tile is tall.
//   phase 3: pointer jumping flattens the trees (each linked run start
//            repeatedly takes its parent's parent, all at once, so depths
//            halve per step), then the run's other neighbour runs above are
//            joined by union-find -- only rows where two branches meet.
//   phase 4: each run start walks to its root and stores it; a run with a
//            strong pixel sets its root's strong bit, and a run on the tile
//            border raises its root's border index -- per run, from the
//            run's extent, instead of per pixel
// Phases 3 and 4 spread their run starts over the lanes of the wave
// (wave_spread): a segment holds 0 to 8 of them, so per lane the counts are
// uneven while a wave's total is small.
template <int T>
__device__ __forceinline__ TileLabel<T> tile_label(SegMasks masks, const TileGeom& g, int* L,
                                                   uint64_t* cm, uint64_t* smk, uint32_t* strong,
                                                   uint32_t* list) {
    using TL = Tile<T>;
    static_assert(TL::kPPT == 16, "row masks assume 16-pixel segments");
    const int t = g.t;
    const int r = t / TL::kTPR;
    const int seg = t % TL::kTPR;
    const int cb = seg * TL::kPPT;
    const int me = r * kHystCols;
    const int up = me - kHystCols;
    TileLabel<T> st;
    st.cand = masks.cand;
    st.strong = masks.strong;
    reinterpret_cast<uint16_t*>(cm)[r * 4 + seg] = (uint16_t)st.cand;
    reinterpret_cast<uint16_t*>(smk)[r * 4 + seg] = (uint16_t)st.strong;
    __syncthreads();
    st.m = cm[r];
    st.S = st.m & ~(st.m << 1);
    const uint32_t starts = (uint32_t)(st.S >> cb) & 0xFFFFu;
    uint64_t A = 0, SA = 0;
    uint32_t linked = 0;  // run starts of the segment (bit k: column cb + k) that point up
    uint32_t more = 0;    // ... and have more than one neighbour run above
    if (r > 0) {
        A = cm[r - 1];
        SA = A & ~(A << 1);
    }
    // only run starts' entries are ever read (every pointer, union and
    // lookup goes through a run start), so each run start writes its own
    // entry here: the run it points at, or itself
    for (uint32_t b = starts; b; b &= b - 1) {
        const int k = __ffs(b) - 1;
        const uint64_t win = adj_window(st.m, cb + k);
        const uint64_t ov = A & win;
        int target = me + cb + k;
        if (ov) {
            const int lo = ctz64(ov);
            target = up + run_start(SA, lo);
            linked |= 1u << k;
            if (SA & win & ~((2ull << lo) - 1ull)) more |= 1u << k;
        }
        L[me + cb + k] = target;
    }
    __syncthreads();
    volatile lds_i32* V = lds_volatile(L);
    // pointer jumping: every entry only ever moves to an ancestor (a smaller
    // index), so a jump stays within i + 1 steps, and a concurrent union's
    // path halving or linking leaves every pointer an ancestor as well
    wave_spread(
        t & (kWave - 1), linked, list, [&](int pos) -> uint32_t { return (uint32_t)(me + cb + pos); },
        [&](uint32_t it) {
            const int i = (int)it;
            int x = V[i];
            for (int steps = i; steps >= 0; --steps) {
                const int gp = V[x];
                if (gp == x) break;
                x = gp;
                V[i] = x;
            }
        });
    // the run's other neighbour runs above: those starting after the run
    // that phase 2 linked to, up to column c1 + 1
    for (uint32_t b = more; b; b &= b - 1) {
        const int c0 = cb + __ffs(b) - 1;
        const uint64_t win = adj_window(st.m, c0);
        const int lo = ctz64(A & win);
        for (uint64_t e = SA & win & ~((2ull << lo) - 1ull); e; e &= e - 1)
            lds_union(L, me + c0, up + ctz64(e));
    }
    __syncthreads();
    // all unions are in: each run start walks to its root (pointers only
    // decrease, so within i + 1 steps).  A walk reads either an old pointer (an
    // ancestor), a root, or a root entry whose border bits another run has
    // already raised, hence the mask; a run start that is itself a root keeps
    // its entry (another run may be raising its border bits).
    const int th = g.th, tw = g.tw;
    wave_spread(
        t & (kWave - 1), starts, list, [&](int pos) -> uint32_t { return (uint32_t)(me + cb + pos); },
        [&](uint32_t it) {
            const int i = (int)it;
            const int rr = i >> 6, c0 = i & (kHystCols - 1);
            const uint64_t mrow = cm[rr];
            const uint64_t srow = smk[rr];
            int x = V[i] & kRootMask;
            for (int steps = i; steps >= 0; --steps) {
                const int p = V[x] & kRootMask;
                if (p == x) break;
                x = p;
            }
            if (x != i) V[i] = x;
            // the run covers columns c0 .. c1 (its first 0 bit above c0, minus one)
            const uint64_t rest = ~mrow >> c0;
            const int c1 = c0 + (rest ? __ffsll((long long)rest) - 1 : 64 - c0) - 1;
            const uint64_t span = (c1 - c0 >= 63) ? ~0ull : (((2ull << (c1 - c0)) - 1ull) << c0);
            if (srow & span) atomicOr(&strong[x >> 5], 1u << (x & 31));
            const int bmax = run_border_max(rr, c0, c1, th, tw);
            if (bmax >= 0) atomicMax(&L[x], x | ((1 + bmax) << kBrepShift));
        });
    __syncthreads();
    return st;
}

// global names of border components: tile * kNamesPerTile + border index
constexpr int kNamesPerTile = 256;

template <int T>
struct LocalSmem {
    alignas(16) int L[Tile<T>::kPx];
    uint64_t cm[T];                      // candidate mask of each tile row
    uint64_t smk[T];                     // strong mask of each tile row
    uint32_t strong[Tile<T>::kPx / 32];  // strong bit of each root
    uint32_t list[kWGThreads];           // per wave: the items of a wave_spread round
    uint32_t wmax[kWGThreads / kWave];   // per wave: largest strength slot seen
};

// border pixel index b of tile pixel (r, c), or -1 inside (see the file comment)
__device__ __forceinline__ int border_index(int r, int c, int th, int tw) {
    if (r == 0) return c;
    if (r == th - 1) return kHystCols + c;
    if (c == 0) return 2 * kHystCols - 1 + r;
    if (c == tw - 1) return 3 * kHystCols - 3 + r;
    return -1;
}

// the border slot holding the global name of border pixel index b
template <int T>
__device__ __forceinline__ int border_slot(int b) {
    if (b < 2 * kHystCols) return b;                                      // top / bottom row
    if (b < 3 * kHystCols - 2) return 2 * kHystCols + (b - 2 * kHystCols + 1);  // left column
    return 2 * kHystCols + T + (b - (3 * kHystCols - 2) + 1);               // right column
}

// A thread's 16 output bytes (row segment of a tile) as two little-endian
// 64-bit words; byte k is pixel k.  Helpers take compile-time or run-time k
// without a dynamically indexed array (which would live in scratch or LDS).
struct Seg16 {
    uint64_t lo = 0, hi = 0;
    __device__ __forceinline__ uint32_t get(int k) const {
        return (uint32_t)((k < 8 ? lo >> (8 * k) : hi >> (8 * (k - 8))) & 0xFFu);
    }
    __device__ __forceinline__ void set(int k, uint32_t v) {  // byte k must be 0
        if (k < 8) lo |= (uint64_t)v << (8 * k);
        else hi |= (uint64_t)v << (8 * (k - 8));
    }
    __device__ __forceinline__ void put(int k, uint32_t v) {
        if (k < 8) lo = (lo & ~(0xFFull << (8 * k))) | ((uint64_t)v << (8 * k));
        else hi = (hi & ~(0xFFull << (8 * (k - 8)))) | ((uint64_t)v << (8 * (k - 8)));
    }
};

// A full 16-byte segment at any alignment: one 16-byte store when aligned;
// otherwise the bytes before the first 4-byte boundary, three aligned dwords
// and the bytes after them (every byte written lies inside the segment, so
// neighbouring segments of other threads are never touched).  Rows whose
// pitch is not a multiple of 16 (uneven widths) take this path.
__device__ __forceinline__ void store_seg(uint8_t* dst, const Seg16& o, int valid, int vec16) {
    const uint32_t w[4] = {(uint32_t)o.lo, (uint32_t)(o.lo >> 32), (uint32_t)o.hi, (uint32_t)(o.hi >> 32)};
    if (vec16 && valid == 16) {
        *reinterpret_cast<uint4*>(dst) = make_uint4(w[0], w[1], w[2], w[3]);
    } else if (valid == 16) {
        const int k = (int)((uintptr_t)dst & 3);
        if (k == 0) {
#pragma unroll
            for (int i = 0; i < 4; ++i) reinterpret_cast<uint32_t*>(dst)[i] = w[i];
        } else {
            const int h = 4 - k;  // bytes up to the first 4-byte boundary
#pragma unroll
            for (int b = 0; b < 3; ++b)
                if (b < h) dst[b] = (uint8_t)(w[0] >> (8 * b));
            uint32_t* d32 = reinterpret_cast<uint32_t*>(dst + h);
#pragma unroll
            for (int i = 0; i < 3; ++i) d32[i] = __builtin_amdgcn_alignbyte(w[i + 1], w[i], h);
#pragma unroll
            for (int b = 0; b < 3; ++b)
                if (b < k) dst[16 - k + b] = (uint8_t)(w[3] >> (8 * (h + b)));
        }
    } else {
        for (int k = 0; k < valid; ++k) dst[k] = (uint8_t)o.get(k);
    }
}

// A full segment read at any alignment.  Unaligned: the aligned dwords that
// cover it (up to 3 bytes either side), joined by byte funnel shifts; used
// only where those extra bytes lie inside the row (wide_ok: at least 4
// columns before the segment and 4 after it).
__device__ __forceinline__ Seg16 load_seg(const uint8_t* src, int valid, int vec16, bool wide_ok) {
    Seg16 out;
    if (vec16 && valid == 16) {
        const uint4 v = *reinterpret_cast<const uint4*>(src);
        out.lo = v.x | (uint64_t)v.y << 32;
        out.hi = v.z | (uint64_t)v.w << 32;
    } else if (valid == 16 && (((uintptr_t)src & 3) == 0 || wide_ok)) {
        const int k = (int)((uintptr_t)src & 3);
        const uint32_t* s32 = reinterpret_cast<const uint32_t*>(src - k);
        uint32_t d[5];
#pragma unroll
        for (int i = 0; i < 4; ++i) d[i] = s32[i];
        d[4] = k ? s32[4] : 0u;
        uint32_t w[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) w[i] = __builtin_amdgcn_alignbyte(d[i + 1], d[i], k);
        out.lo = w[0] | (uint64_t)w[1] << 32;
        out.hi = w[2] | (uint64_t)w[3] << 32;
    } else {
        for (int k = 0; k < valid; ++k) out.set(k, src[k]);
    }
    return out;
}

// Pass 1 on one tile (the whole workgroup takes part).
template <int T>
__device__ __forceinline__ void local_tile(const HystArgs& a, const TileGeom& g, const RawSeg& raw,
                                           int vec16, LocalSmem<T>& sm) {
    using TL = Tile<T>;
    static_assert(T <= kHystCols, "border pixel indices assume T <= 64");
    int* L = sm.L;
    const int t = g.t;
    for (int w = t; w < TL::kPx / 32; w += kWGThreads) sm.strong[w] = 0u;
    // the float path's largest strength: one word, or the walk's per-wave
    // slots reduced here (non-negative float bits order as unsigned integers)
    float mx = 0.0f;
    if (a.smag) {
        uint32_t mb;
        if (a.maxslots) {
            // 16-byte loads, all in flight at once (kMaxSlots / 4 / 256 per
            // thread); words past nslots in the last quad are masked
            static_assert(kMaxSlots % (4 * kWGThreads) == 0, "whole quads per thread");
            const uint4* q4 = reinterpret_cast<const uint4*>(a.maxslots);
            uint32_t m = 0;
#pragma unroll
            for (int k = 0; k < kMaxSlots / 4 / kWGThreads; ++k) {
                const int q = t + k * kWGThreads;
                if (4 * q < a.nslots) {
                    const uint4 v = q4[q];
                    const int n = a.nslots - 4 * q;  // valid words of this quad (>= 1)
                    m = max(m, max(max(v.x, n > 1 ? v.y : 0u), max(n > 2 ? v.z : 0u, n > 3 ? v.w : 0u)));
                }
            }
            m = wave_umax(m);
            if ((t & (kWave - 1)) == 0) sm.wmax[t / kWave] = m;
            __syncthreads();
            mb = max(max(sm.wmax[0], sm.wmax[1]), max(sm.wmax[2], sm.wmax[3]));
        } else {
            mb = *a.maxbits;
        }
        mx = __uint_as_float(mb);
        if (a.max_out && g.tile == 0 && t == 0) *a.max_out = mx;
    }
    const TileLabel<T> st = tile_label<T>(raw_masks<T>(a, g, raw, mx), g, L, sm.cm, sm.smk, sm.strong,
                                          sm.list + (t / kWave) * kWave);
    const int r = t / TL::kTPR;
    const int cb = (t % TL::kTPR) * TL::kPPT;
    const int me = r * kHystCols;
    // every candidate: 255 for a component with a strong pixel, 0 for one
    // without that stays inside the tile, the pending code 1 + b for one
    // without that touches the border (b its largest border index); one
    // lookup per run that covers pixels of the segment (the first may start
    // in an earlier segment)
    bool pending = false;
    if (r < g.th) {
        uint32_t w[4] = {0u, 0u, 0u, 0u};
        const uint32_t starts = (uint32_t)(st.S >> cb) & 0xFFFFu;
        for (uint32_t h = starts | (st.cand & 1u); h; h &= h - 1) {
            const int k0 = __ffs(h) - 1;
            const int k1 = k0 + __ffs(~st.cand >> k0) - 2;  // the run's last pixel in the segment
            const int s0 = (starts >> k0) & 1u ? cb + k0 : run_start(st.S, cb);
            const int root = L[me + s0] & kRootMask;
            const uint32_t br = (uint32_t)L[root] >> kBrepShift;
            const bool strong = (sm.strong[root >> 5] >> (root & 31)) & 1u;
            const bool pend = br != 0 && !strong;
            pending |= pend;
            // Byte permutes instead of 32-bit integer multiplies (those issue
            // at a quarter of the VALU rate): selector 0 repeats byte 0 of
            // the second operand, selectors 0x0C / 0x0D give 0x00 / 0xFF.
            const uint32_t v = __builtin_amdgcn_perm(0u, pend ? br : (strong ? 255u : 0u), 0u);
            const uint32_t span = ((2u << k1) - 1u) & ~((1u << k0) - 1u);
#pragma unroll
            for (int q = 0; q < 4; ++q) {  // bit j of a nibble -> byte j (0x00 / 0xFF)
                const uint32_t b = (((span >> (4 * q)) & 15u) * 0x00204081u) & 0x01010101u;  // 24-bit multiply
                w[q] |= __builtin_amdgcn_perm(0u, 0u, b | 0x0C0C0C0Cu) & v;
            }
        }
        Seg16 out;
        out.lo = w[0] | (uint64_t)w[1] << 32;
        out.hi = w[2] | (uint64_t)w[3] << 32;
        const int valid = min(a.W - (g.X0 + cb), TL::kPPT);
        if (valid > 0) store_seg(a.edges + (int64_t)(g.Y0 + r) * a.epitch + g.X0 + cb, out, valid, vec16);
    }
    // one bit per thread segment with pending codes, one word per wave
    const uint64_t pm = __ballot(pending);
    if ((t & (kWave - 1)) == 0) a.pmask[(int64_t)g.tile * (kWGThreads / kWave) + t / kWave] = pm;
    // the union-find key of every border slot's component (-1: no
    // candidate); the slot of the pixel whose border index names the
    // component starts its union-find entry
    const int base = g.tile * TL::kPerim;
    for (int s = t; s < TL::kPerim; s += kWGThreads) {
        int pr, pc;
        bool in;
        if (s < kHystCols) { pr = 0; pc = s; in = pc < g.tw; }
        else if (s < 2 * kHystCols) { pr = g.th - 1; pc = s - kHystCols; in = pc < g.tw; }
        else if (s < 2 * kHystCols + T) { pr = s - 2 * kHystCols; pc = 0; in = pr < g.th; }
        else { pr = s - 2 * kHystCols - T; pc = g.tw - 1; in = pr < g.th; }
        int key = -1;
        const uint64_t mr = in ? sm.cm[pr] : 0ull;
        if ((mr >> pc) & 1ull) {
            const int root = L[pr * kHystCols + run_start(mr & ~(mr << 1), pc)] & kRootMask;
            const int br = (int)((uint32_t)L[root] >> kBrepShift);  // >= 1 on the border
            const int name = g.tile * kNamesPerTile + br - 1;
            key = (sm.strong[root >> 5] >> (root & 31)) & 1u ? name : name | kWeakKey;
            const int bi = border_index(pr, pc, g.th, g.tw);
            if (bi == br - 1 && border_slot<T>(bi) == s) a.parent[name] = key;
        }
        a.blab[base + s] = key;
    }
}

// One tile per workgroup.  Each XCD takes a contiguous range of tiles:
// neighbouring tiles share the cache lines of the class map and the edge map,
// and each XCD has its own L2.  (Persistent forms -- as many workgroups as
// the chip holds, each taking tile after tile, from per-XCD atomic counters
// or in a fixed order -- measured slower: 65.9 and 61.7 against 55 us for the
// integer hysteresis at 4096^2, then in four passes; so did static pairs of
// tiles per workgroup
// with the second one's loads issued early, 44 -> 57 us for the float pass.)
template <int T>
__global__ void __launch_bounds__(kWGThreads) k_hyst_local(HystArgs a, int tiles_x, int vec16) {
    __shared__ LocalSmem<T> sm;
    const TileGeom g = tile_geom<T>(xcd_remap(blockIdx.x, gridDim.x), tiles_x, a.H, a.W);
    local_tile<T>(a, g, load_raw<T>(a, g), vec16, sm);
}

// Unions of border key gp with the keys q[0..2] of its three neighbours across
// the tile edge (-1: none).  Two components that are both strong need no
// union: every set that either one joins is strong anyway.  When the previous
// pixel along the edge has the same key (cont), that pixel's own unions
// already cover q[0] and q[1] (they are its q[1] and q[2]), so only q[2]
// remains, and only if it differs from q[1]; by induction along the run,
// every pixel's three neighbours end up joined.  Repeats among consecutive
// neighbours are skipped as well.
__device__ __forceinline__ void merge_unions(int* parent, int gp, bool cont, const int (&q)[3]) {
    int prev = cont ? q[1] : -1;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (cont && d < 2) continue;
        const int gq = q[d];
        if (gq >= 0 && gq != prev && (gp | gq) >= kWeakKey) g_union(parent, gp, gq);
        prev = gq;
    }
}

// Pass 2 for border pixel k of a tile (k < T: right edge row k; else bottom
// edge column k - T).  All neighbour keys are loaded before the first union.
template <int T>
__device__ __forceinline__ void merge_one(const HystArgs& a, int tile, int k, int tiles_x, int tiles_y) {
    using TL = Tile<T>;
    const TileGeom g = tile_geom<T>(tile, tiles_x, a.H, a.W);
    const int base = tile * TL::kPerim;
    int q[3];
    if (k < T) {  // right tile edge: pixel (k, tw-1) against column X0+64
        if (k >= g.th || g.tx + 1 >= tiles_x) return;
        const int* slots = a.blab + base + 2 * kHystCols + T;  // right column, row r at r
        const int gp = slots[k];
        const int gprev = k > 0 ? slots[k - 1] : -1;
        if (gp < 0) return;
        const int qx_tile = g.tx + 1;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int qy = g.Y0 + k + d - 1;
            q[d] = -1;
            if (qy >= 0 && qy < a.H) {
                const int qty = qy / T, qr = qy - qty * T;
                q[d] = a.blab[(qty * tiles_x + qx_tile) * TL::kPerim + 2 * kHystCols + qr];
            }
        }
        merge_unions(a.parent, gp, gprev == gp, q);
    } else {  // bottom tile edge: pixel (th-1, c) against row Y0+T
        const int c = k - T;
        if (c >= g.tw || g.ty + 1 >= tiles_y) return;
        const int* slots = a.blab + base + kHystCols;  // bottom row, column c at c
        const int gp = slots[c];
        const int gprev = c > 0 ? slots[c - 1] : -1;
        if (gp < 0) return;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int qx = g.X0 + c + d - 1;
            q[d] = -1;
            if (qx >= 0 && qx < a.W) {
                const int qtx = qx / kHystCols, qc = qx - qtx * kHystCols;
                q[d] = a.blab[((g.ty + 1) * tiles_x + qtx) * TL::kPerim + qc];
            }
        }
        merge_unions(a.parent, gp, gprev == gp, q);
    }
}

template <int T>
__global__ void __launch_bounds__(kWGThreads)
k_hyst_merge(HystArgs a, int tiles_x, int tiles_y, int ntiles) {
    const int per_tile = T + kHystCols;
    const int64_t gid = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)ntiles * per_tile) return;
    const int tile = (int)(gid / per_tile);
    merge_one<T>(a, tile, (int)(gid - (int64_t)tile * per_tile), tiles_x, tiles_y);
}

// Whether the set of key k holds a strong pixel: walk towards the root until
// a strong key (then the root's, smaller still, is strong too) or a weak root.
// Path halving: each visited entry gets its grandparent, an ancestor, so the
// long chains that simultaneous unions leave along an edge crossing many
// tiles shrink for the other threads walking them.  No union runs during
// this pass, so a halving store never overwrites a root.
__device__ __forceinline__ bool key_strong(int* parent, int k) {
    for (int steps = k; steps >= 0; --steps) {
        if (k < kWeakKey) return true;
        const int p = parent[k & kNameMask];
        if (p == k) return false;
        if (p < kWeakKey) return true;
        const int gp = parent[p & kNameMask];
        if (gp == p) return false;
        parent[k & kNameMask] = gp;
        k = gp;
    }
    return false;  // not reached: keys fall along a walk
}

// Pass 3 on one tile: pending codes 1..252 become 255 / 0 by whether the set
// of that border component holds a strong pixel; everything else is already
// final.  Only the thread segments the local pass marked in pmask are read
// and rewritten (a tile without any is skipped); the workgroup resolves every
// border pixel index once (res: LDS, 252 entries), so each pending pixel
// costs one LDS read.
template <int T>
__device__ __forceinline__ void resolve_tile(const HystArgs& a, int tile, int tiles_x, int vec16,
                                             uint8_t* res) {
    using TL = Tile<T>;
    static_assert(kWGThreads >= 3 * kHystCols + T - 4, "one thread per border pixel index");
    const int t = threadIdx.x;
    // the border keys are loaded together with the pending masks, so a tile
    // with pending segments waits for two dependent loads (masks and keys,
    // then segments and the keys' parents) where a walk stops at once
    const bool bthr = t < 2 * kHystCols + 2 * (T - 2);
    int key = -1;
    if (bthr) key = a.blab[(int64_t)tile * TL::kPerim + border_slot<T>(t)];
    // segments with pending codes (the local pass's masks; identical reads in
    // every thread, so the early exit below is uniform)
    const uint64_t* pmt = a.pmask + (int64_t)tile * (kWGThreads / kWave);
    uint64_t any_pm = 0;
#pragma unroll
    for (int w = 0; w < kWGThreads / kWave; ++w) any_pm |= pmt[w];
    if (!any_pm) return;
    const bool mine = (pmt[t / kWave] >> (t & (kWave - 1))) & 1ull;
    const TileGeom g = tile_geom<T>(tile, tiles_x, a.H, a.W);
    const int r = t / TL::kTPR;
    const int cb = (t % TL::kTPR) * TL::kPPT;
    const int valid = r < g.th ? min(a.W - (g.X0 + cb), TL::kPPT) : 0;
    uint8_t* dst = a.edges + (int64_t)(g.Y0 + r) * a.epitch + g.X0 + cb;
    Seg16 out;
    if (mine) {
        const int col0 = g.X0 + cb;
        out = load_seg(dst, valid, vec16, col0 >= 4 && col0 + TL::kPPT + 4 <= a.W);
    }
    if (bthr) res[t] = key >= 0 && key_strong(a.parent, key) ? 255 : 0;
    __syncthreads();
    if (!mine) return;
#pragma unroll
    for (int k = 0; k < TL::kPPT; ++k) {
        const uint32_t e = out.get(k);
        if (e == 0 || e == 255) continue;  // final already (bytes past `valid` are 0)
        out.put(k, res[e - 1]);
    }
    store_seg(dst, out, valid, vec16);
}

template <int T>
__global__ void __launch_bounds__(kWGThreads) k_hyst_resolve(HystArgs a, int tiles_x, int vec16) {
    __shared__ uint8_t res[kWGThreads];
    resolve_tile<T>(a, xcd_remap(blockIdx.x, gridDim.x), tiles_x, vec16, res);
}

template <int T>
hipError_t launch_t(const HystArgs& a, hipStream_t s) {
    const int tiles_x = ceil_div(a.W, kHystCols);
    const int tiles_y = ceil_div(a.H, T);
    const int ntiles = tiles_x * tiles_y;
    const int vec16 = ((uintptr_t)a.edges % 16 == 0) && (a.epitch % 16 == 0);
    hipLaunchKernelGGL(k_hyst_local<T>, dim3(ntiles), dim3(kWGThreads), 0, s, a, tiles_x, vec16);
    const int64_t nmerge = (int64_t)ntiles * (T + kHystCols);
    hipLaunchKernelGGL(k_hyst_merge<T>, dim3((unsigned)ceil_div64(nmerge, kWGThreads)),
                       dim3(kWGThreads), 0, s, a, tiles_x, tiles_y, ntiles);
    hipLaunchKernelGGL(k_hyst_resolve<T>, dim3(ntiles), dim3(kWGThreads), 0, s, a, tiles_x, vec16);
    return hipGetLastError();
}

// ------------------------------------------------------------- batches
__device__ __forceinline__ HystArgs batch_args(const BatchImage& im, char* ws) {
    HystArgs a;
    a.cls = reinterpret_cast<const uint8_t*>(ws + im.cls_off);
    a.cpitch = im.cpitch;
    a.H = im.H;
    a.W = im.W;
    a.edges = im.edges;
    a.epitch = im.epitch;
    a.blab = reinterpret_cast<int32_t*>(ws + im.blab_off);
    a.parent = reinterpret_cast<int32_t*>(ws + im.parent_off);
    a.pmask = reinterpret_cast<uint64_t*>(ws + im.pmask_off);
    return a;
}

// Batch passes: flat grids over all images; a tile's image comes from the
// plan's tile -> image table (merge items are 128 per tile, in tile order,
// so they index the same table).
template <int T>
__global__ void __launch_bounds__(kWGThreads)
k_hyst_local_batch(const BatchImage* imgs, const BatchDev* hdr) {
    __shared__ LocalSmem<T> sm;
    const int task = xcd_remap(blockIdx.x, gridDim.x);
    if (task >= hdr->total_tiles) return;
    const BatchImage& im = imgs[hdr->tile_img[task]];
    const int vec16 = ((uintptr_t)im.edges % 16 == 0) && (im.epitch % 16 == 0);
    const HystArgs a = batch_args(im, hdr->ws);
    const TileGeom g = tile_geom<T>(task - im.tile_base, im.tiles_x, im.H, im.W);
    local_tile<T>(a, g, load_raw<T>(a, g), vec16, sm);
}

template <int T>
__global__ void __launch_bounds__(kWGThreads) k_hyst_merge_batch(const BatchImage* imgs, const BatchDev* hdr) {
    const int g = xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (g >= hdr->total_merge) return;
    const BatchImage& im = imgs[hdr->tile_img[g / (T + kHystCols)]];
    const int local = g - im.merge_base;
    const int tile = local / (T + kHystCols);
    merge_one<T>(batch_args(im, hdr->ws), tile, local - tile * (T + kHystCols), im.tiles_x, im.tiles_y);
}

template <int T>
__global__ void __launch_bounds__(kWGThreads)
k_hyst_resolve_batch(const BatchImage* imgs, const BatchDev* hdr) {
    // one workgroup per tile of the batch (most tiles exit at once, so the
    // hardware dispatcher, not a software loop, should pace them)
    __shared__ uint8_t res[kWGThreads];
    const int task = xcd_remap(blockIdx.x, gridDim.x);
    if (task >= hdr->total_tiles) return;
    const BatchImage& im = imgs[hdr->tile_img[task]];
    const int vec16 = ((uintptr_t)im.edges % 16 == 0) && (im.epitch % 16 == 0);
    resolve_tile<T>(batch_args(im, hdr->ws), task - im.tile_base, im.tiles_x, vec16, res);
}

}  // namespace

hipError_t launch_hyst_batch(const BatchImage* imgs, const BatchDev* hdr, int total_tiles,
                             int total_merge, hipStream_t s) {
    constexpr int T = 64;
    hipLaunchKernelGGL(k_hyst_local_batch<T>, dim3(max(total_tiles, 1)), dim3(kWGThreads), 0, s,
                       imgs, hdr);
    hipLaunchKernelGGL(k_hyst_merge_batch<T>, dim3(ceil_div(max(total_merge, 1), kWGThreads)),
                       dim3(kWGThreads), 0, s, imgs, hdr);
    hipLaunchKernelGGL(k_hyst_resolve_batch<T>, dim3(max(total_tiles, 1)), dim3(kWGThreads), 0, s,
                       imgs, hdr);
    return hipGetLastError();
}

int hyst_tile_rows_default() { return 64; }

static int perim(int tile_rows) { return 2 * kHystCols + 2 * tile_rows; }

static size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

// blab: int32 per border slot; parent: int32 per component name (256 per
// tile; only the names of this call's border components are written and
// read); pmask: one 64-bit word per wave of a tile.  About 0.51 B per pixel.
size_t hyst_workspace_bytes(int H, int W, int tile_rows) {
    const size_t ntiles = (size_t)ceil_div(W, kHystCols) * ceil_div(H, tile_rows);
    const size_t nnames = ntiles * (size_t)kNamesPerTile;
    return al256(ntiles * perim(tile_rows) * 4) + al256(nnames * 4) +
           al256(ntiles * (kWGThreads / kWave) * 8);
}

void hyst_carve(void* ws, int H, int W, int tile_rows, HystArgs& a) {
    const size_t ntiles = (size_t)ceil_div(W, kHystCols) * ceil_div(H, tile_rows);
    const size_t nnames = ntiles * (size_t)kNamesPerTile;
    char* p = static_cast<char*>(ws);
    a.blab = reinterpret_cast<int32_t*>(p);
    p += al256(ntiles * perim(tile_rows) * 4);
    a.parent = reinterpret_cast<int32_t*>(p);
    p += al256(nnames * 4);
    a.pmask = reinterpret_cast<uint64_t*>(p);
}

hipError_t launch_hysteresis(const HystArgs& a, int tile_rows, hipStream_t s) {
    (void)tile_rows;  // 64-row tiles (16-pixel thread segments) only
    return launch_t<64>(a, s);
}

}  // namespace canny
