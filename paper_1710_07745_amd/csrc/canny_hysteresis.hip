// Step 4 of the paper (Section 2.2.1), hysteresis, as connected-component
// labelling on the GPU.  An edge pixel is a candidate (class >= 1) that is
// 8-connected through candidates to a strong pixel (class 2); equivalently,
// a candidate whose 8-connected component contains a strong pixel.  The
// paper keeps this step serial; here it is union-find, whose cost does not
// grow with the length of a propagation chain.
//
// The image is cut into 64-column x T-row tiles.  Four launches:
//   1. local:  each workgroup labels its tile in LDS (union-find with
//              atomicMin linking, roots = smallest pixel index), marks which
//              local components hold a strong pixel, and names every
//              component that touches the tile border by its smallest
//              border slot.  It writes, per border pixel, the global id of
//              its component (or -1), and initialises parent/flag for the
//              component representatives.
//   2. merge:  one thread per tile-border pixel on the right and bottom tile
//              edges unions its component with the 8-connected candidates
//              across the edge (global union-find, atomicMin linking).
//   3. flags:  every representative finds its root (read-only walk), stores
//              it in its own slot (flattening the forest) and ORs its strong
//              flag into the root's.
//   4. final:  each workgroup relabels its tile (same LDS pass as 1), lifts
//              the global strong flags onto its border components and
//              writes 255 / 0 per pixel.
// Border slots of a tile (clipped to the image): top row x -> x, bottom row
// x -> 64 + x, left column y -> 128 + y, right column y -> 128 + T + y.
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

__device__ __forceinline__ int lds_find(volatile int* L, int x) {
    int p = L[x];
    while (p != x) {
        x = p;
        p = L[x];
    }
    return x;
}

__device__ __forceinline__ void lds_union(int* L, int a, int b) {
    volatile int* V = L;
    while (true) {
        a = lds_find(V, a);
        b = lds_find(V, b);
        if (a == b) return;
        if (a < b) { const int t = a; a = b; b = t; }
        const int old = atomicMin(&L[a], b);
        if (old == a) return;
        a = old;
    }
}

__device__ __forceinline__ int g_load(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int g_find(int* parent, int x) {
    int p = g_load(parent + x);
    while (p != x) {
        x = p;
        p = g_load(parent + x);
    }
    return x;
}

__device__ __forceinline__ void g_union(int* parent, int a, int b) {
    while (true) {
        a = g_find(parent, a);
        b = g_find(parent, b);
        if (a == b) return;
        if (a < b) { const int t = a; a = b; b = t; }
        const int old = atomicMin(parent + a, b);
        if (old == a) return;
        a = old;
    }
}

struct TileGeom {
    int tile, ty, tx, X0, Y0, th, tw;
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
    return g;
}

// Load this thread's class codes and build the tile's LDS union-find.
// On return L[i] is the root (smallest index) of pixel i's component, or -1.
// codes: 2 bits per pixel of the thread's segment (bit 2k = pixel k).
template <int T>
__device__ __forceinline__ uint32_t tile_label(const uint8_t* cls, int64_t cpitch, int W,
                                               const TileGeom& g, int* L) {
    using TL = Tile<T>;
    const int t = threadIdx.x;
    const int r = t / TL::kTPR;
    const int cb = (t % TL::kTPR) * TL::kPPT;
    uint32_t codes = 0;
    if (r < g.th) {
        const uint8_t* row = cls + (int64_t)(g.Y0 + r) * cpitch + ((g.X0 + cb) >> 2);
        const int nbytes = TL::kPPT / 4;
        const int avail = (int)(cpitch - ((g.X0 + cb) >> 2));  // bytes left in the row
        if (avail >= nbytes) {
            if (nbytes == 4) codes = *reinterpret_cast<const uint32_t*>(row);
            else if (nbytes == 2) codes = *reinterpret_cast<const uint16_t*>(row);
            else codes = row[0];
        } else {
            for (int k = 0; k < avail; ++k) codes |= (uint32_t)row[k] << (8 * k);
        }
        // pixels past the image edge are not candidates
        const int valid = min(max(W - (g.X0 + cb), 0), TL::kPPT);
        if (valid < 16) codes &= (valid == 0) ? 0u : (0xFFFFFFFFu >> (32 - 2 * valid));
    }
#pragma unroll
    for (int k = 0; k < TL::kPPT; ++k) {
        const int i = r * kHystCols + cb + k;
        L[i] = ((codes >> (2 * k)) & 3u) ? i : -1;
    }
    __syncthreads();
    if (r < g.th) {
#pragma unroll
        for (int k = 0; k < TL::kPPT; ++k) {
            if (!((codes >> (2 * k)) & 3u)) continue;
            const int c = cb + k;
            const int i = r * kHystCols + c;
            if (c > 0 && L[i - 1] >= 0) lds_union(L, i, i - 1);
            if (r > 0) {
                const int up = i - kHystCols;
                if (c > 0 && L[up - 1] >= 0) lds_union(L, i, up - 1);
                if (L[up] >= 0) lds_union(L, i, up);
                if (c + 1 < kHystCols && L[up + 1] >= 0) lds_union(L, i, up + 1);
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < TL::kPPT; ++k) {
        const int i = r * kHystCols + cb + k;
        if ((codes >> (2 * k)) & 3u) L[i] = lds_find(L, i);
    }
    __syncthreads();
    return codes;
}

// Visit the border slots of pixel (r, c) of a tile clipped to th x tw.
template <int T, typename F>
__device__ __forceinline__ void for_slots(int r, int c, int th, int tw, F f) {
    if (r == 0) f(c);
    if (r == th - 1) f(kHystCols + c);
    if (c == 0) f(2 * kHystCols + r);
    if (c == tw - 1) f(2 * kHystCols + T + r);
}

template <int T>
__global__ void __launch_bounds__(kWGThreads) k_hyst_local(HystArgs a, int tiles_x) {
    using TL = Tile<T>;
    __shared__ int L[TL::kPx];
    __shared__ int rep[TL::kPx];
    __shared__ int sfl[TL::kPx];
    __shared__ int bl[TL::kPerim];  // staged border labels: one global store per slot
    const TileGeom g = tile_geom<T>(blockIdx.x, tiles_x, a.H, a.W);
    const int t = threadIdx.x;
    for (int i = t; i < TL::kPx; i += kWGThreads) { rep[i] = 0x7FFFFFFF; sfl[i] = 0; }
    for (int s = t; s < TL::kPerim; s += kWGThreads) bl[s] = -1;  // "no candidate"
    const uint32_t codes = tile_label<T>(a.cls, a.cpitch, a.W, g, L);
    const int r = t / TL::kTPR;
    const int cb = (t % TL::kTPR) * TL::kPPT;
    const int base = g.tile * TL::kPerim;
    if (r < g.th) {
#pragma unroll
        for (int k = 0; k < TL::kPPT; ++k) {
            const uint32_t code = (codes >> (2 * k)) & 3u;
            if (!code) continue;
            const int c = cb + k;
            const int root = L[r * kHystCols + c];
            if (code == 2) sfl[root] = 1;
            for_slots<T>(r, c, g.th, g.tw, [&](int s) { atomicMin(&rep[root], s); });
        }
    }
    __syncthreads();
    if (r < g.th) {
#pragma unroll
        for (int k = 0; k < TL::kPPT; ++k) {
            if (!((codes >> (2 * k)) & 3u)) continue;
            const int c = cb + k;
            const int root = L[r * kHystCols + c];
            const int rs = rep[root];
            for_slots<T>(r, c, g.th, g.tw, [&](int s) {
                bl[s] = base + rs;
                if (s == rs) {
                    a.parent[base + s] = base + s;
                    a.flag[base + s] = sfl[root];
                }
            });
        }
    }
    __syncthreads();
    for (int s = t; s < TL::kPerim; s += kWGThreads) a.blab[base + s] = bl[s];
}

template <int T>
__global__ void __launch_bounds__(kWGThreads)
k_hyst_merge(HystArgs a, int tiles_x, int tiles_y, int ntiles) {
    using TL = Tile<T>;
    const int per_tile = T + kHystCols;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)ntiles * per_tile) return;
    const int tile = (int)(gid / per_tile);
    const int k = (int)(gid - (int64_t)tile * per_tile);
    const TileGeom g = tile_geom<T>(tile, tiles_x, a.H, a.W);
    const int base = tile * TL::kPerim;
    if (k < T) {  // right tile edge: pixel (k, tw-1) against column X0+64
        if (k >= g.th || g.tx + 1 >= tiles_x) return;
        const int gp = a.blab[base + 2 * kHystCols + T + k];
        if (gp < 0) return;
        const int qx_tile = g.tx + 1;
        for (int dy = -1; dy <= 1; ++dy) {
            const int qy = g.Y0 + k + dy;
            if (qy < 0 || qy >= a.H) continue;
            const int qty = qy / T, qr = qy - qty * T;
            const int gq = a.blab[(qty * tiles_x + qx_tile) * TL::kPerim + 2 * kHystCols + qr];
            if (gq >= 0) g_union(a.parent, gp, gq);
        }
    } else {  // bottom tile edge: pixel (th-1, c) against row Y0+T
        const int c = k - T;
        if (c >= g.tw || g.ty + 1 >= tiles_y) return;
        const int gp = a.blab[base + kHystCols + c];
        if (gp < 0) return;
        for (int dx = -1; dx <= 1; ++dx) {
            const int qx = g.X0 + c + dx;
            if (qx < 0 || qx >= a.W) continue;
            const int qtx = qx / kHystCols, qc = qx - qtx * kHystCols;
            const int gq = a.blab[((g.ty + 1) * tiles_x + qtx) * TL::kPerim + qc];
            if (gq >= 0) g_union(a.parent, gp, gq);
        }
    }
}

template <int T>
__global__ void __launch_bounds__(kWGThreads) k_hyst_flags(HystArgs a, int nslots) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nslots) return;
    if (a.blab[s] != s) return;  // not a component representative
    // Read-only find; each thread then stores only its own slot, so every
    // pointer another thread may follow is either its old value (an ancestor)
    // or the root -- never a non-root written after the root.
    int x = s;
    int p = a.parent[x];
    while (p != x) {
        x = p;
        p = a.parent[x];
    }
    a.parent[s] = x;
    if (a.flag[s]) a.flag[x] = 1;
}

template <int T>
__global__ void __launch_bounds__(kWGThreads) k_hyst_final(HystArgs a, int tiles_x, int vec16) {
    using TL = Tile<T>;
    __shared__ int L[TL::kPx];
    __shared__ int sfl[TL::kPx];
    const TileGeom g = tile_geom<T>(blockIdx.x, tiles_x, a.H, a.W);
    const int t = threadIdx.x;
    for (int i = t; i < TL::kPx; i += kWGThreads) sfl[i] = 0;
    const uint32_t codes = tile_label<T>(a.cls, a.cpitch, a.W, g, L);
    const int r = t / TL::kTPR;
    const int cb = (t % TL::kTPR) * TL::kPPT;
    const int base = g.tile * TL::kPerim;
    if (r < g.th) {
#pragma unroll
        for (int k = 0; k < TL::kPPT; ++k) {
            const uint32_t code = (codes >> (2 * k)) & 3u;
            if (!code) continue;
            const int c = cb + k;
            const int root = L[r * kHystCols + c];
            if (code == 2) sfl[root] = 1;
            for_slots<T>(r, c, g.th, g.tw, [&](int s) {
                const int gl = a.blab[base + s];
                if (gl == base + s) {  // this slot represents the component
                    if (a.flag[a.parent[gl]]) sfl[root] = 1;
                }
            });
        }
    }
    __syncthreads();
    if (r < g.th) {
        uint8_t out[TL::kPPT];
#pragma unroll
        for (int k = 0; k < TL::kPPT; ++k) {
            const uint32_t code = (codes >> (2 * k)) & 3u;
            out[k] = (code && sfl[L[r * kHystCols + cb + k]]) ? 255 : 0;
        }
        uint8_t* dst = a.edges + (int64_t)(g.Y0 + r) * a.epitch + g.X0 + cb;
        const int valid = min(a.W - (g.X0 + cb), TL::kPPT);
        if (vec16 && valid == TL::kPPT) {
            if constexpr (TL::kPPT == 16) {
                uint4 v;
                v.x = out[0] | out[1] << 8 | out[2] << 16 | (uint32_t)out[3] << 24;
                v.y = out[4] | out[5] << 8 | out[6] << 16 | (uint32_t)out[7] << 24;
                v.z = out[8] | out[9] << 8 | out[10] << 16 | (uint32_t)out[11] << 24;
                v.w = out[12] | out[13] << 8 | out[14] << 16 | (uint32_t)out[15] << 24;
                *reinterpret_cast<uint4*>(dst) = v;
            } else {
                uint2 v;
                v.x = out[0] | out[1] << 8 | out[2] << 16 | (uint32_t)out[3] << 24;
                v.y = out[4] | out[5] << 8 | out[6] << 16 | (uint32_t)out[7] << 24;
                *reinterpret_cast<uint2*>(dst) = v;
            }
        } else {
            for (int k = 0; k < valid; ++k) dst[k] = out[k];
        }
    }
}

template <int T>
hipError_t launch_t(const HystArgs& a, hipStream_t s) {
    using TL = Tile<T>;
    const int tiles_x = ceil_div(a.W, kHystCols);
    const int tiles_y = ceil_div(a.H, T);
    const int ntiles = tiles_x * tiles_y;
    const int nslots = ntiles * TL::kPerim;
    const int vec16 = ((uintptr_t)a.edges % 16 == 0) && (a.epitch % 16 == 0);
    hipLaunchKernelGGL(k_hyst_local<T>, dim3(ntiles), dim3(kWGThreads), 0, s, a, tiles_x);
    const int64_t nmerge = (int64_t)ntiles * (T + kHystCols);
    hipLaunchKernelGGL(k_hyst_merge<T>, dim3((unsigned)ceil_div64(nmerge, kWGThreads)),
                       dim3(kWGThreads), 0, s, a, tiles_x, tiles_y, ntiles);
    hipLaunchKernelGGL(k_hyst_flags<T>, dim3(ceil_div(nslots, kWGThreads)), dim3(kWGThreads), 0, s,
                       a, nslots);
    hipLaunchKernelGGL(k_hyst_final<T>, dim3(ntiles), dim3(kWGThreads), 0, s, a, tiles_x, vec16);
    return hipGetLastError();
}

}  // namespace

int hyst_tile_rows_default() { return 64; }

static int perim(int tile_rows) { return 2 * kHystCols + 2 * tile_rows; }

size_t hyst_workspace_bytes(int H, int W, int tile_rows) {
    const size_t ntiles = (size_t)ceil_div(W, kHystCols) * ceil_div(H, tile_rows);
    const size_t nslots = ntiles * perim(tile_rows);
    return 3 * ((nslots * sizeof(int32_t) + 255) & ~(size_t)255);
}

void hyst_carve(void* ws, int H, int W, int tile_rows, HystArgs& a) {
    const size_t ntiles = (size_t)ceil_div(W, kHystCols) * ceil_div(H, tile_rows);
    const size_t bytes = ((ntiles * perim(tile_rows) * sizeof(int32_t)) + 255) & ~(size_t)255;
    char* p = static_cast<char*>(ws);
    a.blab = reinterpret_cast<int32_t*>(p);
    a.parent = reinterpret_cast<int32_t*>(p + bytes);
    a.flag = reinterpret_cast<int32_t*>(p + 2 * bytes);
}

hipError_t launch_hysteresis(const HystArgs& a, int tile_rows, hipStream_t s) {
    if (tile_rows == 32) return launch_t<32>(a, s);
    return launch_t<64>(a, s);
}

}  // namespace canny
