// Batched integer Canny over many images of uneven sizes (the same operator
// as canny_u8, Section 2.2.1 Steps 1-4, per image).
//
// A plan fixes the sizes and thresholds and lays out one workspace region per
// image (class map + hysteresis state).  Every phase of the detector runs as
// ONE flat launch over all images: one wave per forward task (a strip and row
// block of one image), one workgroup per hysteresis tile for the local and
// resolve passes, one thread per right or bottom border pixel for merge.
// Work items are uniform, so large and small images interleave freely and no
// shared counter is touched; a tile's image comes from a per-plan
// tile -> image table.  The launches are recorded once into a HIP graph
//     forward -> local -> merge -> resolve
// whose kernels read a device descriptor table; a call uploads the table
// (the caller's image pointers and workspace) and replays the graph, so new
// buffers never need a new recording.
//
// Tuning: the forward's tile height (output rows per wave) is picked by
// timing the candidates on the plan's own sizes with synthetic content, when
// asked, within a time budget; results are kept per process and, if
// CANNY_TUNE_CACHE names a file, in that file as "key rows" lines.  The key
// is a size bucket (arch, CU count, and the image count, total pixels, mean
// height and mean width, each on a logarithmic grid), so batches of a
// similar make-up share one entry instead of re-tuning per exact size list.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/canny.h"
#include "canny_internal.h"

namespace canny {
bool device_ok();
bool size_ok(int H, int W);
int64_t class_pitch(int W);
}  // namespace canny

using namespace canny;

struct canny_batch_plan {
    int n = 0;
    int low = 0, high = 0;
    int fwd_rows = 32;
    int cus = 256;
    int device = 0;
    size_t ws_bytes = 0;
    std::vector<BatchImage> imgs;
    BatchDev hdr{};
    BatchImage* d_imgs = nullptr;
    BatchDev* d_hdr = nullptr;
    int32_t* d_tile_img = nullptr;  // per tile: index of its image (fixed by the sizes)
    // pinned staging of the descriptor table, a ring of kStage copies: a call
    // waits only for the upload kStage calls back (normally long done)
    static constexpr int kStage = 4;
    BatchImage* h_stage[kStage] = {};
    BatchDev* h_stage_hdr[kStage] = {};
    hipEvent_t uploaded[kStage] = {};
    bool pending[kStage] = {};
    int next_stage = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

constexpr int kT = 64;  // hysteresis tile rows
constexpr double kTuneBudgetSeconds = 0.5;  // time box of one tuning run
constexpr int kPerimT = 2 * kHystCols + 2 * kT;

size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

// deterministic texture for tuning runs: smooth ramps plus hashed noise
__global__ void k_fill_texture(uint8_t* p, int64_t n, uint32_t seed) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t h = (uint32_t)i * 2654435761u ^ seed;
    h ^= h >> 13;
    h *= 0x5bd1e995u;
    h ^= h >> 15;
    p[i] = (uint8_t)(((i >> 6) & 0x7F) + (h & 0x3F));
}

void layout(canny_batch_plan& p, const int32_t* H, const int32_t* W) {
    size_t off = 0;
    int tile_base = 0, merge_base = 0;
    p.imgs.resize(p.n);
    for (int i = 0; i < p.n; ++i) {
        BatchImage& m = p.imgs[i];
        std::memset(&m, 0, sizeof(m));
        m.H = H[i];
        m.W = W[i];
        m.cpitch = class_pitch(W[i]);
        m.cls_off = (int64_t)off;
        off += al256((size_t)m.H * m.cpitch);
        HystArgs h;
        char* base = reinterpret_cast<char*>((uintptr_t)4096);
        hyst_carve(base, m.H, m.W, kT, h);
        m.blab_off = (int64_t)off + (reinterpret_cast<char*>(h.blab) - base);
        m.parent_off = (int64_t)off + (reinterpret_cast<char*>(h.parent) - base);
        m.pmask_off = (int64_t)off + (reinterpret_cast<char*>(h.pmask) - base);
        off += al256(hyst_workspace_bytes(m.H, m.W, kT));
        m.tiles_x = ceil_div(m.W, kHystCols);
        m.tiles_y = ceil_div(m.H, kT);
        const int ntiles = m.tiles_x * m.tiles_y;
        m.tile_base = tile_base;
        m.merge_base = merge_base;
        tile_base += ntiles;
        merge_base += ntiles * (kT + kHystCols);
    }
    p.ws_bytes = off;
    p.hdr.n = p.n;
    p.hdr.low = p.low;
    p.hdr.high = p.high;
    p.hdr.total_tiles = tile_base;
    p.hdr.total_merge = merge_base;
}

void set_fwd_rows(canny_batch_plan& p, int rows) {
    p.fwd_rows = rows;
    int base = 0;
    for (BatchImage& m : p.imgs) {
        m.fwd_strips_x = ceil_div(m.W, kU8StripCols);
        m.fwd_base = base;
        base += m.fwd_strips_x * ceil_div(m.H, rows);
    }
    p.hdr.total_fwd = base;
}

hipError_t enqueue(const canny_batch_plan& p, hipStream_t s) {
    hipError_t e = launch_u8_forward_batch(p.d_imgs, p.d_hdr, p.fwd_rows, p.hdr.total_fwd, s);
    if (e != hipSuccess) return e;
    return launch_hyst_batch(p.d_imgs, p.d_hdr, p.hdr.total_tiles, p.hdr.total_merge, s);
}

// synchronous upload of the table (plan creation and tuning only)
hipError_t upload_sync(canny_batch_plan& p) {
    hipError_t e = hipMemcpy(p.d_imgs, p.imgs.data(), sizeof(BatchImage) * p.n, hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
    return hipMemcpy(p.d_hdr, &p.hdr, sizeof(BatchDev), hipMemcpyHostToDevice);
}

std::mutex g_tune_mu;
std::map<std::string, int> g_tune_cache;

// bucket of a positive quantity on a grid of 2^(1/steps) (steps per octave)
int log_bucket(double v, int steps) { return v > 0.0 ? (int)std::floor(std::log2(v) * steps) : -1; }

std::string tune_key(const canny_batch_plan& p) {
    double px = 0.0, sh = 0.0, sw = 0.0;
    for (const BatchImage& m : p.imgs) {
        px += (double)m.H * m.W;
        sh += m.H;
        sw += m.W;
    }
    char buf[96];
    std::snprintf(buf, sizeof(buf), "gfx950:%d:n%d:px%d:h%d:w%d", p.cus, log_bucket(p.n, 2),
                  log_bucket(px, 4), log_bucket(sh / p.n, 2), log_bucket(sw / p.n, 2));
    return buf;
}

bool tune_lookup(const std::string& key, int& rows) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it == g_tune_cache.end()) {
        const char* path = std::getenv("CANNY_TUNE_CACHE");
        if (!path) return false;
        FILE* f = std::fopen(path, "r");
        if (!f) return false;
        char k[128];
        int r;
        while (std::fscanf(f, "%127s %d", k, &r) == 2)
            if (u8_forward_supported_rows(r)) g_tune_cache[k] = r;
        std::fclose(f);
        it = g_tune_cache.find(key);
        if (it == g_tune_cache.end()) return false;
    }
    rows = it->second;
    return true;
}

void tune_store(const std::string& key, int rows) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = rows;
    if (const char* path = std::getenv("CANNY_TUNE_CACHE")) {
        if (FILE* f = std::fopen(path, "a")) {
            std::fprintf(f, "%s %d\n", key.c_str(), rows);
            std::fclose(f);
        }
    }
}

// Time every tile height candidate on the plan's sizes; keep the best.
hipError_t autotune(canny_batch_plan& p) {
    const std::string key = tune_key(p);
    int rows;
    if (tune_lookup(key, rows)) {
        set_fwd_rows(p, rows);
        return hipSuccess;
    }
    // synthetic inputs / outputs laid out back to back, plus a workspace
    size_t in_bytes = 0;
    for (const BatchImage& m : p.imgs) in_bytes += al256((size_t)m.H * m.W);
    uint8_t *in = nullptr, *out = nullptr;
    char* ws = nullptr;
    hipError_t e = hipMalloc(&in, in_bytes);
    if (e == hipSuccess) e = hipMalloc(&out, in_bytes);
    if (e == hipSuccess) e = hipMalloc(&ws, p.ws_bytes);
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    if (e == hipSuccess) {
        const int64_t nb = (int64_t)in_bytes;
        hipLaunchKernelGGL(k_fill_texture, dim3((unsigned)ceil_div64(nb, 256)), dim3(256), 0, nullptr,
                           in, nb, 12345u);
        size_t off = 0;
        for (BatchImage& m : p.imgs) {
            m.in = in + off;
            m.pitch = m.W;
            m.edges = out + off;
            m.epitch = m.W;
            off += al256((size_t)m.H * m.W);
        }
        p.hdr.ws = ws;
        float best = 1e30f;
        int best_rows = 32;
        // taller blocks spread the 8 halo rows of each block over more output
        // rows; shorter ones give more waves.  Candidates in order of how
        // often they won, tried until the budget (wall clock, including the
        // warm-up replay of each) runs out; the default is always timed.
        const int cand_rows[] = {64, 96, 48, 128, 32};
        const auto t_start = std::chrono::steady_clock::now();
        for (int r : cand_rows) {
            if (e != hipSuccess) break;
            const double spent =
                std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
            if (r != cand_rows[0] && spent > kTuneBudgetSeconds) break;
            set_fwd_rows(p, r);
            e = upload_sync(p);
            float t = 1e30f;
            for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {
                (void)hipEventRecord(t0, nullptr);
                e = enqueue(p, nullptr);
                (void)hipEventRecord(t1, nullptr);
                if (e == hipSuccess) e = hipEventSynchronize(t1);
                float ms = 0.0f;
                if (e == hipSuccess && rep > 0 && hipEventElapsedTime(&ms, t0, t1) == hipSuccess)
                    t = ms < t ? ms : t;
            }
            if (t < best) {
                best = t;
                best_rows = r;
            }
        }
        if (e == hipSuccess) {
            set_fwd_rows(p, best_rows);
            tune_store(key, best_rows);
        }
    }
    (void)hipDeviceSynchronize();
    for (BatchImage& m : p.imgs) {
        m.in = nullptr;
        m.edges = nullptr;
    }
    p.hdr.ws = nullptr;
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    if (in) (void)hipFree(in);
    if (out) (void)hipFree(out);
    if (ws) (void)hipFree(ws);
    return e;
}

void release(canny_batch_plan* p) {
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    for (int k = 0; k < canny_batch_plan::kStage; ++k) {
        if (p->uploaded[k]) (void)hipEventDestroy(p->uploaded[k]);
        if (p->h_stage[k]) (void)hipHostFree(p->h_stage[k]);
        if (p->h_stage_hdr[k]) (void)hipHostFree(p->h_stage_hdr[k]);
    }
    if (p->d_imgs) (void)hipFree(p->d_imgs);
    if (p->d_hdr) (void)hipFree(p->d_hdr);
    if (p->d_tile_img) (void)hipFree(p->d_tile_img);
    delete p;
}

}  // namespace

extern "C" {

int canny_batch_plan_create(int n, const int32_t* H, const int32_t* W, int32_t low, int32_t high,
                            int autotune_flag, canny_batch_plan** out) {
    if (!out) return CANNY_ERR_INVALID;
    *out = nullptr;
    if (n < 1 || n > (1 << 20) || !H || !W || low < 0 || low > high) return CANNY_ERR_INVALID;
    int64_t tiles = 0, px = 0;
    for (int i = 0; i < n; ++i) {
        if (!size_ok(H[i], W[i])) return CANNY_ERR_INVALID;
        tiles += (int64_t)ceil_div(H[i], kT) * ceil_div(W[i], kHystCols);
        px += (int64_t)H[i] * W[i];
    }
    // flat per-pixel / per-merge-item grids of the batch use 31-bit indices
    if (tiles * (kT + kHystCols) >= ((int64_t)1 << 31) || tiles * kPerimT >= ((int64_t)1 << 31) ||
        px / 16 >= ((int64_t)1 << 31))
        return CANNY_ERR_INVALID;
    if (!device_ok()) return CANNY_ERR_UNSUPPORTED;
    canny_batch_plan* p = new canny_batch_plan();
    p->n = n;
    p->low = low > 2041 ? 2041 : low;
    p->high = high > 2040 ? 2040 : high;
    hipError_t e = hipGetDevice(&p->device);
    hipDeviceProp_t prop;
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, p->device);
    if (e != hipSuccess) {
        release(p);
        return CANNY_ERR_HIP;
    }
    p->cus = prop.multiProcessorCount;
    layout(*p, H, W);
    set_fwd_rows(*p, 32);
    e = hipMalloc(&p->d_imgs, sizeof(BatchImage) * n);
    if (e == hipSuccess) e = hipMalloc(&p->d_hdr, sizeof(BatchDev));
    if (e == hipSuccess && p->hdr.total_tiles > 0) {  // tile -> image: one load, no search
        std::vector<int32_t> ti((size_t)p->hdr.total_tiles);
        for (int i = 0; i < n; ++i) {
            const BatchImage& m = p->imgs[i];
            for (int k = 0; k < m.tiles_x * m.tiles_y; ++k) ti[(size_t)m.tile_base + k] = i;
        }
        e = hipMalloc(&p->d_tile_img, sizeof(int32_t) * ti.size());
        if (e == hipSuccess)
            e = hipMemcpy(p->d_tile_img, ti.data(), sizeof(int32_t) * ti.size(), hipMemcpyHostToDevice);
        p->hdr.tile_img = p->d_tile_img;
    }
    for (int k = 0; k < canny_batch_plan::kStage && e == hipSuccess; ++k) {
        e = hipHostMalloc(&p->h_stage[k], sizeof(BatchImage) * n, hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc(&p->h_stage_hdr[k], sizeof(BatchDev), hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->uploaded[k], hipEventDisableTiming);
    }
    if (e == hipSuccess && autotune_flag) e = autotune(*p);
    hipStream_t cs = nullptr;
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    // Launch every kernel of the graph once, outside any capture, on an empty
    // table (all totals zero, so each kernel exits at once): the runtime loads
    // the library's code object on the first launch, and that must not happen
    // inside the capture below.
    if (e == hipSuccess) {
        BatchDev empty{};
        e = hipMemcpy(p->d_hdr, &empty, sizeof(BatchDev), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = enqueue(*p, cs);
    if (e == hipSuccess) e = hipStreamSynchronize(cs);
    // record the graph on the private stream
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t le = enqueue(*p, cs);
        e = hipStreamEndCapture(cs, &p->graph);
        if (e == hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (cs) (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        release(p);
        return CANNY_ERR_HIP;
    }
    *out = p;
    return CANNY_OK;
}

size_t canny_batch_workspace_bytes(const canny_batch_plan* p) { return p ? p->ws_bytes : 0; }

int canny_batch_plan_info(const canny_batch_plan* p, int32_t* fwd_rows, int32_t* hyst_rows) {
    if (!p) return CANNY_ERR_INVALID;
    if (fwd_rows) *fwd_rows = p->fwd_rows;
    if (hyst_rows) *hyst_rows = kT;
    return CANNY_OK;
}

int canny_batch(canny_batch_plan* p, const uint8_t* const* in, const int64_t* in_pitch,
                uint8_t* const* edges, const int64_t* edges_pitch, void* ws, size_t ws_bytes,
                void* stream) {
    if (!p || !in || !in_pitch || !edges || !edges_pitch) return CANNY_ERR_INVALID;
    for (int i = 0; i < p->n; ++i) {
        if (!in[i] || !edges[i] || in_pitch[i] < p->imgs[i].W || edges_pitch[i] < p->imgs[i].W)
            return CANNY_ERR_INVALID;
    }
    if (!ws || ws_bytes < p->ws_bytes || ((uintptr_t)ws % 256)) return CANNY_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // this call's staging copy was last read by the upload kStage calls ago
    const int k = p->next_stage;
    p->next_stage = (k + 1) % canny_batch_plan::kStage;
    if (p->pending[k] && hipEventSynchronize(p->uploaded[k]) != hipSuccess) return CANNY_ERR_HIP;
    BatchImage* st = p->h_stage[k];
    for (int i = 0; i < p->n; ++i) {
        st[i] = p->imgs[i];
        st[i].in = in[i];
        st[i].pitch = in_pitch[i];
        st[i].edges = edges[i];
        st[i].epitch = edges_pitch[i];
    }
    *p->h_stage_hdr[k] = p->hdr;
    p->h_stage_hdr[k]->ws = static_cast<char*>(ws);
    hipError_t e = hipMemcpyAsync(p->d_imgs, st, sizeof(BatchImage) * p->n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->d_hdr, p->h_stage_hdr[k], sizeof(BatchDev), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(p->uploaded[k], s);
    if (e == hipSuccess) p->pending[k] = true;
    if (e == hipSuccess) e = hipGraphLaunch(p->exec, s);
    return e == hipSuccess ? CANNY_OK : CANNY_ERR_HIP;
}

void canny_batch_plan_destroy(canny_batch_plan* p) {
    if (!p) return;
    (void)hipDeviceSynchronize();
    release(p);
}

}  // extern "C"
