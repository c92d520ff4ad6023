// Batched form of the two-buffer update (declared in include/lbm.h): independent
// lattices with their own sizes and constants advanced by one launch per step.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lbm_ctx.hpp"
#include "thermo.hpp"

namespace {

thread_local std::string g_create_error;

size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

constexpr int kQueueCounters = 16;  // 2 parities x 8 XCD queues

}  // namespace

struct lbm_batch {
    std::vector<lbm_ctx*> m;
    int prec = 0;
    hipStream_t stream = nullptr;
    size_t desc_size = 0;
    void* desc_dev = nullptr;
    int32_t* starts_dev = nullptr;
    unsigned* queue_dev = nullptr;
    uint32_t* steps_dev = nullptr;         // 2 step counters per member (launch parity)
    std::vector<unsigned char> desc_host;  // as uploaded
    std::vector<int32_t> starts_host;
    std::vector<uint32_t> steps_host;
    std::vector<int64_t> dev_steps;        // each member's step count as the device counters hold it
    bool sr = false;                       // stochastic rounding of the 16-bit stores
    int parity = 0;          // parity of the next launch; flips every launch
    bool queue_clean[2] = {true, true};
    bool uploaded = false;
    lbm_batch_shape shape{32, 4, 0, 0};
    lbm_dev::BatchLaunch bl{};
    int64_t nitems = 0, nodes = 0;
    int cus = 0;
    int graph_steps = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::string err;
};

namespace {

int bfail(lbm_batch* b, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (b) b->err = buf;
    else g_create_error = buf;
    return code;
}

int bhip(lbm_batch* b, hipError_t e, const char* what) {
    return bfail(b, LBM_EHIP, "%s: %s", what, hipGetErrorString(e));
}

void drop_graph(lbm_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

bool shape_valid(const lbm_batch_shape* s) {
    return s->rows_per_wave >= 1 && s->rows_per_wave <= (1 << 20) &&
           (s->waves_per_block == 1 || s->waves_per_block == 2 || s->waves_per_block == 4) &&
           (s->queue == 0 || s->queue == 1) && s->blocks >= 0;
}

// Item offsets and grid of the current shape (host side only).
int plan(lbm_batch* b) {
    const int rows = b->shape.rows_per_wave;
    b->starts_host.assign(b->m.size() + 1, 0);
    int64_t acc = 0, nodes = 0;
    for (size_t i = 0; i < b->m.size(); ++i) {
        const lbm_ctx* c = b->m[i];
        b->starts_host[i] = (int32_t)acc;
        const int width = 64 * c->shape.columns_per_lane;  // strip width of the member's kernel form
        acc += (int64_t)((c->lat.nx + width - 1) / width) * ((c->lat.ny + rows - 1) / rows);
        nodes += (int64_t)c->lat.nx * c->lat.ny;
        if (acc >= ((int64_t)1 << 31)) return bfail(b, LBM_EINVAL, "too many work items for 32-bit indices");
    }
    b->starts_host[b->m.size()] = (int32_t)acc;
    b->nitems = acc;
    b->nodes = nodes;
    const int wpb = b->shape.waves_per_block;
    const int64_t need = (acc + wpb - 1) / wpb;
    b->bl.waves_per_block = wpb;
    b->bl.queue = b->shape.queue;
    if (!b->shape.queue) {
        b->bl.blocks = (int)need;
        b->bl.groups = 1;
    } else {
        int64_t blocks = b->shape.blocks;
        if (blocks == 0) {
            const int per_cu = lbm_dev::batch_blocks_per_cu(b->prec, wpb, 1, b->sr);
            if (per_cu <= 0) return bfail(b, LBM_EHIP, "occupancy query failed for the batched kernel");
            blocks = (int64_t)b->cus * per_cu;
        }
        if (blocks > need) blocks = need;
        if (blocks >= 8) blocks -= blocks % 8;  // equal block counts on every XCD queue
        if (blocks < 1) blocks = 1;
        b->bl.blocks = (int)blocks;
        b->bl.groups = blocks < 8 ? (int)blocks : 8;
    }
    return LBM_OK;
}

template <typename C>
void fill_desc(const lbm_batch* b, unsigned char* dst) {
    for (size_t i = 0; i < b->m.size(); ++i) {
        const lbm_ctx* c = b->m[i];
        lbm_dev::BatchDesc<C> d;
        std::memset(&d, 0, sizeof d);
        d.P = *static_cast<const lbm_dev::Consts<C>*>(c->consts);
        // the next launch has parity b->parity and reads buf[b->parity]
        d.buf[b->parity] = c->buf[c->cur];
        d.buf[b->parity ^ 1] = c->buf[c->cur ^ 1];
        d.cols = c->shape.columns_per_lane;
        d.nstrips = (c->lat.nx + 64 * d.cols - 1) / (64 * d.cols);
        d.rows = b->shape.rows_per_wave;
        std::memcpy(dst + i * sizeof d, &d, sizeof d);
    }
}

// Descriptor and offset tables on the device; synchronising.
int upload(lbm_batch* b) {
    b->desc_host.assign(b->m.size() * b->desc_size, 0);
    if (b->prec == LBM_F64) fill_desc<double>(b, b->desc_host.data());
    else fill_desc<float>(b, b->desc_host.data());
    b->steps_host.assign(2 * b->m.size(), 0u);
    b->dev_steps.assign(b->m.size(), 0);
    for (size_t i = 0; i < b->m.size(); ++i) {
        b->steps_host[2 * i] = b->steps_host[2 * i + 1] = (uint32_t)b->m[i]->steps;
        b->dev_steps[i] = b->m[i]->steps;
    }
    hipError_t e = hipMemcpyAsync(b->desc_dev, b->desc_host.data(), b->desc_host.size(), hipMemcpyHostToDevice,
                                  b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->starts_dev, b->starts_host.data(), b->starts_host.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->steps_dev, b->steps_host.data(), b->steps_host.size() * sizeof(uint32_t),
                           hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bhip(b, e, "descriptor upload");
    b->uploaded = true;
    return LBM_OK;
}

// True when every member's current buffer is the one the next launch will read and its
// step count is the one the device counters hold.
bool descriptors_fresh(const lbm_batch* b) {
    if (!b->uploaded) return false;
    const size_t off = b->prec == LBM_F64 ? offsetof(lbm_dev::BatchDesc<double>, buf)
                                          : offsetof(lbm_dev::BatchDesc<float>, buf);
    for (size_t i = 0; i < b->m.size(); ++i) {
        const void* bufs[2];
        std::memcpy(bufs, b->desc_host.data() + i * b->desc_size + off, sizeof bufs);
        const lbm_ctx* c = b->m[i];
        if (bufs[b->parity] != c->buf[c->cur] || bufs[b->parity ^ 1] != c->buf[c->cur ^ 1]) return false;
        if (c->steps != b->dev_steps[i]) return false;
    }
    return true;
}

int ready(lbm_batch* b) {
    for (size_t i = 0; i < b->m.size(); ++i)
        if (!b->m[i]->fields_set) return bfail(b, LBM_ESTATE, "member %zu has no fields (lbm_set_fields)", i);
    if (!descriptors_fresh(b)) return upload(b);
    return LBM_OK;
}

void advance_members(lbm_batch* b, int64_t n) {
    for (size_t i = 0; i < b->m.size(); ++i) {
        lbm_ctx* c = b->m[i];
        c->steps += n;
        c->cur ^= (int)(n & 1);
        b->dev_steps[i] += n;
    }
}

// One eager launch at the current parity.
int launch_one(lbm_batch* b) {
    hipError_t e;
    if (b->bl.queue && !b->queue_clean[b->parity]) {
        e = hipMemsetAsync(b->queue_dev + b->parity * 8, 0, 8 * sizeof(unsigned), b->stream);
        if (e != hipSuccess) return bhip(b, e, "queue reset");
    }
    e = lbm_dev::launch_step_ab_batch(b->prec, b->desc_dev, b->starts_dev, b->queue_dev, b->steps_dev,
                                      (int)b->m.size(), (int)b->nitems, b->parity, b->bl, b->sr, b->stream);
    if (e != hipSuccess) return bhip(b, e, "batched step launch");
    if (b->bl.queue) {
        b->queue_clean[b->parity] = false;
        b->queue_clean[b->parity ^ 1] = true;  // the launch clears the other parity's counters
    }
    b->parity ^= 1;
    advance_members(b, 1);
    return LBM_OK;
}

// Captures graph_steps launches starting at parity 0 (kernel launches only).
int capture(lbm_batch* b) {
    drop_graph(b);
    hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return bhip(b, e, "begin capture");
    hipError_t le = hipSuccess;
    for (int k = 0; k < b->graph_steps && le == hipSuccess; ++k)
        le = lbm_dev::launch_step_ab_batch(b->prec, b->desc_dev, b->starts_dev, b->queue_dev, b->steps_dev,
                                           (int)b->m.size(), (int)b->nitems, k & 1, b->bl, b->sr, b->stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->stream, &g);
    if (le != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return bhip(b, le, "launch during capture");
    }
    if (e != hipSuccess) return bhip(b, e, "end capture");
    b->graph = g;
    e = hipGraphInstantiateWithFlags(&b->exec, g, 0);
    if (e != hipSuccess) {
        drop_graph(b);
        return bhip(b, e, "graph instantiate");
    }
    return LBM_OK;
}

int step_n(lbm_batch* b, int64_t n) {
    if (b->graph_steps > 0 && n >= b->graph_steps + (b->parity & 1)) {
        if (b->parity) {  // graphs start at parity 0
            int r = launch_one(b);
            if (r) return r;
            --n;
        }
        if (b->bl.queue && !b->queue_clean[0]) {
            hipError_t e = hipMemsetAsync(b->queue_dev, 0, 8 * sizeof(unsigned), b->stream);
            if (e != hipSuccess) return bhip(b, e, "queue reset");
            b->queue_clean[0] = true;
        }
        if (!b->exec) {
            int r = capture(b);
            if (r) return r;
        }
        while (n >= b->graph_steps) {
            hipError_t e = hipGraphLaunch(b->exec, b->stream);
            if (e != hipSuccess) return bhip(b, e, "graph launch");
            if (b->bl.queue) {  // the last captured launch has parity 1
                b->queue_clean[1] = false;
                b->queue_clean[0] = true;
            }
            advance_members(b, b->graph_steps);
            n -= b->graph_steps;
        }
    }
    for (int64_t k = 0; k < n; ++k) {
        int r = launch_one(b);
        if (r) return r;
    }
    return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_maxwell(const lbm_eos* eos, double Tr, double out[4]) {
    if (!eos || !out) return LBM_EINVAL;
    if (!(Tr > 0 && Tr < 1)) return LBM_EINVAL;
    if (!(eos->kind == LBM_EOS_CS || eos->kind == LBM_EOS_VDW)) return LBM_EINVAL;
    if (!(eos->a_t > 0 && eos->b_t > 0 && eos->R > 0 && eos->K_eos > 0)) return LBM_EINVAL;
    lbm_host::Eos e{eos->kind, eos->a_t, eos->b_t, eos->R, eos->K_eos};
    long double Tc, pc, rv, rl, ps;
    lbm_host::critical(e, &Tc, &pc);
    std::string why;
    if (!lbm_host::coexistence(e, (long double)Tr * Tc, &rv, &rl, &ps, &why)) return LBM_EINVAL;
    out[0] = (double)rv;
    out[1] = (double)rl;
    out[2] = (double)ps;
    out[3] = (double)Tc;
    return LBM_OK;
}

int lbm_batch_workspace_bytes(int32_t n, int32_t precision, size_t* bytes) {
    if (!bytes) return bfail(nullptr, LBM_EINVAL, "bytes is NULL");
    if (n < 1) return bfail(nullptr, LBM_EINVAL, "a batch needs at least one member");
    if (precision < LBM_F64 || precision > LBM_BF16) return bfail(nullptr, LBM_EINVAL, "unknown precision");
    *bytes = round256((size_t)n * lbm_dev::batch_desc_size(precision)) + round256(((size_t)n + 1) * sizeof(int32_t)) +
             round256(kQueueCounters * sizeof(unsigned)) + round256(2 * (size_t)n * sizeof(uint32_t));
    return LBM_OK;
}

int lbm_batch_create(lbm_batch** out, lbm_ctx* const* members, int32_t n, void* workspace,
                     size_t workspace_bytes) {
    g_create_error.clear();
    if (!out) return bfail(nullptr, LBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!members || n < 1) return bfail(nullptr, LBM_EINVAL, "a batch needs at least one member");
    const lbm_ctx* m0 = members[0];
    if (!m0) return bfail(nullptr, LBM_EINVAL, "member 0 is NULL");
    for (int32_t i = 0; i < n; ++i) {
        const lbm_ctx* c = members[i];
        if (!c) return bfail(nullptr, LBM_EINVAL, "member %d is NULL", i);
        if (c->host_only) return bfail(nullptr, LBM_ESTATE, "member %d is a host-only context", i);
        if (c->p.scheme != LBM_SCHEME_AB) return bfail(nullptr, LBM_EINVAL, "member %d: batches need LBM_SCHEME_AB", i);
        if (c->lat.bc_x != LBM_BC_PERIODIC)
            return bfail(nullptr, LBM_EINVAL, "member %d: batches need periodic lattices", i);
        if (c->p.precision != m0->p.precision)
            return bfail(nullptr, LBM_EINVAL, "member %d: all members must share one precision", i);
        if (c->stream != m0->stream) return bfail(nullptr, LBM_EINVAL, "member %d: all members must share one stream", i);
        if (c->p.rounding != m0->p.rounding)
            return bfail(nullptr, LBM_EINVAL, "member %d: all members must share one rounding mode", i);
        if (((size_t)18 * c->lat.ny + 17) * c->lat.nx * lbm_dev::storage_bytes(c->p.precision) + 64 >= ((size_t)1 << 32))
            return bfail(nullptr, LBM_EINVAL, "member %d: %d x %d is too large for a batch (its state must stay below 4 GiB)",
                         i, c->lat.nx, c->lat.ny);
        for (int32_t j = 0; j < i; ++j)
            if (members[j] == c) return bfail(nullptr, LBM_EINVAL, "member %d appears twice", i);
    }
    size_t need = 0;
    lbm_batch_workspace_bytes(n, m0->p.precision, &need);
    if (!workspace) return bfail(nullptr, LBM_EINVAL, "workspace is NULL");
    if (workspace_bytes < need)
        return bfail(nullptr, LBM_ESPACE, "workspace has %zu bytes, %zu needed", workspace_bytes, need);
    if (reinterpret_cast<uintptr_t>(workspace) & 255)
        return bfail(nullptr, LBM_EINVAL, "workspace must be 256-byte aligned");
    lbm_batch* b = new (std::nothrow) lbm_batch();
    if (!b) return bfail(nullptr, LBM_EINVAL, "out of host memory");
    b->m.assign(members, members + n);
    b->prec = m0->p.precision;
    b->sr = m0->p.rounding == LBM_ROUND_STOCHASTIC;
    b->shape = lbm_batch_shape{lbm_dev::default_rows(b->prec), lbm_dev::default_waves(b->prec), 0, 0};
    b->stream = m0->stream;
    b->desc_size = lbm_dev::batch_desc_size(b->prec);
    char* w = static_cast<char*>(workspace);
    b->desc_dev = w;
    w += round256((size_t)n * b->desc_size);
    b->starts_dev = reinterpret_cast<int32_t*>(w);
    w += round256(((size_t)n + 1) * sizeof(int32_t));
    b->queue_dev = reinterpret_cast<unsigned*>(w);
    w += round256(kQueueCounters * sizeof(unsigned));
    b->steps_dev = reinterpret_cast<uint32_t*>(w);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipMemsetAsync(b->queue_dev, 0, kQueueCounters * sizeof(unsigned), b->stream);
    if (e != hipSuccess) {
        bhip(nullptr, e, "batch set-up");
        delete b;
        return LBM_EHIP;
    }
    int r = plan(b);
    if (!r) r = upload(b);
    if (r) {
        g_create_error = b->err;
        delete b;
        return r;
    }
    *out = b;
    return LBM_OK;
}

int lbm_batch_set_shape(lbm_batch* b, const lbm_batch_shape* shape) {
    if (!b) return bfail(nullptr, LBM_EINVAL, "batch is NULL");
    if (!shape || !shape_valid(shape))
        return bfail(b, LBM_EINVAL, "shape: rows_per_wave >= 1, waves_per_block 1/2/4, queue 0/1, blocks >= 0");
    const lbm_batch_shape old = b->shape;
    b->shape = *shape;
    int r = plan(b);
    if (r) {
        b->shape = old;
        plan(b);
        return r;
    }
    drop_graph(b);
    b->uploaded = false;  // item offsets and rows changed
    if (b->bl.queue) b->queue_clean[0] = b->queue_clean[1] = false;
    return LBM_OK;
}

int lbm_batch_get_shape(const lbm_batch* b, lbm_batch_shape* shape) {
    if (!b || !shape) return LBM_EINVAL;
    *shape = b->shape;
    if (b->shape.queue) shape->blocks = b->bl.blocks;
    return LBM_OK;
}

int lbm_batch_set_graph(lbm_batch* b, int32_t steps_per_graph) {
    if (!b) return bfail(nullptr, LBM_EINVAL, "batch is NULL");
    if (steps_per_graph < 0 || (steps_per_graph > 0 && (steps_per_graph & 1)))
        return bfail(b, LBM_EINVAL, "steps_per_graph must be 0 or even");
    if (steps_per_graph > 0 && b->stream == nullptr)
        return bfail(b, LBM_EINVAL, "graph capture needs a created stream, not the null stream");
    if (steps_per_graph != b->graph_steps) drop_graph(b);
    b->graph_steps = steps_per_graph;
    return LBM_OK;
}

int lbm_batch_step(lbm_batch* b, int64_t n) {
    if (!b) return bfail(nullptr, LBM_EINVAL, "batch is NULL");
    if (n < 0) return bfail(b, LBM_EINVAL, "n must be >= 0");
    int r = ready(b);
    if (r) return r;
    return step_n(b, n);
}

int lbm_batch_autotune(lbm_batch* b, int32_t steps_per_candidate, lbm_batch_shape* best, double* ms_per_step) {
    if (!b) return bfail(nullptr, LBM_EINVAL, "batch is NULL");
    if (steps_per_candidate < 1) return bfail(b, LBM_EINVAL, "steps_per_candidate must be >= 1");
    int r = ready(b);
    if (r) return r;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return bhip(b, e, "event create");
    }
    const int graph_steps = b->graph_steps;
    b->graph_steps = 0;  // candidates run eagerly
    lbm_batch_shape win = b->shape;
    double win_ms = 0;
    bool have = false;
    static const int kRows[] = {2, 4, 8, 16, 32, 64, 128};
    static const int kWpb[] = {1, 2, 4};
    for (int q = 0; q < 2 && !r; ++q)
        for (int ri : kRows)
            for (int wi : kWpb) {
                if (r) break;
                lbm_batch_shape s{ri, wi, q, 0};
                if ((r = lbm_batch_set_shape(b, &s))) break;
                if ((r = ready(b))) break;
                if ((r = step_n(b, 2))) break;
                e = hipEventRecord(e0, b->stream);
                if (e == hipSuccess && (r = step_n(b, steps_per_candidate))) break;
                if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess) {
                    r = bhip(b, e, "autotune timing");
                    break;
                }
                const double per = (double)ms / steps_per_candidate;
                if (!have || per < win_ms) {
                    have = true;
                    win = s;
                    win_ms = per;
                }
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->graph_steps = graph_steps;
    if (r) return r;
    if ((r = lbm_batch_set_shape(b, &win))) return r;
    if (best) lbm_batch_get_shape(b, best);
    if (ms_per_step) *ms_per_step = win_ms;
    return LBM_OK;
}

int lbm_batch_size(const lbm_batch* b, int64_t* items, int64_t* nodes) {
    if (!b) return LBM_EINVAL;
    if (items) *items = b->nitems;
    if (nodes) *nodes = b->nodes;
    return LBM_OK;
}

int lbm_batch_destroy(lbm_batch* b) {
    if (!b) return LBM_OK;
    drop_graph(b);
    delete b;
    return LBM_OK;
}

const char* lbm_batch_last_error(const lbm_batch* b) { return b ? b->err.c_str() : g_create_error.c_str(); }

}  // extern "C"
