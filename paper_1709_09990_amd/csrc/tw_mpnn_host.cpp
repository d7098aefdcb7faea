// Host side of the message-passing network: features, parameters, Adam state,
// prediction, gradients and training steps (declared in include/tw.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "tw.h"
#include "tw_mpnn.h"

struct tw_mpnn {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    float *params = nullptr, *m = nullptr, *v = nullptr, *grads = nullptr;
    uint16_t *wsb = nullptr, *wsbt = nullptr, *wnb = nullptr, *wnbt = nullptr;
    // per-call buffers, grown as needed
    size_t cap = 0;
    uint64_t *adj = nullptr;
    float *feat = nullptr;
    int32_t *n = nullptr;
    float *targets = nullptr, *pred = nullptr, *sq = nullptr, *partial = nullptr;
    uint64_t step = 0;
};

namespace {

#define MP_TRY(expr)                                            \
    do {                                                        \
        if ((expr) != hipSuccess) {                             \
            (void)hipGetLastError();                            \
            return TW_EDEVICE;                                  \
        }                                                       \
    } while (0)

bool valid_graph(const tw_graph *g)
{
    if (!g || !g->adj || g->n < 1 || g->n > 64)
        return false;
    const int n = (int)g->n;
    const uint64_t all = n == 64 ? ~0ull : ((1ull << n) - 1);
    for (int i = 0; i < n; ++i) {
        if ((g->adj[i] & ~all) || ((g->adj[i] >> i) & 1ull))
            return false;
        for (int j = 0; j < n; ++j)
            if (((g->adj[i] >> j) & 1ull) != ((g->adj[j] >> i) & 1ull))
                return false;
    }
    return true;
}

// [1, deg/8, core/8, n/64] per vertex; core(v) = the largest c such that v is
// in a subgraph of minimum degree c (repeatedly delete a min-degree vertex,
// lowest index first).
void node_features(const tw_graph *g, float *out)
{
    const int n = (int)g->n;
    std::memset(out, 0, sizeof(float) * 64 * twk::MpnnFeat);
    int core[64] = {0};
    uint64_t alive = n == 64 ? ~0ull : ((1ull << n) - 1);
    int cur = 0;
    while (alive) {
        int best = -1, bd = 1 << 20;
        for (uint64_t a = alive; a; a &= a - 1) {
            const int x = __builtin_ctzll(a);
            const int d = __builtin_popcountll(g->adj[x] & alive);
            if (d < bd) {
                bd = d;
                best = x;
            }
        }
        cur = std::max(cur, bd);
        core[best] = cur;
        alive &= ~(1ull << best);
    }
    for (int v = 0; v < n; ++v) {
        float *x = out + v * twk::MpnnFeat;
        x[0] = 1.f;
        x[1] = (float)__builtin_popcountll(g->adj[v]) / 8.f;
        x[2] = (float)core[v] / 8.f;
        x[3] = (float)n / 64.f;
    }
}

template <typename T>
hipError_t dmalloc(T **p, size_t count)
{
    return hipMalloc((void **)p, std::max<size_t>(count, 1) * sizeof(T));
}

tw_status ensure(tw_mpnn *m, size_t count)
{
    if (count <= m->cap)
        return TW_OK;
    (void)hipStreamSynchronize(m->stream);
    (void)hipFree(m->adj);
    (void)hipFree(m->feat);
    (void)hipFree(m->n);
    (void)hipFree(m->targets);
    (void)hipFree(m->pred);
    (void)hipFree(m->sq);
    (void)hipFree(m->partial);
    m->adj = nullptr;
    m->feat = nullptr;
    m->n = nullptr;
    m->targets = m->pred = m->sq = m->partial = nullptr;
    m->cap = 0;
    size_t c = std::max<size_t>(count, 64);
    if (dmalloc(&m->adj, c * 64) != hipSuccess || dmalloc(&m->feat, c * 64 * twk::MpnnFeat) != hipSuccess ||
        dmalloc(&m->n, c) != hipSuccess || dmalloc(&m->targets, c * 2) != hipSuccess ||
        dmalloc(&m->pred, c * 2) != hipSuccess || dmalloc(&m->sq, c * 2) != hipSuccess ||
        dmalloc(&m->partial, c * (size_t)twk::MpnnParams) != hipSuccess) {
        (void)hipGetLastError();
        return TW_ENOMEM;
    }
    m->cap = c;
    return TW_OK;
}

tw_status upload_graphs(tw_mpnn *m, const tw_graph *gs, uint32_t count)
{
    for (uint32_t t = 0; t < count; ++t)
        if (!valid_graph(&gs[t]))
            return TW_EINVAL;
    tw_status s = ensure(m, count);
    if (s != TW_OK)
        return s;
    std::vector<uint64_t> adj((size_t)count * 64, 0);
    std::vector<float> feat((size_t)count * 64 * twk::MpnnFeat);
    std::vector<int32_t> ns(count);
    for (uint32_t t = 0; t < count; ++t) {
        for (uint32_t j = 0; j < gs[t].n; ++j)
            adj[(size_t)t * 64 + j] = gs[t].adj[j];
        node_features(&gs[t], feat.data() + (size_t)t * 64 * twk::MpnnFeat);
        ns[t] = (int32_t)gs[t].n;
    }
    MP_TRY(hipMemcpyAsync(m->adj, adj.data(), adj.size() * 8, hipMemcpyHostToDevice, m->stream));
    MP_TRY(hipMemcpyAsync(m->feat, feat.data(), feat.size() * 4, hipMemcpyHostToDevice, m->stream));
    MP_TRY(hipMemcpyAsync(m->n, ns.data(), ns.size() * 4, hipMemcpyHostToDevice, m->stream));
    MP_TRY(hipStreamSynchronize(m->stream));
    return TW_OK;
}

twk::MpnnArgs base_args(tw_mpnn *m)
{
    twk::MpnnArgs a{};
    a.adj = m->adj;
    a.feat = m->feat;
    a.n = m->n;
    a.params = m->params;
    a.wsb = m->wsb;
    a.wsbt = m->wsbt;
    a.wnb = m->wnb;
    a.wnbt = m->wnbt;
    return a;
}

// y = network(graphs); with targets also per-graph squared errors and the
// summed gradient in m->grads.
tw_status run(tw_mpnn *m, uint32_t count, const float *targets, bool grads, float *out_loss)
{
    twk::MpnnArgs a = base_args(m);
    a.pred = m->pred;
    if (targets) {
        MP_TRY(hipMemcpyAsync(m->targets, targets, (size_t)count * 2 * 4, hipMemcpyHostToDevice, m->stream));
        a.targets = m->targets;
        a.sq_err = m->sq;
        a.grad_scale = 1.f / (float)(2 * count);
    }
    if (grads)
        a.grads = m->partial;
    MP_TRY(twk::launch_mpnn(a, (int)count, m->stream));
    if (grads)
        MP_TRY(twk::launch_mpnn_reduce(m->partial, (int)count, m->grads, m->stream));
    if (out_loss && targets) {
        std::vector<float> sq((size_t)count * 2);
        MP_TRY(hipMemcpyAsync(sq.data(), m->sq, sq.size() * 4, hipMemcpyDeviceToHost, m->stream));
        MP_TRY(hipStreamSynchronize(m->stream));
        double sum = 0;
        for (float e : sq)
            sum += e;
        *out_loss = (float)(sum / (double)sq.size());
    }
    MP_TRY(hipStreamSynchronize(m->stream));
    return TW_OK;
}

tw_status pack(tw_mpnn *m)
{
    MP_TRY(twk::launch_mpnn_pack(m->params, m->wsb, m->wsbt, m->wnb, m->wnbt, m->stream));
    MP_TRY(hipStreamSynchronize(m->stream));
    return TW_OK;
}

}  // namespace

extern "C" {

uint32_t tw_mpnn_param_count(void) { return (uint32_t)twk::MpnnParams; }

tw_status tw_mpnn_features(const tw_graph *g, float *out)
{
    if (!out || !valid_graph(g))
        return TW_EINVAL;
    node_features(g, out);
    return TW_OK;
}

void tw_mpnn_destroy(tw_mpnn *m)
{
    if (!m)
        return;
    (void)hipSetDevice(m->device);
    if (m->stream)
        (void)hipStreamSynchronize(m->stream);
    for (void *p : {(void *)m->params, (void *)m->m, (void *)m->v, (void *)m->grads, (void *)m->wsb,
                    (void *)m->wsbt, (void *)m->wnb, (void *)m->wnbt, (void *)m->adj, (void *)m->feat,
                    (void *)m->n, (void *)m->targets, (void *)m->pred, (void *)m->sq, (void *)m->partial})
        if (p)
            (void)hipFree(p);
    if (m->own_stream && m->stream)
        (void)hipStreamDestroy(m->stream);
    delete m;
}

tw_status tw_mpnn_create(int device, void *stream, const float *params, tw_mpnn **out)
{
    if (!out || !params)
        return TW_EINVAL;
    *out = nullptr;
    tw_mpnn *m = new (std::nothrow) tw_mpnn();
    if (!m)
        return TW_ENOMEM;
    m->device = device;
    if (hipSetDevice(device) != hipSuccess) {
        delete m;
        return TW_EDEVICE;
    }
    if (stream) {
        m->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&m->stream, hipStreamNonBlocking) != hipSuccess) {
            delete m;
            return TW_EDEVICE;
        }
        m->own_stream = true;
    }
    const size_t P = twk::MpnnParams;
    if (dmalloc(&m->params, P) != hipSuccess || dmalloc(&m->m, P) != hipSuccess ||
        dmalloc(&m->v, P) != hipSuccess || dmalloc(&m->grads, P) != hipSuccess ||
        dmalloc(&m->wsb, 3 * 4096) != hipSuccess || dmalloc(&m->wsbt, 3 * 4096) != hipSuccess ||
        dmalloc(&m->wnb, 3 * 4096) != hipSuccess || dmalloc(&m->wnbt, 3 * 4096) != hipSuccess) {
        (void)hipGetLastError();
        tw_mpnn_destroy(m);
        return TW_ENOMEM;
    }
    tw_status s = tw_mpnn_set_params(m, params);
    if (s != TW_OK) {
        tw_mpnn_destroy(m);
        return s;
    }
    *out = m;
    return TW_OK;
}

tw_status tw_mpnn_set_params(tw_mpnn *m, const float *params)
{
    if (!m || !params)
        return TW_EINVAL;
    (void)hipSetDevice(m->device);
    const size_t P = twk::MpnnParams;
    std::vector<float> zeros(P, 0.f);
    MP_TRY(hipMemcpyAsync(m->params, params, P * 4, hipMemcpyHostToDevice, m->stream));
    MP_TRY(hipMemcpyAsync(m->m, zeros.data(), P * 4, hipMemcpyHostToDevice, m->stream));
    MP_TRY(hipMemcpyAsync(m->v, zeros.data(), P * 4, hipMemcpyHostToDevice, m->stream));
    m->step = 0;
    return pack(m);
}

tw_status tw_mpnn_get_params(tw_mpnn *m, float *params)
{
    if (!m || !params)
        return TW_EINVAL;
    (void)hipSetDevice(m->device);
    MP_TRY(hipMemcpyAsync(params, m->params, (size_t)twk::MpnnParams * 4, hipMemcpyDeviceToHost, m->stream));
    MP_TRY(hipStreamSynchronize(m->stream));
    return TW_OK;
}

tw_status tw_mpnn_predict(tw_mpnn *m, const tw_graph *gs, uint32_t count, float *out)
{
    if (!m || (count && (!gs || !out)))
        return TW_EINVAL;
    if (!count)
        return TW_OK;
    (void)hipSetDevice(m->device);
    tw_status s = upload_graphs(m, gs, count);
    if (s != TW_OK)
        return s;
    s = run(m, count, nullptr, false, nullptr);
    if (s != TW_OK)
        return s;
    MP_TRY(hipMemcpyAsync(out, m->pred, (size_t)count * 2 * 4, hipMemcpyDeviceToHost, m->stream));
    MP_TRY(hipStreamSynchronize(m->stream));
    return TW_OK;
}

tw_status tw_mpnn_gradients(tw_mpnn *m, const tw_graph *gs, uint32_t count, const float *targets,
                            float *out_loss, float *out_grads)
{
    if (!m || !count || !gs || !targets || !out_grads)
        return TW_EINVAL;
    (void)hipSetDevice(m->device);
    tw_status s = upload_graphs(m, gs, count);
    if (s != TW_OK)
        return s;
    s = run(m, count, targets, true, out_loss);
    if (s != TW_OK)
        return s;
    MP_TRY(hipMemcpyAsync(out_grads, m->grads, (size_t)twk::MpnnParams * 4, hipMemcpyDeviceToHost, m->stream));
    MP_TRY(hipStreamSynchronize(m->stream));
    return TW_OK;
}

uint32_t tw_mpnn_trace_floats(void) { return (uint32_t)twk::MpnnTraceFloats; }

tw_status tw_mpnn_trace(tw_mpnn *m, const tw_graph *g, const float *target, float *out_trace, float *out_grads)
{
    if (!m || !g || !target || !out_trace || !out_grads)
        return TW_EINVAL;
    (void)hipSetDevice(m->device);
    tw_status s = upload_graphs(m, g, 1);
    if (s != TW_OK)
        return s;
    float *dtr = nullptr;
    if (dmalloc(&dtr, (size_t)twk::MpnnTraceFloats) != hipSuccess) {
        (void)hipGetLastError();
        return TW_ENOMEM;
    }
    twk::MpnnArgs a = base_args(m);
    a.pred = m->pred;
    a.trace = dtr;
    a.grads = m->partial;
    a.sq_err = m->sq;
    a.grad_scale = 0.5f;  // one graph, two outputs: the loss is their mean
    tw_status st = TW_OK;
    if (hipMemcpyAsync(m->targets, target, 2 * 4, hipMemcpyHostToDevice, m->stream) != hipSuccess ||
        (a.targets = m->targets, twk::launch_mpnn(a, 1, m->stream)) != hipSuccess ||
        hipMemcpyAsync(out_trace, dtr, (size_t)twk::MpnnTraceFloats * 4, hipMemcpyDeviceToHost, m->stream) !=
            hipSuccess ||
        hipMemcpyAsync(out_grads, m->partial, (size_t)twk::MpnnParams * 4, hipMemcpyDeviceToHost, m->stream) !=
            hipSuccess ||
        hipStreamSynchronize(m->stream) != hipSuccess) {
        (void)hipGetLastError();
        st = TW_EDEVICE;
    }
    (void)hipFree(dtr);
    return st;
}

tw_status tw_mpnn_train_step(tw_mpnn *m, const tw_graph *gs, uint32_t count, const float *targets, float lr,
                             float weight_decay, float *out_loss)
{
    if (!m || !count || !gs || !targets)
        return TW_EINVAL;
    (void)hipSetDevice(m->device);
    tw_status s = upload_graphs(m, gs, count);
    if (s != TW_OK)
        return s;
    s = run(m, count, targets, true, out_loss);
    if (s != TW_OK)
        return s;
    m->step++;
    twk::MpnnOptArgs o{};
    o.params = m->params;
    o.m = m->m;
    o.v = m->v;
    o.grads = m->grads;
    o.lr = lr;
    o.beta1 = 0.9f;
    o.beta2 = 0.999f;
    o.eps = 1e-8f;
    o.weight_decay = weight_decay;
    o.bc1 = 1.f - std::pow(0.9f, (float)m->step);
    o.bc2 = 1.f - std::pow(0.999f, (float)m->step);
    MP_TRY(twk::launch_mpnn_adamw(o, m->stream));
    return pack(m);
}

}  // extern "C"
