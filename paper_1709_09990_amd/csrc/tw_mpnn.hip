// The small message-passing network that predicts a graph's treewidth and the
// size of its largest certifying level (used to pick the first bound k and to
// size per-graph memory).  bfloat16 MFMA on gfx950, float32 accumulation.
//
//   x_v     = [1, deg(v)/8, core(v)/8, n/64, 0...]          (64 wide, host)
//   H_{l+1} = ReLU(H_l Ws_l^T + (A H_l) Wn_l^T + b_l) * mask   l = 0, 1, 2
//   r       = [sum_v H3_v ; max_v H3_v],  y = Wo r + bo       (2 outputs)
//   loss    = mean over graphs and outputs of (y - t)^2
//
// One workgroup (4 waves) per graph, padded to 64 nodes: every product is a
// 64x64 output with K = 64, and wave w computes the 32x32 quadrant
// (rows 32*(w/2), cols 32*(w%2)) with v_mfma_f32_32x32x16_bf16.  Operands sit
// in LDS (or, for weights, global memory) with K contiguous, so each lane
// fetches its 8 bf16 operand values with one 16-byte load.
//
// bfloat16 rounding points (the CPU reference rounds at the same ones):
// H_l, A H_l and the weights in the forward pass; dZ_l and dZ_l Wn_l in the
// backward pass.  Gradients of every graph are written to their own slot and
// summed by a second kernel in a fixed order (deterministic).
#include "tw_mpnn.h"

namespace twk {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int NP = 64;       // padded nodes
constexpr int HD = 64;       // hidden width
constexpr int LD = HD + 8;   // LDS row stride in bf16 elements (16-byte pad against bank conflicts)
constexpr int LDF = HD + 1;  // fp32 LDS row stride

__device__ __forceinline__ uint16_t to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest, ties to even
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float from_bf16(uint16_t b)
{
    return __uint_as_float((uint32_t)b << 16);
}

// acc += A[32 rows][K] * B^T[32 cols][K], A and Bt with K contiguous.
// Lane l supplies A[l%32][8*(l/32) .. +7] and Bt[l%32][8*(l/32) .. +7] per
// K step of 16.
__device__ __forceinline__ f32x16 mma32(const uint16_t *A, int sa, const uint16_t *Bt, int sb, int K,
                                        f32x16 acc, int lane)
{
    const int r = lane & 31, h = lane >> 5;
    for (int k0 = 0; k0 < K; k0 += 16) {
        const bf16x8 a = *(const bf16x8 *)(A + r * sa + k0 + 8 * h);
        const bf16x8 b = *(const bf16x8 *)(Bt + r * sb + k0 + 8 * h);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    return acc;
}

// Row/column of accumulator element e (0..15) of lane `lane` in a 32x32 tile.
__device__ __forceinline__ int acc_row(int e, int lane) { return 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3); }
__device__ __forceinline__ int acc_col(int lane) { return lane & 31; }

__device__ __forceinline__ f32x16 zero16()
{
    f32x16 z;
#pragma unroll
    for (int e = 0; e < 16; ++e)
        z[e] = 0.f;
    return z;
}

struct Smem {
    uint16_t adj[NP * LD];          // A[v][u] (symmetric)
    uint16_t hn[NP * LD];           // H_l node-major [v][f] (current layer input)
    uint16_t hf[4][HD * LD];        // H_l feature-major [f][v], l = 0..3 (kept for backward)
    uint16_t mn[NP * LD];           // (A H_l) node-major
    uint16_t mf[3][HD * LD];        // (A H_l) feature-major, l = 0..2
    uint16_t dzn[NP * LD];          // dZ node-major
    uint16_t dzf[HD * LD];          // dZ feature-major
    uint16_t pf[HD * LD];           // (dZ Wn) feature-major
    float f32[NP * LDF];            // H3 (forward), then dH / dZ (backward), fp32
    float r[2 * HD];
    float dr[2 * HD];
    int amax[HD];
    float mask[NP];
    float y[2], dy[2];
};

__global__ __launch_bounds__(256) void mpnn_kernel(MpnnArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    Smem &s = *reinterpret_cast<Smem *>(smem_raw);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const int rq = 32 * (w >> 1), cq = 32 * (w & 1);
    const int g = blockIdx.x;
    const int n = a.n[g];
    const uint64_t *rows = a.adj + (size_t)g * 64;
    const float *x = a.feat + (size_t)g * NP * MpnnFeat;
    float *tr = a.trace ? a.trace + (size_t)g * MpnnTraceFloats : nullptr;

    // adjacency, mask, H0 (node- and feature-major)
    for (int e = tid; e < NP * NP; e += 256) {
        const int v = e >> 6, u = e & 63;
        const bool edge = v < n && ((rows[v] >> u) & 1ull);
        s.adj[v * LD + u] = edge ? (uint16_t)0x3F80 : (uint16_t)0;  // 1.0 or 0.0
        const float xv = (v < n && u < MpnnFeat) ? x[v * MpnnFeat + u] : 0.f;
        const uint16_t xb = to_bf16(xv);
        s.hn[v * LD + u] = xb;
        s.hf[0][u * LD + v] = xb;
    }
    if (tid < NP)
        s.mask[tid] = tid < n ? 1.f : 0.f;
    __syncthreads();

    // ---------------- forward ----------------
    for (int l = 0; l < 3; ++l) {
        // M = A H_l  (K = nodes; B operand = H feature-major)
        f32x16 acc = mma32(s.adj + rq * LD, LD, s.hf[l] + cq * LD, LD, NP, zero16(), lane);
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int v = rq + acc_row(e, lane), f = cq + acc_col(lane);
            const uint16_t b = to_bf16(acc[e]);
            s.mn[v * LD + f] = b;
            s.mf[l][f * LD + v] = b;
            if (tr)
                tr[MpnnTrM + l * 4096 + v * 64 + f] = acc[e];
        }
        __syncthreads();
        // Z = H_l Ws^T + M Wn^T + b  (K = features; B operands = weights [out][in])
        const uint16_t *Ws = a.wsb + (size_t)l * HD * HD;
        const uint16_t *Wn = a.wnb + (size_t)l * HD * HD;
        acc = mma32(s.hn + rq * LD, LD, Ws + cq * HD, HD, HD, zero16(), lane);
        acc = mma32(s.mn + rq * LD, LD, Wn + cq * HD, HD, HD, acc, lane);
        __syncthreads();  // every wave has read hn / mn
        const float *bias = a.params + (size_t)l * MpnnLayerParams + 2 * HD * HD;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int v = rq + acc_row(e, lane), o = cq + acc_col(lane);
            float z = acc[e] + bias[o];
            if (tr)
                tr[MpnnTrZ + l * 4096 + v * 64 + o] = z;
            z = z > 0.f ? z : 0.f;
            z *= s.mask[v];
            const uint16_t b = to_bf16(z);
            s.hn[v * LD + o] = b;
            s.hf[l + 1][o * LD + v] = b;
            if (l == 2)
                s.f32[v * LDF + o] = z;
        }
        __syncthreads();
    }

    // ---------------- readout and heads (fp32) ----------------
    if (tid < HD) {
        float sum = 0.f;
        for (int v = 0; v < n; ++v)
            sum += s.f32[v * LDF + tid];
        s.r[tid] = sum;
    } else if (tid < 2 * HD) {
        const int j = tid - HD;
        float best = -1.f;
        int arg = 0;
        for (int v = 0; v < n; ++v) {
            const float h = s.f32[v * LDF + j];
            if (h > best) {
                best = h;
                arg = v;
            }
        }
        s.r[HD + j] = n > 0 ? best : 0.f;
        s.amax[j] = arg;
    }
    __syncthreads();
    if (tr && tid < 2 * HD)
        tr[MpnnTrR + tid] = s.r[tid];
    const float *Wo = a.params + 3 * MpnnLayerParams;
    const float *bo = Wo + 2 * 2 * HD;
    if (tid < 2) {
        float y = bo[tid];
        for (int j = 0; j < 2 * HD; ++j)
            y += Wo[tid * 2 * HD + j] * s.r[j];
        s.y[tid] = y;
        if (tr)
            tr[MpnnTrR + 2 * HD + tid] = y;
        if (a.pred)
            a.pred[(size_t)g * 2 + tid] = y;
        if (a.targets) {
            const float d = y - a.targets[(size_t)g * 2 + tid];
            s.dy[tid] = 2.f * d * a.grad_scale;
            if (a.sq_err)
                a.sq_err[(size_t)g * 2 + tid] = d * d;
        }
    }
    if (!a.grads)
        return;
    __syncthreads();

    // ---------------- backward ----------------
    float *gslot = a.grads + (size_t)g * MpnnParams;
    float *gWo = gslot + 3 * MpnnLayerParams;
    for (int e = tid; e < 2 * 2 * HD; e += 256)
        gWo[e] = s.dy[e / (2 * HD)] * s.r[e % (2 * HD)];
    if (tid < 2)
        gWo[2 * 2 * HD + tid] = s.dy[tid];
    if (tid < 2 * HD)
        s.dr[tid] = Wo[tid] * s.dy[0] + Wo[2 * HD + tid] * s.dy[1];
    __syncthreads();
    // dH3 into f32 (fp32)
    for (int e = tid; e < NP * HD; e += 256) {
        const int v = e >> 6, j = e & 63;
        float d = s.mask[v] * s.dr[j];
        if (v < n && s.amax[j] == v)
            d += s.dr[HD + j];
        s.f32[v * LDF + j] = d;
        if (tr)
            tr[MpnnTrDH3 + v * 64 + j] = d;
    }
    __syncthreads();

    for (int l = 2; l >= 0; --l) {
        float *gl = gslot + (size_t)l * MpnnLayerParams;
        // dZ = dH * [H_{l+1} > 0] * mask; bias gradient from fp32 dZ
        for (int e = tid; e < NP * HD; e += 256) {
            const int v = e >> 6, o = e & 63;
            const bool on = from_bf16(s.hf[l + 1][o * LD + v]) > 0.f;
            const float dz = on ? s.f32[v * LDF + o] * s.mask[v] : 0.f;
            s.f32[v * LDF + o] = dz;
            if (tr)
                tr[MpnnTrDZ + l * 4096 + v * 64 + o] = dz;
            const uint16_t b = to_bf16(dz);
            s.dzn[v * LD + o] = b;
            s.dzf[o * LD + v] = b;
        }
        __syncthreads();
        if (tid < HD) {
            float sum = 0.f;
            for (int v = 0; v < NP; ++v)
                sum += s.f32[v * LDF + tid];
            gl[2 * HD * HD + tid] = sum;
        }
        // dWs = dZ^T H_l, dWn = dZ^T M_l  (K = nodes; A = dZ feature-major)
        f32x16 acc = mma32(s.dzf + rq * LD, LD, s.hf[l] + cq * LD, LD, NP, zero16(), lane);
#pragma unroll
        for (int e = 0; e < 16; ++e)
            gl[(rq + acc_row(e, lane)) * HD + cq + acc_col(lane)] = acc[e];
        acc = mma32(s.dzf + rq * LD, LD, s.mf[l] + cq * LD, LD, NP, zero16(), lane);
#pragma unroll
        for (int e = 0; e < 16; ++e)
            gl[HD * HD + (rq + acc_row(e, lane)) * HD + cq + acc_col(lane)] = acc[e];
        if (l == 0)
            break;
        // P = bf16(dZ Wn) (K = out; B operand = Wn^T stored [in][out])
        const uint16_t *WsT = a.wsbt + (size_t)l * HD * HD;
        const uint16_t *WnT = a.wnbt + (size_t)l * HD * HD;
        acc = mma32(s.dzn + rq * LD, LD, WnT + cq * HD, HD, HD, zero16(), lane);
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            s.pf[(cq + acc_col(lane)) * LD + rq + acc_row(e, lane)] = to_bf16(acc[e]);
            if (tr)
                tr[MpnnTrP + (l - 1) * 4096 + (rq + acc_row(e, lane)) * 64 + cq + acc_col(lane)] = acc[e];
        }
        __syncthreads();
        // dH_l = dZ Ws + A P
        acc = mma32(s.dzn + rq * LD, LD, WsT + cq * HD, HD, HD, zero16(), lane);
        acc = mma32(s.adj + rq * LD, LD, s.pf + cq * LD, LD, NP, acc, lane);
        __syncthreads();  // f32 (dZ) fully consumed
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            s.f32[(rq + acc_row(e, lane)) * LDF + cq + acc_col(lane)] = acc[e];
            if (tr)
                tr[MpnnTrDH + (l - 1) * 4096 + (rq + acc_row(e, lane)) * 64 + cq + acc_col(lane)] = acc[e];
        }
        __syncthreads();
    }
}

// grads[p] = sum over graphs of partial[g][p], in graph order.
__global__ void mpnn_reduce_kernel(const float *partial, int graphs, float *grads)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= MpnnParams)
        return;
    float s = 0.f;
    for (int g = 0; g < graphs; ++g)
        s += partial[(size_t)g * MpnnParams + p];
    grads[p] = s;
}

// AdamW on the fp32 master parameters (decoupled weight decay on the
// matrices, not on biases), then the bf16 working copies in both layouts.
__global__ void mpnn_adamw_kernel(MpnnOptArgs o)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= MpnnParams)
        return;
    const float g = o.grads[p];
    float m = o.m[p] = o.beta1 * o.m[p] + (1.f - o.beta1) * g;
    float v = o.v[p] = o.beta2 * o.v[p] + (1.f - o.beta2) * g * g;
    const float mh = m / o.bc1, vh = v / o.bc2;
    float th = o.params[p];
    int layer = p / MpnnLayerParams;
    int within = p % MpnnLayerParams;
    const bool is_bias = (layer < 3 && within >= 2 * HD * HD) || (layer >= 3 && p >= 3 * MpnnLayerParams + 2 * 2 * HD);
    if (!is_bias)
        th -= o.lr * o.weight_decay * th;
    th -= o.lr * mh / (sqrtf(vh) + o.eps);
    o.params[p] = th;
}

__global__ void mpnn_pack_kernel(const float *params, uint16_t *wsb, uint16_t *wsbt, uint16_t *wnb,
                                 uint16_t *wnbt)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 3 * HD * HD)
        return;
    const int l = e / (HD * HD), r = (e / HD) % HD, c = e % HD;
    const float *P = params + (size_t)l * MpnnLayerParams;
    const uint16_t s = to_bf16(P[r * HD + c]);
    const uint16_t nn = to_bf16(P[HD * HD + r * HD + c]);
    wsb[(size_t)l * HD * HD + r * HD + c] = s;
    wsbt[(size_t)l * HD * HD + c * HD + r] = s;
    wnb[(size_t)l * HD * HD + r * HD + c] = nn;
    wnbt[(size_t)l * HD * HD + c * HD + r] = nn;
}

}  // namespace

size_t mpnn_smem_bytes() { return sizeof(Smem); }

hipError_t launch_mpnn(const MpnnArgs &a, int graphs, hipStream_t s)
{
    if (graphs <= 0)
        return hipSuccess;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)mpnn_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(Smem));
        if (e != hipSuccess)
            return e;
        attr_set = true;
    }
    hipLaunchKernelGGL(mpnn_kernel, dim3(graphs), dim3(256), sizeof(Smem), s, a);
    return hipGetLastError();
}

hipError_t launch_mpnn_reduce(const float *partial, int graphs, float *grads, hipStream_t s)
{
    hipLaunchKernelGGL(mpnn_reduce_kernel, dim3((MpnnParams + 255) / 256), dim3(256), 0, s, partial, graphs,
                       grads);
    return hipGetLastError();
}

hipError_t launch_mpnn_adamw(const MpnnOptArgs &o, hipStream_t s)
{
    hipLaunchKernelGGL(mpnn_adamw_kernel, dim3((MpnnParams + 255) / 256), dim3(256), 0, s, o);
    return hipGetLastError();
}

hipError_t launch_mpnn_pack(const float *params, uint16_t *wsb, uint16_t *wsbt, uint16_t *wnb, uint16_t *wnbt,
                            hipStream_t s)
{
    hipLaunchKernelGGL(mpnn_pack_kernel, dim3((3 * 64 * 64 + 255) / 256), dim3(256), 0, s, params, wsb, wsbt,
                       wnb, wnbt);
    return hipGetLastError();
}

}  // namespace twk
