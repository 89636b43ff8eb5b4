// Batched uneven workload: the whole hot path (preprocessing, MoP paths,
// path search and argmin, precoding) for groups of subcarriers with
// different user counts N, perturbation intervals and path counts, as one
// captured HIP graph per slot.
//
// Stages, each one launch over all groups (descriptor per group, looked up
// per workgroup or per vector):
//   fill      reset the per-vector argmin keys and the tile queue
//   preprocess / MoP   one workgroup per subcarrier (vp_preprocess.hip, vp_mop.hip)
//   search    persistent: one wave per workgroup, a grid that fills the chip
//             once; each wave takes the next tile from an atomic counter.  A
//             tile is (vt vectors of one subcarrier) x (a chunk of 64/vt * pl
//             consecutive paths): each of the vt lane segments walks its
//             vector's paths, reduces the segment's (cost, k) key and merges
//             it into the vector's key with a 64-bit atomic minimum.
//   finish    one lane per vector: re-walk the winning path for l (user
//             order), the cost, and the precoded vector x = G (s + tau l)
// The walk, start residual and key are those of the per-call search
// (vp_walk.hpp), so every vector gets exactly the per-call result.
//
// The tile shape (vt, pl) is chosen per class of groups with equal K; the
// tile list is built on the host in decreasing order of estimated work
// (longest first) so that the queue's tail holds the short tiles.
#include <math.h>

#include <algorithm>
#include <new>
#include <vector>

#include "../../include/vp_batch.h"
#include "vp_walk.hpp"

namespace vp {
namespace {

constexpr int kBW = 64;    // threads of a persistent search workgroup (one wave)
constexpr int kFT = 256;   // threads of the fill and finish kernels
constexpr int kMaxBatchK = 512;

__global__ __launch_bounds__(kFT) void k_batch_fill(unsigned long long *__restrict__ best, int n_vec,
                                                    uint32_t *__restrict__ counter) {
    const int v = blockIdx.x * kFT + threadIdx.x;
    if (v < n_vec) best[v] = ~0ull;
    if (v == 0) *counter = 0u;
}

template <int N>
__device__ __forceinline__ void batch_tile(const BatchGroup &g, int vfirst, int k0, int lane,
                                           const float2 *__restrict__ W, const uint8_t *__restrict__ perm,
                                           const float2 *__restrict__ s, const uint8_t *__restrict__ paths,
                                           int n_sym, unsigned flags, unsigned long long *__restrict__ best,
                                           float2 (*s_r0)[kMaxN], float *s_nlinv, float *s_wdiag) {
    constexpr int NP = VP_PACKED(N);
    const int lpv = kBW / g.vt;                    // lanes per vector (64, 32 or 16)
    const int seg = lane / lpv, sl = lane % lpv;
    const int sc = vfirst / n_sym;                 // every vector of a tile is on this subcarrier
    const int v = vfirst + seg;
    const bool vok = (v < g.n_vec) && (v / n_sym == sc);
    const float2 *__restrict__ Wc = W + g.offW + (long long)sc * NP;
    const float w00 = Wc[0].x;
    if (!(w00 > 0.f) || !isfinite(w00)) return;   // failed preprocessing: the key stays unset
    const uint8_t *pm = perm + g.offN + (long long)sc * N;
    if (lane < N) {
        s_wdiag[lane] = Wc[vp_pidx(N, lane, lane)].x;
        s_nlinv[lane] = -(1.0f / s_wdiag[lane]);
    }
    if (vok && sl < N)
        s_r0[seg][sl] = stilde_over_tau<N>(Wc, pm, s + g.offS, (size_t)v, (size_t)g.n_vec, sl, 1.0f / g.tau);
    __syncthreads();
    const uint8_t *P = paths + g.offP + (long long)sc * g.K * N;
    const float tau2 = g.tau * g.tau;
    unsigned long long key = ~0ull;
    const int kend = min(g.K, k0 + lpv * g.pl);
    if (vok) {
        for (int k = k0 + sl; k < kend; k += lpv) {
            const unsigned long long wd = load_word<N>(P, k);
            float2 r[N];
#pragma unroll
            for (int i = 0; i < N; ++i) r[i] = s_r0[seg][i];
            const float ped = walk<N, kTierAny, false>(Wc, s_nlinv, s_wdiag, r, wd, 0ull, VP_DEMAP_LUT, nullptr, nullptr);
            key = umin64(key, ((unsigned long long)__float_as_uint(ped * tau2) << 32) | (unsigned)k);
        }
        if ((flags & VP_INCLUDE_ZERO) && k0 == 0 && sl == 0) {
            float z = 0.f;
            for (int i = 0; i < N; ++i) {
                z = fmaf(s_r0[seg][i].x, s_r0[seg][i].x, z);
                z = fmaf(s_r0[seg][i].y, s_r0[seg][i].y, z);
            }
            key = umin64(key, ((unsigned long long)__float_as_uint(z * tau2) << 32) | (unsigned)g.K);
        }
    }
    for (int off = lpv >> 1; off > 0; off >>= 1) key = umin64(key, __shfl_xor(key, off));
    if (vok && sl == 0 && key != ~0ull) atomicMin(best + g.v0 + v, key);
    __syncthreads();   // the next tile rewrites the LDS state
}

__global__ __launch_bounds__(kBW) void k_batch_search(const BatchGroup *__restrict__ groups,
                                                      const uint2 *__restrict__ tiles,
                                                      const uint32_t *__restrict__ ntiles,
                                                      uint32_t *__restrict__ counter, const float2 *__restrict__ W,
                                                      const uint8_t *__restrict__ perm,
                                                      const float2 *__restrict__ s,
                                                      const uint8_t *__restrict__ paths, int n_sym, unsigned flags,
                                                      unsigned long long *__restrict__ best) {
    __shared__ float2 s_r0[4][kMaxN];
    __shared__ float s_nlinv[kMaxN];
    __shared__ float s_wdiag[kMaxN];
    const int lane = threadIdx.x;
    const uint32_t nt = *ntiles;
    for (;;) {   // every wave leaves once the counter has passed the last tile
        uint32_t ti = 0;
        if (lane == 0) ti = atomicAdd(counter, 1u);
        ti = __builtin_amdgcn_readfirstlane(ti);
        if (ti >= nt) break;
        const uint2 tl = tiles[ti];
        const BatchGroup g = groups[tl.x >> 16];
        const int vfirst = (int)(tl.x & 0xffffu), k0 = (int)tl.y;
        switch (g.U) {
#define VP_CASE(n)                                                                                             \
    case n:                                                                                                    \
        batch_tile<n>(g, vfirst, k0, lane, W, perm, s, paths, n_sym, flags, best, s_r0, s_nlinv, s_wdiag); \
        break;
            VP_CASE(1) VP_CASE(2) VP_CASE(3) VP_CASE(4) VP_CASE(5) VP_CASE(6) VP_CASE(7) VP_CASE(8)
            VP_CASE(9) VP_CASE(10) VP_CASE(11) VP_CASE(12) VP_CASE(13) VP_CASE(14) VP_CASE(15) VP_CASE(16)
#undef VP_CASE
            default: break;
        }
    }
}

template <int N>
__device__ __forceinline__ void batch_finish_one(const BatchGroup &g, int vloc, unsigned long long key,
                                                 const float2 *__restrict__ W, const uint8_t *__restrict__ perm,
                                                 const float2 *__restrict__ s, const uint8_t *__restrict__ paths,
                                                 const float2 *__restrict__ G, int n_sym, int M, float P_T,
                                                 int8_t *__restrict__ l_out, float *__restrict__ cost_out,
                                                 float2 *__restrict__ x_out) {
    constexpr int NP = VP_PACKED(N);
    const int sc = vloc / n_sym;
    const uint32_t k = (uint32_t)(key & 0xffffffffull);
    const float2 *__restrict__ Wc = W + g.offW + (long long)sc * NP;
    const uint8_t *pm = perm + g.offN + (long long)sc * N;
    const float2 *sg = s + g.offS;
    float ra[N], rb[N];
#pragma unroll
    for (int i = 0; i < N; ++i) ra[i] = rb[i] = 0.f;
    if (k < (uint32_t)g.K) {
        float nlinv[N], wdiag[N];
        float2 r[N];
        const float inv_tau = 1.0f / g.tau;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            wdiag[i] = Wc[vp_pidx(N, i, i)].x;
            nlinv[i] = -(1.0f / wdiag[i]);
            r[i] = stilde_over_tau<N>(Wc, pm, sg, (size_t)vloc, (size_t)g.n_vec, i, inv_tau);
        }
        const uint8_t *P = paths + g.offP + ((long long)sc * g.K + k) * N;
        unsigned long long wd = 0;
        for (int i = 0; i < N; ++i) wd |= (unsigned long long)(P[i] & 15) << (4 * i);
        (void)walk<N, kTierLut, true>(Wc, nlinv, wdiag, r, wd, 0ull, VP_DEMAP_LUT, ra, rb);
    }
    const bool ok = k <= (uint32_t)g.K;   // a path or the zero perturbation
    const float c = ok ? __uint_as_float((uint32_t)(key >> 32)) : __int_as_float(0x7fc00000);
    cost_out[g.v0 + vloc] = c;
    int pu[N];
#pragma unroll
    for (int i = 0; i < N; ++i) pu[i] = pm[i] < N ? pm[i] : N - 1;
    float lr[N], li[N];   // l in user order
#pragma unroll
    for (int u = 0; u < N; ++u) {
        float a = 0.f, b = 0.f;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const bool hit = pu[i] == u;
            a = hit ? ra[i] : a;
            b = hit ? rb[i] : b;
        }
        lr[u] = a;
        li[u] = b;
        int8_t *o = l_out + 2 * (g.offS + (long long)u * g.n_vec + vloc);
        o[0] = (int8_t)a;
        o[1] = (int8_t)b;
    }
    // x = G (s + tau l), the arithmetic of vp_precode
    float scale = 1.f;
    if (P_T > 0.f) scale = (c > 0.f && isfinite(c)) ? sqrtf(P_T / c) : __int_as_float(0x7fc00000);
    const float2 *Gs = G + g.offG + (long long)sc * M * N;
    float2 *xo = x_out + (long long)(g.v0 + vloc) * M;
    for (int m = 0; m < M; ++m) {
        float re = 0.f, im = 0.f;
#pragma unroll
        for (int u = 0; u < N; ++u) {
            const float2 su = sg[(long long)u * g.n_vec + vloc];
            const float ur = fmaf(g.tau, lr[u], su.x);
            const float ui = fmaf(g.tau, li[u], su.y);
            const float2 gi = Gs[(long long)m * N + u];
            re = fmaf(gi.x, ur, fmaf(-gi.y, ui, re));
            im = fmaf(gi.x, ui, fmaf(gi.y, ur, im));
        }
        if (P_T > 0.f) {
            re *= scale;
            im *= scale;
        }
        xo[m] = make_float2(re, im);
    }
}

__global__ __launch_bounds__(kFT) void k_batch_finish(const BatchGroup *__restrict__ groups, int n_groups,
                                                      int n_vec_total, const unsigned long long *__restrict__ best,
                                                      const float2 *__restrict__ W, const uint8_t *__restrict__ perm,
                                                      const float2 *__restrict__ s,
                                                      const uint8_t *__restrict__ paths,
                                                      const float2 *__restrict__ G, int n_sym, int M, float P_T,
                                                      int8_t *__restrict__ l, float *__restrict__ cost,
                                                      float2 *__restrict__ x) {
    const int v = blockIdx.x * kFT + threadIdx.x;
    if (v >= n_vec_total) return;
    int lo = 0, hi = n_groups - 1;   // the group holding vector v
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (groups[mid].v0 <= v) lo = mid;
        else hi = mid - 1;
    }
    const BatchGroup g = groups[lo];
    const int vloc = v - g.v0;
    const unsigned long long key = best[v];
    switch (g.U) {
#define VP_CASE(n)                                                                                                  \
    case n: batch_finish_one<n>(g, vloc, key, W, perm, s, paths, G, n_sym, M, P_T, l, cost, x); break;
        VP_CASE(1) VP_CASE(2) VP_CASE(3) VP_CASE(4) VP_CASE(5) VP_CASE(6) VP_CASE(7) VP_CASE(8)
        VP_CASE(9) VP_CASE(10) VP_CASE(11) VP_CASE(12) VP_CASE(13) VP_CASE(14) VP_CASE(15) VP_CASE(16)
#undef VP_CASE
        default: break;
    }
}

bool exceeds_box(int K, int N) {   // K > 9^N ?
    long long cap = 1;
    for (int i = 0; i < N; ++i) {
        cap *= 9;
        if (cap >= K) return false;
    }
    return cap < K;
}

}  // namespace
}  // namespace vp

using namespace vp;

struct vp_batch {
    int device = 0;
    int n_groups = 0, M = 0, n_sym = 0, n_sc = 0, n_vec = 0;
    float P_T = 0.f;
    uint32_t flags = 0;
    std::vector<BatchGroup> hg;
    std::vector<int> classK;
    std::vector<int> cls_vt, cls_pl;
    int lpt = 1;
    int n_tiles = 0, max_tiles = 0, grid = 0;
    float default_ms = 0.f, tuned_ms = 0.f;
    // device memory owned by the plan
    BatchGroup *d_groups = nullptr;
    int32_t *d_sc_group = nullptr;
    float2 *W = nullptr, *G = nullptr;
    float *w2 = nullptr;
    uint8_t *perm = nullptr, *paths = nullptr;
    int32_t *status = nullptr;
    unsigned long long *best = nullptr;
    uint2 *tiles = nullptr;
    uint32_t *counter = nullptr, *ntiles = nullptr;
    // caller's arrays
    const float2 *H = nullptr, *s = nullptr;
    float2 *x = nullptr;
    int8_t *l = nullptr;
    float *cost = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

void free_plan(vp_batch *p) {
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    void *bufs[] = {p->d_groups, p->d_sc_group, p->W, p->G, p->w2, p->perm, p->paths, p->status,
                    p->best, p->tiles, p->counter, p->ntiles};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    delete p;
}

int class_of(const vp_batch *p, int K) {
    for (size_t c = 0; c < p->classK.size(); ++c)
        if (p->classK[c] == K) return (int)c;
    return -1;
}

// Default tile shape for K paths: the fewest paths per lane that cover K with
// one tile per vector, several vectors per wave when K is small.
void default_shape(int K, int &vt, int &pl) {
    vt = K <= 16 ? 4 : (K <= 32 ? 2 : 1);
    const int lpv = kBW / vt;
    pl = std::min(8, (K + lpv - 1) / lpv);
    int p2 = 1;
    while (p2 < pl) p2 <<= 1;
    pl = p2;
}

// Builds the tile list of the current shapes; longest tiles first (LPT) or
// group order.  Returns the number of tiles.
int build_tiles(vp_batch *p, std::vector<uint2> &out) {
    out.clear();
    std::vector<std::pair<float, uint2>> withw;
    for (int gi = 0; gi < p->n_groups; ++gi) {
        const BatchGroup &g = p->hg[gi];
        const int lpv = kBW / g.vt, chunk = lpv * g.pl;
        for (int sc = 0; sc < g.n_sc; ++sc)
            for (int b = 0; b < p->n_sym; b += g.vt) {
                const int vfirst = sc * p->n_sym + b;
                for (int k0 = 0; k0 < g.K; k0 += chunk) {
                    const int kn = std::min(chunk, g.K - k0);
                    const float work = (float)((kn + lpv - 1) / lpv) * (float)(g.U * (g.U + 3));
                    withw.push_back({work, make_uint2(((uint32_t)gi << 16) | (uint32_t)vfirst, (uint32_t)k0)});
                }
            }
    }
    if (p->lpt)
        std::stable_sort(withw.begin(), withw.end(),
                         [](const std::pair<float, uint2> &a, const std::pair<float, uint2> &b) {
                             return a.first > b.first;
                         });
    out.reserve(withw.size());
    for (auto &w : withw) out.push_back(w.second);
    return (int)out.size();
}

// Applies the class shapes to the groups and uploads groups and tiles.
int upload_shapes(vp_batch *p) {
    for (auto &g : p->hg) {
        const int c = class_of(p, g.K);
        g.vt = p->cls_vt[c];
        g.pl = p->cls_pl[c];
    }
    std::vector<uint2> tiles;
    const int nt = build_tiles(p, tiles);
    if (nt > p->max_tiles) return VP_EINVAL;
    p->n_tiles = nt;
    if (hipMemcpy(p->d_groups, p->hg.data(), sizeof(BatchGroup) * p->hg.size(), hipMemcpyHostToDevice) != hipSuccess)
        return VP_ELAUNCH;
    if (nt > 0 && hipMemcpy(p->tiles, tiles.data(), sizeof(uint2) * nt, hipMemcpyHostToDevice) != hipSuccess)
        return VP_ELAUNCH;
    const uint32_t n32 = (uint32_t)nt;
    if (hipMemcpy(p->ntiles, &n32, sizeof(n32), hipMemcpyHostToDevice) != hipSuccess) return VP_ELAUNCH;
    return VP_OK;
}

int enqueue_slot(vp_batch *p, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_fill, dim3((unsigned)((p->n_vec + kFT - 1) / kFT)), dim3(kFT), 0, st, p->best,
                       p->n_vec, p->counter);
    int rc = launch_batch_preprocess(p->d_groups, p->d_sc_group, p->n_sc, p->M, p->H, p->W, p->w2, p->perm, p->G,
                                     p->status, st);
    if (rc != VP_OK) return rc;
    int max_K = 0;
    for (const auto &g : p->hg) max_K = g.K > max_K ? g.K : max_K;
    rc = launch_batch_mop(p->d_groups, p->d_sc_group, p->n_sc, max_K, p->w2, p->paths, st);
    if (rc != VP_OK) return rc;
    hipLaunchKernelGGL(k_batch_search, dim3((unsigned)p->grid), dim3(kBW), 0, st, p->d_groups, p->tiles, p->ntiles,
                       p->counter, p->W, p->perm, p->s, p->paths, p->n_sym, p->flags, p->best);
    hipLaunchKernelGGL(k_batch_finish, dim3((unsigned)((p->n_vec + kFT - 1) / kFT)), dim3(kFT), 0, st, p->d_groups,
                       p->n_groups, p->n_vec, p->best, p->W, p->perm, p->s, p->paths, p->G, p->n_sym, p->M, p->P_T,
                       p->l, p->cost, p->x);
    return launch_status();
}

float time_slots(vp_batch *p, int reps, hipStream_t st) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -1.f;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -1.f;
    }
    (void)hipGraphLaunch(p->exec, st);   // warm
    (void)hipEventRecord(e0, st);
    for (int r = 0; r < reps; ++r) (void)hipGraphLaunch(p->exec, st);
    (void)hipEventRecord(e1, st);
    float ms = -1.f;
    if (hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) ms /= reps;
    else ms = -1.f;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms;
}

}  // namespace

extern "C" {

int vp_batch_create(const vp_group *groups, int n_groups, int n_t, int n_sym, float P_T, uint32_t flags,
                    const vp_c32 *H, const vp_c32 *s, vp_c32 *x, int8_t *l, float *cost, vp_batch **plan) {
    if (!plan) return VP_EINVAL;
    *plan = nullptr;
    if (!groups || n_groups < 1 || n_sym < 1 || n_t < 1 || !H || !s || !x || !l || !cost) return VP_EINVAL;
    if (!(P_T >= 0.f) || !isfinite(P_T) || (flags & ~(uint32_t)VP_INCLUDE_ZERO)) return VP_EINVAL;
    if (n_t > kMaxM || n_groups > 65535) return VP_EUNSUPPORTED;
    std::vector<int> classes;
    for (int g = 0; g < n_groups; ++g) {
        const vp_group &d = groups[g];
        if (d.n_sc < 1 || d.K < 1 || d.n_users < 1) return VP_EINVAL;
        if (d.n_users > kMaxN || d.K > kMaxBatchK) return VP_EUNSUPPORTED;
        if (exceeds_box(d.K, d.n_users)) return VP_EINVAL;
        if (!(d.tau > 0.f) || !isfinite(d.tau) || !(d.alpha >= 0.f) || !isfinite(d.alpha)) return VP_EINVAL;
        if (d.alpha == 0.f && d.n_users > n_t) return VP_EINVAL;
        if ((long long)d.n_sc * n_sym > 65535) return VP_EINVAL;
        if (std::find(classes.begin(), classes.end(), d.K) == classes.end()) classes.push_back(d.K);
    }
    if ((int)classes.size() > VP_BATCH_MAX_CLASSES) return VP_EUNSUPPORTED;

    vp_batch *p = new (std::nothrow) vp_batch;
    if (!p) return VP_ELAUNCH;
    (void)hipGetDevice(&p->device);
    p->n_groups = n_groups;
    p->M = n_t;
    p->n_sym = n_sym;
    p->P_T = P_T;
    p->flags = flags;
    p->H = (const float2 *)H;
    p->s = (const float2 *)s;
    p->x = (float2 *)x;
    p->l = l;
    p->cost = cost;
    p->classK = classes;
    long long offH = 0, offW = 0, offN = 0, offG = 0, offP = 0, offS = 0, max_tiles = 0;
    int sc0 = 0, v0 = 0;
    std::vector<int32_t> sc_group;
    for (int gi = 0; gi < n_groups; ++gi) {
        const vp_group &d = groups[gi];
        BatchGroup g;
        g.U = d.n_users;
        g.K = d.K;
        g.n_sc = d.n_sc;
        g.n_vec = d.n_sc * n_sym;
        g.vt = 1;
        g.pl = 1;
        g.tau = d.tau;
        g.alpha = d.alpha;
        g.sc0 = sc0;
        g.v0 = v0;
        g.offH = offH;
        g.offW = offW;
        g.offN = offN;
        g.offG = offG;
        g.offP = offP;
        g.offS = offS;
        p->hg.push_back(g);
        for (int j = 0; j < d.n_sc; ++j) sc_group.push_back(gi);
        offH += (long long)d.n_sc * g.U * n_t;
        offW += (long long)d.n_sc * VP_PACKED(g.U);
        offN += (long long)d.n_sc * g.U;
        offG += (long long)d.n_sc * n_t * g.U;
        offP += (long long)d.n_sc * g.K * g.U;
        offS += (long long)g.U * g.n_vec;
        max_tiles += (long long)g.n_vec * ((g.K + 15) / 16);   // smallest chunk: 16 paths
        sc0 += d.n_sc;
        v0 += g.n_vec;
    }
    p->n_sc = sc0;
    p->n_vec = v0;
    if (max_tiles > (1ll << 30)) {
        free_plan(p);
        return VP_EUNSUPPORTED;
    }
    p->max_tiles = (int)max_tiles;
    p->cls_vt.resize(classes.size());
    p->cls_pl.resize(classes.size());
    for (size_t c = 0; c < classes.size(); ++c) default_shape(classes[c], p->cls_vt[c], p->cls_pl[c]);

    bool ok = hipMalloc((void **)&p->d_groups, sizeof(BatchGroup) * n_groups) == hipSuccess &&
              hipMalloc((void **)&p->d_sc_group, sizeof(int32_t) * p->n_sc) == hipSuccess &&
              hipMalloc((void **)&p->W, sizeof(float2) * offW) == hipSuccess &&
              hipMalloc((void **)&p->G, sizeof(float2) * offG) == hipSuccess &&
              hipMalloc((void **)&p->w2, sizeof(float) * offN) == hipSuccess &&
              hipMalloc((void **)&p->perm, offN) == hipSuccess &&
              hipMalloc((void **)&p->paths, offP) == hipSuccess &&
              hipMalloc((void **)&p->status, sizeof(int32_t) * p->n_sc) == hipSuccess &&
              hipMalloc((void **)&p->best, sizeof(unsigned long long) * p->n_vec) == hipSuccess &&
              hipMalloc((void **)&p->tiles, sizeof(uint2) * p->max_tiles) == hipSuccess &&
              hipMalloc((void **)&p->counter, sizeof(uint32_t)) == hipSuccess &&
              hipMalloc((void **)&p->ntiles, sizeof(uint32_t)) == hipSuccess;
    ok = ok && hipMemcpy(p->d_sc_group, sc_group.data(), sizeof(int32_t) * p->n_sc, hipMemcpyHostToDevice) ==
                   hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        free_plan(p);
        return VP_ELAUNCH;
    }
    int rc = upload_shapes(p);
    if (rc != VP_OK) {
        free_plan(p);
        return rc;
    }
    // persistent grid: as many one-wave workgroups as fit on the chip at once
    int n_cu = 0, per_cu = 0;
    (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, p->device);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_batch_search, kBW, 0);
    p->grid = std::max(1, n_cu) * std::max(1, per_cu);
    prepare_batch_kernels();
    // capture the slot
    hipStream_t cs = nullptr;
    ok = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
        rc = enqueue_slot(p, cs);
        const bool ended = hipStreamEndCapture(cs, &p->graph) == hipSuccess;
        ok = rc == VP_OK && ended && p->graph &&
             hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) == hipSuccess;
    }
    if (cs) (void)hipStreamDestroy(cs);
    if (!ok) {
        (void)hipGetLastError();
        free_plan(p);
        return VP_ELAUNCH;
    }
    *plan = p;
    return VP_OK;
}

int vp_batch_run(vp_batch *plan, void *stream) {
    if (!plan) return VP_EINVAL;
    if (hipGraphLaunch(plan->exec, (hipStream_t)stream) != hipSuccess) return launch_status();
    return VP_OK;
}

int vp_batch_tune(vp_batch *plan, int reps, void *stream) {
    if (!plan || reps < 1) return VP_EINVAL;
    vp_batch *p = plan;
    hipStream_t st = (hipStream_t)stream;
    if (hipStreamSynchronize(st) != hipSuccess) return launch_status();
    p->default_ms = time_slots(p, reps, st);
    if (p->default_ms < 0.f) return VP_ELAUNCH;
    float best_ms = p->default_ms;
    for (size_t c = 0; c < p->classK.size(); ++c) {
        const int K = p->classK[c];
        int bvt = p->cls_vt[c], bpl = p->cls_pl[c];
        for (int vt : {1, 2, 4})
            for (int pl : {1, 2, 4, 8}) {
                const int chunk = (kBW / vt) * pl;
                if (chunk > 2 * K || 8 * chunk < K || (vt == bvt && pl == bpl)) continue;
                p->cls_vt[c] = vt;
                p->cls_pl[c] = pl;
                int rc = upload_shapes(p);
                if (rc != VP_OK) return rc;
                const float ms = time_slots(p, reps, st);
                if (ms < 0.f) return VP_ELAUNCH;
                if (ms < best_ms) {
                    best_ms = ms;
                    bvt = vt;
                    bpl = pl;
                }
            }
        p->cls_vt[c] = bvt;
        p->cls_pl[c] = bpl;
    }
    // queue order
    p->lpt ^= 1;
    int rc = upload_shapes(p);
    if (rc != VP_OK) return rc;
    const float ms = time_slots(p, reps, st);
    if (ms >= 0.f && ms < best_ms) best_ms = ms;
    else p->lpt ^= 1;
    rc = upload_shapes(p);
    if (rc != VP_OK) return rc;
    p->tuned_ms = best_ms;
    (void)hipGraphLaunch(p->exec, st);   // outputs of the chosen configuration
    return hipStreamSynchronize(st) == hipSuccess ? VP_OK : launch_status();
}

int vp_batch_get_info(const vp_batch *plan, vp_batch_info *info) {
    if (!plan || !info) return VP_EINVAL;
    vp_batch_info r = {};
    r.n_groups = plan->n_groups;
    r.n_sc = plan->n_sc;
    r.n_vec = plan->n_vec;
    r.n_tiles = plan->n_tiles;
    r.persistent_workgroups = plan->grid;
    r.n_classes = (int32_t)plan->classK.size();
    for (size_t c = 0; c < plan->classK.size(); ++c) {
        r.class_K[c] = plan->classK[c];
        r.class_vt[c] = plan->cls_vt[c];
        r.class_pl[c] = plan->cls_pl[c];
    }
    r.lpt_order = plan->lpt;
    r.default_ms = plan->default_ms;
    r.tuned_ms = plan->tuned_ms;
    *info = r;
    return VP_OK;
}

int vp_batch_buffers(const vp_batch *plan, const vp_c32 **W, const float **w2, const uint8_t **perm,
                     const vp_c32 **G, const int32_t **status, const uint8_t **paths) {
    if (!plan) return VP_EINVAL;
    if (W) *W = (const vp_c32 *)plan->W;
    if (w2) *w2 = plan->w2;
    if (perm) *perm = plan->perm;
    if (G) *G = (const vp_c32 *)plan->G;
    if (status) *status = plan->status;
    if (paths) *paths = plan->paths;
    return VP_OK;
}

int vp_batch_destroy(vp_batch *plan) {
    free_plan(plan);
    return VP_OK;
}

}  // extern "C"
