// Native driver of the warm-start CNN: parameters, activations, forward, backward and Adam, all as HIP kernel
// launches on one stream (k_cnn.hip). The network is a 4-level 3D encoder-decoder (U-Net) on an S^3 volume,
// channels 16/32/64/64, 3x3x3 convolutions with bias and ReLU, 2x average pooling, nearest upsampling with
// skip concatenation, and a 1x1x1 linear head: 2 input channels (contrast, source) -> 2 output channels
// (Re u, Im u).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "helm_internal.h"

namespace helm {
hipError_t cnn_conv_fwd(int bf16, const float *in, long long in_bs, int Ci, int S, int taps, const void *wt, int Kp,
                        int COP, const float *bias, int Co, float *out, long long out_bs, int relu, int B, hipStream_t s);
hipError_t cnn_bias_grad(const float *g, long long g_bs, int B, long long V, int Co, float *part, float *db,
                         hipStream_t s);
hipError_t cnn_pack_weights(int bf16, const float *W, int Co, int Ci, int taps, int transpose, int COP, int Kp,
                            void *wt, hipStream_t s);
hipError_t cnn_relu_bwd(float *g, long long g_bs, const float *y, long long y_bs, long long per, int B, hipStream_t s);
hipError_t cnn_pool_fwd(const float *in, long long in_bs, float *out, long long out_bs, int C, int S, int B, hipStream_t s);
hipError_t cnn_pool_bwd(const float *gout, long long gout_bs, float *gin, long long gin_bs, int C, int S, int B,
                        int accumulate, hipStream_t s);
hipError_t cnn_up_fwd(const float *in, long long in_bs, float *out, long long out_bs, int C, int S, int B, hipStream_t s);
hipError_t cnn_up_bwd(const float *gout, long long gout_bs, float *gin, long long gin_bs, int C, int S, int B, hipStream_t s);
hipError_t cnn_mse(const float *y, const float *t, long long n, float *g, double *part, double *loss, hipStream_t s);
hipError_t cnn_adam(float *w, const float *g, float *m, float *v, long long n, float lr, float b1, float b2, float eps,
                    float c1, float c2, hipStream_t s);
hipError_t cnn_prolong(const float *coarse, int nc, double scale, double gre, double gim, int cubic, double2 *fine,
                       int nf, double2 *work, hipStream_t s);
hipError_t cnn_conv_direct(int use_bf16, const float *in, long long in_bs, int Ci, int S, const void *wt, int COP,
                           const float *bias, int Co, float *out, long long out_bs, int relu, int B, float *part,
                           long long part_elems, hipStream_t s);
long long cnn_direct_size(int Co, int Ci);
hipError_t cnn_wgrad_1x1(const float *g, long long g_bs, int Co, const float *in, long long in_bs, int Ci, int V, int B,
                         float *part, long long part_elems, float *dW, hipStream_t s);
hipError_t cnn_wgrad_direct(int use_bf16, const float *g, long long g_bs, int Co, const float *in, long long in_bs,
                            int Ci, int S, int B, float *part, long long part_elems, float *dW, hipStream_t s);
hipError_t cnn_pack_direct(int use_bf16, const float *W, int Co, int Ci, int transpose, void *wt, hipStream_t s);
hipError_t cnn_features(const double *k2h, const double2 *fh, int halo, int nf, int S, double k0sq, double cs,
                        double fs, float *x, hipStream_t s);
}  // namespace helm

using namespace helm;

namespace {

constexpr int NL = 12;
// (ci, co, taps, relu, level) of the twelve convolutions
const int LAYERS[NL][5] = {
    {2, 16, 27, 1, 0},  {16, 16, 27, 1, 0},            // encoder level 0 (the second writes the skip s1)
    {16, 32, 27, 1, 1}, {32, 32, 27, 1, 1},            // level 1 (skip s2)
    {32, 64, 27, 1, 2}, {64, 64, 27, 1, 2},            // level 2 (skip s3)
    {64, 64, 27, 1, 3}, {64, 64, 27, 1, 3},            // bottleneck, level 3
    {128, 64, 27, 1, 2}, {96, 32, 27, 1, 1}, {48, 16, 27, 1, 0},   // decoder on [up | skip]
    {16, 2, 1, 0, 0}};                                 // linear 1x1x1 head

inline int pad16(int v) { return (v + 15) / 16 * 16; }
inline int pad64(int v) { return (v + 63) / 64 * 64; }

struct View {           // a channel slice of a buffer: channel c of sample b at p + b*bs + c*V
    float *p;
    long long bs;
};

}  // namespace

struct helm_cnn {
    int S0 = 0, maxB = 0, bf16 = 1;
    hipStream_t stream = nullptr;
    std::string err;
    std::vector<void *> allocs;
    long long nparams = 0;
    long long woff[NL], boff[NL];
    int COP[NL], Kp[NL], COPt[NL], Kpt[NL];
    void *wt[NL], *wtT[NL];
    float *params = nullptr, *grads = nullptr, *am = nullptr, *av = nullptr;
    int step = 0;
    // activations and their gradients (see the forward sequence)
    enum { X, C1A, CAT1, P1, C2A, CAT2, P2, C3A, CAT3, P3, C4A, C4B, D3, D2, D1, OUT, NBUF };
    float *act[NBUF] = {}, *grd[NBUF] = {};
    int bch[NBUF], blev[NBUF];
    float *part = nullptr;
    long long part_elems = 0;
    double *mse_part = nullptr, *loss_dev = nullptr;
    float *bias_part = nullptr;      // 64 slices per channel of the bias-gradient reduction
    double2 *pwork = nullptr;        // separable cubic prolongation intermediates (grown on demand)
    long long pwork_elems = 0;
};

namespace {

template <typename T> hipError_t nalloc(helm_cnn &n, T **p, size_t count) {
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(1, count) * sizeof(T));
    if (e == hipSuccess) { n.allocs.push_back(q); *p = (T *)q; }
    return e;
}

inline int S_of(const helm_cnn &n, int lev) { return n.S0 >> lev; }
inline long long V_of(const helm_cnn &n, int lev) { long long s = S_of(n, lev); return s * s * s; }

View view(helm_cnn &n, float *const *arr, int buf, int ch0) {
    long long V = V_of(n, n.blev[buf]);
    return View{arr[buf] + (long long)ch0 * V, (long long)n.bch[buf] * V};
}

#define NTRY(expr)                                                                                      \
    do {                                                                                                \
        hipError_t _e = (expr);                                                                         \
        if (_e != hipSuccess) {                                                                         \
            n.err = std::string(#expr) + ": " + hipGetErrorString(_e);                                  \
            return HELM_EDEVICE;                                                                        \
        }                                                                                               \
    } while (0)

// 27-tap layers: direct-convolution format (forward, and the data gradient with mirrored taps); the 1-tap head:
// implicit-GEMM format
helm_status pack_all(helm_cnn &n) {
    for (int l = 0; l < NL; ++l) {
        const int ci = LAYERS[l][0], co = LAYERS[l][1], taps = LAYERS[l][2];
        if (taps == 27) {
            NTRY(cnn_pack_direct(n.bf16, n.params + n.woff[l], co, ci, 0, n.wt[l], n.stream));
            NTRY(cnn_pack_direct(n.bf16, n.params + n.woff[l], ci, co, 1, n.wtT[l], n.stream));
        } else {
            NTRY(cnn_pack_weights(n.bf16, n.params + n.woff[l], co, ci, taps, 0, n.COP[l], n.Kp[l], n.wt[l], n.stream));
            NTRY(cnn_pack_weights(n.bf16, n.params + n.woff[l], co, ci, taps, 1, n.COPt[l], n.Kpt[l], n.wtT[l], n.stream));
        }
    }
    return HELM_OK;
}

helm_status conv_fwd(helm_cnn &n, int l, View in, View out, int B) {
    const int ci = LAYERS[l][0], co = LAYERS[l][1], taps = LAYERS[l][2], relu = LAYERS[l][3];
    if (taps == 27)
        NTRY(cnn_conv_direct(n.bf16, in.p, in.bs, ci, S_of(n, LAYERS[l][4]), n.wt[l], n.COP[l], n.params + n.boff[l],
                             co, out.p, out.bs, relu, B, n.part, n.part_elems, n.stream));
    else
        NTRY(cnn_conv_fwd(n.bf16, in.p, in.bs, ci, S_of(n, LAYERS[l][4]), taps, n.wt[l], n.Kp[l], n.COP[l],
                          n.params + n.boff[l], co, out.p, out.bs, relu, B, n.stream));
    return HELM_OK;
}

// gradients of layer l given dL/d(out) in g (already ReLU-masked); dL/d(in) into gin (may be null)
helm_status conv_bwd(helm_cnn &n, int l, View in, View g, View *gin, int B) {
    const int ci = LAYERS[l][0], co = LAYERS[l][1], taps = LAYERS[l][2], lev = LAYERS[l][4];
    const int S = S_of(n, lev);
    if (taps == 27) {
        NTRY(cnn_wgrad_direct(n.bf16, g.p, g.bs, co, in.p, in.bs, ci, S, B, n.part, n.part_elems, n.grads + n.woff[l],
                              n.stream));
    } else {
        NTRY(cnn_wgrad_1x1(g.p, g.bs, co, in.p, in.bs, ci, (int)V_of(n, lev), B, n.part, n.part_elems,
                           n.grads + n.woff[l], n.stream));
    }
    NTRY(cnn_bias_grad(g.p, g.bs, B, V_of(n, lev), co, n.bias_part, n.grads + n.boff[l], n.stream));
    if (gin && taps == 27)
        NTRY(cnn_conv_direct(n.bf16, g.p, g.bs, co, S, n.wtT[l], n.COPt[l], nullptr, ci, gin->p, gin->bs, 0, B,
                             n.part, n.part_elems, n.stream));
    else if (gin)
        NTRY(cnn_conv_fwd(n.bf16, g.p, g.bs, co, S, taps, n.wtT[l], n.Kpt[l], n.COPt[l], nullptr, ci, gin->p, gin->bs,
                          0, B, n.stream));
    return HELM_OK;
}

helm_status relu_mask(helm_cnn &n, View g, View y, int C, int lev, int B) {
    NTRY(cnn_relu_bwd(g.p, g.bs, y.p, y.bs, (long long)C * V_of(n, lev), B, n.stream));
    return HELM_OK;
}

helm_status forward(helm_cnn &n, const float *x, int B) {
    float **A = n.act;
    View vx{(float *)x, 2 * V_of(n, 0)};
    auto v = [&](int buf, int c0) { return view(n, A, buf, c0); };
    helm_status st;
#define F(expr) if ((st = (expr)) != HELM_OK) return st
    F(conv_fwd(n, 0, vx, v(helm_cnn::C1A, 0), B));
    F(conv_fwd(n, 1, v(helm_cnn::C1A, 0), v(helm_cnn::CAT1, 32), B));
    NTRY(cnn_pool_fwd(v(helm_cnn::CAT1, 32).p, v(helm_cnn::CAT1, 32).bs, A[helm_cnn::P1], v(helm_cnn::P1, 0).bs, 16, n.S0, B, n.stream));
    F(conv_fwd(n, 2, v(helm_cnn::P1, 0), v(helm_cnn::C2A, 0), B));
    F(conv_fwd(n, 3, v(helm_cnn::C2A, 0), v(helm_cnn::CAT2, 64), B));
    NTRY(cnn_pool_fwd(v(helm_cnn::CAT2, 64).p, v(helm_cnn::CAT2, 64).bs, A[helm_cnn::P2], v(helm_cnn::P2, 0).bs, 32, S_of(n, 1), B, n.stream));
    F(conv_fwd(n, 4, v(helm_cnn::P2, 0), v(helm_cnn::C3A, 0), B));
    F(conv_fwd(n, 5, v(helm_cnn::C3A, 0), v(helm_cnn::CAT3, 64), B));
    NTRY(cnn_pool_fwd(v(helm_cnn::CAT3, 64).p, v(helm_cnn::CAT3, 64).bs, A[helm_cnn::P3], v(helm_cnn::P3, 0).bs, 64, S_of(n, 2), B, n.stream));
    F(conv_fwd(n, 6, v(helm_cnn::P3, 0), v(helm_cnn::C4A, 0), B));
    F(conv_fwd(n, 7, v(helm_cnn::C4A, 0), v(helm_cnn::C4B, 0), B));
    NTRY(cnn_up_fwd(A[helm_cnn::C4B], v(helm_cnn::C4B, 0).bs, v(helm_cnn::CAT3, 0).p, v(helm_cnn::CAT3, 0).bs, 64, S_of(n, 3), B, n.stream));
    F(conv_fwd(n, 8, v(helm_cnn::CAT3, 0), v(helm_cnn::D3, 0), B));
    NTRY(cnn_up_fwd(A[helm_cnn::D3], v(helm_cnn::D3, 0).bs, v(helm_cnn::CAT2, 0).p, v(helm_cnn::CAT2, 0).bs, 64, S_of(n, 2), B, n.stream));
    F(conv_fwd(n, 9, v(helm_cnn::CAT2, 0), v(helm_cnn::D2, 0), B));
    NTRY(cnn_up_fwd(A[helm_cnn::D2], v(helm_cnn::D2, 0).bs, v(helm_cnn::CAT1, 0).p, v(helm_cnn::CAT1, 0).bs, 32, S_of(n, 1), B, n.stream));
    F(conv_fwd(n, 10, v(helm_cnn::CAT1, 0), v(helm_cnn::D1, 0), B));
    F(conv_fwd(n, 11, v(helm_cnn::D1, 0), v(helm_cnn::OUT, 0), B));
    return HELM_OK;
}

helm_status backward(helm_cnn &n, const float *x, int B) {
    // grd[OUT] holds dL/d(out)
    float **A = n.act, **G = n.grd;
    auto va = [&](int buf, int c0) { return view(n, A, buf, c0); };
    auto vg = [&](int buf, int c0) { return view(n, G, buf, c0); };
    View vx{(float *)x, 2 * V_of(n, 0)};
    helm_status st;
    View g;
    g = vg(helm_cnn::D1, 0);
    F(conv_bwd(n, 11, va(helm_cnn::D1, 0), vg(helm_cnn::OUT, 0), &g, B));
    F(relu_mask(n, vg(helm_cnn::D1, 0), va(helm_cnn::D1, 0), 16, 0, B));
    g = vg(helm_cnn::CAT1, 0);
    F(conv_bwd(n, 10, va(helm_cnn::CAT1, 0), vg(helm_cnn::D1, 0), &g, B));
    NTRY(cnn_up_bwd(vg(helm_cnn::CAT1, 0).p, vg(helm_cnn::CAT1, 0).bs, G[helm_cnn::D2], vg(helm_cnn::D2, 0).bs, 32, S_of(n, 1), B, n.stream));
    F(relu_mask(n, vg(helm_cnn::D2, 0), va(helm_cnn::D2, 0), 32, 1, B));
    g = vg(helm_cnn::CAT2, 0);
    F(conv_bwd(n, 9, va(helm_cnn::CAT2, 0), vg(helm_cnn::D2, 0), &g, B));
    NTRY(cnn_up_bwd(vg(helm_cnn::CAT2, 0).p, vg(helm_cnn::CAT2, 0).bs, G[helm_cnn::D3], vg(helm_cnn::D3, 0).bs, 64, S_of(n, 2), B, n.stream));
    F(relu_mask(n, vg(helm_cnn::D3, 0), va(helm_cnn::D3, 0), 64, 2, B));
    g = vg(helm_cnn::CAT3, 0);
    F(conv_bwd(n, 8, va(helm_cnn::CAT3, 0), vg(helm_cnn::D3, 0), &g, B));
    NTRY(cnn_up_bwd(vg(helm_cnn::CAT3, 0).p, vg(helm_cnn::CAT3, 0).bs, G[helm_cnn::C4B], vg(helm_cnn::C4B, 0).bs, 64, S_of(n, 3), B, n.stream));
    F(relu_mask(n, vg(helm_cnn::C4B, 0), va(helm_cnn::C4B, 0), 64, 3, B));
    g = vg(helm_cnn::C4A, 0);
    F(conv_bwd(n, 7, va(helm_cnn::C4A, 0), vg(helm_cnn::C4B, 0), &g, B));
    F(relu_mask(n, vg(helm_cnn::C4A, 0), va(helm_cnn::C4A, 0), 64, 3, B));
    g = vg(helm_cnn::P3, 0);
    F(conv_bwd(n, 6, va(helm_cnn::P3, 0), vg(helm_cnn::C4A, 0), &g, B));
    // skip s3 = CAT3[64:128): its gradient already holds the concat part; add the pooling path
    NTRY(cnn_pool_bwd(G[helm_cnn::P3], vg(helm_cnn::P3, 0).bs, vg(helm_cnn::CAT3, 64).p, vg(helm_cnn::CAT3, 64).bs, 64, S_of(n, 2), B, 1, n.stream));
    F(relu_mask(n, vg(helm_cnn::CAT3, 64), va(helm_cnn::CAT3, 64), 64, 2, B));
    g = vg(helm_cnn::C3A, 0);
    F(conv_bwd(n, 5, va(helm_cnn::C3A, 0), vg(helm_cnn::CAT3, 64), &g, B));
    F(relu_mask(n, vg(helm_cnn::C3A, 0), va(helm_cnn::C3A, 0), 64, 2, B));
    g = vg(helm_cnn::P2, 0);
    F(conv_bwd(n, 4, va(helm_cnn::P2, 0), vg(helm_cnn::C3A, 0), &g, B));
    NTRY(cnn_pool_bwd(G[helm_cnn::P2], vg(helm_cnn::P2, 0).bs, vg(helm_cnn::CAT2, 64).p, vg(helm_cnn::CAT2, 64).bs, 32, S_of(n, 1), B, 1, n.stream));
    F(relu_mask(n, vg(helm_cnn::CAT2, 64), va(helm_cnn::CAT2, 64), 32, 1, B));
    g = vg(helm_cnn::C2A, 0);
    F(conv_bwd(n, 3, va(helm_cnn::C2A, 0), vg(helm_cnn::CAT2, 64), &g, B));
    F(relu_mask(n, vg(helm_cnn::C2A, 0), va(helm_cnn::C2A, 0), 32, 1, B));
    g = vg(helm_cnn::P1, 0);
    F(conv_bwd(n, 2, va(helm_cnn::P1, 0), vg(helm_cnn::C2A, 0), &g, B));
    NTRY(cnn_pool_bwd(G[helm_cnn::P1], vg(helm_cnn::P1, 0).bs, vg(helm_cnn::CAT1, 32).p, vg(helm_cnn::CAT1, 32).bs, 16, n.S0, B, 1, n.stream));
    F(relu_mask(n, vg(helm_cnn::CAT1, 32), va(helm_cnn::CAT1, 32), 16, 0, B));
    g = vg(helm_cnn::C1A, 0);
    F(conv_bwd(n, 1, va(helm_cnn::C1A, 0), vg(helm_cnn::CAT1, 32), &g, B));
    F(relu_mask(n, vg(helm_cnn::C1A, 0), va(helm_cnn::C1A, 0), 16, 0, B));
    F(conv_bwd(n, 0, vx, vg(helm_cnn::C1A, 0), nullptr, B));
    return HELM_OK;
#undef F
}

void cnn_free(helm_cnn *n) {
    if (!n) return;
    if (n->stream) hipStreamSynchronize(n->stream);
    else hipDeviceSynchronize();
    for (void *p : n->allocs) hipFree(p);
    delete n;
}

thread_local std::string g_cnn_err;

}  // namespace

extern "C" {

helm_status helm_cnn_create(helm_cnn **out, int size, int max_batch, int bf16, unsigned long long seed, void *stream) {
    g_cnn_err.clear();
    if (!out || size < 8 || size % 8 != 0 || max_batch < 1) {
        g_cnn_err = "size must be a positive multiple of 8 and max_batch >= 1";
        return HELM_EINVAL;
    }
    *out = nullptr;
    helm_cnn *n = new helm_cnn();
    n->S0 = size;
    n->maxB = max_batch;
    n->bf16 = bf16 ? 1 : 0;
    n->stream = (hipStream_t)stream;
    auto fail = [&](helm_status s, const std::string &m) { g_cnn_err = m; cnn_free(n); return s; };
    long long off = 0;
    for (int l = 0; l < NL; ++l) {
        const int ci = LAYERS[l][0], co = LAYERS[l][1], taps = LAYERS[l][2];
        n->woff[l] = off; off += (long long)co * ci * taps;
        n->boff[l] = off; off += co;
        n->COP[l] = pad16(co);  n->Kp[l] = pad64(ci * taps);
        n->COPt[l] = pad16(ci); n->Kpt[l] = pad64(co * taps);
    }
    n->nparams = off;
    const size_t esz = n->bf16 ? 2 : 4;
    for (int l = 0; l < NL; ++l) {
        const int ci = LAYERS[l][0], co = LAYERS[l][1], taps = LAYERS[l][2];
        const size_t nf = taps == 27 ? (size_t)cnn_direct_size(co, ci) : (size_t)n->COP[l] * n->Kp[l];
        const size_t nt = taps == 27 ? (size_t)cnn_direct_size(ci, co) : (size_t)n->COPt[l] * n->Kpt[l];
        if (hipMalloc(&n->wt[l], esz * nf) != hipSuccess) return fail(HELM_ENOMEM, "weights");
        n->allocs.push_back(n->wt[l]);
        if (hipMalloc(&n->wtT[l], esz * nt) != hipSuccess) return fail(HELM_ENOMEM, "weights");
        n->allocs.push_back(n->wtT[l]);
    }
    if (nalloc(*n, &n->params, off) || nalloc(*n, &n->grads, off) || nalloc(*n, &n->am, off) || nalloc(*n, &n->av, off))
        return fail(HELM_ENOMEM, "parameters");
    const int ch[helm_cnn::NBUF] = {2, 16, 48, 16, 32, 96, 32, 64, 128, 64, 64, 64, 64, 32, 16, 2};
    const int lv[helm_cnn::NBUF] = {0, 0, 0, 1, 1, 1, 2, 2, 2, 3, 3, 3, 2, 1, 0, 0};
    for (int b = 0; b < helm_cnn::NBUF; ++b) {
        n->bch[b] = ch[b];
        n->blev[b] = lv[b];
        if (b == helm_cnn::X) continue;     // the input is the caller's
        size_t cnt = (size_t)ch[b] * V_of(*n, lv[b]) * max_batch;
        if (nalloc(*n, &n->act[b], cnt) || nalloc(*n, &n->grd[b], cnt)) return fail(HELM_ENOMEM, "activations");
    }
    // wgrad partials: up to 128 chunks of pad16(co) x pad64(ci taps)
    long long pe = 0;
    for (int l = 0; l < NL; ++l) pe = std::max(pe, 129LL * pad16(LAYERS[l][1]) * pad64(LAYERS[l][0] * LAYERS[l][2]));
    n->part_elems = pe;
    if (nalloc(*n, &n->part, pe) || nalloc(*n, &n->bias_part, 64 * 64)) return fail(HELM_ENOMEM, "partials");
    long long mp = ((long long)2 * V_of(*n, 0) * max_batch + 255) / 256;
    if (nalloc(*n, &n->mse_part, mp) || nalloc(*n, &n->loss_dev, 1)) return fail(HELM_ENOMEM, "loss");
    // He-uniform initial weights (fan-in), zero biases, from a 64-bit LCG seeded by `seed`
    std::vector<float> h(off, 0.0f);
    unsigned long long st = seed * 6364136223846793005ULL + 1442695040888963407ULL;
    auto uni = [&]() {
        st = st * 6364136223846793005ULL + 1442695040888963407ULL;
        return (double)(st >> 11) * (1.0 / 9007199254740992.0);
    };
    for (int l = 0; l < NL; ++l) {
        const int ci = LAYERS[l][0], co = LAYERS[l][1], taps = LAYERS[l][2];
        double a = std::sqrt(6.0 / (ci * taps));
        if (l == NL - 1) a *= 0.1;
        for (long long i = 0; i < (long long)co * ci * taps; ++i) h[n->woff[l] + i] = (float)((2.0 * uni() - 1.0) * a);
    }
    if (hipMemcpy(n->params, h.data(), off * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(n->am, 0, off * sizeof(float)) != hipSuccess || hipMemset(n->av, 0, off * sizeof(float)) != hipSuccess)
        return fail(HELM_EDEVICE, "parameter upload");
    if (pack_all(*n) != HELM_OK) return fail(HELM_EDEVICE, n->err);
    *out = n;
    return HELM_OK;
}

long long helm_cnn_num_params(const helm_cnn *n) { return n ? n->nparams : 0; }

const char *helm_cnn_last_error(const helm_cnn *n) { return n ? n->err.c_str() : g_cnn_err.c_str(); }

helm_status helm_cnn_get_params(helm_cnn *n_, float *host) {
    if (!n_ || !host) return HELM_EINVAL;
    helm_cnn &n = *n_;
    NTRY(hipMemcpyAsync(host, n.params, n.nparams * sizeof(float), hipMemcpyDeviceToHost, n.stream));
    NTRY(hipStreamSynchronize(n.stream));
    return HELM_OK;
}

helm_status helm_cnn_set_params(helm_cnn *n_, const float *host) {
    if (!n_ || !host) return HELM_EINVAL;
    helm_cnn &n = *n_;
    NTRY(hipMemcpyAsync(n.params, host, n.nparams * sizeof(float), hipMemcpyHostToDevice, n.stream));
    NTRY(hipStreamSynchronize(n.stream));
    return pack_all(n);
}

helm_status helm_cnn_get_grads(helm_cnn *n_, float *host) {
    if (!n_ || !host) return HELM_EINVAL;
    helm_cnn &n = *n_;
    NTRY(hipMemcpyAsync(host, n.grads, n.nparams * sizeof(float), hipMemcpyDeviceToHost, n.stream));
    NTRY(hipStreamSynchronize(n.stream));
    return HELM_OK;
}

helm_status helm_cnn_forward(helm_cnn *n_, const float *x, float *y, int B) {
    if (!n_ || !x || B < 1 || B > n_->maxB) return HELM_EINVAL;
    helm_cnn &n = *n_;
    helm_status st = forward(n, x, B);
    if (st != HELM_OK) return st;
    if (y) NTRY(hipMemcpyAsync(y, n.act[helm_cnn::OUT], (size_t)2 * V_of(n, 0) * B * sizeof(float),
                               hipMemcpyDeviceToDevice, n.stream));
    return HELM_OK;
}

helm_status helm_cnn_loss_grad(helm_cnn *n_, const float *x, const float *t, int B, double *loss) {
    if (!n_ || !x || !t || B < 1 || B > n_->maxB) return HELM_EINVAL;
    helm_cnn &n = *n_;
    helm_status st = forward(n, x, B);
    if (st != HELM_OK) return st;
    const long long N = 2 * V_of(n, 0) * B;
    NTRY(cnn_mse(n.act[helm_cnn::OUT], t, N, n.grd[helm_cnn::OUT], n.mse_part, n.loss_dev, n.stream));
    st = backward(n, x, B);
    if (st != HELM_OK) return st;
    if (loss) {
        NTRY(hipMemcpyAsync(loss, n.loss_dev, sizeof(double), hipMemcpyDeviceToHost, n.stream));
        NTRY(hipStreamSynchronize(n.stream));
    }
    return HELM_OK;
}

helm_status helm_cnn_adam_step(helm_cnn *n_, double lr) {
    if (!n_ || !(lr > 0.0)) return HELM_EINVAL;
    helm_cnn &n = *n_;
    n.step += 1;
    const double b1 = 0.9, b2 = 0.999;
    NTRY(cnn_adam(n.params, n.grads, n.am, n.av, n.nparams, (float)lr, (float)b1, (float)b2, 1e-8f,
                  (float)(1.0 - std::pow(b1, n.step)), (float)(1.0 - std::pow(b2, n.step)), n.stream));
    return pack_all(n);
}

helm_status helm_cnn_train_step(helm_cnn *n, const float *x, const float *t, int B, double lr, double *loss) {
    helm_status st = helm_cnn_loss_grad(n, x, t, B, loss);
    if (st != HELM_OK) return st;
    return helm_cnn_adam_step(n, lr);
}

helm_status helm_cnn_prolong(helm_cnn *n_, const float *coarse, int nc, double scale, double gamma_re,
                             double gamma_im, int cubic, void *fine, int nf) {
    if (!n_ || !coarse || !fine || nc < 1 || nf < 1) return HELM_EINVAL;
    helm_cnn &n = *n_;
    double2 *work = nullptr;
    if (cubic) {
        const long long need = (long long)nf * nc * nc + (long long)nf * nf * nc;
        if (need > n.pwork_elems) {
            if (n.pwork) {
                NTRY(hipStreamSynchronize(n.stream));
                NTRY(hipFree(n.pwork));
                n.allocs.erase(std::find(n.allocs.begin(), n.allocs.end(), (void *)n.pwork));
                n.pwork = nullptr;
                n.pwork_elems = 0;
            }
            void *q = nullptr;
            NTRY(hipMalloc(&q, need * sizeof(double2)));
            n.allocs.push_back(q);
            n.pwork = (double2 *)q;
            n.pwork_elems = need;
        }
        work = n.pwork;
    }
    NTRY(cnn_prolong(coarse, nc, scale, gamma_re, gamma_im, cubic, (double2 *)fine, nf, work, n.stream));
    return HELM_OK;
}

helm_status helm_cnn_features(helm_cnn *n_, const double *k2_halo, const void *f_halo, int halo, int nf, double k0,
                              double c_scale, double f_scale, float *x) {
    if (!n_ || !k2_halo || !f_halo || !x || !(k0 > 0.0)) return HELM_EINVAL;
    helm_cnn &n = *n_;
    if (halo < 1 || nf < n.S0) {
        n.err = "features: need halo >= 1 and a solver grid at least as fine as the network grid";
        return HELM_EINVAL;
    }
    NTRY(cnn_features(k2_halo, (const double2 *)f_halo, halo, nf, n.S0, k0 * k0, c_scale, f_scale, x, n.stream));
    return HELM_OK;
}

void helm_cnn_destroy(helm_cnn *n) { cnn_free(n); }

}  // extern "C"
