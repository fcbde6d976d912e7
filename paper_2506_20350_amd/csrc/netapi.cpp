// Learned correction of the block-circulant preconditioner: network state,
// inference inside flexible GMRES, and the C ABI of forward, gradients and
// training.  Kernels are in net.hip.
#include <algorithm>
#include <cmath>
#include <utility>
#include <vector>

#include "lib.h"
#include "net.h"

using namespace mlfft;

#define HIPCHK(call, what)                                   \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return c->hip_fail(e_, what);  \
    } while (0)

static int pad32(int c) { return (c + 31) / 32 * 32; }

struct Net {
    int b = 0, hidden = 0;
    int cin[4], cout[4], cinp[4], coutp[4];
    size_t woff[4];            // offsets of the layers in the flat FP32 master array
    size_t nweights = 0;
    Buf wmaster, m, v, dw;     // FP32, flat [layer][co][ci][3][3]
    Buf wbf[4];                // bf16 [coutp][9][cinp]
    Buf dwp[4];                // FP32 padded gradients
    int adam_t = 0;
    // workspaces (grown on demand)
    Buf act[4], out, yhat, scale, phase, tgt, g0, g1, loss, fb, wpart;
    int fb_w = 0;
};

bool Ctx::net_ready() const { return net != nullptr; }

void Ctx::net_release() {
    delete net;
    net = nullptr;
}

static mlfft_status ensure_ws(Ctx* c, Net& n, int W, int npix, bool train) {
    const size_t P = (size_t)W * npix;
    const size_t N = P * n.b;
    for (int l = 0; l < 4; ++l) HIPCHK(n.act[l].ensure(P * n.cinp[l] * 2), "network activations");
    HIPCHK(n.out.ensure(P * n.coutp[3] * 4), "network output");
    HIPCHK(n.yhat.ensure(N * 8), "network input");
    HIPCHK(n.scale.ensure((size_t)W * 8), "network scales");
    HIPCHK(n.phase.ensure((size_t)W * 16), "network phases");
    if (train) {
        int cmax = 0;
        for (int l = 0; l < 4; ++l) cmax = std::max(cmax, std::max(n.cinp[l], n.coutp[l]));
        HIPCHK(n.tgt.ensure(P * n.coutp[3] * 4), "training targets");
        HIPCHK(n.g0.ensure(P * cmax * 4), "gradients");
        HIPCHK(n.g1.ensure(P * cmax * 4), "gradients");
        HIPCHK(n.loss.ensure((size_t)W * 8), "loss");
        size_t pmax = 0;
        for (int l = 0; l < 4; ++l)
            pmax = std::max(pmax, (size_t)n_wgrad_chunks((long)P, n.cinp[l], n.coutp[l]) * n.coutp[l] * 9 * n.cinp[l]);
        HIPCHK(n.wpart.ensure(pmax * 4), "gradient partial sums");
    }
    return MLFFT_OK;
}

// forward through the four convolutions; input already in act[0]
static mlfft_status forward_convs(Ctx* c, Net& n, int W, int H, int Wd) {
    for (int l = 0; l < 4; ++l) {
        void* dst = l < 3 ? n.act[l + 1].p : n.out.p;
        const int pr = c->prof_begin(PK_NET_FWD, MLFFT_FP32_BF16GEMM, 0,
                                     2.0 * W * H * Wd * 9.0 * n.cin[l] * n.cout[l]);
        HIPCHK(n_conv_fwd((const unsigned short*)n.act[l].p, (const unsigned short*)n.wbf[l].p, dst, W, H, Wd,
                          n.cinp[l], n.coutp[l], l < 3 ? 1 : 0, c->stream), "convolution");
        c->prof_end(pr);
    }
    return MLFFT_OK;
}

// y, e: complex64 vectors (W columns, H x Wd cells of b); computes loss per sample and padded gradients
static mlfft_status forward_backward(Ctx* c, Net& n, int W, int H, int Wd, const void* y, const void* e) {
    hipStream_t s = c->stream;
    const int npix = H * Wd;
    const size_t N = (size_t)npix * n.b;
    mlfft_status st = ensure_ws(c, n, W, npix, true);
    if (st < 0) return st;
    HIPCHK(n_normalise((const float2*)y, N, W, npix, n.b, n.cinp[0], (float2*)n.yhat.p, (unsigned short*)n.act[0].p,
                       (double*)n.scale.p, (double2*)n.phase.p, s), "normalise");
    st = forward_convs(c, n, W, H, Wd);
    if (st < 0) return st;
    HIPCHK(n_target((const float2*)e, N, W, npix, n.b, n.coutp[3], (double*)n.scale.p, (double2*)n.phase.p,
                    (float*)n.tgt.p, s), "targets");
    HIPCHK(n_loss_grad((const float2*)n.yhat.p, (const float*)n.out.p, (const float*)n.tgt.p, N, W, n.b, n.coutp[3],
                       (float*)n.g0.p, (double*)n.loss.p, s), "loss");
    float* g = (float*)n.g0.p;
    float* gnext = (float*)n.g1.p;
    for (int l = 3; l >= 0; --l) {
        const int pr = c->prof_begin(PK_NET_BWD, MLFFT_FP32, 0, 4.0 * W * npix * 9.0 * n.cin[l] * n.cout[l]);
        HIPCHK(n_wgrad(g, (const unsigned short*)n.act[l].p, (float*)n.dwp[l].p, (float*)n.wpart.p, W, H, Wd, n.cinp[l],
                       n.coutp[l], s), "weight gradient");
        if (l > 0) {
            HIPCHK(n_dgrad(g, (const unsigned short*)n.wbf[l].p, (const unsigned short*)n.act[l].p, gnext, W, H, Wd,
                           n.cinp[l], n.coutp[l], s), "input gradient");
            std::swap(g, gnext);
        }
        c->prof_end(pr);
    }
    return MLFFT_OK;
}

mlfft_status Ctx::net_correct(const Array* a, int W, const void* y, void* z, int prec, int* fallbacks) {
    Ctx* c = this;
    (void)fallbacks;
    if (!net) return fail(MLFFT_E_STATE, "no network");
    if (prec == MLFFT_FP64) return fail(MLFFT_E_ARG, "the learned correction runs on complex64 data");
    Net& n = *net;
    if (a->b != n.b) return fail(MLFFT_E_ARG, "network built for b = %d, array has b = %d", n.b, a->b);
    const int H = a->Ny, Wd = a->Nx, npix = H * Wd;
    const size_t N = (size_t)npix * n.b;
    mlfft_status st = ensure_ws(c, n, W, npix, false);
    if (st < 0) return st;
    if (n.fb_w < W) {
        HIPCHK(n.fb.ensure((size_t)W * sizeof(int)), "fallback flags");
        HIPCHK(hipMemsetAsync(n.fb.p, 0, (size_t)W * sizeof(int), stream), "fallback flags");
        n.fb_w = W;
    }
    HIPCHK(n_normalise((const float2*)y, N, W, npix, n.b, n.cinp[0], (float2*)n.yhat.p, (unsigned short*)n.act[0].p,
                       (double*)n.scale.p, (double2*)n.phase.p, stream), "normalise");
    st = forward_convs(c, n, W, H, Wd);
    if (st < 0) return st;
    HIPCHK(n_finish((const float2*)y, (const float2*)n.yhat.p, (const float*)n.out.p, N, W, n.b, n.coutp[3],
                    (double*)n.scale.p, (double2*)n.phase.p, (float2*)z, (int*)n.fb.p, stream), "finish");
    return MLFFT_OK;
}

int Ctx::net_fallbacks_take() {
    if (!net || !net->fb.p || net->fb_w == 0) return 0;
    std::vector<int> h(net->fb_w);
    if (hipMemcpyAsync(h.data(), net->fb.p, h.size() * sizeof(int), hipMemcpyDeviceToHost, stream) != hipSuccess) return 0;
    if (hipStreamSynchronize(stream) != hipSuccess) return 0;
    (void)hipMemsetAsync(net->fb.p, 0, h.size() * sizeof(int), stream);
    int s = 0;
    for (int v : h) s += v;
    return s;
}

static mlfft_status pack_all(Ctx* c, Net& n) {
    for (int l = 0; l < 4; ++l)
        HIPCHK(n_pack_weights((const float*)n.wmaster.p + n.woff[l], (unsigned short*)n.wbf[l].p, n.cin[l], n.cout[l],
                              n.cinp[l], n.coutp[l], c->stream), "pack weights");
    return MLFFT_OK;
}

extern "C" {

// splitmix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators", 2014) of a counter: the i-th 64-bit value of stream `seed`
static uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// standard normal number i of stream seed (Box-Muller on two counter-based uniforms in (0, 1))
static double normal_draw(uint64_t seed, uint64_t i) {
    const uint64_t base = splitmix64(seed) ^ (i * 2);
    const double u1 = ((splitmix64(base) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    const double u2 = ((splitmix64(base ^ 1) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
}

mlfft_status mlfft_net_create(mlfft_ctx ctx, int b, int hidden, unsigned seed) {
    if (!ctx) return MLFFT_E_ARG;
    Ctx* c = ctx;
    if (b < 1 || b > 256) return c->fail(MLFFT_E_ARG, "b must be in [1, 256]");
    if (hidden < 1 || hidden > 512) return c->fail(MLFFT_E_ARG, "hidden must be in [1, 512]");
    HIPCHK(hipSetDevice(c->device), "set device");
    HIPCHK(hipStreamSynchronize(c->stream), "net create");
    c->net_release();
    Net* n = new Net();
    for (Buf* x : {&n->wmaster, &n->m, &n->v, &n->dw, &n->out, &n->yhat, &n->scale, &n->phase, &n->tgt, &n->g0, &n->g1,
                   &n->loss, &n->fb, &n->wpart})
        x->bind(&c->alloc);
    for (int l = 0; l < 4; ++l) {
        n->wbf[l].bind(&c->alloc);
        n->dwp[l].bind(&c->alloc);
        n->act[l].bind(&c->alloc);
    }
    n->b = b;
    n->hidden = hidden;
    const int ch[5] = {2 * b, hidden, hidden, hidden, 2 * b};
    size_t off = 0;
    for (int l = 0; l < 4; ++l) {
        n->cin[l] = ch[l];
        n->cout[l] = ch[l + 1];
        n->cinp[l] = pad32(ch[l]);
        n->coutp[l] = pad32(ch[l + 1]);
        n->woff[l] = off;
        off += (size_t)ch[l] * ch[l + 1] * 9;
    }
    n->nweights = off;
    c->net = n;
    HIPCHK(n->wmaster.ensure(off * 4), "weights");
    HIPCHK(n->m.ensure(off * 4), "weights");
    HIPCHK(n->v.ensure(off * 4), "weights");
    HIPCHK(n->dw.ensure(off * 4), "weights");
    // He-normal weights (standard deviation sqrt(2 / (9 c_in))) for the first three
    // layers from the seed, zeros for the last one; seed 0: all zeros
    std::vector<float> w0(off, 0.f);
    if (seed != 0)
        for (int l = 0; l < 3; ++l) {
            const double sd = std::sqrt(2.0 / (9.0 * n->cin[l]));
            const size_t cnt = (size_t)n->cin[l] * n->cout[l] * 9;
            for (size_t i = 0; i < cnt; ++i) w0[n->woff[l] + i] = (float)(sd * normal_draw(seed, n->woff[l] + i));
        }
    HIPCHK(hipMemcpyAsync(n->wmaster.p, w0.data(), off * 4, hipMemcpyHostToDevice, c->stream), "weights");
    HIPCHK(hipMemsetAsync(n->m.p, 0, off * 4, c->stream), "weights");
    HIPCHK(hipMemsetAsync(n->v.p, 0, off * 4, c->stream), "weights");
    for (int l = 0; l < 4; ++l) {
        HIPCHK(n->wbf[l].ensure((size_t)n->coutp[l] * 9 * n->cinp[l] * 2), "weights");
        HIPCHK(n->dwp[l].ensure((size_t)n->coutp[l] * 9 * n->cinp[l] * 4), "weights");
    }
    mlfft_status st = pack_all(c, *n);
    if (st < 0) return st;
    HIPCHK(hipStreamSynchronize(c->stream), "net create");
    return MLFFT_OK;
}

size_t mlfft_net_num_weights(mlfft_ctx ctx) {
    return (ctx && ctx->net) ? ctx->net->nweights : 0;
}

mlfft_status mlfft_net_set_weights(mlfft_ctx ctx, const float* host, size_t n) {
    if (!ctx) return MLFFT_E_ARG;
    Ctx* c = ctx;
    if (!c->net) return c->fail(MLFFT_E_STATE, "no network");
    if (!host || n != c->net->nweights) return c->fail(MLFFT_E_ARG, "expected %zu weights", c->net->nweights);
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(host[i])) return c->fail(MLFFT_E_ARG, "non-finite weight at %zu", i);
    Net& nt = *c->net;
    HIPCHK(hipMemcpyAsync(nt.wmaster.p, host, n * 4, hipMemcpyHostToDevice, c->stream), "weights");
    HIPCHK(hipMemsetAsync(nt.m.p, 0, n * 4, c->stream), "weights");
    HIPCHK(hipMemsetAsync(nt.v.p, 0, n * 4, c->stream), "weights");
    nt.adam_t = 0;
    mlfft_status st = pack_all(c, nt);
    if (st < 0) return st;
    HIPCHK(hipStreamSynchronize(c->stream), "weights");
    return MLFFT_OK;
}

mlfft_status mlfft_net_get_weights(mlfft_ctx ctx, float* host, size_t n) {
    if (!ctx) return MLFFT_E_ARG;
    Ctx* c = ctx;
    if (!c->net) return c->fail(MLFFT_E_STATE, "no network");
    if (!host || n != c->net->nweights) return c->fail(MLFFT_E_ARG, "expected %zu weights", c->net->nweights);
    HIPCHK(hipMemcpyAsync(host, c->net->wmaster.p, n * 4, hipMemcpyDeviceToHost, c->stream), "weights");
    HIPCHK(hipStreamSynchronize(c->stream), "weights");
    return MLFFT_OK;
}

mlfft_status mlfft_net_forward(mlfft_ctx ctx, int W, int H, int Wd, const void* x, void* out) {
    if (!ctx) return MLFFT_E_ARG;
    Ctx* c = ctx;
    if (!c->net) return c->fail(MLFFT_E_STATE, "no network");
    if (W < 1 || H < 1 || Wd < 1 || !x || !out) return c->fail(MLFFT_E_ARG, "bad forward arguments");
    Net& n = *c->net;
    mlfft_status st = ensure_ws(c, n, W, H * Wd, false);
    if (st < 0) return st;
    const long P = (long)W * H * Wd;
    HIPCHK(n_pack_nhwc((const float*)x, (unsigned short*)n.act[0].p, P, n.cin[0], n.cinp[0], c->stream), "pack input");
    st = forward_convs(c, n, W, H, Wd);
    if (st < 0) return st;
    HIPCHK(n_unpack_nhwc((const float*)n.out.p, (float*)out, P, n.cout[3], n.coutp[3], c->stream), "unpack output");
    return MLFFT_OK;
}

mlfft_status mlfft_net_apply(mlfft_ctx ctx, int array_id, int W, const void* y, void* z) {
    if (!ctx) return MLFFT_E_ARG;
    Ctx* c = ctx;
    Array* a = c->find(array_id);
    if (!a) return c->fail(MLFFT_E_STATE, "unknown array id %d", array_id);
    if (W < 1 || !y || !z) return c->fail(MLFFT_E_ARG, "bad apply arguments");
    if (a->Nc > 0) return c->fail(MLFFT_E_ARG, "the learned correction is not defined for arrays with border unknowns");
    return c->net_correct(a, W, y, z, MLFFT_FP32, nullptr);
}

static mlfft_status grads_common(Ctx* c, int W, int H, int Wd, const void* y, const void* e, double* mean_loss) {
    if (!c->net) return c->fail(MLFFT_E_STATE, "no network");
    if (W < 1 || H < 1 || Wd < 1 || !y || !e) return c->fail(MLFFT_E_ARG, "bad training arguments");
    Net& n = *c->net;
    mlfft_status st = forward_backward(c, n, W, H, Wd, y, e);
    if (st < 0) return st;
    std::vector<double> l(W);
    HIPCHK(hipMemcpyAsync(l.data(), n.loss.p, W * 8, hipMemcpyDeviceToHost, c->stream), "loss");
    HIPCHK(hipStreamSynchronize(c->stream), "loss");
    double s = 0.0;
    for (double v : l) s += v;
    *mean_loss = s / W;
    return MLFFT_OK;
}

mlfft_status mlfft_net_grads(mlfft_ctx ctx, int W, int H, int Wd, const void* y, const void* e, float* host_grads,
                             float* loss) {
    if (!ctx) return MLFFT_E_ARG;
    Ctx* c = ctx;
    double ml = 0.0;
    mlfft_status st = grads_common(c, W, H, Wd, y, e, &ml);
    if (st < 0) return st;
    Net& n = *c->net;
    for (int l = 0; l < 4; ++l)
        HIPCHK(n_unpack_grad((const float*)n.dwp[l].p, (float*)n.dw.p + n.woff[l], n.cin[l], n.cout[l], n.cinp[l],
                             c->stream), "gradients");
    if (host_grads)
        HIPCHK(hipMemcpyAsync(host_grads, n.dw.p, n.nweights * 4, hipMemcpyDeviceToHost, c->stream), "gradients");
    HIPCHK(hipStreamSynchronize(c->stream), "gradients");
    if (loss) *loss = (float)ml;
    return MLFFT_OK;
}

mlfft_status mlfft_net_train_step(mlfft_ctx ctx, int W, int H, int Wd, const void* y, const void* e, float lr,
                                  float* loss) {
    if (!ctx) return MLFFT_E_ARG;
    Ctx* c = ctx;
    if (!(lr > 0.f)) return c->fail(MLFFT_E_ARG, "lr must be positive");
    double ml = 0.0;
    mlfft_status st = grads_common(c, W, H, Wd, y, e, &ml);
    if (st < 0) return st;
    Net& n = *c->net;
    n.adam_t += 1;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - std::pow(b1, (float)n.adam_t), c2 = 1.f - std::pow(b2, (float)n.adam_t);
    for (int l = 0; l < 4; ++l)
        HIPCHK(n_adam((float*)n.wmaster.p + n.woff[l], (float*)n.m.p + n.woff[l], (float*)n.v.p + n.woff[l],
                      (const float*)n.dwp[l].p, (unsigned short*)n.wbf[l].p, n.cin[l], n.cout[l], n.cinp[l], lr, b1, b2,
                      eps, c1, c2, c->stream), "adam");
    HIPCHK(hipStreamSynchronize(c->stream), "train step");
    if (loss) *loss = (float)ml;
    return MLFFT_OK;
}

}  // extern "C"
