// Host orchestration of the learned-guess U-Net (C-ABI of jacobi_guess.h):
// workspace carve-up, the layer order of the forward and backward passes, and
// the Adam step.  Every step runs in the kernels of kernels_nn.hip.

#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "jacobi.h"
#include "jacobi_guess.h"
#include "nn_internal.h"
#include "runtime_common.h"

using namespace jacobi_impl;
using namespace jacobi_impl::nn;

namespace {

struct Layout {
    size_t total = 0;
    // byte offsets
    size_t w = 0, wt = 0, woff = 0, in = 0, out = 0, blend = 0, loss = 0, lpart = 0,
           gpart = 0, wpart = 0, sines = 0, mpart = 0, acoef = 0;
    std::vector<size_t> ea, eb, dn, sm, da, db, ga, gb, gs;
};

int n_layers(int L) { return 3 * L - 1 + 2 * (L - 1); }

size_t add(size_t& off, size_t bytes)
{
    const size_t at = off;
    off = (size_t)round_up((int64_t)(off + bytes), 256);
    return at;
}

bool plan(int64_t n, int L, Layout* lay)
{
    if (L < 2 || L > 6 || n < (1 << (L - 1)) || n % (1 << (L - 1)) || n > 2048) return false;
    Layout l;
    size_t off = 0;
    const int nl = n_layers(L);
    l.w = add(off, (size_t)nl * kConvW * 2);
    l.wt = add(off, (size_t)nl * kConvW * 2);
    l.woff = add(off, (size_t)nl * 8);
    auto vox = [&](int lev) { const int64_t d = n >> lev; return (size_t)(d * d * d); };
    l.in = add(off, vox(0) * kC * 2);
    l.out = add(off, vox(0) * 4);
    l.blend = add(off, vox(0) * 4);
    l.loss = add(off, 8);
    l.lpart = add(off, (size_t)head_blocks((int64_t)vox(0)) * 8);
    l.gpart = add(off, (size_t)head_blocks((int64_t)vox(0)) * 17 * 4);
    l.wpart = add(off, (size_t)kMaxWgradBlocks * (kConvW + kC) * 4);
    l.sines = add(off, (size_t)2 * n * 4);
    l.mpart = add(off, (size_t)head_blocks((int64_t)vox(0)) * 8 * 8);
    l.acoef = add(off, 8 * 8);
    for (int lev = 0; lev < L; ++lev) {
        l.ea.push_back(add(off, vox(lev) * kC * 2));
        l.eb.push_back(add(off, vox(lev) * kC * 2));
        l.dn.push_back(lev < L - 1 ? add(off, vox(lev + 1) * kC * 2) : 0);
        l.sm.push_back(lev < L - 1 ? add(off, vox(lev) * kC * 2) : 0);
        l.da.push_back(lev < L - 1 ? add(off, vox(lev) * kC * 2) : 0);
        l.db.push_back(lev < L - 1 ? add(off, vox(lev) * kC * 2) : 0);
        l.ga.push_back(add(off, vox(lev) * kC * 4));
        l.gb.push_back(add(off, vox(lev) * kC * 4));
        l.gs.push_back(lev < L - 1 ? add(off, vox(lev) * kC * 4) : 0);
    }
    l.total = off;
    *lay = l;
    return true;
}

// Index of each conv layer in the parameter vector (oracle/layer order).
struct Index {
    std::vector<int> enc_a, enc_b, down, dec_a, dec_b;
};

Index layer_index(int L)
{
    Index ix;
    ix.enc_a.assign(L, -1);
    ix.enc_b.assign(L, -1);
    ix.down.assign(L, -1);
    ix.dec_a.assign(L, -1);
    ix.dec_b.assign(L, -1);
    int q = 0;
    for (int l = 0; l < L; ++l) {
        ix.enc_a[l] = q++;
        ix.enc_b[l] = q++;
        if (l < L - 1) ix.down[l] = q++;
    }
    for (int l = L - 2; l >= 0; --l) {
        ix.dec_a[l] = q++;
        ix.dec_b[l] = q++;
    }
    return ix;
}

}  // namespace

struct jg_net_s {
    int64_t n = 0;
    int L = 0;
    int nl = 0;
    int64_t nparams = 0;
    float* params = nullptr;
    float* grads = nullptr;
    float* m = nullptr;
    float* v = nullptr;
    char* ws = nullptr;
    hipStream_t s = nullptr;
    Layout lay;
    Index ix;
    std::vector<int64_t> woff_host;
    std::vector<float> sines_host;
    float low_weight = 0.f;  // weight of the low-mode term of the loss
};

namespace {

template <typename T>
T* at(jg_net* h, size_t off) { return reinterpret_cast<T*>(h->ws + off); }

const uint16_t* W(jg_net* h, int layer) { return at<uint16_t>(h, h->lay.w) + (size_t)layer * kConvW; }
const uint16_t* WT(jg_net* h, int layer) { return at<uint16_t>(h, h->lay.wt) + (size_t)layer * kConvW; }
const float* B(jg_net* h, int layer) { return h->params + (size_t)layer * kConvP + kConvW; }
float* G(jg_net* h, int layer) { return h->grads + (size_t)layer * kConvP; }
uint16_t* A(jg_net* h, size_t off) { return at<uint16_t>(h, off); }
float* F(jg_net* h, size_t off) { return at<float>(h, off); }

}  // namespace

extern "C" {

int jg_param_count(int32_t levels, int64_t* count)
{
    if (!count) return fail(JACOBI_EINVAL, "null argument");
    if (levels < 2 || levels > 6) return fail(JACOBI_EINVAL, "levels must be 2..6");
    *count = (int64_t)n_layers(levels) * kConvP + kC + 1;
    return JACOBI_OK;
}

int jg_workspace_size(int64_t n, int32_t levels, size_t* bytes)
{
    if (!bytes) return fail(JACOBI_EINVAL, "null argument");
    Layout l;
    if (!plan(n, levels, &l))
        return fail(JACOBI_EINVAL, "n=%lld must be a multiple of 2^(levels-1), levels 2..6",
                    (long long)n);
    *bytes = l.total;
    return JACOBI_OK;
}

int jg_create(int64_t n, int32_t levels, float* params, float* grads, float* adam_m,
              float* adam_v, void* workspace, size_t workspace_bytes, void* stream,
              jg_net** out)
{
    if (!out) return fail(JACOBI_EINVAL, "null output handle pointer");
    *out = nullptr;
    Layout l;
    if (!plan(n, levels, &l))
        return fail(JACOBI_EINVAL, "n=%lld must be a multiple of 2^(levels-1), levels 2..6",
                    (long long)n);
    if (!params) return fail(JACOBI_EINVAL, "params is null");
    if (!workspace || workspace_bytes < l.total)
        return fail(JACOBI_EWORKSPACE, "workspace of %zu bytes needed", l.total);
    if (reinterpret_cast<uintptr_t>(workspace) % 256)
        return fail(JACOBI_EINVAL, "workspace must be 256-byte aligned");
    jg_net* h = new (std::nothrow) jg_net_s();
    if (!h) return fail(JACOBI_EINVAL, "out of host memory");
    h->n = n;
    h->L = levels;
    h->nl = n_layers(levels);
    jg_param_count(levels, &h->nparams);
    h->params = params;
    h->grads = grads;
    h->m = adam_m;
    h->v = adam_v;
    h->ws = static_cast<char*>(workspace);
    h->s = static_cast<hipStream_t>(stream);
    h->lay = l;
    h->ix = layer_index(levels);
    h->woff_host.resize(h->nl);
    for (int q = 0; q < h->nl; ++q) h->woff_host[q] = (int64_t)q * kConvP;
    // S_p(i) = sin(pi p (i+1)/(n+1)), p = 1, 2: the sine modes of the
    // low-mode loss term.
    h->sines_host.resize(2 * n);
    for (int p = 1; p <= 2; ++p)
        for (int64_t i = 0; i < n; ++i)
            h->sines_host[(p - 1) * n + i] =
                (float)std::sin(M_PI * p * (double)(i + 1) / (double)(n + 1));
    hipError_t e = hipMemcpyAsync(at<int64_t>(h, l.woff), h->woff_host.data(),
                                  sizeof(int64_t) * h->nl, hipMemcpyHostToDevice, h->s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(F(h, l.sines), h->sines_host.data(), sizeof(float) * 2 * n,
                           hipMemcpyHostToDevice, h->s);
    if (e == hipSuccess) e = hipStreamSynchronize(h->s);
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e, "network set-up");
    }
    *out = h;
    return JACOBI_OK;
}

int jg_forward(jg_net* h, const double* box, float* out)
{
    if (!h || !box) return fail(JACOBI_EINVAL, "null argument");
    const Layout& l = h->lay;
    const Index& ix = h->ix;
    const int L = h->L;
    hipError_t e = prep_weights(h->params, at<int64_t>(h, l.woff), h->nl,
                                at<uint16_t>(h, l.w), at<uint16_t>(h, l.wt), h->s);
    if (e == hipSuccess) e = lift(box, (int)h->n, A(h, l.in), F(h, l.blend), h->s);
    const uint16_t* x = A(h, l.in);
    for (int lev = 0; lev < L && e == hipSuccess; ++lev) {
        const int d = (int)(h->n >> lev);
        e = conv_fwd(x, d, W(h, ix.enc_a[lev]), B(h, ix.enc_a[lev]), A(h, l.ea[lev]), 1, true, h->s);
        if (e == hipSuccess)
            e = conv_fwd(A(h, l.ea[lev]), d, W(h, ix.enc_b[lev]), B(h, ix.enc_b[lev]),
                         A(h, l.eb[lev]), 1, true, h->s);
        if (e == hipSuccess && lev < L - 1) {
            e = conv_fwd(A(h, l.eb[lev]), d, W(h, ix.down[lev]), B(h, ix.down[lev]),
                         A(h, l.dn[lev]), 2, true, h->s);
            x = A(h, l.dn[lev]);
        } else {
            x = A(h, l.eb[lev]);
        }
    }
    for (int lev = L - 2; lev >= 0 && e == hipSuccess; --lev) {
        const int d = (int)(h->n >> lev);
        e = up_add(x, A(h, l.eb[lev]), A(h, l.sm[lev]), d, h->s);
        if (e == hipSuccess)
            e = conv_fwd(A(h, l.sm[lev]), d, W(h, ix.dec_a[lev]), B(h, ix.dec_a[lev]),
                         A(h, l.da[lev]), 1, true, h->s);
        if (e == hipSuccess)
            e = conv_fwd(A(h, l.da[lev]), d, W(h, ix.dec_b[lev]), B(h, ix.dec_b[lev]),
                         A(h, l.db[lev]), 1, true, h->s);
        x = A(h, l.db[lev]);
    }
    const float* hw = h->params + (size_t)h->nl * kConvP;
    const int64_t nv = h->n * h->n * h->n;
    if (e == hipSuccess)
        e = head(x, nv, (int)h->n, hw, hw + kC, F(h, l.blend), F(h, l.out), nullptr,
                 nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, LowModeLoss{}, h->s);
    if (e == hipSuccess && out)
        e = hipMemcpyAsync(out, F(h, l.out), nv * sizeof(float), hipMemcpyDeviceToDevice, h->s);
    if (e != hipSuccess) return hip_fail(e, "network forward");
    return JACOBI_OK;
}

int jg_backward(jg_net* h, const float* target, double* loss)
{
    if (!h || !target) return fail(JACOBI_EINVAL, "null argument");
    if (!h->grads) return fail(JACOBI_ESTATE, "network created without gradient buffer");
    const Layout& l = h->lay;
    const Index& ix = h->ix;
    const int L = h->L;
    const int64_t nv = h->n * h->n * h->n;
    float* gparam_head = h->grads + (size_t)h->nl * kConvP;
    const float* hw = h->params + (size_t)h->nl * kConvP;
    float* wpart = F(h, l.wpart);
    const uint16_t* last = A(h, l.db[0]);
    // head: dx into ga[0] (masked by the last ReLU output), head gradients
    LowModeLoss low;
    low.weight = h->low_weight;
    low.sines = F(h, l.sines);
    low.mpart = at<double>(h, l.mpart);
    low.acoef = at<double>(h, l.acoef);
    hipError_t e = head(last, nv, (int)h->n, hw, hw + kC, F(h, l.blend), F(h, l.out), target,
                        F(h, l.ga[0]),
                        at<double>(h, l.lpart), F(h, l.gpart), at<double>(h, l.loss),
                        gparam_head, gparam_head + kC, low, h->s);
    // decoder, from level 0 up: ga[lev] holds the gradient of dec_b's output
    for (int lev = 0; lev <= L - 2 && e == hipSuccess; ++lev) {
        const int d = (int)(h->n >> lev);
        e = conv_bwd_weight(A(h, l.da[lev]), d, F(h, l.ga[lev]), d, 1, wpart,
                            G(h, ix.dec_b[lev]), h->s);
        if (e == hipSuccess)
            e = conv_bwd_data(F(h, l.ga[lev]), d, W(h, ix.dec_b[lev]), WT(h, ix.dec_b[lev]), F(h, l.gb[lev]), d, 1,
                              false, A(h, l.da[lev]), h->s);
        if (e == hipSuccess)
            e = conv_bwd_weight(A(h, l.sm[lev]), d, F(h, l.gb[lev]), d, 1, wpart,
                                G(h, ix.dec_a[lev]), h->s);
        if (e == hipSuccess)
            e = conv_bwd_data(F(h, l.gb[lev]), d, W(h, ix.dec_a[lev]), WT(h, ix.dec_a[lev]), F(h, l.gs[lev]), d, 1,
                              false, nullptr, h->s);
        // the upsampled input came from dec_b of level lev+1, or from the
        // bottom encoder output
        const uint16_t* prev = lev + 1 <= L - 2 ? A(h, l.db[lev + 1]) : A(h, l.eb[L - 1]);
        if (e == hipSuccess) e = up_bwd(F(h, l.gs[lev]), F(h, l.ga[lev + 1]), d, prev, h->s);
    }
    // encoder, from the bottom up; ga[lev] = gradient of enc_b's output (for
    // lev < L-1 it arrives through the down conv and the skip)
    for (int lev = L - 1; lev >= 0 && e == hipSuccess; --lev) {
        const int d = (int)(h->n >> lev);
        float* cur = F(h, l.ga[lev]);
        if (lev < L - 1) {
            const int dd = d / 2;
            e = conv_bwd_weight(A(h, l.eb[lev]), d, F(h, l.ga[lev + 1]), dd, 2, wpart,
                                G(h, ix.down[lev]), h->s);
            if (e == hipSuccess)
                e = conv_bwd_data(F(h, l.ga[lev + 1]), dd, W(h, ix.down[lev]), WT(h, ix.down[lev]), F(h, l.gs[lev]),
                                  d, 2, true, A(h, l.eb[lev]), h->s);
            cur = F(h, l.gs[lev]);
        }
        if (e == hipSuccess)
            e = conv_bwd_weight(A(h, l.ea[lev]), d, cur, d, 1, wpart, G(h, ix.enc_b[lev]), h->s);
        if (e == hipSuccess)
            e = conv_bwd_data(cur, d, W(h, ix.enc_b[lev]), WT(h, ix.enc_b[lev]), F(h, l.gb[lev]), d, 1, false,
                              A(h, l.ea[lev]), h->s);
        const uint16_t* in = lev == 0 ? A(h, l.in) : A(h, l.dn[lev - 1]);
        if (e == hipSuccess)
            e = conv_bwd_weight(in, d, F(h, l.gb[lev]), d, 1, wpart, G(h, ix.enc_a[lev]), h->s);
        if (e == hipSuccess && lev > 0)
            e = conv_bwd_data(F(h, l.gb[lev]), d, W(h, ix.enc_a[lev]), WT(h, ix.enc_a[lev]), F(h, l.ga[lev]), d, 1,
                              false, A(h, l.dn[lev - 1]), h->s);
    }
    if (e != hipSuccess) return hip_fail(e, "network backward");
    if (loss) {
        e = hipMemcpyAsync(loss, at<double>(h, l.loss), sizeof(double), hipMemcpyDeviceToHost,
                           h->s);
        if (e == hipSuccess) e = hipStreamSynchronize(h->s);
        if (e != hipSuccess) return hip_fail(e, "loss copy");
    }
    return JACOBI_OK;
}

int jg_set_low_mode_weight(jg_net* h, double weight)
{
    if (!h) return fail(JACOBI_EINVAL, "null handle");
    if (!(weight >= 0.0) || weight > 1e12) return fail(JACOBI_EINVAL, "weight must be in [0, 1e12]");
    h->low_weight = (float)weight;
    return JACOBI_OK;
}

int jg_zero_grads(jg_net* h)
{
    if (!h || !h->grads) return fail(JACOBI_EINVAL, "no gradient buffer");
    hipError_t e = zero_f32(h->grads, h->nparams, h->s);
    return e == hipSuccess ? JACOBI_OK : hip_fail(e, "zero grads");
}

int jg_adam(jg_net* h, float lr, float beta1, float beta2, float eps, int64_t step)
{
    if (!h || !h->grads || !h->m || !h->v)
        return fail(JACOBI_EINVAL, "network has no gradient / Adam buffers");
    if (step < 1) return fail(JACOBI_EINVAL, "step must be >= 1");
    hipError_t e = adam(h->params, h->grads, h->m, h->v, h->nparams, lr, beta1, beta2, eps,
                        step, h->s);
    return e == hipSuccess ? JACOBI_OK : hip_fail(e, "adam");
}

int jg_write_guess(jg_net* h, double* box)
{
    if (!h || !box) return fail(JACOBI_EINVAL, "null argument");
    hipError_t e = write_guess(F(h, h->lay.out), (int)h->n, box, h->s);
    return e == hipSuccess ? JACOBI_OK : hip_fail(e, "write guess");
}

int jg_write_blend(jg_net* h, double* box)
{
    if (!h || !box) return fail(JACOBI_EINVAL, "null argument");
    const Layout& l = h->lay;
    hipError_t e = lift(box, (int)h->n, A(h, l.in), F(h, l.blend), h->s);
    if (e == hipSuccess) e = write_guess(F(h, l.blend), (int)h->n, box, h->s);
    return e == hipSuccess ? JACOBI_OK : hip_fail(e, "write blend");
}

int jg_destroy(jg_net* h)
{
    delete h;
    return JACOBI_OK;
}

}  // extern "C"

namespace {

// Layer workspace: the transposed weights, then the weight-gradient partials.
size_t layer_ws(int64_t d, int stride, size_t* part_off)
{
    const int dout = (int)(d / stride);
    *part_off = (size_t)round_up(kConvW * 2, 256);
    (void)dout;
    return *part_off + (size_t)round_up((int64_t)kMaxWgradBlocks * kConvP * 4, 256);
}

int layer_args(const void* a, const void* b, const void* c, int64_t d, int stride)
{
    if (!a || !b || !c) return fail(JACOBI_EINVAL, "null argument");
    if ((stride != 1 && stride != 2) || d < stride || d % stride || d > 1024)
        return fail(JACOBI_EINVAL, "need stride 1 or 2 and 1 <= d <= 1024 divisible by it");
    return JACOBI_OK;
}

int layer_ws_check(void* ws, size_t bytes, int64_t d, int stride, size_t* part_off)
{
    const size_t need = layer_ws(d, stride, part_off);
    if (!ws || bytes < need)
        return fail(JACOBI_EWORKSPACE, "workspace of %zu bytes needed", need);
    if (reinterpret_cast<uintptr_t>(ws) % 256)
        return fail(JACOBI_EINVAL, "workspace must be 256-byte aligned");
    return JACOBI_OK;
}

}  // namespace

extern "C" {

int jg_conv3_workspace_size(int64_t d, int32_t stride, size_t* bytes)
{
    if (!bytes) return fail(JACOBI_EINVAL, "null argument");
    int rc = layer_args(bytes, bytes, bytes, d, stride);
    if (rc != JACOBI_OK) return rc;
    size_t off = 0;
    *bytes = layer_ws(d, stride, &off);
    return JACOBI_OK;
}

int jg_conv3_forward(const uint16_t* x, int64_t d, const uint16_t* w, const float* bias,
                     int32_t stride, float* y, void* stream)
{
    int rc = layer_args(x, w, y, d, stride);
    if (rc != JACOBI_OK) return rc;
    if (!bias) return fail(JACOBI_EINVAL, "null argument");
    hipError_t e = conv_fwd_f32(x, (int)d, w, bias, y, stride, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? JACOBI_OK : hip_fail(e, "conv forward");
}

int jg_conv3_backward_data(const float* dy, int64_t d, const uint16_t* w, int32_t stride,
                           float* dx, void* workspace, size_t workspace_bytes, void* stream)
{
    int rc = layer_args(dy, w, dx, d, stride);
    if (rc != JACOBI_OK) return rc;
    size_t off = 0;
    rc = layer_ws_check(workspace, workspace_bytes, d, stride, &off);
    if (rc != JACOBI_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint16_t* wt = static_cast<uint16_t*>(workspace);
    hipError_t e = transpose_w(w, wt, s);
    if (e == hipSuccess)
        e = conv_bwd_data(dy, (int)(d / stride), w, wt, dx, (int)d, stride, false, nullptr, s);
    return e == hipSuccess ? JACOBI_OK : hip_fail(e, "conv data gradient");
}

int jg_conv3_backward_weight(const uint16_t* x, int64_t d, const float* dy, int32_t stride,
                             float* grad, void* workspace, size_t workspace_bytes,
                             void* stream)
{
    int rc = layer_args(x, dy, grad, d, stride);
    if (rc != JACOBI_OK) return rc;
    size_t off = 0;
    rc = layer_ws_check(workspace, workspace_bytes, d, stride, &off);
    if (rc != JACOBI_OK) return rc;
    float* part = reinterpret_cast<float*>(static_cast<char*>(workspace) + off);
    hipError_t e = conv_bwd_weight(x, (int)d, dy, (int)(d / stride), stride, part, grad,
                                   static_cast<hipStream_t>(stream));
    return e == hipSuccess ? JACOBI_OK : hip_fail(e, "conv weight gradient");
}

}  // extern "C"
