// C ABI of the mask network: layer plan, buffer layouts and the forward /
// backward schedules over the kernels of mask_kernels.hip.
//
// Layer plan (parameter order): enc0a, enc0b, ..., enc(L-1)a, enc(L-1)b,
// dec(L-2)a, dec(L-2)b, ..., dec0a, dec0b, then the head.  Inputs: enc0a reads
// the scans (as 8 channels: one scan in channel 0, or for the dual-input
// network f in channel 0 and g in channel 1), enc{l}a reads the max-pool
// of enc{l-1}b's activation, every b conv reads its a conv's activation,
// dec{l}a reads concat[up2(deeper), enc{l}b] where deeper is dec{l+1}b (or
// enc{L-1}b at the bottom).  The head reads the last conv's activation.
#include <math.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "internal.hpp"
#include "profile.hpp"
#include "mask_kernels.hpp"
#include "mask_net.hpp"

namespace fmbym {
namespace {

struct ConvL {
    int cin, cout, cink, level;
    bool enc, first_of_level;
    size_t w, gamma, beta;   // float offsets in params
    size_t pf, pb;           // bf16 element offsets in packed (pb unused for the first conv)
    int bn;                  // first channel in the running statistics
};

struct Net {
    int levels = 0, base = 0, chans = 1;   // chans: input scans and output masks per sample
    float eps = 0.f, momentum = 0.f;
    std::vector<ConvL> convs;
    size_t n_params = 0, n_packed = 0, head_w = 0, head_b = 0;
    int bn_channels = 0;
    int ch(int l) const { return base << l; }
    // index of a conv by (enc/dec, level, part b?)
    int enc_a(int l) const { return 2 * l; }
    int enc_b(int l) const { return 2 * l + 1; }
    int dec_a(int l) const { return 2 * levels + 2 * (levels - 2 - l); }
    int dec_b(int l) const { return dec_a(l) + 1; }
    int last() const { return (int)convs.size() - 1; }
    // activation feeding dec{l}a's upsampling
    int deeper(int l) const { return l + 1 == levels - 1 ? enc_b(levels - 1) : dec_b(l + 1); }
};

size_t al64(size_t x) { return (x + 63) & ~(size_t)63; }

bool build_net(const fmbym_mask_desc* d, Net& net) {
    if (!d || d->levels < 1 || d->levels > 6 || d->base_channels != 8) return false;
    if (d->channels != 0 && d->channels != 1 && d->channels != 2) return false;
    net = Net();
    net.levels = d->levels;
    net.base = d->base_channels;
    net.chans = d->channels == 2 ? 2 : 1;
    net.eps = d->bn_eps;
    net.momentum = d->bn_momentum;
    size_t po = 0, pk = 0;
    int bn = 0;
    auto add = [&](int cin, int cout, int level, bool enc, bool first) {
        ConvL c{};
        c.cin = cin;
        c.cout = cout;
        c.cink = cin < 8 ? 8 : cin;
        c.level = level;
        c.enc = enc;
        c.first_of_level = first;
        c.w = po;
        po += (size_t)cout * cin * 9;
        c.gamma = po;
        po += cout;
        c.beta = po;
        po += cout;
        c.pf = pk;
        pk = al64(pk + (size_t)cout * 9 * c.cink);
        c.pb = pk;
        if (!net.convs.empty()) pk = al64(pk + (size_t)cin * 9 * cout);
        c.bn = bn;
        bn += cout;
        net.convs.push_back(c);
    };
    for (int l = 0; l < net.levels; ++l) {
        add(l == 0 ? net.chans : net.ch(l - 1), net.ch(l), l, true, true);
        add(net.ch(l), net.ch(l), l, true, false);
    }
    for (int l = net.levels - 2; l >= 0; --l) {
        add(net.ch(l + 1) + net.ch(l), net.ch(l), l, false, true);
        add(net.ch(l), net.ch(l), l, false, false);
    }
    net.head_w = po;
    po += (size_t)net.chans * net.base * 9;
    net.head_b = po;
    po += net.chans;
    net.n_params = po;
    net.n_packed = pk;
    net.bn_channels = bn;
    return true;
}

bool size_ok(const Net& net, int images, int n) {
    if (images < 1 || images > (1 << 16)) return false;
    if (n != 128 && n != 256 && n != 512) return false;
    return (n >> (net.levels - 1)) >= 16;
}

struct Bump {
    size_t off = 0;
    size_t take(size_t bytes) {
        const size_t o = off;
        off = (off + bytes + 255) & ~(size_t)255;
        return o;
    }
};

struct ActLayout {
    size_t x8 = 0, mask = 0, part = 0, tmp = 0, total = 0;
    std::vector<size_t> z, a, stat, pool, cat;
};

ActLayout act_layout(const Net& net, int I, int n) {
    ActLayout L;
    Bump b;
    const size_t bf = 2, fl = 4;
    auto pix = [&](int l) { return (size_t)I * (size_t)(n >> l) * (size_t)(n >> l); };
    L.x8 = b.take(pix(0) * 8 * bf);
    size_t part_max = 0;
    for (const ConvL& c : net.convs) {
        L.z.push_back(b.take(pix(c.level) * c.cout * bf));
        L.a.push_back(b.take(pix(c.level) * c.cout * bf));
        L.stat.push_back(b.take(4 * (size_t)c.cout * fl));
        const size_t p = (size_t)conv_part_blocks(I, n >> c.level) * 2 * c.cout * fl;
        if (p > part_max) part_max = p;
    }
    L.pool.assign(net.levels, 0);
    for (int l = 1; l < net.levels; ++l) L.pool[l] = b.take(pix(l) * net.ch(l - 1) * bf);
    L.cat.assign(net.levels, 0);
    for (int l = 0; l + 1 < net.levels; ++l) L.cat[l] = b.take(pix(l) * (net.ch(l + 1) + net.ch(l)) * bf);
    L.mask = b.take(pix(0) * net.chans * fl);
    L.part = b.take(part_max);
    L.tmp = b.take(colsum_tmp_floats(2 * 256) * fl);
    L.total = b.off;
    return L;
}

struct WsLayout {
    size_t dz[2] = {0, 0}, part = 0, coef = 0, wpart = 0, hpart = 0, tmp = 0, total = 0;
    std::vector<size_t> g, dpool, dcat;
};

WsLayout ws_layout(const Net& net, int I, int n) {
    WsLayout L;
    Bump b;
    const size_t fl = 4;
    auto pix = [&](int l) { return (size_t)I * (size_t)(n >> l) * (size_t)(n >> l); };
    size_t dz_max = 0, part_max = 0, wpart_max = 0;
    for (const ConvL& c : net.convs) {
        L.g.push_back(b.take(pix(c.level) * c.cout * fl));
        dz_max = std::max(dz_max, pix(c.level) * c.cout * 2);
        part_max = std::max(part_max, (size_t)bn_part_blocks((long long)pix(c.level), c.cout) * 2 * c.cout * fl);
        int nb, tpb;
        wgrad_grid(I, n >> c.level, &nb, &tpb);
        wpart_max = std::max(wpart_max, (size_t)nb * c.cout * 9 * c.cink * fl);
    }
    L.dpool.assign(net.levels, 0);
    for (int l = 1; l < net.levels; ++l) L.dpool[l] = b.take(pix(l) * net.ch(l - 1) * fl);
    L.dcat.assign(net.levels, 0);
    for (int l = 0; l + 1 < net.levels; ++l) L.dcat[l] = b.take(pix(l) * (net.ch(l + 1) + net.ch(l)) * fl);
    L.dz[0] = b.take(dz_max);   // layers alternate: a weight gradient may still read the other
    L.dz[1] = b.take(dz_max);
    L.part = b.take(part_max);
    L.coef = b.take(3 * 256 * fl);   // per-channel coefficients of the widest BN layer
    L.wpart = b.take(wpart_max);
    L.hpart = b.take(((pix(0) + 4095) / 4096) * net.chans * (9 * net.base + 1) * fl);   // rows of every output channel
    size_t cols = 2 * 256;
    for (const ConvL& c : net.convs) cols = std::max(cols, (size_t)c.cout * 9 * c.cink);
    L.tmp = b.take(colsum_tmp_floats((int)cols) * fl);
    L.total = b.off;
    return L;
}

template <class T>
T* at(void* base, size_t off) {
    return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}
template <class T>
const T* at(const void* base, size_t off) {
    return reinterpret_cast<const T*>(static_cast<const char*>(base) + off);
}

int finish(hipStream_t) {
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? FMBYM_OK : hip_fail(e);
}

// The backward's weight gradients run on a second stream per device, beside
// the chain of data gradients on the caller's stream: the weight gradient of
// layer j waits for that layer's dz (event dz), and the chain waits for it
// (event w[j % 2]) before it overwrites that dz buffer two layers later and
// at the end.  Enqueueing holds g_lane_mu, so calls from several host threads
// take the events in turn (a wait uses the event's state when it is enqueued).
constexpr int kMaxLanes = 64;
struct WgradLane {
    hipStream_t s = nullptr;
    hipEvent_t dz = nullptr;
    hipEvent_t w[2] = {nullptr, nullptr};
};
std::mutex g_lane_mu;
WgradLane g_lanes[kMaxLanes];

// The lane of the current device, created on first use (call with g_lane_mu held).
hipError_t wgrad_lane(WgradLane** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxLanes) return hipErrorInvalidDevice;
    WgradLane& L = g_lanes[dev];
    if (!L.s) {
        WgradLane n;
        e = hipStreamCreateWithFlags(&n.s, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&n.dz, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&n.w[0], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&n.w[1], hipEventDisableTiming);
        if (e != hipSuccess) {
            for (hipEvent_t ev : {n.dz, n.w[0], n.w[1]})
                if (ev) (void)hipEventDestroy(ev);
            if (n.s) (void)hipStreamDestroy(n.s);
            return e;
        }
        L = n;
    }
    *out = &L;
    return hipSuccess;
}

}  // namespace
}  // namespace fmbym

using namespace fmbym;

extern "C" {

size_t fmbym_mask_param_count(const fmbym_mask_desc* d) {
    Net net;
    return build_net(d, net) ? net.n_params : 0;
}

size_t fmbym_mask_packed_bytes(const fmbym_mask_desc* d) {
    Net net;
    return build_net(d, net) ? net.n_packed * sizeof(bf16) : 0;
}

size_t fmbym_mask_bn_channels(const fmbym_mask_desc* d) {
    Net net;
    return build_net(d, net) ? (size_t)net.bn_channels : 0;
}

int fmbym_mask_pack(const fmbym_mask_desc* d, void* stream) {
    const TraceRange trace_range("fmbym_mask_pack");
    Net net;
    if (!build_net(d, net)) return FMBYM_EUNSUPPORTED;
    if (!d->params || !d->packed) return FMBYM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    PackLayers t{};
    t.n = (int)net.convs.size();
    if (t.n > kMaxPackLayers) return FMBYM_EUNSUPPORTED;
    for (int j = 0; j < t.n; ++j) {
        const ConvL& c = net.convs[j];
        t.cin[j] = c.cin;
        t.cout[j] = c.cout;
        t.cink[j] = c.cink;
        t.start[j + 1] = t.start[j] + c.cout * 9 * c.cink;
        t.w[j] = (long long)c.w;
        t.pf[j] = (long long)c.pf;
        t.pb[j] = j ? (long long)c.pb : -1;   // the first conv has no data gradient
    }
    launch_pack(t, d->params, (bf16*)d->packed, s);
    return finish(s);
}

size_t fmbym_mask_activation_bytes(const fmbym_mask_desc* d, int32_t images, int32_t n) {
    Net net;
    if (!build_net(d, net) || !size_ok(net, images, n)) return 0;
    return act_layout(net, images, n).total;
}

size_t fmbym_mask_workspace_bytes(const fmbym_mask_desc* d, int32_t images, int32_t n) {
    Net net;
    if (!build_net(d, net) || !size_ok(net, images, n)) return 0;
    return ws_layout(net, images, n).total;
}

int fmbym_mask_fwd(const fmbym_mask_desc* d, int32_t I, int32_t n, const float* x, float* mask, void* act,
                   size_t act_bytes, int training, void* stream) {
    const TraceRange trace_range("fmbym_mask_fwd");
    return mask_forward(d, I, n, x, nullptr, mask, act, act_bytes, training, (hipStream_t)stream);
}

int fmbym_mask_bwd(const fmbym_mask_desc* d, int32_t I, int32_t n, const float* d_mask, const void* act,
                   size_t act_bytes, float* d_params, float* d_x, void* ws, size_t ws_bytes, void* stream) {
    const TraceRange trace_range("fmbym_mask_bwd");
    Net net;
    if (!d) return FMBYM_EINVAL;
    if (!build_net(d, net)) return FMBYM_EUNSUPPORTED;
    if (!size_ok(net, I, n)) return FMBYM_EUNSUPPORTED;
    if (!d_mask || !d_params || !d->params || !d->packed) return FMBYM_EINVAL;
    const ActLayout A = act_layout(net, I, n);
    const WsLayout W = ws_layout(net, I, n);
    if (!act || act_bytes < A.total) return FMBYM_EWORKSPACE;
    if (!ws || ws_bytes < W.total) return FMBYM_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    const bf16* pk = (const bf16*)d->packed;
    const float* P = d->params;
    void* wsp = ws;
    const int last = net.last();
    std::lock_guard<std::mutex> lane_lock(g_lane_mu);
    WgradLane* lane = nullptr;
    if (const hipError_t e = wgrad_lane(&lane); e != hipSuccess) return hip_fail(e);
    bool side_used = false;
    // the caller's stream waits for every weight gradient before any return
    auto join = [&](int rc) {
        if (side_used) {
            const hipError_t e = hipStreamWaitEvent(s, lane->w[0], 0);
            if (e != hipSuccess && rc == FMBYM_OK) rc = hip_fail(e);
        }
        return rc;
    };
    launch_head_bwd(d_mask, at<float>(act, A.mask), at<bf16>(act, A.a[last]), P + net.head_w,
                    at<float>(wsp, W.g[last]), at<float>(wsp, W.hpart),
                    at<float>(wsp, W.tmp), d_params + net.head_w, d_params + net.head_b, I, n, net.base,
                    net.chans, s);
    for (int j = last; j >= 0; --j) {
        const ConvL& c = net.convs[j];
        const int S = n >> c.level;
        const long long M = (long long)I * S * S;
        bf16* dz = at<bf16>(wsp, W.dz[j & 1]);
        // dz[j % 2] was last read by the weight gradient of layer j + 2
        if (j + 2 <= last && hipStreamWaitEvent(s, lane->w[j & 1], 0) != hipSuccess) return join(finish(s));
        launch_bn_relu_bwd(at<float>(wsp, W.g[j]), at<bf16>(act, A.z[j]), at<float>(act, A.stat[j]),
                           P + c.gamma, at<float>(wsp, W.part), at<float>(wsp, W.tmp), at<float>(wsp, W.coef),
                           d_params + c.gamma,
                           d_params + c.beta, dz, M, c.cout, s);
        const bf16* in;
        if (j == 0)
            in = at<bf16>(act, A.x8);
        else if (c.enc && c.first_of_level)
            in = at<bf16>(act, A.pool[c.level]);
        else if (!c.enc && c.first_of_level)
            in = at<bf16>(act, A.cat[c.level]);
        else
            in = at<bf16>(act, A.a[j - 1]);
        if (hipEventRecord(lane->dz, s) != hipSuccess || hipStreamWaitEvent(lane->s, lane->dz, 0) != hipSuccess)
            return join(finish(s));
        side_used = true;
        const bool ok = launch_wgrad(c.cink, c.cout, dz, in, at<float>(wsp, W.wpart), at<float>(wsp, W.tmp),
                                     d_params + c.w, c.cin, I, S, lane->s);
        if (hipEventRecord(lane->w[j & 1], lane->s) != hipSuccess) return join(finish(s));
        if (!ok) {   // w[0] then marks the lane's last work, which the join waits for
            (void)hipEventRecord(lane->w[0], lane->s);
            return join(FMBYM_EUNSUPPORTED);
        }
        if (j == 0) {
            if (d_x) launch_input_grad(dz, P + c.w, d_x, I, S, c.cout, net.chans, s);
            break;
        }
        // data gradient into the buffer of this conv's input
        float* din;
        if (c.enc && c.first_of_level)
            din = at<float>(wsp, W.dpool[c.level]);
        else if (!c.enc && c.first_of_level)
            din = at<float>(wsp, W.dcat[c.level]);
        else
            din = at<float>(wsp, W.g[j - 1]);
        if (!launch_conv3x3(c.cout, c.cin, kConvDgrad, dz, pk + c.pb, din, nullptr, BnInfer{}, I, S, s)) {
            (void)hipEventRecord(lane->w[0], lane->s);
            return join(FMBYM_EUNSUPPORTED);
        }
        // the gradient of the next conv down (parameter order j - 1) when it is a b conv
        if (!c.enc && c.first_of_level) {
            // deeper activation of dec{l}a: dec{l+1}b or enc{L-1}b
            launch_up_bwd(din, at<float>(wsp, W.g[net.deeper(c.level)]), I, S, net.ch(c.level + 1),
                          net.ch(c.level), s);
        } else if (c.enc && c.first_of_level) {
            const int l = c.level;   // >= 1: enc{l-1}b gets the pool adjoint plus its skip gradient
            launch_pool_bwd(din, at<bf16>(act, A.a[net.enc_b(l - 1)]), at<float>(wsp, W.dcat[l - 1]),
                            net.ch(l) + net.ch(l - 1), net.ch(l), at<float>(wsp, W.g[net.enc_b(l - 1)]), I,
                            n >> (l - 1), net.ch(l - 1), s);
        }
    }
    return join(finish(s));   // layer 0's weight gradient recorded w[0] last
}

int fmbym_adam(float* params, const float* grad, float* m, float* v, int64_t count, int32_t step, float lr,
               float beta1, float beta2, float eps, void* stream) {
    const TraceRange trace_range("fmbym_adam");
    if (!params || !grad || !m || !v || count < 1 || step < 1) return FMBYM_EINVAL;
    if (!(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return FMBYM_EINVAL;
    const float c1 = (float)(1.0 - pow((double)beta1, step));
    const float c2 = (float)(1.0 - pow((double)beta2, step));
    hipStream_t s = (hipStream_t)stream;
    launch_adam(params, grad, m, v, count, lr, beta1, beta2, eps, c1, c2, s);
    return finish(s);
}

int fmbym_pose_loss(int32_t batch, const float* pose, const float* target, int32_t kind, float* loss,
                    float* d_pose, void* stream) {
    const TraceRange trace_range("fmbym_pose_loss");
    if (batch < 1 || !pose || !target || !loss || !d_pose) return FMBYM_EINVAL;
    if (kind != FMBYM_LOSS_L1 && kind != FMBYM_LOSS_L2) return FMBYM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    launch_pose_loss(batch, pose, target, kind, loss, d_pose, s);
    return finish(s);
}

}  // extern "C"

namespace fmbym {

int mask_forward(const fmbym_mask_desc* d, int I, int n, const float* x, const float* const* x_tab,
                 float* mask, void* act, size_t act_bytes, int training, hipStream_t s) {
    Net net;
    if (!d) return FMBYM_EINVAL;
    if (!build_net(d, net)) return FMBYM_EUNSUPPORTED;
    if (!size_ok(net, I, n)) return FMBYM_EUNSUPPORTED;
    if ((!x && !x_tab) || !mask || !d->params || !d->packed || !d->bn_running) return FMBYM_EINVAL;
    if (x_tab && net.chans != 1) return FMBYM_EUNSUPPORTED;   // scan tables hold one scan per image
    if (!(d->bn_eps > 0.f) || !(d->bn_momentum >= 0.f && d->bn_momentum <= 1.f)) return FMBYM_EINVAL;
    const ActLayout A = act_layout(net, I, n);
    if (!act || act_bytes < A.total) return FMBYM_EWORKSPACE;
    const bf16* pk = (const bf16*)d->packed;
    float* run_mean = d->bn_running;
    float* run_var = d->bn_running + net.bn_channels;
    if (!training) {
        // Inference: BN on the running statistics and ReLU inside each convolution;
        // the first reads the scans, every encoder b convolution above the bottom
        // also writes the max pooling its level's successor reads, and every
        // decoder a convolution forms concat[up2(deeper), skip] while staging.
        for (int j = 0; j <= net.last(); ++j) {
            const ConvL& c = net.convs[j];
            const int S = n >> c.level;
            ConvSrc src{nullptr, nullptr, nullptr, nullptr, 0, 0};
            int kind = kSrcPlain;
            if (j == 0) {
                kind = kSrcScan;
                src.x = x;
                src.x_tab = x_tab;
                src.plane = (long long)I * n * n;
                src.ch = net.chans;
            } else if (c.enc && c.first_of_level) {
                src.in = at<bf16>(act, A.pool[c.level]);
            } else if (!c.enc && c.first_of_level) {
                kind = kSrcUpCat;
                src.in = at<bf16>(act, A.a[net.deeper(c.level)]);
                src.skip = at<bf16>(act, A.a[net.enc_b(c.level)]);
            } else {
                src.in = at<bf16>(act, A.a[j - 1]);
            }
            bf16* pool = c.enc && !c.first_of_level && c.level + 1 < net.levels ? at<bf16>(act, A.pool[c.level + 1])
                                                                                : nullptr;
            const BnInfer bn{d->params + c.gamma, d->params + c.beta, run_mean + c.bn, run_var + c.bn, net.eps};
            if (!launch_conv_infer(c.cink, c.cout, kind, src, pk + c.pf, at<bf16>(act, A.a[j]), pool, bn, I, S, s))
                return FMBYM_EUNSUPPORTED;
        }
        if (!launch_head_fwd(at<bf16>(act, A.a[net.last()]), d->params + net.head_w, d->params + net.head_b, mask, I,
                             n, net.base, net.chans, s))
            return FMBYM_EUNSUPPORTED;
        return finish(s);
    }
    launch_input8(x, x_tab, at<bf16>(act, A.x8), I, n, net.chans, s);
    for (int j = 0; j <= net.last(); ++j) {
        const ConvL& c = net.convs[j];
        const int S = n >> c.level;
        const bf16* in;
        if (j == 0) {
            in = at<bf16>(act, A.x8);
        } else if (c.enc && c.first_of_level) {
            in = at<bf16>(act, A.pool[c.level]);   // written by the previous level's BN + ReLU pass
        } else if (!c.enc && c.first_of_level) {
            launch_up_concat(at<bf16>(act, A.a[net.deeper(c.level)]), at<bf16>(act, A.a[net.enc_b(c.level)]),
                             at<bf16>(act, A.cat[c.level]), I, S, net.ch(c.level + 1), net.ch(c.level), s);
            in = at<bf16>(act, A.cat[c.level]);
        } else {
            in = at<bf16>(act, A.a[j - 1]);
        }
        if (!launch_conv3x3(c.cink, c.cout, kConvTrain, in, pk + c.pf, at<bf16>(act, A.z[j]), at<float>(act, A.part),
                            BnInfer{}, I, S, s))
            return FMBYM_EUNSUPPORTED;
        const long long M = (long long)I * S * S;
        launch_bn_stats(at<float>(act, A.part), conv_part_blocks(I, S), c.cout, M, d->params + c.gamma,
                        d->params + c.beta, net.eps, net.momentum, 1, run_mean + c.bn,
                        run_var + c.bn, at<float>(act, A.stat[j]), at<float>(act, A.tmp), s);
        if (c.enc && !c.first_of_level && c.level + 1 < net.levels)   // with the next level's input
            launch_bn_relu_pool(at<bf16>(act, A.z[j]), at<float>(act, A.stat[j]), at<bf16>(act, A.a[j]),
                                at<bf16>(act, A.pool[c.level + 1]), I, S, c.cout, s);
        else
            launch_bn_relu(at<bf16>(act, A.z[j]), at<float>(act, A.stat[j]), at<bf16>(act, A.a[j]), M, c.cout, s);
    }
    if (!launch_head_fwd(at<bf16>(act, A.a[net.last()]), d->params + net.head_w, d->params + net.head_b, mask, I,
                         n, net.base, net.chans, s))
        return FMBYM_EUNSUPPORTED;
    (void)hipMemcpyAsync(at<float>(act, A.mask), mask, (size_t)net.chans * I * n * n * sizeof(float),
                         hipMemcpyDeviceToDevice, s);
    return finish(s);
}

}  // namespace fmbym
