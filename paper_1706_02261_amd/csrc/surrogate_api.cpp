// C-ABI host layer of the learned PSF surrogate: the network's architecture
// table, the parameter / training-state / weight-blob / workspace layouts, and
// the forward, backward and Adam sequences built from the kernels in
// surrogate.hip.  Contracts: include/psf_surrogate.h and, for inference,
// include/bpm.h.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstring>

#include "../../include/bpm.h"
#include "../../include/psf_surrogate.h"
#include "abi_util.hpp"
#include "internal.hpp"

namespace {

using namespace bpm;
using namespace bpm::abi;

// ---------------------------------------------------------------------------
// architecture: five strided 3-D convolutions down to a 2-D map, nearest x2
// upsampling and a 3x3 convolution whose 32 output channels are the PSF planes

constexpr int kLayers = 6;
constexpr int kPatchD = 64, kPatchHW = 32, kPlanes = 32, kInCh = 8;
constexpr int kHeadC = 64;             // channels of the map the error head pools
constexpr int kInferChunk = 1024;      // samples per inference pass
constexpr int kMaxTrainBatch = 1024;

struct LayerSpec {
    int Ci, Co, kd, kh, kw, sd, sh, sw, pd, ph, pw, D, H, W;
};
constexpr LayerSpec kSpec[kLayers] = {
    {kInCh, 32, 3, 3, 3, 2, 2, 2, 1, 1, 1, kPatchD, kPatchHW, kPatchHW},  // c1 -> 32 x 16 x 16
    {32, 32, 3, 3, 3, 2, 1, 1, 1, 1, 1, 32, 16, 16},                     // c2 -> 16
    {32, 32, 3, 3, 3, 2, 1, 1, 1, 1, 1, 16, 16, 16},                     // c3 -> 8
    {32, 32, 3, 3, 3, 2, 1, 1, 1, 1, 1, 8, 16, 16},                      // c4 -> 4
    {32, kHeadC, 4, 3, 3, 1, 1, 1, 0, 1, 1, 4, 16, 16},                  // d1 -> 1 x 16 x 16
    {kHeadC, kPlanes, 1, 3, 3, 1, 1, 1, 0, 1, 1, 1, 32, 32},             // d2 -> 1 x 32 x 32
};

// Completes a geometry from its 15 defining integers; false if degenerate.
bool make_geo(const int g[15], ConvGeo* c) {
    ConvGeo r{};
    r.N = g[0]; r.D = g[1]; r.H = g[2]; r.W = g[3]; r.Ci = g[4]; r.Co = g[5];
    r.kd = g[6]; r.kh = g[7]; r.kw = g[8]; r.sd = g[9]; r.sh = g[10]; r.sw = g[11];
    r.pd = g[12]; r.ph = g[13]; r.pw = g[14];
    if (r.N < 1 || r.D < 1 || r.H < 1 || r.W < 1 || r.Ci < 1 || r.Co < 1 || r.kd < 1 ||
        r.kh < 1 || r.kw < 1 || r.sd < 1 || r.sh < 1 || r.sw < 1 || r.pd < 0 || r.ph < 0 ||
        r.pw < 0)
        return false;
    const long Do = ((long)r.D + 2L * r.pd - r.kd) / r.sd + 1;
    const long Ho = ((long)r.H + 2L * r.ph - r.kh) / r.sh + 1;
    const long Wo = ((long)r.W + 2L * r.pw - r.kw) / r.sw + 1;
    if (r.D + 2L * r.pd < r.kd || r.H + 2L * r.ph < r.kh || r.W + 2L * r.pw < r.kw) return false;
    if (Do > (1 << 20) || Ho > (1 << 20) || Wo > (1 << 20)) return false;
    r.Do = (int)Do; r.Ho = (int)Ho; r.Wo = (int)Wo;
    r.taps = r.kd * r.kh * r.kw;
    r.K = r.taps * r.Ci;
    r.Kp = (r.K + 15) / 16 * 16;
    *c = r;
    return true;
}

ConvGeo layer_geo(int l, int N) {
    const LayerSpec& s = kSpec[l];
    const int g[15] = {N, s.D, s.H, s.W, s.Ci, s.Co, s.kd, s.kh, s.kw,
                       s.sd, s.sh, s.sw, s.pd, s.ph, s.pw};
    ConvGeo c{};
    make_geo(g, &c);
    return c;
}

size_t out_elems(int l) {  // per sample
    const ConvGeo c = layer_geo(l, 1);
    return (size_t)c.Do * c.Ho * c.Wo * c.Co;
}
size_t in_elems(int l) {
    const ConvGeo c = layer_geo(l, 1);
    return (size_t)c.D * c.H * c.W * c.Ci;
}

// ---------------------------------------------------------------------------
// parameter vector: all conv weights [Co][Kp] (layer order), then all biases,
// then the error head (weights [kHeadC], bias)

struct ParamLayout {
    size_t w[kLayers], b[kLayers], we, be, bias_begin, total;
};

ParamLayout param_layout() {
    ParamLayout p{};
    size_t o = 0;
    for (int l = 0; l < kLayers; ++l) {
        const ConvGeo c = layer_geo(l, 1);
        p.w[l] = o;
        o += (size_t)c.Co * c.Kp;
    }
    p.bias_begin = o;
    for (int l = 0; l < kLayers; ++l) {
        p.b[l] = o;
        o += kSpec[l].Co;
    }
    p.we = o;
    o += kHeadC;
    p.be = o;
    o += 1;
    p.total = o;
    return p;
}

// bf16 weights, transposed bf16 weights and tap tables of every layer
struct PackLayout {
    size_t wb[kLayers], wt[kLayers], taps[kLayers], taps_t[kLayers], end;
};

PackLayout pack_layout(size_t o, bool with_transposed) {
    PackLayout k{};
    for (int l = 0; l < kLayers; ++l) {
        const ConvGeo c = layer_geo(l, 1);
        k.wb[l] = o;
        o += align_up(2 * (size_t)c.Co * c.Kp);
        k.wt[l] = o;
        if (with_transposed && l > 0) o += align_up(2 * (size_t)c.Ci * c.taps * c.Co);
        k.taps[l] = o;
        o += align_up(sizeof(int4) * (size_t)(c.K / 8));
        k.taps_t[l] = o;
        if (with_transposed && l > 0) o += align_up(sizeof(int4) * (size_t)(c.taps * c.Co / 8));
    }
    k.end = o;
    return k;
}

// training state: params, grads, Adam m and v (fp32), then the packed layers
struct StateLayout {
    size_t params, grads, m, v;
    PackLayout pack;
    size_t total;
};

StateLayout state_layout() {
    const size_t P = align_up(sizeof(float) * param_layout().total);
    StateLayout s{};
    s.params = 0;
    s.grads = P;
    s.m = 2 * P;
    s.v = 3 * P;
    s.pack = pack_layout(4 * P, true);
    s.total = s.pack.end;
    return s;
}

// inference blob: the fp32 biases and head, then bf16 weights and tap tables
struct BlobLayout {
    size_t bias;
    PackLayout pack;
    size_t total;
};

BlobLayout blob_layout() {
    const ParamLayout p = param_layout();
    BlobLayout b{};
    b.bias = 0;
    b.pack = pack_layout(align_up(sizeof(float) * (p.total - p.bias_begin)), false);
    b.total = b.pack.end;
    return b;
}

// Per-sample activation / gradient buffers of one pass.
struct WsLayout {
    size_t act[kLayers];  // act[0] = input x0, act[l] = output of layer l - 1 (bf16)
    size_t a5, up;        // d1 output and its upsampling (bf16)
    size_t psf, z;        // fp32 [n][planes][32][32]
    size_t gd[kLayers];   // gradient at the pre-activation output of layer l (bf16)
    size_t du;            // gradient at the upsampled map
    size_t pooled, epre, err, derr, dpool;  // fp32 error-head buffers
    size_t total;
};

WsLayout ws_layout(int B, bool training) {
    WsLayout w{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += align_up(bytes);
        return at;
    };
    // inference forms the input channels and the upsampled map while staging
    for (int l = training ? 0 : 1; l < kLayers - 1; ++l) w.act[l] = take(2 * in_elems(l) * B);
    w.a5 = take(2 * out_elems(4) * B);
    if (training) w.up = take(2 * in_elems(5) * B);
    w.pooled = take(sizeof(float) * kHeadC * B);
    w.epre = take(sizeof(float) * B);
    if (training) {
        w.psf = take(sizeof(float) * out_elems(5) * B);
        w.z = take(sizeof(float) * out_elems(5) * B);
        for (int l = 0; l < kLayers; ++l) w.gd[l] = take(2 * out_elems(l) * B);
        w.du = take(2 * in_elems(5) * B);
        w.err = take(sizeof(float) * B);
        w.derr = take(sizeof(float) * B);
        w.dpool = take(sizeof(float) * kHeadC * B);
    }
    w.total = o;
    return w;
}

template <typename T>
T* at(void* base, size_t off) {
    return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}
template <typename T>
const T* at(const void* base, size_t off) {
    return reinterpret_cast<const T*>(static_cast<const char*>(base) + off);
}

// bf16 weights (and, with wt, their transposes) of every layer from fp32
hipError_t pack_all(const float* params, void* base, const PackLayout& k, bool transposed,
                    hipStream_t s) {
    const ParamLayout p = param_layout();
    for (int l = 0; l < kLayers; ++l) {
        const ConvGeo c = layer_geo(l, 1);
        void* wt = transposed && l > 0 ? at<void>(base, k.wt[l]) : nullptr;
        hipError_t e = sg::pack_weights(params + p.w[l], c.Co, c.Ci, c.taps, c.Kp,
                                        at<void>(base, k.wb[l]), wt, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t tables_all(void* base, const PackLayout& k, bool transposed, hipStream_t s) {
    for (int l = 0; l < kLayers; ++l) {
        const ConvGeo c = layer_geo(l, 1);
        int4* tt = transposed && l > 0 ? at<int4>(base, k.taps_t[l]) : nullptr;
        hipError_t e = sg::tap_tables(c, at<int4>(base, k.taps[l]), tt, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Forward pass of B samples.  Weights, tap tables and biases come from `wbase`
// (packed layout k) and `bias` (fp32 biases then head, param-layout order from
// bias_begin).  The PSF goes to psf (fp32 [B][planes][32][32]), its
// pre-activation to z (may be null), the predicted error to err.
// With `training`, the stored input x0 and the upsampled map (which the
// weight gradients read) are materialised; inference forms both on the fly
// while staging the first and the last convolution's input tiles.  Either
// way the convolutions see the same bf16 values.
hipError_t forward(const void* wbase, const PackLayout& k, const float* bias, const float* dn,
                   const float* depth, int B, void* ws, const WsLayout& w, float* psf, float* z,
                   float* err, hipStream_t s, bool training) {
    const ParamLayout p = param_layout();
    auto bias_of = [&](int l) { return bias + (p.b[l] - p.bias_begin); };
    hipError_t e = hipSuccess;
    if (training) e = sg::prep_input(dn, depth, B, at<void>(ws, w.act[0]), s);
    for (int l = 0; l < 5 && e == hipSuccess; ++l) {
        void* out = l < 4 ? at<void>(ws, w.act[l + 1]) : at<void>(ws, w.a5);
        const bool patch = l == 0 && !training;
        e = sg::conv_forward(layer_geo(l, B), patch ? (const void*)dn : at<void>(ws, w.act[l]),
                             at<void>(wbase, k.wb[l]), bias_of(l), at<int4>(wbase, k.taps[l]), 0,
                             out, nullptr, nullptr, s, patch ? 1 : 0, depth);
    }
    if (e == hipSuccess && training)
        e = sg::upsample(at<void>(ws, w.a5), B, 16, 16, kHeadC, at<void>(ws, w.up), s);
    if (e == hipSuccess)
        e = sg::conv_forward(layer_geo(5, B),
                             training ? at<void>(ws, w.up) : at<void>(ws, w.a5),
                             at<void>(wbase, k.wb[5]), bias_of(5), at<int4>(wbase, k.taps[5]), 1,
                             nullptr, psf, z, s, training ? 0 : 2, depth);
    if (e == hipSuccess)
        e = sg::head_forward(at<void>(ws, w.a5), B, 16 * 16, kHeadC, bias + (p.we - p.bias_begin),
                             bias + (p.be - p.bias_begin), at<float>(ws, w.pooled),
                             at<float>(ws, w.epre), err, s);
    return e;
}

int check_ptr(const void* p, size_t align, const char* name) {
    if (!p) return fail(BPM_ERR_INVALID_ARG, "%s must be non-null", name);
    if (!aligned(p, align))
        return fail(BPM_ERR_INVALID_ARG, "%s must be %zu-byte aligned", name, align);
    return BPM_OK;
}

// Validation shared by the building-block entries.
int check_conv_geo(const int* geom, ConvGeo* c, bool data_grad) {
    if (!geom) return fail(BPM_ERR_INVALID_ARG, "geom must be non-null");
    if (!make_geo(geom, c))
        return fail(BPM_ERR_INVALID_ARG, "degenerate convolution geometry");
    if (c->Ci % 8 != 0 || (data_grad && c->Ci % 32 != 0))
        return fail(BPM_ERR_UNSUPPORTED_SIZE, "Ci=%d must be a multiple of %d", c->Ci,
                    data_grad ? 32 : 8);
    if (c->Co % 32 != 0 || 256 % c->Co != 0)
        return fail(BPM_ERR_UNSUPPORTED_SIZE, "Co=%d must be 32, 64, 128 or 256", c->Co);
    const double in = (double)c->N * c->D * c->H * c->W * c->Ci;
    const double out = (double)c->N * c->Do * c->Ho * c->Wo * c->Co;
    const double P = (double)c->N * c->Do * c->Ho * c->Wo;
    if (in > 2e9 || out > 2e9 || P > 65535.0 * 2048.0 || c->K > (1 << 24))
        return fail(BPM_ERR_UNSUPPORTED_SIZE, "convolution too large");
    if (c->Wo > 128 || sg::fwd_lds_bytes(*c) > sg::kMaxConvLds ||
        (double)c->N * c->Do * sg::fwd_tile(*c).tiles_y > 2e9)
        return fail(BPM_ERR_UNSUPPORTED_SIZE,
                    "Wo=%d: output rows of at most 128 and an input tile of at most %zu bytes",
                    c->Wo, sg::kMaxConvLds);
    return BPM_OK;
}

size_t conv_ws_bytes(const ConvGeo& c) {
    return align_up(2 * (size_t)c.Co * c.Kp) + align_up(2 * (size_t)c.Ci * c.taps * c.Co) +
           align_up(sizeof(int4) * (size_t)(c.K / 8)) +
           align_up(sizeof(int4) * (size_t)(c.taps * c.Co / 8));
}

struct ConvWs {
    void *wb, *wt;
    int4 *taps, *taps_t;
};
ConvWs conv_ws_carve(const ConvGeo& c, void* ws) {
    ConvWs r{};
    char* b = static_cast<char*>(ws);
    r.wb = b;
    b += align_up(2 * (size_t)c.Co * c.Kp);
    r.wt = b;
    b += align_up(2 * (size_t)c.Ci * c.taps * c.Co);
    r.taps = reinterpret_cast<int4*>(b);
    b += align_up(sizeof(int4) * (size_t)(c.K / 8));
    r.taps_t = reinterpret_cast<int4*>(b);
    return r;
}

}  // namespace

extern "C" {

size_t psf_surrogate_param_count(void) { return param_layout().total; }

int psf_surrogate_layer_geometry(int layer, int* geom_out) {
    if (layer < 0 || layer >= kLayers)
        return fail(BPM_ERR_INVALID_ARG, "layer=%d must be in [0, %d)", layer, kLayers);
    if (!geom_out) return fail(BPM_ERR_INVALID_ARG, "geom_out must be non-null");
    const LayerSpec& s = kSpec[layer];
    const int g[15] = {1, s.D, s.H, s.W, s.Ci, s.Co, s.kd, s.kh, s.kw,
                       s.sd, s.sh, s.sw, s.pd, s.ph, s.pw};
    for (int i = 0; i < 15; ++i) geom_out[i] = g[i];
    return BPM_OK;
}
size_t psf_surrogate_weights_bytes(void) { return blob_layout().total; }
size_t psf_surrogate_state_bytes(void) { return state_layout().total; }

size_t psf_surrogate_workspace_size(int batch, int training) {
    if (batch < 0) return 0;
    if (training) return ws_layout(batch < 1 ? 1 : batch, true).total;
    const int chunk = batch < kInferChunk ? (batch < 1 ? 1 : batch) : kInferChunk;
    return ws_layout(chunk, false).total;
}

int psf_surrogate_train_init(void* state, const float* init_params, void* hip_stream) {
    if (int rc = check_ptr(state, kAlign, "state")) return rc;
    if (int rc = check_ptr(init_params, 4, "init_params")) return rc;
    const hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const StateLayout L = state_layout();
    const size_t n = param_layout().total;
    hipError_t e = hipMemcpyAsync(at<float>(state, L.params), init_params, sizeof(float) * n,
                                  hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = sg::fill_zero(at<float>(state, L.grads), (long)n, s);
    if (e == hipSuccess) e = sg::fill_zero(at<float>(state, L.m), (long)n, s);
    if (e == hipSuccess) e = sg::fill_zero(at<float>(state, L.v), (long)n, s);
    if (e == hipSuccess) e = tables_all(state, L.pack, true, s);
    if (e == hipSuccess) e = pack_all(at<float>(state, L.params), state, L.pack, true, s);
    return device_status(e, "surrogate init");
}

int psf_surrogate_train_step(void* state, const float* dn, const float* depth,
                             const float* target, int batch, float lr, float err_weight, int step,
                             float* loss_out, float* err_true, void* workspace,
                             size_t workspace_bytes, void* hip_stream) {
    if (int rc = check_ptr(state, kAlign, "state")) return rc;
    if (batch < 1 || batch > kMaxTrainBatch)
        return fail(BPM_ERR_INVALID_ARG, "batch=%d must be in [1, %d]", batch, kMaxTrainBatch);
    if (int rc = check_ptr(dn, 4, "dn")) return rc;
    if (int rc = check_ptr(depth, 4, "depth")) return rc;
    if (int rc = check_ptr(target, 4, "target")) return rc;
    if (int rc = check_ptr(loss_out, 4, "loss_out")) return rc;
    if (err_true && !aligned(err_true, 4))
        return fail(BPM_ERR_INVALID_ARG, "err_true must be 4-byte aligned");
    if (!(lr >= 0.f) || !(err_weight >= 0.f) || !std::isfinite(lr) || !std::isfinite(err_weight))
        return fail(BPM_ERR_NOT_FINITE, "lr=%g and err_weight=%g must be finite and >= 0",
                    (double)lr, (double)err_weight);
    if (lr > 0.f && step < 1)
        return fail(BPM_ERR_INVALID_ARG, "step=%d must be >= 1 for an update", step);
    const WsLayout w = ws_layout(batch, true);
    if (int rc = check_workspace(workspace, workspace_bytes, w.total)) return rc;
    const hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const StateLayout L = state_layout();
    const ParamLayout p = param_layout();
    const int B = batch;
    float* params = at<float>(state, L.params);
    float* grads = at<float>(state, L.grads);
    void* ws = workspace;

    hipError_t e = forward(state, L.pack, params + p.bias_begin, dn, depth, B, ws, w,
                           at<float>(ws, w.psf), at<float>(ws, w.z), at<float>(ws, w.err), s,
                           true);
    if (e == hipSuccess) e = sg::fill_zero(grads, (long)p.total, s);
    if (e == hipSuccess) e = sg::fill_zero(loss_out, 2, s);
    if (e == hipSuccess)
        e = sg::loss_and_grad(at<float>(ws, w.psf), at<float>(ws, w.z), target,
                              at<float>(ws, w.epre), at<float>(ws, w.err), B, err_weight,
                              at<void>(ws, w.gd[5]), at<float>(ws, w.derr), loss_out, err_true, s);
    if (e == hipSuccess)
        e = sg::head_backward(at<float>(ws, w.pooled), at<float>(ws, w.derr), params + p.we, B,
                              kHeadC, grads + p.we, grads + p.be, at<float>(ws, w.dpool), s);
    // d2: weights from the upsampled map, data gradient back to it
    if (e == hipSuccess) {
        const ConvGeo c = layer_geo(5, B);
        e = sg::conv_backward_weight(c, at<void>(ws, w.up), at<void>(ws, w.gd[5]),
                                     at<int4>(state, L.pack.taps[5]), grads + p.w[5],
                                     grads + p.b[5], s);
        if (e == hipSuccess)
            e = sg::conv_backward_data(c, at<void>(ws, w.gd[5]), at<void>(state, L.pack.wt[5]),
                                       nullptr, at<int4>(state, L.pack.taps_t[5]),
                                       at<void>(ws, w.du), s);
    }
    if (e == hipSuccess)
        e = sg::upsample_backward(at<void>(ws, w.du), at<void>(ws, w.a5), at<float>(ws, w.dpool),
                                  B, 16, 16, kHeadC, at<void>(ws, w.gd[4]), s);
    for (int l = 4; l >= 0 && e == hipSuccess; --l) {
        const ConvGeo c = layer_geo(l, B);
        e = sg::conv_backward_weight(c, at<void>(ws, w.act[l]), at<void>(ws, w.gd[l]),
                                     at<int4>(state, L.pack.taps[l]), grads + p.w[l],
                                     grads + p.b[l], s);
        if (e == hipSuccess && l > 0)  // the input of layer l is the ReLU output of layer l - 1
            e = sg::conv_backward_data(c, at<void>(ws, w.gd[l]), at<void>(state, L.pack.wt[l]),
                                       at<void>(ws, w.act[l]), at<int4>(state, L.pack.taps_t[l]),
                                       at<void>(ws, w.gd[l - 1]), s);
    }
    if (e == hipSuccess && lr > 0.f) {
        e = sg::adam_update(params, grads, at<float>(state, L.m), at<float>(state, L.v),
                            (long)p.total, lr, step, s);
        if (e == hipSuccess) e = pack_all(params, state, L.pack, true, s);
    }
    return device_status(e, "surrogate train step");
}

int psf_surrogate_gradients(const void* state, float* grads_out, void* hip_stream) {
    if (int rc = check_ptr(state, kAlign, "state")) return rc;
    if (int rc = check_ptr(grads_out, 4, "grads_out")) return rc;
    return device_status(hipMemcpyAsync(grads_out, at<float>(state, state_layout().grads),
                                        sizeof(float) * param_layout().total,
                                        hipMemcpyDeviceToDevice,
                                        static_cast<hipStream_t>(hip_stream)),
                         "surrogate gradients");
}

int psf_surrogate_params(const void* state, float* params_out, void* hip_stream) {
    if (int rc = check_ptr(state, kAlign, "state")) return rc;
    if (int rc = check_ptr(params_out, 4, "params_out")) return rc;
    return device_status(hipMemcpyAsync(params_out, at<float>(state, state_layout().params),
                                        sizeof(float) * param_layout().total,
                                        hipMemcpyDeviceToDevice,
                                        static_cast<hipStream_t>(hip_stream)),
                         "surrogate params");
}

int psf_surrogate_export(const void* state, void* weights_blob, void* hip_stream) {
    if (int rc = check_ptr(state, kAlign, "state")) return rc;
    if (int rc = check_ptr(weights_blob, kAlign, "weights_blob")) return rc;
    const hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const StateLayout L = state_layout();
    const BlobLayout b = blob_layout();
    const ParamLayout p = param_layout();
    hipError_t e = hipMemcpyAsync(at<void>(weights_blob, b.bias),
                                  at<float>(state, L.params) + p.bias_begin,
                                  sizeof(float) * (p.total - p.bias_begin),
                                  hipMemcpyDeviceToDevice, s);
    for (int l = 0; l < kLayers && e == hipSuccess; ++l) {
        const ConvGeo c = layer_geo(l, 1);
        e = hipMemcpyAsync(at<void>(weights_blob, b.pack.wb[l]), at<void>(state, L.pack.wb[l]),
                           2 * (size_t)c.Co * c.Kp, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(at<void>(weights_blob, b.pack.taps[l]),
                               at<void>(state, L.pack.taps[l]), sizeof(int4) * (size_t)(c.K / 8),
                               hipMemcpyDeviceToDevice, s);
    }
    return device_status(e, "surrogate export");
}

int psf_surrogate_infer(const void* weights_bf16, size_t weights_bytes, const float* dn_patches,
                        const float* depth, int batch, float* psf_out, float* pred_err,
                        void* workspace, size_t workspace_bytes, void* hip_stream) {
    if (int rc = check_ptr(weights_bf16, kAlign, "weights")) return rc;
    const BlobLayout b = blob_layout();
    if (weights_bytes != b.total)
        return fail(BPM_ERR_INVALID_ARG, "weights_bytes=%zu; this network's blob has %zu bytes",
                    weights_bytes, b.total);
    if (batch < 0) return fail(BPM_ERR_INVALID_ARG, "batch=%d must be >= 0", batch);
    if (batch == 0) return BPM_OK;
    if (int rc = check_ptr(dn_patches, 4, "dn_patches")) return rc;
    if (int rc = check_ptr(depth, 4, "depth")) return rc;
    if (int rc = check_ptr(psf_out, 4, "psf_out")) return rc;
    if (int rc = check_ptr(pred_err, 4, "pred_err")) return rc;
    const int chunk = batch < kInferChunk ? batch : kInferChunk;
    const WsLayout w = ws_layout(chunk, false);
    if (int rc = check_workspace(workspace, workspace_bytes, w.total)) return rc;
    const hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const size_t per_dn = (size_t)kPatchD * kPatchHW * kPatchHW;
    const size_t per_psf = (size_t)kPlanes * kPatchHW * kPatchHW;
    hipError_t e = hipSuccess;
    for (int n0 = 0; n0 < batch && e == hipSuccess; n0 += chunk) {
        const int B = batch - n0 < chunk ? batch - n0 : chunk;
        e = forward(weights_bf16, b.pack, at<float>(weights_bf16, b.bias), dn_patches + n0 * per_dn,
                    depth + n0, B, workspace, w, psf_out + n0 * per_psf, nullptr, pred_err + n0, s,
                    false);
    }
    return device_status(e, "surrogate inference");
}

int psf_extract_patches(const float* dn, int nz, int ny, int nx, int z0, const int* sources,
                        int n, float* patches, void* hip_stream) {
    if (ny < kPatchHW || nx < kPatchHW || z0 < 0 || z0 + kPatchD > nz)
        return fail(BPM_ERR_INVALID_ARG,
                    "nz=%d ny=%d nx=%d z0=%d: need ny, nx >= %d and z0 + %d <= nz", nz, ny, nx,
                    z0, kPatchHW, kPatchD);
    if ((double)nz * ny * nx > 4e10) return fail(BPM_ERR_UNSUPPORTED_SIZE, "dn volume too large");
    if (n < 0) return fail(BPM_ERR_INVALID_ARG, "n=%d must be >= 0", n);
    if (n == 0) return BPM_OK;
    if (int rc = check_ptr(dn, 4, "dn")) return rc;
    if (int rc = check_ptr(sources, 4, "sources")) return rc;
    if (int rc = check_ptr(patches, 16, "patches")) return rc;
    return device_status(sg::extract_patches(dn, ny, nx, z0, sources, n, patches,
                                             static_cast<hipStream_t>(hip_stream)),
                         "extract patches");
}

size_t psf_conv_workspace_size(const int* geom) {
    ConvGeo c{};
    if (!geom || !make_geo(geom, &c)) return 0;
    return conv_ws_bytes(c);
}

int psf_conv_forward(const void* x, const float* w, const float* bias, const int* geom,
                     int epilogue, void* y_bf16, float* y_f32, float* z_f32, void* workspace,
                     size_t workspace_bytes, void* hip_stream) {
    ConvGeo c{};
    if (int rc = check_conv_geo(geom, &c, false)) return rc;
    if (int rc = check_ptr(x, 16, "x")) return rc;
    if (int rc = check_ptr(w, 4, "w")) return rc;
    if (int rc = check_ptr(bias, 4, "bias")) return rc;
    if (epilogue == 0) {
        if (int rc = check_ptr(y_bf16, 8, "y_bf16")) return rc;
    } else if (epilogue == 1) {
        if (c.Do != 1) return fail(BPM_ERR_INVALID_ARG, "epilogue 1 needs Do == 1 (Do=%d)", c.Do);
        if (int rc = check_ptr(y_f32, 4, "y_f32")) return rc;
        if (z_f32 && !aligned(z_f32, 4))
            return fail(BPM_ERR_INVALID_ARG, "z_f32 must be 4-byte aligned");
    } else {
        return fail(BPM_ERR_INVALID_ARG, "epilogue=%d must be 0 or 1", epilogue);
    }
    if (int rc = check_workspace(workspace, workspace_bytes, conv_ws_bytes(c))) return rc;
    const hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const ConvWs k = conv_ws_carve(c, workspace);
    hipError_t e = sg::tap_tables(c, k.taps, nullptr, s);
    if (e == hipSuccess) e = sg::pack_weights(w, c.Co, c.Ci, c.taps, c.Kp, k.wb, nullptr, s);
    if (e == hipSuccess)
        e = sg::conv_forward(c, x, k.wb, bias, k.taps, epilogue, y_bf16, y_f32, z_f32, s);
    return device_status(e, "conv forward");
}

int psf_conv_backward(const void* x, const float* w, const void* dy, const void* xmask,
                      const int* geom, void* dx, float* dw, float* db, void* workspace,
                      size_t workspace_bytes, void* hip_stream) {
    ConvGeo c{};
    if (int rc = check_conv_geo(geom, &c, dx != nullptr)) return rc;
    if (int rc = check_ptr(dy, 16, "dy")) return rc;
    if (dx) {
        if (int rc = check_ptr(w, 4, "w")) return rc;
        if (int rc = check_ptr(dx, 8, "dx")) return rc;
        if (xmask && !aligned(xmask, 2))
            return fail(BPM_ERR_INVALID_ARG, "xmask must be 2-byte aligned");
    }
    if (dw) {
        if (int rc = check_ptr(x, 2, "x")) return rc;
        if (!aligned(dw, 4)) return fail(BPM_ERR_INVALID_ARG, "dw must be 4-byte aligned");
    }
    if (db && !aligned(db, 4)) return fail(BPM_ERR_INVALID_ARG, "db must be 4-byte aligned");
    if (int rc = check_workspace(workspace, workspace_bytes, conv_ws_bytes(c))) return rc;
    const hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const ConvWs k = conv_ws_carve(c, workspace);
    hipError_t e = sg::tap_tables(c, k.taps, k.taps_t, s);
    if (e == hipSuccess && dw) e = sg::fill_zero(dw, (long)c.Co * c.Kp, s);
    if (e == hipSuccess && db) e = sg::fill_zero(db, c.Co, s);
    if (e == hipSuccess && (dw || db))
        e = sg::conv_backward_weight(c, x, dy, k.taps, dw, db, s);
    if (e == hipSuccess && dx) {
        e = sg::pack_weights(w, c.Co, c.Ci, c.taps, c.Kp, k.wb, k.wt, s);
        if (e == hipSuccess) e = sg::conv_backward_data(c, dy, k.wt, xmask, k.taps_t, dx, s);
    }
    return device_status(e, "conv backward");
}

}  // extern "C"
