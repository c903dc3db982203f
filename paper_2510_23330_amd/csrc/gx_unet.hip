// gx_unet.hip -- the supernova surrogate's 3-D U-Net (Sec. 3.3) as whole-
// network calls: the layer sequence of the forward pass (inference or
// training) and of the backward pass, run in C++ over the convolution,
// pooling, upsampling and concatenation blocks of gx_nn.hip, plus the
// channel standardisation coefficients of the network's inputs and targets.
//
// Network (per level l < L: 2 3^3 convolutions with bias and LeakyReLU 0.1;
// 2^3 average pooling down; nearest x2 upsampling + 3^3 convolution up; skip
// by channel concatenation; a linear 1^3 head).  Layer order, which also
// fixes the flat parameter layout (every layer's weights [Cout][kvol][Cin],
// then every layer's bias):
//   e0a e0b e1a e1b ... e{L-1}a e{L-1}b, then for l = L-2 .. 0: u{l}c d{l}a
//   d{l}b, then head.
// Activations are held in the context (grow-only scratch) from a forward
// pass with save = 1 until the next forward pass; the backward pass reads
// them.
#include "gx_internal.hpp"

#include <cmath>
#include <cstring>
#include <map>
#include <set>
#include <string>
#include <vector>

// fused backward steps (gx_nn.hip); channel counts multiples of 8
int gx_split_dact(gx_ctx* ctx, const uint16_t* gc, int64_t V, int Ca, int Cb, const uint16_t* ya,
                  uint16_t* ga, uint16_t* gb);
int gx_upsample2_bwd_dact(gx_ctx* ctx, const uint16_t* dout, int B, int S, int C,
                          const uint16_t* y, uint16_t* din);
int gx_avgpool2_bwd_combine(gx_ctx* ctx, const uint16_t* dout, int B, int S, int C,
                            const uint16_t* skip, const uint16_t* y, uint16_t* din);

namespace {

struct ULayer {
    std::string name;
    int cin, cout, ksize, act;
    int64_t w_off, b_off;
    int64_t n_w() const { return (int64_t)cout * (ksize == 3 ? 27 : 1) * cin; }
};

int unet_layers(int levels, int base, int cin, int cout, std::vector<ULayer>& L, int64_t* n_par) {
    if (levels < 2 || levels > 6 || base < 16 || base % 16 || cin < 8 || cin % 8 || cout < 16 ||
        cout % 16)
        return GX_EINVAL;
    L.clear();
    std::vector<int> ch(levels);
    for (int l = 0; l < levels; l++) ch[l] = base << l;
    int c = cin;
    for (int l = 0; l < levels; l++) {
        L.push_back({"e" + std::to_string(l) + "a", c, ch[l], 3, 1, 0, 0});
        L.push_back({"e" + std::to_string(l) + "b", ch[l], ch[l], 3, 1, 0, 0});
        c = ch[l];
    }
    for (int l = levels - 2; l >= 0; l--) {
        L.push_back({"u" + std::to_string(l) + "c", ch[l + 1], ch[l], 3, 1, 0, 0});
        L.push_back({"d" + std::to_string(l) + "a", 2 * ch[l], ch[l], 3, 1, 0, 0});
        L.push_back({"d" + std::to_string(l) + "b", ch[l], ch[l], 3, 1, 0, 0});
    }
    L.push_back({"head", ch[0], cout, 1, 0, 0, 0});
    int64_t off = 0;
    for (auto& ly : L) {
        ly.w_off = off;
        off += ly.n_w();
    }
    for (auto& ly : L) {
        ly.b_off = off;
        off += ly.cout;
    }
    *n_par = off;
    return GX_OK;
}

}  // namespace

// Per-context network state: the saved activations and gradients by name.
struct gx_unet_state {
    int levels = 0, base = 0, cin = 0, cout = 0, B = 0, S = 0, saved = 0;
    std::map<std::string, Buf> act, grad;
    std::set<std::string> fresh_act, fresh_grad;  // written by the last pass
};

static gx_unet_state& ustate(gx_ctx* ctx) {
    if (!ctx->unet) ctx->unet = new gx_unet_state();
    return *ctx->unet;
}

void gx_unet_free(gx_ctx* ctx) {
    if (!ctx->unet) return;
    for (auto* m : {&ctx->unet->act, &ctx->unet->grad})
        for (auto& kv : *m)
            if (kv.second.p) (void)hipFree(kv.second.p);
    delete ctx->unet;
    ctx->unet = nullptr;
}

static int ubuf(gx_ctx* ctx, std::map<std::string, Buf>& m, std::set<std::string>& fresh,
                const std::string& name, int64_t elems, uint16_t** out) {
    GX_TRY(gx_reserve(ctx, m[name], (size_t)elems * sizeof(uint16_t)));
    *out = (uint16_t*)m[name].p;
    fresh.insert(name);
    return GX_OK;
}

extern "C" int gx_unet_sizes(int levels, int base, int cin, int cout, int64_t* n_params,
                             int64_t* n_layers) {
    std::vector<ULayer> L;
    int64_t n = 0;
    int rc = unet_layers(levels, base, cin, cout, L, &n);
    if (rc != GX_OK) return rc;
    if (n_params) *n_params = n;
    if (n_layers) *n_layers = (int64_t)L.size();
    return GX_OK;
}

extern "C" int gx_unet_layer(int levels, int base, int cin, int cout, int index, char* name,
                             int name_cap, int* lcin, int* lcout, int* ksize, int64_t* w_off,
                             int64_t* b_off) {
    std::vector<ULayer> L;
    int64_t n = 0;
    int rc = unet_layers(levels, base, cin, cout, L, &n);
    if (rc != GX_OK) return rc;
    if (index < 0 || index >= (int)L.size()) return GX_EINVAL;
    const ULayer& ly = L[index];
    if (name && name_cap > 0) {
        std::strncpy(name, ly.name.c_str(), (size_t)name_cap - 1);
        name[name_cap - 1] = 0;
    }
    if (lcin) *lcin = ly.cin;
    if (lcout) *lcout = ly.cout;
    if (ksize) *ksize = ly.ksize;
    if (w_off) *w_off = ly.w_off;
    if (b_off) *b_off = ly.b_off;
    return GX_OK;
}

extern "C" int gx_unet_forward(gx_ctx* ctx, const gx_unet* net, const uint16_t* in, int B, int S,
                               int save, float* out_f32, int nc, const float* scale,
                               const float* shift, float* out_phys) {
    if (!ctx || !net || !net->w_bf16 || !net->w_f32 || !in || B < 1 || (!out_f32 && !out_phys))
        return GX_EINVAL;
    if (out_phys && (!scale || !shift || nc < 1 || nc > net->cout)) return GX_EINVAL;
    std::vector<ULayer> L;
    int64_t npar = 0;
    if (unet_layers(net->levels, net->base, net->cin, net->cout, L, &npar) != GX_OK)
        return gx_fail(ctx, GX_EINVAL, "unet_forward: bad network description");
    if (S < (1 << (net->levels - 1)) || S % (1 << (net->levels - 1)))
        return gx_fail(ctx, GX_EINVAL, "unet_forward: S = %d not divisible by 2^(levels-1)", S);
    std::map<std::string, const ULayer*> by;
    for (auto& ly : L) by[ly.name] = &ly;
    gx_unet_state& st = ustate(ctx);
    st.saved = 0;
    st.S = 0;
    st.fresh_act.clear();
    st.fresh_grad.clear();
    const int lv = net->levels;
    auto w = [&](const char* nm) { return net->w_bf16 + by.at(nm)->w_off; };
    auto b = [&](const char* nm) { return net->w_f32 + by.at(nm)->b_off; };
    auto A = [&](const std::string& nm, int64_t elems, uint16_t** p) {
        return ubuf(ctx, st.act, st.fresh_act, nm, elems, p);
    };
    std::vector<int> ch(lv);
    for (int l = 0; l < lv; l++) ch[l] = net->base << l;
    const uint16_t* h = in;
    for (int l = 0; l < lv; l++) {
        const int s = S >> l;
        const int64_t V = (int64_t)B * s * s * s;
        const std::string ea = "e" + std::to_string(l) + "a", eb = "e" + std::to_string(l) + "b";
        uint16_t *pa, *pb;
        GX_TRY(A(ea, V * ch[l], &pa));
        GX_TRY(A(eb, V * ch[l], &pb));
        const ULayer& la = *by.at(ea);
        GX_TRY(gx_conv3d_fwd(ctx, h, B, s, la.cin, w(ea.c_str()), b(ea.c_str()), 3, la.cout, 1, pa,
                             nullptr));
        if (l < lv - 1) {  // the pooled copy comes from the same launch
            uint16_t* pp;
            GX_TRY(A("p" + std::to_string(l), V / 8 * ch[l], &pp));
            GX_TRY(gx_conv3d_fwd_pool(ctx, pa, B, s, ch[l], w(eb.c_str()), b(eb.c_str()), ch[l], 1,
                                      pb, pp));
            h = pp;
        } else {
            GX_TRY(gx_conv3d_fwd(ctx, pa, B, s, ch[l], w(eb.c_str()), b(eb.c_str()), 3, ch[l], 1, pb,
                                 nullptr));
            h = pb;
        }
    }
    for (int l = lv - 2; l >= 0; l--) {
        const int s = S >> l;
        const int64_t V = (int64_t)B * s * s * s;
        const std::string ls = std::to_string(l);
        const std::string uc = "u" + ls + "c", da = "d" + ls + "a", db = "d" + ls + "b";
        uint16_t *pu, *pda, *pdb, *pe;
        GX_TRY(A(uc, V * ch[l], &pu));
        GX_TRY(A(da, V * ch[l], &pda));
        GX_TRY(A(db, V * ch[l], &pdb));
        pe = (uint16_t*)st.act["e" + ls + "b"].p;
        // the backward pass needs the upsampled and concatenated inputs of
        // the up path as copies only where its weight gradient cannot read
        // them from their sources (gx_wgrad_fused_ok)
        if (save && !gx_wgrad_fused_ok(s, ch[l + 1], ch[l])) {
            uint16_t* pup;
            GX_TRY(A("up" + ls, V * ch[l + 1], &pup));
            GX_TRY(gx_upsample2(ctx, h, B, s / 2, ch[l + 1], pup, 0));
            GX_TRY(gx_conv3d_fwd(ctx, pup, B, s, ch[l + 1], w(uc.c_str()), b(uc.c_str()), 3, ch[l], 1,
                                 pu, nullptr));
        } else {
            GX_TRY(gx_conv3d_fwd_fused(ctx, h, ch[l + 1], nullptr, 1, B, s, ch[l + 1], w(uc.c_str()),
                                       b(uc.c_str()), ch[l], 1, pu, nullptr));
        }
        if (save && !gx_wgrad_fused_ok(s, 2 * ch[l], ch[l])) {
            uint16_t* pc;
            GX_TRY(A("c" + ls, V * 2 * ch[l], &pc));
            GX_TRY(gx_concat(ctx, pu, ch[l], pe, ch[l], V, pc, 0));
            GX_TRY(gx_conv3d_fwd(ctx, pc, B, s, 2 * ch[l], w(da.c_str()), b(da.c_str()), 3, ch[l], 1,
                                 pda, nullptr));
        } else {
            GX_TRY(gx_conv3d_fwd_fused(ctx, pu, ch[l], pe, 0, B, s, 2 * ch[l], w(da.c_str()),
                                       b(da.c_str()), ch[l], 1, pda, nullptr));
        }
        GX_TRY(gx_conv3d_fwd(ctx, pda, B, s, ch[l], w(db.c_str()), b(db.c_str()), 3, ch[l], 1, pdb,
                             nullptr));
        h = pdb;
    }
    if (out_phys)
        GX_TRY(gx_conv_head(ctx, h, B, S, ch[0], w("head"), b("head"), net->cout, nc, scale, shift,
                            out_phys, nc));
    if (out_f32)
        GX_TRY(gx_conv3d_fwd(ctx, h, B, S, ch[0], w("head"), b("head"), 1, net->cout, 0, nullptr,
                             out_f32));
    st.levels = lv;
    st.base = net->base;
    st.cin = net->cin;
    st.cout = net->cout;
    st.B = B;
    st.S = S;
    st.saved = save ? 1 : 0;
    return GX_OK;
}

extern "C" int gx_unet_backward(gx_ctx* ctx, const gx_unet* net, const uint16_t* in, int B, int S,
                                const uint16_t* dout, float* grad) {
    if (!ctx || !net || !net->w_bf16 || !in || !dout || !grad) return GX_EINVAL;
    std::vector<ULayer> L;
    int64_t npar = 0;
    if (unet_layers(net->levels, net->base, net->cin, net->cout, L, &npar) != GX_OK)
        return gx_fail(ctx, GX_EINVAL, "unet_backward: bad network description");
    gx_unet_state& st = ustate(ctx);
    if (!st.saved || st.levels != net->levels || st.base != net->base || st.cin != net->cin ||
        st.cout != net->cout || st.B != B || st.S != S)
        return gx_fail(ctx, GX_ESTALE,
                       "unet_backward: needs a saving forward pass of the same network and shape");
    st.fresh_grad.clear();
    std::map<std::string, const ULayer*> by;
    for (auto& ly : L) by[ly.name] = &ly;
    const int lv = net->levels, top = lv - 1;
    std::vector<int> ch(lv);
    for (int l = 0; l < lv; l++) ch[l] = net->base << l;
    auto act = [&](const std::string& nm) { return (uint16_t*)st.act.at(nm).p; };
    auto G = [&](const std::string& nm, int64_t elems, uint16_t** p) {
        return ubuf(ctx, st.grad, st.fresh_grad, nm, elems, p);
    };
    auto wgrad = [&](const std::string& nm, const uint16_t* x, const uint16_t* dy, int s) {
        const ULayer& ly = *by.at(nm);
        return gx_conv3d_bwd_weight(ctx, x, dy, B, s, ly.cin, ly.ksize, ly.cout, grad + ly.w_off,
                                    grad + ly.b_off);
    };
    auto dgrad = [&](const std::string& nm, const uint16_t* dy, int s, const uint16_t* y_in,
                     uint16_t* dx) {
        const ULayer& ly = *by.at(nm);
        return gx_conv3d_bwd_data(ctx, dy, B, s, ly.cin, net->w_bf16 + ly.w_off, ly.ksize, ly.cout,
                                  y_in, dx);
    };
    // gradient buffers (one per activation, plus the skip share of each level)
    std::map<std::string, uint16_t*> g;
    for (int l = 0; l < lv; l++) {
        const int s = S >> l;
        const int64_t V = (int64_t)B * s * s * s;
        const std::string ls = std::to_string(l);
        GX_TRY(G("e" + ls + "a", V * ch[l], &g["e" + ls + "a"]));
        GX_TRY(G("e" + ls + "b", V * ch[l], &g["e" + ls + "b"]));
        if (l < lv - 1) {
            GX_TRY(G("p" + ls, V / 8 * ch[l], &g["p" + ls]));
            GX_TRY(G("skip" + ls, V * ch[l], &g["skip" + ls]));
            GX_TRY(G("up" + ls, V * ch[l + 1], &g["up" + ls]));
            GX_TRY(G("c" + ls, V * 2 * ch[l], &g["c" + ls]));
            GX_TRY(G("u" + ls + "c", V * ch[l], &g["u" + ls + "c"]));
            GX_TRY(G("d" + ls + "a", V * ch[l], &g["d" + ls + "a"]));
            GX_TRY(G("d" + ls + "b", V * ch[l], &g["d" + ls + "b"]));
        }
    }
    // head
    GX_TRY(wgrad("head", act("d0b"), dout, S));
    GX_TRY(dgrad("head", dout, S, act("d0b"), g["d0b"]));
    // decoder, finest level first
    for (int l = 0; l < top; l++) {
        const int s = S >> l;
        const int64_t V = (int64_t)B * s * s * s;
        const std::string ls = std::to_string(l);
        const std::string uc = "u" + ls + "c", da = "d" + ls + "a", db = "d" + ls + "b";
        GX_TRY(wgrad(db, act(da), g[db], s));
        GX_TRY(dgrad(db, g[db], s, act(da), g[da]));
        if (gx_wgrad_fused_ok(s, 2 * ch[l], ch[l])) {
            const ULayer& ly = *by.at(da);
            GX_TRY(gx_conv3d_bwd_weight_fused(ctx, act(uc), ch[l], act("e" + ls + "b"), 0, g[da], B,
                                              s, ly.cin, ly.ksize, ly.cout, grad + ly.w_off,
                                              grad + ly.b_off));
        } else {
            GX_TRY(wgrad(da, act("c" + ls), g[da], s));
        }
        GX_TRY(dgrad(da, g[da], s, nullptr, g["c" + ls]));
        if (ch[l] % 8 == 0) {
            GX_TRY(gx_split_dact(ctx, g["c" + ls], V, ch[l], ch[l], act(uc), g[uc],
                                 g["skip" + ls]));
        } else {
            GX_TRY(gx_concat(ctx, g[uc], ch[l], g["skip" + ls], ch[l], V, g["c" + ls], 1));
            GX_TRY(gx_grad_combine(ctx, V * ch[l], g[uc], nullptr, act(uc), g[uc]));
        }
        // the coarser level's output, whose upsampling is this layer's input
        const std::string below =
            l + 1 < top ? "d" + std::to_string(l + 1) + "b" : "e" + std::to_string(top) + "b";
        if (gx_wgrad_fused_ok(s, ch[l + 1], ch[l])) {
            const ULayer& ly = *by.at(uc);
            GX_TRY(gx_conv3d_bwd_weight_fused(ctx, act(below), ch[l + 1], nullptr, 1, g[uc], B, s,
                                              ly.cin, ly.ksize, ly.cout, grad + ly.w_off,
                                              grad + ly.b_off));
        } else {
            GX_TRY(wgrad(uc, act("up" + ls), g[uc], s));
        }
        GX_TRY(dgrad(uc, g[uc], s, nullptr, g["up" + ls]));
        // into the next coarser level's output
        const int sc = s / 2;
        const int64_t Vc = (int64_t)B * sc * sc * sc;
        if (ch[l + 1] % 8 == 0) {
            GX_TRY(gx_upsample2_bwd_dact(ctx, g["up" + ls], B, sc, ch[l + 1], act(below),
                                         g[below]));
        } else {
            GX_TRY(gx_upsample2(ctx, g["up" + ls], B, sc, ch[l + 1], g[below], 1));
            GX_TRY(gx_grad_combine(ctx, Vc * ch[l + 1], g[below], nullptr, act(below), g[below]));
        }
    }
    // encoder, coarsest level first
    for (int l = top; l >= 0; l--) {
        const int s = S >> l;
        const std::string ls = std::to_string(l);
        const std::string ea = "e" + ls + "a", eb = "e" + ls + "b";
        GX_TRY(wgrad(eb, act(ea), g[eb], s));
        GX_TRY(dgrad(eb, g[eb], s, act(ea), g[ea]));
        if (l == 0) {
            GX_TRY(wgrad("e0a", in, g["e0a"], s));
            break;
        }
        const std::string pl = "p" + std::to_string(l - 1), ebl = "e" + std::to_string(l - 1) + "b";
        GX_TRY(wgrad(ea, act(pl), g[ea], s));
        GX_TRY(dgrad(ea, g[ea], s, nullptr, g[pl]));
        // through the pooling into level l-1's output, plus its skip gradient
        const int sf = 2 * s;
        const int64_t Vf = (int64_t)B * sf * sf * sf;
        if (ch[l - 1] % 8 == 0) {
            GX_TRY(gx_avgpool2_bwd_combine(ctx, g[pl], B, sf, ch[l - 1],
                                           g["skip" + std::to_string(l - 1)], act(ebl), g[ebl]));
        } else {
            GX_TRY(gx_avgpool2(ctx, g[pl], B, sf, ch[l - 1], g[ebl], 1));
            GX_TRY(gx_grad_combine(ctx, Vf * ch[l - 1], g[ebl], g["skip" + std::to_string(l - 1)],
                                   act(ebl), g[ebl]));
        }
    }
    return GX_OK;
}

extern "C" int gx_unet_saved(gx_ctx* ctx, const char* name, int gradient, uint16_t* dst,
                             int64_t cap, int64_t* count) {
    if (!ctx || !name || !count || cap < 0) return GX_EINVAL;
    gx_unet_state& st = ustate(ctx);
    if (st.S == 0) return gx_fail(ctx, GX_ESTALE, "unet_saved: no forward pass");
    auto& m = gradient ? st.grad : st.act;
    auto& fresh = gradient ? st.fresh_grad : st.fresh_act;
    auto it = m.find(name);
    const std::string nm = name;
    // the up path's upsampled ("up{l}") and concatenated ("c{l}") inputs are
    // kept only where their weight gradient cannot read them from their
    // sources; otherwise they are formed again here from the kept activations
    const bool rebuild = !gradient && (it == m.end() || !fresh.count(name)) &&
                         (nm.rfind("up", 0) == 0 || (nm[0] == 'c' && nm.size() > 1));
    if (!rebuild && (it == m.end() || !fresh.count(name)))
        return gx_fail(ctx, GX_EINVAL, "unet_saved: %s not written by the last pass", name);
    // element count of the tensor at the last pass's shape
    const int lv = st.levels;
    int l = -1;
    int64_t cmul = 1;
    if (nm.rfind("skip", 0) == 0) l = std::atoi(nm.c_str() + 4);
    else if (nm.rfind("up", 0) == 0) {
        l = std::atoi(nm.c_str() + 2);
        cmul = -1;  // channels of the level below
    } else l = std::atoi(nm.c_str() + 1);
    if (l < 0 || l >= lv) return gx_fail(ctx, GX_EINVAL, "unet_saved: bad name %s", name);
    int s = st.S >> l;
    int64_t C = (int64_t)st.base << l;
    if (nm[0] == 'p') s /= 2;
    if (nm[0] == 'c') C *= 2;
    if (cmul < 0) C = (int64_t)st.base << (l + 1);
    const int64_t n = (int64_t)st.B * s * s * s * C;
    *count = n;
    if (!dst) return GX_OK;
    if (cap < n) return gx_fail(ctx, GX_EINVAL, "unet_saved: %s needs %lld elements", name, (long long)n);
    if (rebuild) {
        if (l >= lv - 1) return gx_fail(ctx, GX_EINVAL, "unet_saved: bad name %s", name);
        const int top = lv - 1;
        auto kept = [&](const std::string& k) -> uint16_t* {
            auto a = st.act.find(k);
            return (a != st.act.end() && st.fresh_act.count(k)) ? (uint16_t*)a->second.p : nullptr;
        };
        const std::string ls = std::to_string(l);
        if (nm[0] == 'u') {
            const std::string below =
                l + 1 < top ? "d" + std::to_string(l + 1) + "b" : "e" + std::to_string(top) + "b";
            uint16_t* src = kept(below);
            if (!src) return gx_fail(ctx, GX_EINVAL, "unet_saved: %s not written by the last pass", name);
            return gx_upsample2(ctx, src, st.B, s / 2, (int)C, dst, 0);
        }
        uint16_t *pu = kept("u" + ls + "c"), *pe = kept("e" + ls + "b");
        if (!pu || !pe) return gx_fail(ctx, GX_EINVAL, "unet_saved: %s not written by the last pass", name);
        const int64_t V = (int64_t)st.B * s * s * s;
        return gx_concat(ctx, pu, (int)(C / 2), pe, (int)(C / 2), V, dst, 0);
    }
    GX_HIP(ctx, hipMemcpyAsync(dst, it->second.p, (size_t)n * sizeof(uint16_t),
                               hipMemcpyDeviceToDevice, ctx->stream));
    return GX_OK;
}

// ---------------------------------------------------------------------------
// Standardisation coefficients from FP64 channel sums (gx_chan_stats): mean,
// standard deviation floored at min_std, and the affine maps x -> (x - mean)
// / std (scale = 1 / std, shift = -mean / std).
// ---------------------------------------------------------------------------
__global__ void k_chan_moments(const double* __restrict__ sums, int nc, double count,
                               double min_std, float* __restrict__ mean, float* __restrict__ sd,
                               float* __restrict__ scale, float* __restrict__ shift) {
    const int c = threadIdx.x;
    if (c >= nc) return;
    const double m = sums[c] / count;
    const double var = fmax(sums[nc + c] / count - m * m, 0.0);
    const double s = fmax(sqrt(var), min_std);
    if (mean) mean[c] = (float)m;
    if (sd) sd[c] = (float)s;
    if (scale) scale[c] = (float)(1.0 / s);
    if (shift) shift[c] = (float)(-m / s);
}

extern "C" int gx_chan_moments(gx_ctx* ctx, const double* sums, int nc, double count,
                               double min_std, float* mean, float* std_out, float* scale,
                               float* shift) {
    if (!ctx || !sums || nc < 1 || nc > 64 || !(count > 0) || !(min_std >= 0)) return GX_EINVAL;
    GX_HIP(ctx, hipSetDevice(ctx->device));
    hipLaunchKernelGGL(k_chan_moments, dim3(1), dim3(64), 0, ctx->stream, sums, nc, count, min_std,
                       mean, std_out, scale, shift);
    GX_LAUNCH_CHECK(ctx);
    return GX_OK;
}
