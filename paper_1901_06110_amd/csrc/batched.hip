// Batched DSG-NLM forward over images of uneven sizes: one launch per sweep
// for the whole batch.  Blocks index a flat tile list that spans every image,
// so small and large images share the machine and each image keeps its own
// maximum row sum m (one packed key per image).
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "internal.h"

namespace dsnlm {

int check_denoiser_args(int n1, int n2, int S, int P, float h, const char* who);
bool overlaps(const void* a, const void* b, size_t bytes);

namespace {

// Grow-only device workspace reused across calls (per process).
struct BatchWorkspace {
    std::mutex mu;
    float* arrays = nullptr;  // c, delta, B' for every image
    size_t arrays_cap = 0;    // floats
    unsigned long long* keys = nullptr;
    size_t keys_cap = 0;
    ImgDesc* descs = nullptr;
    size_t descs_cap = 0;
    TileRef* tiles = nullptr;
    size_t tiles_cap = 0;
    float* part = nullptr;    // partial buffers of the half-window sweeps
    size_t part_cap = 0;
    std::vector<ImgDesc> last_descs;
    std::vector<TileRef> last_tiles;
    int last_S = -1, last_P = -1;  // of the last forward (for the backward)
};

BatchWorkspace g_ws;

template <class T>
hipError_t grow(T** p, size_t* cap, size_t need) {
    if (need <= *cap) return hipSuccess;
    if (*p) {
        hipError_t e = hipFree(*p);
        if (e != hipSuccess) return e;
        *p = nullptr;
    }
    size_t n = need + need / 4 + 16;
    hipError_t e = hipMalloc(p, n * sizeof(T));
    if (e != hipSuccess) {
        *cap = 0;
        return e;
    }
    *cap = n;
    return hipSuccess;
}

bool same_descs(const std::vector<ImgDesc>& a, const std::vector<ImgDesc>& b) {
    return a.size() == b.size() &&
           (a.empty() || std::memcmp(a.data(), b.data(), a.size() * sizeof(ImgDesc)) == 0);
}

bool same_tiles(const std::vector<TileRef>& a, const std::vector<TileRef>& b) {
    return a.size() == b.size() &&
           (a.empty() || std::memcmp(a.data(), b.data(), a.size() * sizeof(TileRef)) == 0);
}

}  // namespace

}  // namespace dsnlm

using namespace dsnlm;

extern "C" int dsnlm_forward_batched(const dsnlm_image* imgs, int count, int S, int P, void* stream) {
    if (count < 0) return fail(DSNLM_EINVAL, "dsnlm_forward_batched: negative count");
    if (count == 0) return DSNLM_OK;
    if (!imgs) return fail(DSNLM_EINVAL, "dsnlm_forward_batched: null descriptor array");
    size_t total = 0;
    for (int k = 0; k < count; ++k) {
        const dsnlm_image& im = imgs[k];
        if (!im.guide || !im.x || !im.y)
            return fail(DSNLM_EINVAL, "dsnlm_forward_batched: null pointer in image " + std::to_string(k));
        int rc = check_denoiser_args(im.n1, im.n2, S, P, im.h, "dsnlm_forward_batched");
        if (rc) return rc;
        const size_t bytes = (size_t)im.n1 * im.n2 * sizeof(float);
        if (overlaps(im.x, im.y, bytes) || overlaps(im.guide, im.y, bytes))
            return fail(DSNLM_EINVAL, "dsnlm_forward_batched: y overlaps x or the guide in image " +
                                          std::to_string(k));
        total += (size_t)im.n1 * im.n2;
    }
    const TileCfg cfg = sweep_tile_cfg(P, kPassA);
    std::lock_guard<std::mutex> lk(g_ws.mu);
    int rc = check_hip(grow(&g_ws.arrays, &g_ws.arrays_cap, 3 * total), "batch workspace");
    if (!rc) rc = check_hip(grow(&g_ws.keys, &g_ws.keys_cap, (size_t)count), "batch keys");
    if (!rc) rc = check_hip(grow(&g_ws.descs, &g_ws.descs_cap, (size_t)count), "batch descriptors");
    if (rc) return rc;

    std::vector<ImgDesc> descs(count);
    std::vector<TileRef> tiles;
    size_t part_total = 0;
    for (int k = 0; k < count; ++k) part_total += half_part_floats(imgs[k].n1, imgs[k].n2, S, P);
    rc = check_hip(grow(&g_ws.part, &g_ws.part_cap, part_total), "batch partial buffers");
    if (rc) return rc;
    size_t off = 0, part_off = 0;
    const double log2e = 1.4426950408889634;
    for (int k = 0; k < count; ++k) {
        const dsnlm_image& im = imgs[k];
        const size_t n = (size_t)im.n1 * im.n2;
        ImgDesc d{};
        d.z = im.guide;
        d.x = im.x;
        d.y = im.y;
        d.c = g_ws.arrays + off;
        d.delta = g_ws.arrays + total + off;
        d.bp = g_ws.arrays + 2 * total + off;
        d.key = g_ws.keys + k;
        d.part = g_ws.part + part_off;
        d.zpad = half_zpad(d.part, im.n1, im.n2, S, P);
        part_off += half_part_floats(im.n1, im.n2, S, P);
        d.n1 = im.n1;
        d.n2 = im.n2;
        const double np = 2.0 * P + 1.0;
        const double kappa = 1.0 / (2.0 * np * np * (double)im.h * (double)im.h);
        d.kappa = (float)kappa;
        d.beta = (float)(kappa * log2e);
        d.h = im.h;
        d.tile_base = (int)tiles.size();
        descs[k] = d;
        const int nty = (im.n1 + cfg.TH - 1) / cfg.TH, ntx = (im.n2 + cfg.TW - 1) / cfg.TW;
        for (int ty = 0; ty < nty; ++ty)
            for (int tx = 0; tx < ntx; ++tx)
                tiles.push_back(TileRef{k, ty * cfg.TH, tx * cfg.TW, (ty == 0 && tx == 0) ? 1 : 0});
        off += n;
    }
    rc = check_hip(grow(&g_ws.tiles, &g_ws.tiles_cap, tiles.size()), "batch tiles");
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    // descriptors only change when the batch does; re-upload in stream order
    // (the host copies kept in the workspace stay alive as copy sources)
    if (!same_descs(descs, g_ws.last_descs)) {
        g_ws.last_descs = descs;
        rc = check_hip(hipMemcpyAsync(g_ws.descs, g_ws.last_descs.data(),
                                      descs.size() * sizeof(ImgDesc), hipMemcpyHostToDevice, st),
                       "upload descriptors");
        if (rc) {
            g_ws.last_descs.clear();
            return rc;
        }
    }
    if (!same_tiles(tiles, g_ws.last_tiles)) {
        g_ws.last_tiles = tiles;
        rc = check_hip(hipMemcpyAsync(g_ws.tiles, g_ws.last_tiles.data(),
                                      tiles.size() * sizeof(TileRef), hipMemcpyHostToDevice, st),
                       "upload tiles");
        if (rc) {
            g_ws.last_tiles.clear();
            return rc;
        }
    }
    const int nt = (int)tiles.size();
    g_ws.last_S = S;
    g_ws.last_P = P;
    ImgDesc none{};
    none.part = g_ws.part;  // every descriptor carries a partial buffer
    rc = check_hip(launch_sweep(kPassA, S, P, none, g_ws.descs, g_ws.tiles, nt, st), "batch pass A");
    if (!rc) rc = check_hip(launch_sweep(kPassBApply, S, P, none, g_ws.descs, g_ws.tiles, nt, st), "batch pass B");
    if (!rc) rc = check_hip(launch_epilogue(none, g_ws.descs, g_ws.tiles, nt, S, P, st), "batch epilogue");
    return rc;
}

extern "C" int dsnlm_batched_state(int image, float* m, int* argmax, const float** c, const float** delta,
                                   void* stream) {
    std::lock_guard<std::mutex> lk(g_ws.mu);
    if (image < 0 || image >= (int)g_ws.last_descs.size())
        return fail(DSNLM_EINVAL, "dsnlm_batched_state: no such image in the last dsnlm_forward_batched");
    const ImgDesc& d = g_ws.last_descs[image];
    if (c) *c = d.c;
    if (delta) *delta = d.delta;
    if (!m && !argmax) return DSNLM_OK;
    unsigned long long key = 0;
    hipStream_t st = static_cast<hipStream_t>(stream);
    int rc = check_hip(hipMemcpyAsync(&key, d.key, sizeof(key), hipMemcpyDeviceToHost, st), "copy key");
    if (!rc) rc = check_hip(hipStreamSynchronize(st), "synchronise");
    if (rc) return rc;
    const unsigned bits = (unsigned)(key >> 32);
    float mv;
    std::memcpy(&mv, &bits, sizeof(mv));
    if (m) *m = mv;
    if (argmax) *argmax = (int)(~(unsigned)(key & 0xffffffffu));
    return DSNLM_OK;
}

extern "C" int dsnlm_backward_batched(const dsnlm_image_grad* grads, int count, void* stream) {
    if (count < 0 || (count > 0 && !grads)) return fail(DSNLM_EINVAL, "dsnlm_backward_batched: bad arguments");
    std::lock_guard<std::mutex> lk(g_ws.mu);
    if (count != (int)g_ws.last_descs.size() || g_ws.last_S < 0)
        return fail(DSNLM_EINVAL, "dsnlm_backward_batched: count differs from the last dsnlm_forward_batched");
    if (count == 0) return DSNLM_OK;
    const int S = g_ws.last_S, P = g_ws.last_P;
    if (!sweep_d2_fits(S, P))
        for (int k = 0; k < count; ++k)
            if (grads[k].dguide || grads[k].dh)
                return fail(DSNLM_EUNSUPPORTED, "dsnlm_backward_batched: guide/bandwidth gradients need S <= 24");
    std::vector<BwdImage> ims(count);
    for (int k = 0; k < count; ++k) {
        const ImgDesc& f = g_ws.last_descs[k];
        if (!grads[k].dy) return fail(DSNLM_EINVAL, "dsnlm_backward_batched: null dy in image " + std::to_string(k));
        const size_t bytes = (size_t)f.n1 * f.n2 * sizeof(float);
        for (float* o : {grads[k].dx, grads[k].dguide})
            if (o && (overlaps(o, f.x, bytes) || overlaps(o, f.z, bytes) || overlaps(o, grads[k].dy, bytes)))
                return fail(DSNLM_EINVAL, "dsnlm_backward_batched: an output overlaps an input in image " +
                                              std::to_string(k));
        ims[k] = BwdImage{&g_ws.last_descs[k], grads[k].dy, grads[k].dx, grads[k].dguide, grads[k].dh};
    }
    return enqueue_backward_batch(ims.data(), count, S, P, g_ws.tiles, (int)g_ws.last_tiles.size(),
                                  static_cast<hipStream_t>(stream));
}
