// Backward pass (vector-Jacobian product) of y = W(z, h) x on gfx950.
//
// The paper defines the forward map only (Section 3: eq. NLM, steps S1-S3,
// Algorithm 2); the backward below is the chain rule through it, written in
// gather form so that no pixel is ever updated by two threads (no atomics).
// With a_{s,d} = Lambda_d exp(-kappa D_{s,d}), omega_s = sum_d a_{s,d},
// c_s = omega_s^(-1/2), B'_s = c_s sum_d a c_{s+d} (x_{s+d} - x_s),
// delta_s = c_s sum_d a c_{s+d}, m = delta_{s*} and y = x + B'/m:
//
//   B'bar = ybar / m,   mbar = -sum ybar B' / m^2,   f_s = [s = s*] mbar
//   t_r = c_r B'bar_r,  w_r = c_r (f_r - B'bar_r x_r)
//   U_s = sum_d a t_{s+d},  Wc_s = sum_d a w_{s+d}                 (sweep C)
//   xbar = ybar - delta B'bar + c U                                 (= W ybar)
//   cbar = B'bar B'/c + f delta/c + x U + Wc,  omegabar = -cbar c^3 / 2
//   abar_{s,d} = omegabar_s + c_{s+d} (beta_s x_{s+d} + gamma_s),
//        beta_s = c_s B'bar_s,  gamma_s = c_s (f_s - x_s B'bar_s)
//   Dbar_{s,d} = -kappa a (abar_{s,d} + abar_{s+d,-d})            (both orders)
//   hbar = -(1/h) sum_{s,d} Dbar_{s,d} D_{s,d}
//   zbar(p) = 2 sum_d (z(p) - z(p+d)) sum_{|s-p| <= P} Dbar_{s,d}  (padded grid)
//   dguide = fold of zbar through the mirror padding.
// Sweep D (dsnlm_sweep_d.hip) recomputes D_{s,d} on the forward's tiles,
// forms Dbar_{s,d} in LDS, box-sums it over the patch and scatters zbar.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

namespace dsnlm {

namespace {

__device__ __forceinline__ int reflect_clamp_b(int k, int n) {
    if (k < 0) k = -k - 1;
    if (k >= n) k = 2 * n - 1 - k;
    k = k < 0 ? 0 : k;
    k = k >= n ? n - 1 : k;
    return k;
}

struct BwdArgs {
    const float* x;      // image of the forward
    const float* dy;     // cotangent of y
    const float* c;      // c_s
    const float* delta;  // delta_s
    const float* bp;     // B'_s
    const unsigned long long* key;  // (m, s*)
    float* pairs;        // [2n] t, w  (input of sweep C)
    float* cw;           // [2n] U, Wc (output of sweep C)
    float* aux5;         // sweep-D factors: float4 (omegabar, c, B'bar, x) per pixel,
                         // column-major after a lead pad of kAux4Lead entries
    float* dx;           // W ybar (nullable)
    float* partials;     // per-block partial sums
    float* mbar;         // device scalar
    int n;
    // batched form only
    float* gz;           // padded-grid guide gradient
    float* dguide;       // guide gradient (nullable)
    float* dh;           // device scalar (nullable)
    float* hpart;        // sweep-D block partials of this image
    int n1, n2, P, nd;
    float h;
};

// B'bar, the (t, w) pairs, and per-block sums of ybar B'.
__global__ void __launch_bounds__(256) k_bwd_prep(BwdArgs a) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    const float m = __uint_as_float((unsigned)(*a.key >> 32));
    float part = 0.f;
    if (idx < a.n) {
        const float yb = a.dy[idx];
        const float bb = yb / m;
        const float cc = a.c[idx];
        a.pairs[2 * idx] = cc * bb;
        a.pairs[2 * idx + 1] = -cc * bb * a.x[idx];
        part = yb * a.bp[idx];
    }
    __shared__ double sh[256];
    sh[threadIdx.x] = part;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) a.partials[blockIdx.x] = (float)sh[0];
}

// mbar = -sum / m^2 (fixed-order reduction) and the f term of w at s*.
__global__ void __launch_bounds__(256) k_bwd_mbar(BwdArgs a, int nblk) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) acc += a.partials[b];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const unsigned long long key = *a.key;
        const float m = __uint_as_float((unsigned)(key >> 32));
        const int sstar = (int)(~(unsigned)(key & 0xffffffffu));
        const float mb = (float)(-sh[0] / ((double)m * m));
        *a.mbar = mb;
        a.pairs[2 * sstar + 1] += a.c[sstar] * mb;
    }
}

// xbar, cbar and the per-pixel factors of sweep D for a 16 x 16 tile (256
// threads).  The float4 factors are written column-major through an LDS
// transpose, so both the row-major reads and the column-major writes of a
// wave are contiguous.
__device__ __forceinline__ void mid_tile(const BwdArgs& a, int i0, int j0) {
    __shared__ float4 tile[16][17];
    const int n1 = a.n1, n2 = a.n2;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int i = i0 + ty, j = j0 + tx;
    float4 val = make_float4(0.f, 0.f, 0.f, 0.f);
    if (i < n1 && j < n2) {
        const int idx = i * n2 + j;
        const unsigned long long key = *a.key;
        const float m = __uint_as_float((unsigned)(key >> 32));
        const int sstar = (int)(~(unsigned)(key & 0xffffffffu));
        const float f = idx == sstar ? *a.mbar : 0.f;
        const float yb = a.dy[idx];
        const float bb = yb / m;
        const float cc = a.c[idx];
        const float dl = a.delta[idx];
        const float xv = a.x[idx];
        const float U = a.cw[2 * idx];
        const float Wc = a.cw[2 * idx + 1];
        if (a.dx) a.dx[idx] = yb - dl * bb + cc * U;
        const float cbar = bb * a.bp[idx] / cc + f * dl / cc + xv * U + Wc;
        const float obar = -0.5f * cbar * cc * cc * cc;
        val = make_float4(obar, cc, bb, xv);
    }
    tile[tx][ty] = val;
    __syncthreads();
    const int wc = threadIdx.x >> 4, wr = threadIdx.x & 15;  // lanes walk down a column
    const int gi = i0 + wr, gj = j0 + wc;
    if (gi < n1 && gj < n2) reinterpret_cast<float4*>(a.aux5)[kAux4Lead + (size_t)gj * n1 + gi] = tile[wc][wr];
}

__global__ void __launch_bounds__(256) k_bwd_mid(BwdArgs a) { mid_tile(a, blockIdx.y * 16, blockIdx.x * 16); }


// ---- segmented forms for a batch: block b of the grid works on image
// map[b].x, its local block map[b].y ------------------------------------------
__global__ void __launch_bounds__(256) k_bwd_prep_seg(const BwdArgs* __restrict__ imgs,
                                                      const int2* __restrict__ map) {
    const int2 mb = map[blockIdx.x];
    const BwdArgs a = imgs[mb.x];
    const int idx = mb.y * 256 + threadIdx.x;
    const float m = __uint_as_float((unsigned)(*a.key >> 32));
    float part = 0.f;
    if (idx < a.n) {
        const float yb = a.dy[idx];
        const float bb = yb / m;
        const float cc = a.c[idx];
        a.pairs[2 * idx] = cc * bb;
        a.pairs[2 * idx + 1] = -cc * bb * a.x[idx];
        part = yb * a.bp[idx];
    }
    __shared__ double sh[256];
    sh[threadIdx.x] = part;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) a.partials[mb.y] = (float)sh[0];
}

// one block per image
__global__ void __launch_bounds__(256) k_bwd_mbar_seg(const BwdArgs* __restrict__ imgs) {
    const BwdArgs a = imgs[blockIdx.x];
    const int nblk = (a.n + 255) / 256;
    __shared__ double sh[256];
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) acc += a.partials[b];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const unsigned long long key = *a.key;
        const float m = __uint_as_float((unsigned)(key >> 32));
        const int sstar = (int)(~(unsigned)(key & 0xffffffffu));
        const float mb = (float)(-sh[0] / ((double)m * m));
        *a.mbar = mb;
        a.pairs[2 * sstar + 1] += a.c[sstar] * mb;
    }
}

// tmap[b] = (image, 16 x 16 tile index in row-major tile order)
__global__ void __launch_bounds__(256) k_bwd_mid_seg(const BwdArgs* __restrict__ imgs,
                                                     const int2* __restrict__ tmap) {
    const int2 mb = tmap[blockIdx.x];
    const BwdArgs a = imgs[mb.x];
    const int ntx = (a.n2 + 15) / 16;
    const int ti = mb.y / ntx, tj = mb.y - ti * ntx;
    mid_tile(a, ti * 16, tj * 16);
}

__global__ void __launch_bounds__(256) k_fold_seg(const BwdArgs* __restrict__ imgs, const int2* __restrict__ map) {
    const int2 mb = map[blockIdx.x];
    const BwdArgs a = imgs[mb.x];
    const int idx = mb.y * 256 + threadIdx.x;
    if (idx >= a.n || !a.dguide) return;
    const int n1 = a.n1, n2 = a.n2, P = a.P;
    const int i = idx / n2, j = idx - i * n2;
    int pi[3], pj[3];
    int ci = 0, cj = 0;
    pi[ci++] = i;
    if (i <= P - 1) pi[ci++] = -1 - i;
    if (i >= n1 - P) pi[ci++] = 2 * n1 - 1 - i;
    pj[cj++] = j;
    if (j <= P - 1) pj[cj++] = -1 - j;
    if (j >= n2 - P) pj[cj++] = 2 * n2 - 1 - j;
    const int W2 = n2 + 2 * P;
    float acc = 0.f;
    for (int x = 0; x < ci; ++x)
        for (int y = 0; y < cj; ++y) acc += a.gz[(size_t)(pi[x] + P) * W2 + pj[y] + P];
    a.dguide[idx] = acc;
}

// one block per image: dh = -(1/h) sum of its sweep-D partials
__global__ void __launch_bounds__(256) k_dh_seg(const BwdArgs* __restrict__ imgs) {
    const BwdArgs a = imgs[blockIdx.x];
    if (!a.dh) return;
    __shared__ double sh[256];
    double acc = 0.0;
    for (int b = threadIdx.x; b < a.nd; b += 256) acc += a.hpart[b];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *a.dh = (float)(-sh[0] / a.h);
}

// dguide(q) = sum of zbar over the padded positions that mirror onto q.
__global__ void __launch_bounds__(256) k_fold(const float* __restrict__ gz, float* __restrict__ dz, int n1,
                                              int n2, int P) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= n1 * n2) return;
    const int i = idx / n2, j = idx - i * n2;
    int pi[3], pj[3];
    int ci = 0, cj = 0;
    pi[ci++] = i;
    if (i <= P - 1) pi[ci++] = -1 - i;
    if (i >= n1 - P) pi[ci++] = 2 * n1 - 1 - i;
    pj[cj++] = j;
    if (j <= P - 1) pj[cj++] = -1 - j;
    if (j >= n2 - P) pj[cj++] = 2 * n2 - 1 - j;
    const int W2 = n2 + 2 * P;
    float acc = 0.f;
    for (int a = 0; a < ci; ++a)
        for (int b = 0; b < cj; ++b) acc += gz[(size_t)(pi[a] + P) * W2 + pj[b] + P];
    dz[idx] = acc;
}

// dh = -(1/h) sum of the block partials (fixed order).
__global__ void __launch_bounds__(256) k_dh(const float* __restrict__ hpart, int nblk, float h,
                                            float* __restrict__ dh) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) acc += hpart[b];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *dh = (float)(-sh[0] / h);
}

inline int blocks256(size_t n) { return (int)((n + 255) / 256); }

}  // namespace

ImgDesc base_desc(const dsnlm_weights* w);
bool overlaps(const void* a, const void* b, size_t bytes);

// Scratch (floats) needed by dsnlm_apply_backward for an n1 x n2 image.
size_t backward_scratch_floats(int n1, int n2, int S, int P) {
    const size_t n = (size_t)n1 * n2;
    const size_t tiles = (size_t)((n1 + 31) / 32) * ((n2 + 63) / 64) * sweep_d2_groups(n1, n2, S);
    return 2 * (size_t)kFacLead + 2 * n + 2 * n + aux4_floats(n) + (size_t)(n1 + 2 * P) * (n2 + 2 * P) +
           blocks256(n) + tiles + 8 + sweep_d2_part_floats(n1, n2, S, P);
}

int enqueue_backward(dsnlm_weights* w, const float* x, const float* dy, float* dx, float* dguide, float* dh,
                     float* scratch, hipStream_t st) {
    const int n1 = w->n1, n2 = w->n2, S = w->S, P = w->P;
    const size_t n = (size_t)n1 * n2;
    float* pairs = scratch + 2 * kFacLead;  // read by the half-window sweep C as partner factors
    float* cw = pairs + 2 * n;
    float* aux5 = cw + 2 * n;               // 16-byte aligned: read as float4
    float* gz = aux5 + aux4_floats(n);
    float* partials = gz + (size_t)(n1 + 2 * P) * (n2 + 2 * P);
    const int nb = blocks256(n);
    // sweep-D blocks (tiles x dx groups), one partial of hbar each
    const int nd = ((n1 + 31) / 32) * ((n2 + 63) / 64) * sweep_d2_groups(n1, n2, S);
    float* hpart = partials + nb;
    float* mbar = hpart + nd;
    float* dpart = mbar + 8;  // sweep-D partial regions

    BwdArgs a{};
    a.x = x;
    a.dy = dy;
    a.c = w->c;
    a.delta = w->delta;
    a.bp = w->bp;
    a.key = w->key;
    a.pairs = pairs;
    a.cw = cw;
    a.aux5 = aux5;
    a.n1 = n1;
    a.n2 = n2;
    a.dx = dx;
    a.partials = partials;
    a.mbar = mbar;
    a.n = (int)n;
    {
        ProfScope prof(DSNLM_K_BWD_PREP, st);
        hipLaunchKernelGGL(k_bwd_prep, dim3(nb), dim3(256), 0, st, a);
        hipLaunchKernelGGL(k_bwd_mbar, dim3(1), dim3(256), 0, st, a, nb);
        int rc = check_hip(hipGetLastError(), "backward prep");
        if (rc) return rc;
    }
    ImgDesc d = base_desc(w);
    d.x = x;
    d.aux_in = pairs;
    d.aux_out = cw;
    int rc = check_hip(launch_sweep(kPassC, S, P, d, nullptr, nullptr, 0, st), "backward sweep C");
    if (rc) return rc;
    {
        ProfScope prof(DSNLM_K_BWD_PREP, st);
        hipLaunchKernelGGL(k_bwd_mid, dim3((n2 + 15) / 16, (n1 + 15) / 16), dim3(256), 0, st, a);
        rc = check_hip(hipGetLastError(), "backward mid");
        if (rc) return rc;
    }
    if (!dguide && !dh) return DSNLM_OK;
    d.aux5 = aux5;
    d.mbar = mbar;
    d.gz = gz;
    d.hpart = hpart;
    d.dpart = dpart;
    rc = check_hip(launch_sweep_d2(S, P, d, nullptr, nullptr, 0, st), "backward sweep D");
    if (!rc) rc = check_hip(launch_d2_gather(S, P, d, nullptr, nullptr, 0, st), "backward sweep D gather");
    if (rc) return rc;
    ProfScope prof(DSNLM_K_BWD_TAIL, st);
    if (dguide) hipLaunchKernelGGL(k_fold, dim3(nb), dim3(256), 0, st, gz, dguide, n1, n2, P);
    if (dh) hipLaunchKernelGGL(k_dh, dim3(1), dim3(256), 0, st, hpart, nd, w->h, dh);
    return check_hip(hipGetLastError(), "backward tail");
}

namespace {

// Grow-only workspace of the batched backward.
struct BwdBatchWs {
    float* arrays = nullptr;
    size_t arrays_cap = 0;
    BwdArgs* args = nullptr;
    size_t args_cap = 0;
    ImgDesc* descs = nullptr;
    size_t descs_cap = 0;
    int2* map = nullptr;
    size_t map_cap = 0;
    int2* gmap = nullptr;
    size_t gmap_cap = 0;
    int2* tmap = nullptr;
    size_t tmap_cap = 0;
    std::vector<int2> h_tmap;
    std::vector<BwdArgs> h_args;
    std::vector<ImgDesc> h_descs;
    std::vector<int2> h_map;
    std::vector<int2> h_gmap;
};
BwdBatchWs g_bws;

template <class T>
hipError_t grow_b(T** p, size_t* cap, size_t need) {
    if (need <= *cap) return hipSuccess;
    if (*p) {
        hipError_t e = hipFree(*p);
        if (e != hipSuccess) return e;
        *p = nullptr;
    }
    const size_t n = need + need / 4 + 16;
    hipError_t e = hipMalloc(p, n * sizeof(T));
    *cap = e == hipSuccess ? n : 0;
    return e;
}

template <class T>
int upload_if_changed(T* dev, std::vector<T>& keep, const std::vector<T>& now, hipStream_t st, const char* what) {
    if (keep.size() == now.size() && !now.empty() &&
        std::memcmp(keep.data(), now.data(), now.size() * sizeof(T)) == 0)
        return DSNLM_OK;
    keep = now;
    if (keep.empty()) return DSNLM_OK;
    const int rc =
        check_hip(hipMemcpyAsync(dev, keep.data(), keep.size() * sizeof(T), hipMemcpyHostToDevice, st), what);
    if (rc) keep.clear();  // force a fresh upload next time
    return rc;
}

}  // namespace

int enqueue_backward_batch(const BwdImage* ims, int count, int S, int P, const TileRef* fwd_tiles, int nfwd_tiles,
                           hipStream_t st) {
    // workspace layout per image: pairs 2n | cw 2n | sweep-D factors | gz | partials nb | hpart nd | mbar
    size_t total = 0;
    std::vector<size_t> base(count);
    std::vector<int> nd(count), nb(count);
    for (int k = 0; k < count; ++k) {
        const ImgDesc& f = *ims[k].fwd;
        const size_t n = (size_t)f.n1 * f.n2;
        nb[k] = (int)((n + 255) / 256);
        nd[k] = ((f.n1 + 31) / 32) * ((f.n2 + 63) / 64);  // forward tiles
        base[k] = total;  // 256-byte aligned: the factors are read as float4
        total += 2 * (size_t)kFacLead + 4 * n + aux4_floats(n) + (size_t)(f.n1 + 2 * P) * (f.n2 + 2 * P) +
                 nb[k] + nd[k] + 4 + sweep_d2_part_floats(f.n1, f.n2, S, P);
        total = (total + 63) & ~(size_t)63;
    }
    int rc = check_hip(grow_b(&g_bws.arrays, &g_bws.arrays_cap, total), "batched backward workspace");
    if (!rc) rc = check_hip(grow_b(&g_bws.args, &g_bws.args_cap, (size_t)count), "batched backward args");
    if (!rc) rc = check_hip(grow_b(&g_bws.descs, &g_bws.descs_cap, (size_t)count), "batched backward descriptors");
    if (rc) return rc;
    std::vector<BwdArgs> args(count);
    std::vector<ImgDesc> descs(count);
    std::vector<int2> map, tmap;
    std::vector<int2> gmap;
    for (int k = 0; k < count; ++k) {
        const ImgDesc& f = *ims[k].fwd;
        const size_t n = (size_t)f.n1 * f.n2;
        float* b = g_bws.arrays + base[k] + 2 * kFacLead;  // lead pad before the (t, w) pairs
        BwdArgs a{};
        a.x = f.x;
        a.dy = ims[k].dy;
        a.c = f.c;
        a.delta = f.delta;
        a.bp = f.bp;
        a.key = f.key;
        a.pairs = b;
        a.cw = b + 2 * n;
        a.aux5 = b + 4 * n;
        a.gz = b + 4 * n + aux4_floats(n);
        a.partials = a.gz + (size_t)(f.n1 + 2 * P) * (f.n2 + 2 * P);
        a.hpart = a.partials + nb[k];
        a.mbar = a.hpart + nd[k];
        float* dpart = a.mbar + 4;
        a.n = (int)n;
        a.dx = ims[k].dx;
        a.dguide = ims[k].dguide;
        a.dh = ims[k].dh;
        a.n1 = f.n1;
        a.n2 = f.n2;
        a.P = P;
        a.nd = nd[k];
        a.h = f.h;
        args[k] = a;
        ImgDesc d = f;
        d.aux_in = a.pairs;
        d.aux_out = a.cw;
        d.aux5 = a.aux5;
        d.mbar = a.mbar;
        d.gz = a.gz;
        d.hpart = a.hpart;
        d.dpart = dpart;
        descs[k] = d;
        for (int b2 = 0; b2 < nb[k]; ++b2) map.push_back(make_int2(k, b2));
        const int nt16 = ((f.n1 + 15) / 16) * ((f.n2 + 15) / 16);
        for (int t = 0; t < nt16; ++t) tmap.push_back(make_int2(k, t));
        const int ng = (int)(((size_t)(f.n1 + 2 * P) * (f.n2 + 2 * P) + 255) / 256);
        for (int g = 0; g < ng; ++g) gmap.push_back(make_int2(k, g));
    }
    rc = check_hip(grow_b(&g_bws.map, &g_bws.map_cap, map.size()), "batched backward map");
    if (!rc) rc = check_hip(grow_b(&g_bws.gmap, &g_bws.gmap_cap, gmap.size()), "batched backward gather map");
    if (!rc) rc = check_hip(grow_b(&g_bws.tmap, &g_bws.tmap_cap, tmap.size()), "batched backward tile map");
    if (!rc) rc = upload_if_changed(g_bws.args, g_bws.h_args, args, st, "upload backward args");
    if (!rc) rc = upload_if_changed(g_bws.descs, g_bws.h_descs, descs, st, "upload backward descriptors");
    if (!rc) rc = upload_if_changed(g_bws.map, g_bws.h_map, map, st, "upload backward map");
    if (!rc) rc = upload_if_changed(g_bws.gmap, g_bws.h_gmap, gmap, st, "upload backward gather map");
    if (!rc) rc = upload_if_changed(g_bws.tmap, g_bws.h_tmap, tmap, st, "upload backward tile map");
    if (rc) return rc;
    const int nmap = (int)map.size();
    {
        ProfScope prof(DSNLM_K_BWD_PREP, st);
        hipLaunchKernelGGL(k_bwd_prep_seg, dim3(nmap), dim3(256), 0, st, g_bws.args, g_bws.map);
        hipLaunchKernelGGL(k_bwd_mbar_seg, dim3(count), dim3(256), 0, st, g_bws.args);
        rc = check_hip(hipGetLastError(), "batched backward prep");
        if (rc) return rc;
    }
    ImgDesc none{};
    none.part = descs[0].part;  // non-null: the forward's descriptors carry partial buffers
    rc = check_hip(launch_sweep(kPassC, S, P, none, g_bws.descs, fwd_tiles, nfwd_tiles, st), "batched sweep C");
    if (rc) return rc;
    {
        ProfScope prof(DSNLM_K_BWD_PREP, st);
        hipLaunchKernelGGL(k_bwd_mid_seg, dim3((unsigned)tmap.size()), dim3(256), 0, st, g_bws.args, g_bws.tmap);
        rc = check_hip(hipGetLastError(), "batched backward mid");
        if (rc) return rc;
    }
    bool need_d = false;
    for (int k = 0; k < count; ++k) need_d = need_d || ims[k].dguide || ims[k].dh;
    if (!need_d) return DSNLM_OK;
    rc = check_hip(launch_sweep_d2(S, P, none, g_bws.descs, fwd_tiles, nfwd_tiles, st), "batched sweep D");
    if (!rc)
        rc = check_hip(launch_d2_gather(S, P, none, g_bws.descs, g_bws.gmap, (int)gmap.size(), st),
                       "batched sweep D gather");
    if (rc) return rc;
    ProfScope prof(DSNLM_K_BWD_TAIL, st);
    hipLaunchKernelGGL(k_fold_seg, dim3(nmap), dim3(256), 0, st, g_bws.args, g_bws.map);
    hipLaunchKernelGGL(k_dh_seg, dim3(count), dim3(256), 0, st, g_bws.args);
    return check_hip(hipGetLastError(), "batched backward tail");
}

}  // namespace dsnlm

using namespace dsnlm;

extern "C" int dsnlm_apply_backward(const dsnlm_weights* wc, const float* x, const float* dy, float* dx,
                                    float* dguide, float* dh, void* stream) {
    if (!wc || !x || !dy) return fail(DSNLM_EINVAL, "dsnlm_apply_backward: null pointer");
    dsnlm_weights* w = const_cast<dsnlm_weights*>(wc);
    if (!w->applied)
        return fail(DSNLM_EINVAL, "dsnlm_apply_backward: the handle holds no forward to differentiate");
    if (w->P > kMaxP)
        return fail(DSNLM_EUNSUPPORTED, "dsnlm_apply_backward: the backward supports P <= 5");
    if ((dguide || dh) && !sweep_d2_fits(w->S, w->P))
        return fail(DSNLM_EUNSUPPORTED, "dsnlm_apply_backward: guide/bandwidth gradients need S <= 24");
    const size_t bytes = (size_t)w->n1 * w->n2 * sizeof(float);
    if (dx && (overlaps(dx, x, bytes) || overlaps(dx, dy, bytes)))
        return fail(DSNLM_EINVAL, "dsnlm_apply_backward: dx overlaps x or dy");
    if (dguide && (overlaps(dguide, x, bytes) || overlaps(dguide, dy, bytes)))
        return fail(DSNLM_EINVAL, "dsnlm_apply_backward: dguide overlaps x or dy");
    const size_t need = backward_scratch_floats(w->n1, w->n2, w->S, w->P);
    if (w->bscratch_cap < need) {
        if (w->bscratch) (void)hipFree(w->bscratch);
        w->bscratch = nullptr;
        w->bscratch_cap = 0;
        int rc = check_hip(hipMalloc(&w->bscratch, need * sizeof(float)), "backward scratch");
        if (rc) return rc;
        w->bscratch_cap = need;
    }
    return enqueue_backward(w, x, dy, dx, dguide, dh, w->bscratch, static_cast<hipStream_t>(stream));
}
