// Internal declarations of the DSG-NLM / LADMM HIP library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/dsnlm.h"

namespace dsnlm {

constexpr int kMaxS = 24;
constexpr int kMaxP = 5;       // the register-resident sweeps (every entry point)
constexpr int kMaxPWide = 15;  // forward, build, apply and brute force (dsnlm_wide.hip)
// Largest image, and largest guide padded by S + P on every side, in pixels.
// The kernels form element offsets in 32-bit ints and scale them by at most 4
// (float4 records, byte offsets of buffer loads), so 2^28 keeps every such
// offset below 2^31.
constexpr long long kMaxPixels = 1LL << 28;

// log2 of one factor of the separable hat of step S1, for offsets -S..S.
struct HatTable {
    float lg[2 * kMaxS + 1];
};
HatTable make_hat(int S);

// Per-image view used by the sweep kernels.  Unused pointers may be null.
struct ImgDesc {
    const float* z;        // guide (n1 x n2)
    const float* x;        // image being filtered (n1 x n2)
    float* y;              // output of the epilogue
    float* c;              // c_s = omega_s^(-1/2)
    float* delta;          // delta_s = c_s sum_r a c_r
    float* s0;             // sum_r a c_r (d = 0 included) of the last build, kept for the
                           // half-window apply (single image; null: it takes delta / c)
    float* bp;             // B'_s = c_s sum_r a c_r (x_r - x_s)
    unsigned long long* key;  // packed (bits(m) << 32) | (~argmax)
    // backward
    const float* aux_in;   // per-pixel float2 inputs of the backward sweep C
    float* aux_out;        // its per-pixel float2 outputs
    const float* aux5;     // per-pixel factors of the backward sweep D: float4
                           // (omegabar, c, B'bar, x) per pixel
    const float* mbar;     // device scalar mbar of the backward (sweep D)
    float* gz;             // sweep D output: gradient on the padded grid
    float* dpart;          // sweep D: per-tile partner-region partial sums
    float* hpart;          // sweep D output: per-block partial sums for dh
    float* part;           // half-window sweeps: per-tile partner-region partial sums
    float* zpad;           // half-window sweeps: the guide mirrored into a margin of S + P
    float* gpart;          // half-window sweeps split into `groups` dx groups (single image):
    int groups;            // partial regions of groups 1.. (group 0 uses part); 0 or 1: no split
    int n1, n2;
    float beta;            // log2(e) / (2 (2P+1)^2 h^2)
    float kappa;           // 1 / (2 (2P+1)^2 h^2)
    float h;
    int tile_base;         // first entry of this image in a batch tile list
    // Algorithm 1's dual half fused into the gather of a frozen apply
    // (single image, half-window path): with lu set, the gather also forms
    // v_new = x + B'/m (x = the denoiser input), u <- u + lx - v_new,
    // v <- v_new and per-block partial sums of (lx - v_new)^2 and
    // (v_new - v_old)^2 into lres (2 floats per gather block).
    const float* lx;
    float* lv;
    float* lu;
    float* lres;
    // with lstep also set (the 9-tap, factor-2 mirrored super-resolution
    // operator), the gather then takes the next iteration's x-step from lx,
    // lv and lu (sr_step.h)
    const struct SRStepArgs* lstep;
};

// A single-image gather (and epilogue) splits each 32 x 64 tile's rows over
// this many blocks, so that a small image still spreads over the CUs.
constexpr int kGatherSplit = 4;
static_assert(32 / kGatherSplit == 8, "the folded next x-step covers 8 rows per gather block");
inline int gather_blocks(int n1, int n2) { return ((n1 + 31) / 32) * ((n2 + 63) / 64) * kGatherSplit; }

// Per-pixel float4 factors of sweep D are stored with this many zero-cost pad
// pixels before and after each image, so that a thread's run of partners
// never leaves the allocation (partners outside the image are masked).
constexpr int kAux4Lead = 32;
constexpr int kAux4Trail = 128;
inline size_t aux4_floats(size_t n) { return 4 * (n + kAux4Lead + kAux4Trail); }

// One tile of a batch: image index and tile origin.
struct TileRef {
    int img;
    int ti0;
    int tj0;
    int flags;             // bit 0: first tile of its image
};

// Tile of block b in a batched launch of n blocks (one per tile).  The
// dispatcher deals consecutive blocks to the 8 XCDs in turn, so block b runs
// on XCD b mod 8; this gives each XCD a contiguous run of the tile list (the
// tiles of one image in row-major order), so that neighbouring tiles, which
// read the same guide and factor halos, share that XCD's L2.  The mapping is
// a permutation of 0..n-1: any other placement of blocks changes only which
// tiles share an L2, not the results.
__device__ __forceinline__ int xcd_tile(int b, int n) {
    const int x = b & 7, q = n >> 3, r = n & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

enum SweepMode : int {
    kPassA = 0,        // row sums of step S1 -> c
    kPassBApply = 1,   // delta, B' and the running max key (x known)
    kPassBBuild = 2,   // delta and the key only
    kApply = 3,        // B' only (weights already built)
    kPassC = 4,        // backward: sum a t_r, sum a w_r
    kNLM = 6,          // plain NLM (eq. NLM): sums of k and k x, no hat (half window only)
};

// Variant table of the sweeps (tuning.hip).
// 0 plain, 1 software-pipelined, 2 grouped register window (full window);
// 3 half window (accumulating sweeps only; needs ImgDesc::part)
constexpr int kSweepVariants = 4;
constexpr int kHalfVariant = 3;
int sweep_variant(int mode, int S, int P);
void set_sweep_variant(int kind, int S, int P, int v);
void save_tuning();

struct TileCfg {
    int TH, TW, threads;
};

// Launchers (dsnlm_sweep.hip).
TileCfg sweep_tile_cfg(int P, int mode);
size_t sweep_lds_bytes(int S, int P, int mode);
// Set the dynamic-LDS attribute of every single-image sweep kernel for patch
// half-widths S and P (needed once before a stream capture).
hipError_t prepare_sweeps(int S, int P);
hipError_t launch_sweep(int mode, int S, int P, const ImgDesc& one, const ImgDesc* batch,
                        const TileRef* tiles, int ntiles, hipStream_t st);
hipError_t launch_epilogue(const ImgDesc& one, const ImgDesc* batch, const TileRef* tiles,
                           int ntiles, int S, int P, hipStream_t st);

// Half-window sweeps (dsnlm_half.hip).  Floats of the partial buffer of an
// n1 x n2 image; whether the LDS of a mode fits; the launcher (sweep +
// gather).  launch_sweep routes a mode here when variant 3 is selected and a
// partial buffer is given (for a batch launch: one.part non-null means every
// descriptor carries one).
// Lead pad (float2 entries) before the backward's (t, w) pair array.
constexpr int kFacLead = 32;
size_t half_part_floats(int n1, int n2, int S, int P);  // partial regions + mirrored guide
// A single-image sweep splits the half window's shifts over `groups` blocks
// per tile (equal contiguous ranges; ImgDesc::groups, ::gpart, set by
// base_desc from the handle), which fills the GPU for a small image; batch
// launches never split, so a batched result differs from the single-image one
// by summation order only.
// The count comes from the tuning table (dsnlm_tune) when it has an entry for
// the image's size class, else from a default by tile count.
constexpr int kMaxShiftGroups = 8;
int half_split_groups(int n1, int n2, int S, int P);
int tuned_shift_groups(int n1, int n2, int S, int P);  // 0: no table entry
void set_shift_groups(int n1, int n2, int S, int P, int groups);
size_t half_group_floats(int n1, int n2, int S, int groups);        // floats of ImgDesc::gpart
float* half_zpad(float* part, int n1, int n2, int S, int P);  // the mirrored guide inside it
bool half_lds_fits(int S, int P, int mode);
bool half_mode_ok(int mode);
// Whether launch_sweep runs `mode` on the half-window path for this
// descriptor (whose gather of kApply then also writes y = x + B'/m when
// d.y is set, and Algorithm 1's dual half when d.lu is set).
bool sweep_takes_half(int mode, int S, int P, const ImgDesc& one);
hipError_t launch_half(int mode, int S, int P, const ImgDesc& one, const ImgDesc* batch, const TileRef* tiles,
                       int ntiles, hipStream_t st);
hipError_t prepare_half(int S, int P);

// Wide patches, kMaxP < P <= kMaxPWide (dsnlm_wide.hip): single-image passes
// A, B (both forms) and apply; launch_sweep routes such P here.
// The dy range of the window is split into wide_groups() groups whose
// per-pixel sums go to d.part (wide_part_floats() floats).
bool wide_fits(int S, int P);
int wide_groups(int n1, int n2, int S);
size_t wide_part_floats(int n1, int n2, int S);
hipError_t launch_wide(int mode, int S, int P, const ImgDesc& d, hipStream_t st);

// Brute-force DSG-NLM (dsnlm_brute.hip): c, delta, B' and the key of d from
// directly summed patch distances; d.zpad must hold room for the mirrored
// guide (margin S + P).
hipError_t launch_brute(const ImgDesc& d, int S, int P, hipStream_t st);

// Sweep D on the forward's 32 x 64 tiling (dsnlm_sweep_d.hip): every pair
// is evaluated by one tile, whose contributions land in a partial region
// (rows ti0 - P .. ti0 + 32 + P + S, columns tj0 - P - S .. tj0 + 64 + P + S);
// the gather sums the covering regions into gz on the padded grid.  The
// tile list of a batch launch is the forward's; d.hpart gets one entry per
// forward tile of the image.
// A single-image launch splits the dx range into sweep_d2_groups() groups
// (partial regions and hbar partials per (tile, group)); a batch uses one.
bool sweep_d2_fits(int S, int P);
int sweep_d2_groups(int n1, int n2, int S);
size_t sweep_d2_part_floats(int n1, int n2, int S, int P);  // for the single-image groups
hipError_t launch_sweep_d2(int S, int P, const ImgDesc& one, const ImgDesc* batch, const TileRef* tiles, int ntiles,
                           hipStream_t st);
// map[b] = (image, block of 256 padded-grid pixels) for a batch launch
hipError_t launch_d2_gather(int S, int P, const ImgDesc& one, const ImgDesc* batch, const int2* map, int nblocks,
                            hipStream_t st);

// Backward launchers (dsnlm_backward.hip).
int enqueue_backward(dsnlm_weights* w, const float* x, const float* dy, float* dx, float* dguide,
                     float* dh, float* scratch, hipStream_t st);
size_t backward_scratch_floats(int n1, int n2, int S, int P);

// Brackets one kernel launch with events when instrumentation is enabled.
class ProfScope {
  public:
    ProfScope(int kind, hipStream_t st);
    ~ProfScope();
    ProfScope(const ProfScope&) = delete;
    ProfScope& operator=(const ProfScope&) = delete;

  private:
    int kind_;
    hipStream_t st_;
    hipEvent_t ev_;
};

// Batched backward (dsnlm_backward.hip) over the state a batched forward left.
struct BwdImage {
    const ImgDesc* fwd;     // forward descriptor of the image (z, x, c, delta, B', key, sizes)
    const float* dy;
    float* dx;              // nullable
    float* dguide;          // nullable
    float* dh;              // nullable (device scalar)
};
int enqueue_backward_batch(const BwdImage* ims, int count, int S, int P, const TileRef* fwd_tiles,
                           int nfwd_tiles, hipStream_t st);

// Error state.
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
int check_hip(hipError_t e, const char* what);

}  // namespace dsnlm

struct dsnlm_weights {
    int n1, n2, S, P;
    float h;
    int device;
    float* guide;      // copy of the guide
    float* c;
    float* delta;
    float* s0;         // pass B's sum_r a c_r (half-window builds of a single image)
    float* bp;
    unsigned long long* key;
    float* scratch;    // solver scratch (grow-only), freed with the handle
    size_t scratch_cap;
    float* zbuf;       // denoiser input x + u inside the solver (in scratch)
    float* bscratch;   // backward scratch (grow-only), freed with the handle
    size_t bscratch_cap;
    float* part;       // partial buffer of the half-window sweeps (grow-only)
    size_t part_cap;
    float* gpart;      // partial regions of the extra dx groups (grow-only)
    size_t gpart_cap;
    bool applied;      // bp holds B' of the last apply
    bool solver_owned; // owned by a ladmm_solve cache entry: nothing outside the solve
                       // reads its guide copy
};
