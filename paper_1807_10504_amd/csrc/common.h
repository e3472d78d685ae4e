// Shared internals of the ibproj library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/ibproj.h"
#include "freefall.h"

namespace ib {

// ---------------------------------------------------------------------------
// error reporting
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);

#define IB_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return ::ib::fail(IB_EHIP, std::string(#call " failed: ") +                \
                                           hipGetErrorString(e_));                     \
    } while (0)

#define IB_CHECK(cond, code, msg)                                                      \
    do {                                                                               \
        if (!(cond)) return ::ib::fail((code), (msg));                                 \
    } while (0)

#define IB_TRY(call)                                                                   \
    do {                                                                               \
        int r_ = (call);                                                               \
        if (r_ != IB_OK) return r_;                                                    \
    } while (0)

// ---------------------------------------------------------------------------
// grid geometry passed to kernels by value
struct Dims {
    int nx, ny, nz;   // nz = 1 in 2D
    int dim;
    double h;
    __host__ __device__ long cells() const { return (long)nx * ny * nz; }
};

inline Dims make_dims(const ib_grid& g) {
    Dims d;
    d.dim = g.dim;
    d.nx = g.n[0];
    d.ny = g.n[1];
    d.nz = g.dim == 3 ? g.n[2] : 1;
    d.h = g.h;
    return d;
}

constexpr int kBlock = 256;
inline unsigned grid_for(long n, int block = kBlock) {
    return (unsigned)((n + block - 1) / block);
}

__host__ __device__ inline int wrap(int i, int n) {
    int r = i % n;
    return r < 0 ? r + n : r;
}

// the same for -n <= i < 2n, without a division
// (i, j, k) of cell c, x fastest; grids have fewer than 2^31 cells (checked
// where they are made), so 32-bit divisions do, not the emulated 64-bit ones
__device__ __forceinline__ void cell_ijk(long c, int nx, int ny, int& i, int& j, int& k) {
    const unsigned cu = (unsigned)c, r = cu / (unsigned)nx;
    i = (int)(cu - r * (unsigned)nx);
    j = (int)(r % (unsigned)ny);
    k = (int)(r / (unsigned)ny);
}

__host__ __device__ inline int wrap_near(int i, int n) {
    return i < 0 ? i + n : (i >= n ? i - n : i);
}

// fixed tree sum over one block (blockDim.x a power of two, sh of blockDim.x)
__device__ inline double block_reduce_sum(double v, double* sh) {
    int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// body force density on the vertical faces of the free-fall runs:
//   (rho_f - rho_mean) grav + rho_f fa,  rho_mean = *rsum * inv_w
// (rsum: a device sum of the density; NULL when grav is 0)
struct Body {
    double grav, fa, inv_w;
    const double* rsum;
    __device__ double at(double rf) const {
        const double rm = rsum ? *rsum * inv_w : 0.0;
        return (rf - rm) * grav + rf * fa;
    }
    bool on() const { return grav != 0.0 || fa != 0.0; }
};

// fixed-point scale of the deterministic integer accumulation of Heaviside
// contributions: 1.0 (a full cell) maps to 2^56
constexpr double kFixScale = 72057594037927936.0;        // 2^56
constexpr double kFixInv = 1.0 / 72057594037927936.0;

// tile edge (cells) of the marker bins
constexpr int kTile = 4;
// exclusive scan of the tile counts: blocks of 1024 threads x 4 items, the
// block totals scanned by one more block
constexpr int kScanThreads = 1024, kScanItems = 4, kScanTile = kScanThreads * kScanItems;
constexpr long kMaxTiles = (long)kScanTile * kScanTile - 1;

// ---------------------------------------------------------------------------
// context
struct Ctx {
    ib_grid g;
    Dims d;
    int max_markers, max_elems;
    // binning
    int n_tiles, tnx, tny, tnz;
    int32_t* bin_key = nullptr;      // per marker tile key
    int32_t* bin_order = nullptr;    // marker indices in tile order, ascending within a tile
    int32_t* tile_start = nullptr;   // n_tiles + 1
    int32_t* bin_count = nullptr;    // n_tiles + 1: per-tile counts, then scatter cursors
    int32_t* scan_part = nullptr;    // kScanTile + 1: block totals of the two-level scan
    // Heaviside accumulators (int64, zeroed after every use)
    long long* accA = nullptr;
    long long* accS = nullptr;
    // nearest-element keys per face (all ones after every use)
    unsigned long long* best = nullptr;  // dim * cells
    // offset vertices (4 surfaces)
    double* offv = nullptr;              // 4 * max_markers * dim
    // device marker buffers for 2D steps
    double* mX = nullptr;
    double* mfs = nullptr;
    double* mds = nullptr;
    double* mnrm = nullptr;
    // step intermediates
    double* H = nullptr;
    double* F[3] = {nullptr, nullptr, nullptr};
    double* beta[3] = {nullptr, nullptr, nullptr};
    double* rho = nullptr;
    bool beta_from_rho = false;   // the step's beta was not stored: form it from rho
    double* b = nullptr;
    // flags / scalars
    int* flags = nullptr;                // [0] geometry error, [1] band face without element
    double* red = nullptr;               // reduction scratch
    int red_len = 0;
    double* host_red = nullptr;          // pinned host scalars
};

// launchers implemented in the .hip files
int launch_bin_markers(Ctx* c, const ib_surface* s, hipStream_t st);
int launch_interp(Ctx* c, const double* const u[3], const ib_surface* s, double* U, hipStream_t st);
int launch_spread_delta(Ctx* c, const ib_surface* s, double* const F[3], hipStream_t st);
int launch_heaviside(Ctx* c, const ib_surface* s, double* H, hipStream_t st);
int launch_irrot_force(Ctx* c, const ib_surface* s, const double* H, double* const F[3], hipStream_t st);
// beta (dim face arrays) and rho (cell densities) may each be null
int launch_coefficients(Ctx* c, const double* H, double rin, double rout, double* const beta[3],
                        double* rho, hipStream_t st);
// rhs / update: with rho (cell densities) set, the face coefficients are formed
// from it where they are used, 2 / (rho_c + rho_{c-e}), bitwise the stored beta
// (beta is then not read)
int launch_rhs(Ctx* c, const double* const us[3], const double* const F[3], const double* const beta[3],
               double dt, double* b, hipStream_t st, const double* rho = nullptr);
int launch_update(Ctx* c, const double* const us[3], const double* const F[3], const double* const beta[3],
                  const double* p, double dt, double* const un[3], hipStream_t st, const double* rho = nullptr);
int launch_diagnostics(Ctx* c, const double* p, const double* H, const double* const u[3],
                       const double* const F[3], ib_diag* out, hipStream_t st);
int read_flags(Ctx* c, int* host_flags, hipStream_t st);

// deterministic reduction helpers (fixed tree: block partials then one block)
int device_sum(const double* partials_in, int n, double* out_dev, hipStream_t st);
// two independent sums of n partials each in one launch (bitwise those of two
// device_sum calls)
int device_sum2(const double* partials0, const double* partials1, int n, double* out0, double* out1,
                hipStream_t st);

// pieces of the step shared by project_step and flow_step (api.hip)
int spread_impl(Ctx* c, const ib_surface* s, int mode, double* const F[3], double* H, hipStream_t st);
// axis_x: NaN, or the axis of a mirrored axisymmetric meridian curve (adds
// the azimuthal curvature to sigma kappa)
// mass_target: NULL, or the area / volume the relocated markers are corrected
// to (ib_mass_correct; its displacement to *mass_delta when not NULL)
int relocate_2d(Ctx* c, const ib_params* prm, ib_state* stt, const double* U_dev, double* fs_host,
                ib_surface* s, hipStream_t st, double axis_x, const double* mass_target,
                double* mass_delta);

// sum of rho over the cells (weighted == 0) or of rho (i + 1/2) h over the
// cells of an nr-wide meridian plane (weighted == 1), into *out (device);
// part holds at least kMeanParts partials
constexpr int kMeanParts = 1024;
int density_sum(const double* rho, long N, int nr, double h, int weighted, double* part, double* out,
                hipStream_t st);

// validation of the free-fall fields of ib_flow_params
int check_freefall(const ib_flow_params* fp, const char* who);
int coefficients_and_hierarchy(Ctx* c, mg_handle* m, const ib_params* prm, const double* H,
                               hipStream_t st);
int solve_and_update(Ctx* c, mg_handle* m, const ib_params* prm, ib_state* stt, ib_outputs* out,
                     const double* const u_star[3], const double* H, double* const F[3],
                     hipStream_t st);

}  // namespace ib

// the opaque context handle of the C ABI is the library's context
struct ib_ctx : ib::Ctx {};

// 1 when the multigrid's finest level reads cell densities directly (mg.hip)
int mg_takes_density(const mg_handle* m);
// the caller has just zeroed the next solve's initial guess (on the solve's
// stream): its first residual is b, so the first operator application is
// skipped (the same residual and norms bit for bit); cleared by that solve
void mg_hint_zero_guess(mg_handle* m);
// ||b - A x|| / ||b|| and the energy functional E(x) = x . (b + b - A x) of a
// start x (NULL: zero, E = 0); the smaller E, the smaller the error in the
// operator's energy norm; syncs (mg.hip)
int mg_energy(mg_handle* m, const double* b, const double* x, double* rel, double* E, hipStream_t st);
namespace ib {
// WS_NN: the network's guess into out->p, judged by multigrid against the
// fallback (stt->p_prev, or zero) and replaced by it when it loses; sets the
// guess fields of out (api.hip)
int nn_warm_start(mg_handle* m, ib_state* stt, ib_outputs* out, double rho_in, double rho_out,
                  const double* b, const double* H, long N, hipStream_t st);
}  // namespace ib
// cells of the grid the network handle was created for (0 for null)
long nn_cells(const ib_nn* nn);
