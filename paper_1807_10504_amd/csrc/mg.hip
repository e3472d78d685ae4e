// Geometric multigrid for the projection Poisson problem (Section 2.1: the
// centred second-order Laplacian of eq ps, solved by multigrid).
//
// (A p)_c = (1/h^2) sum_faces beta_f (p_nb - p_c), periodic, zero-mean p.
// Cell-centred V(nu1, nu2): red-black Gauss-Seidel (red = i+j+k even first),
// restriction = mean of the 2^dim children of the fine residual, cell-centred
// (bi/tri)linear prolongation (3/4, 1/4 per axis), coarse face coefficient =
// mean of the 2^(dim-1) fine faces on the coarse face, coarsest grid solved
// with the inverse of the bordered matrix [[A, 1], [1^T, 0]] (zero-mean
// constraint; solved through an SPD shift of the constant mode, see the
// coarsest-level kernels), mean of p removed (once, after the last cycle: the
// cycle commutes with adding a constant, so iterates differ from a per-cycle
// removal by a constant only).
//
// Mixed precision: the V-cycle in float32 (float32 coefficients cast from the
// float64 hierarchy) acting on fl32(b - A p), with the defect, the update
// p += e and the coarsest solve in float64.
//
// Memory layout: every level stores p, b and one coefficient array per axis
// (left faces) as SoA with x fastest; a finest level given by cell densities
// (mg_update_density) keeps only rho and its float64 kernels form each face
// coefficient where they use it. The smoother of large 3D levels is a
// single-pass tiled sweep; the others are one-thread-per-cell stencils.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "common.h"

namespace ib {

template <typename T>
struct LevelT {
    T* p = nullptr;
    T* b = nullptr;
    T* beta[3] = {nullptr, nullptr, nullptr};
    T* alt = nullptr;   // second p buffer for the single-pass smoother
};

struct Level {
    Dims d;
    LevelT<double> f64;
    LevelT<float> f32;
    bool own_pb = true;
    bool fused = false;  // single-pass smoother applies
    int tz = 0;          // its z-range per workgroup
    int rtz = 0;         // z-range of the density sweep (nx % 64 == 0)
    // finest level only: cell densities from which the float64 kernels form
    // the face coefficients themselves (f64.beta is then unused)
    const double* rho = nullptr;
    // ... and their float32 roundings, from which the float32 kernels of the
    // mixed-precision cycle form theirs in float32 (stored in f32.beta[0];
    // f32.beta[1..2] are then unused)
    const float* rho32 = nullptr;
    // finest level of the float64 density path inside the flexible CG: the
    // last post-smoothing sweep also leaves the partial inner products of
    // the preconditioned residual with b (and with dots_q when not null)
    bool dots_on = false;
    const double* dots_q = nullptr;
    double* dots_part = nullptr;
    const double* dots_r = nullptr;  // the float64 residual (float32 cycle)
};

}  // namespace ib

struct mg_handle {
    ib_grid g;
    mg_opts o;
    // the next solve starts from a guess its caller has just zeroed
    // (mg_hint_zero_guess): the first residual is then b itself
    bool x_zero = false;
    std::vector<ib::Level> lv;
    // coarsest dense solve
    int nc = 0;                 // coarsest cells
    double* cmat = nullptr;     // (nc+1)^2 bordered matrix
    double* cinv = nullptr;     // its inverse
    double* cwork = nullptr;    // coarsest rhs/solution in float64 (mixed)
    // reductions
    double* red = nullptr;      // block partials + scalars
    double* host = nullptr;     // pinned scalars
    // float64 buffers for the mixed defect loop are the caller's p and b
    bool coeffs_ready = false;
    // finest face arrays formed from densities on grids whose kernels cannot
    // read the densities directly
    double* beta0[3] = {nullptr, nullptr, nullptr};
    // flexible CG (krylov): residual r, preconditioned residual z (float64
    // V-cycle), direction d, q = A d; device scalars
    double* kr = nullptr;
    double* kz = nullptr;
    double* kd = nullptr;
    double* kd2 = nullptr;  // second direction buffer of the fused density-path update
    double* kq = nullptr;
    double* ks = nullptr;
    // first level run by the persistent coarse kernel (-1: none)
    int persist = -1;
};

namespace ib {

constexpr int kRed = 8192;
// residual checks skipped at most in a row on the predicted rate (an early,
// erratic rate must not carry the solve far past its tolerance)
constexpr int kMaxSkip = 4;

// ---------------------------------------------------------------------------
// optional event timing of finest-level launches
struct Prof {
    bool on = false;
    std::vector<hipEvent_t> pool;
    struct Pending {
        hipEvent_t a, b;
        int kind;
    };
    std::vector<Pending> pending;
    long long count[IB_PROF_KINDS] = {0};
    double ms[IB_PROF_KINDS] = {0};
};
static Prof g_prof;

static hipEvent_t prof_event() {
    if (!g_prof.pool.empty()) {
        hipEvent_t e = g_prof.pool.back();
        g_prof.pool.pop_back();
        return e;
    }
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

struct ProfScope {
    hipEvent_t a = nullptr, b = nullptr;
    int kind;
    hipStream_t st;
    ProfScope(int k, hipStream_t s, bool finest) : kind(k), st(s) {
        if (!g_prof.on || !finest) return;
        a = prof_event();
        b = prof_event();
        if (a && b) (void)hipEventRecord(a, st);
    }
    ~ProfScope() {
        if (!a || !b) return;
        (void)hipEventRecord(b, st);
        g_prof.pending.push_back({a, b, kind});
    }
};

// called after a stream synchronisation
static void prof_drain() {
    for (auto& p : g_prof.pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            g_prof.count[p.kind] += 1;
            g_prof.ms[p.kind] += ms;
        }
        g_prof.pool.push_back(p.a);
        g_prof.pool.push_back(p.b);
    }
    g_prof.pending.clear();
}

// ---------------------------------------------------------------------------
// index helpers
struct Nb {
    long c, xm, xp, ym, yp, zm, zp;
};

__device__ __forceinline__ Nb neighbours(const Dims& d, int i, int j, int k, int dim) {
    Nb n;
    n.c = ((long)k * d.ny + j) * d.nx + i;
    n.xm = i == 0 ? n.c + d.nx - 1 : n.c - 1;
    n.xp = i == d.nx - 1 ? n.c - (d.nx - 1) : n.c + 1;
    n.ym = j == 0 ? n.c + (long)(d.ny - 1) * d.nx : n.c - d.nx;
    n.yp = j == d.ny - 1 ? n.c - (long)(d.ny - 1) * d.nx : n.c + d.nx;
    if (dim == 3) {
        long pl = (long)d.nx * d.ny;
        n.zm = k == 0 ? n.c + (long)(d.nz - 1) * pl : n.c - pl;
        n.zp = k == d.nz - 1 ? n.c - (long)(d.nz - 1) * pl : n.c + pl;
    } else {
        n.zm = n.zp = n.c;
    }
    return n;
}

// Face coefficients of a level, read through one of two sources:
// stored per axis (the face on the low side of each cell) ...
template <typename T>
struct CoefArrays {
    const T* __restrict__ b0;
    const T* __restrict__ b1;
    const T* __restrict__ b2;
    __device__ T xl(const Nb& n) const { return b0[n.c]; }
    __device__ T xr(const Nb& n) const { return b0[n.xp]; }
    __device__ T yl(const Nb& n) const { return b1[n.c]; }
    __device__ T yr(const Nb& n) const { return b1[n.yp]; }
    __device__ T zl(const Nb& n) const { return b2[n.c]; }
    __device__ T zr(const Nb& n) const { return b2[n.zp]; }
};

// ... or formed from the cell densities, beta = 2 / (rho_hi + rho_lo) (the
// inverse of the mean density of the two cells; eq indicator with I = H).
// The operands and the division are those of the coefficient kernel, so the
// values are bitwise the stored ones.
struct CoefRho {
    const double* __restrict__ rho;
    __device__ double f(long hi, long lo) const { return 2.0 / (rho[hi] + rho[lo]); }
    __device__ double xl(const Nb& n) const { return f(n.c, n.xm); }
    __device__ double xr(const Nb& n) const { return f(n.xp, n.c); }
    __device__ double yl(const Nb& n) const { return f(n.c, n.ym); }
    __device__ double yr(const Nb& n) const { return f(n.yp, n.c); }
    __device__ double zl(const Nb& n) const { return f(n.c, n.zm); }
    __device__ double zr(const Nb& n) const { return f(n.zp, n.c); }
};

// ... or in float32 from float32 densities (the mixed-precision cycle's finest
// level on the density path), 2 / (rho_hi + rho_lo) rounded in float32
struct CoefRhoF {
    const float* __restrict__ rho;
    __device__ float f(long hi, long lo) const { return 2.0f / (rho[hi] + rho[lo]); }
    __device__ float xl(const Nb& n) const { return f(n.c, n.xm); }
    __device__ float xr(const Nb& n) const { return f(n.xp, n.c); }
    __device__ float yl(const Nb& n) const { return f(n.c, n.ym); }
    __device__ float yr(const Nb& n) const { return f(n.yp, n.c); }
    __device__ float zl(const Nb& n) const { return f(n.c, n.zm); }
    __device__ float zr(const Nb& n) const { return f(n.zp, n.c); }
};

// densities: where all neighbours share the cell's density, every face is
// 2 / (rho + rho) = 1 / rho exactly, and one division serves the six faces
template <int DIM>
__device__ __forceinline__ double apply_row_rho(const double* __restrict__ p, const CoefRho& co,
                                                const Nb& n) {
    const double* __restrict__ r = co.rho;
    const double rc = r[n.c];
    const double rxp = r[n.xp], rxm = r[n.xm], ryp = r[n.yp], rym = r[n.ym];
    const double rzp = DIM == 3 ? r[n.zp] : rc, rzm = DIM == 3 ? r[n.zm] : rc;
    double bxp, bxm, byp, bym, bzp, bzm;
    if (rxp == rc && rxm == rc && ryp == rc && rym == rc && rzp == rc && rzm == rc) {
        bxp = bxm = byp = bym = bzp = bzm = 1.0 / rc;
    } else {
        bxp = 2.0 / (rxp + rc);
        bxm = 2.0 / (rc + rxm);
        byp = 2.0 / (ryp + rc);
        bym = 2.0 / (rc + rym);
        bzp = 2.0 / (rzp + rc);
        bzm = 2.0 / (rc + rzm);
    }
    const double pc = p[n.c];
    double s = bxp * (p[n.xp] - pc) - bxm * (pc - p[n.xm]);
    s += byp * (p[n.yp] - pc) - bym * (pc - p[n.ym]);
    if (DIM == 3) s += bzp * (p[n.zp] - pc) - bzm * (pc - p[n.zm]);
    return s;
}

template <typename T, int DIM, class K>
__device__ __forceinline__ T apply_row(const T* __restrict__ p, const K& co, const Nb& n) {
    if constexpr (std::is_same<K, CoefRho>::value) {
        return apply_row_rho<DIM>(p, co, n);
    } else {
        // sum_d br (p_r - p) - bl (p - p_l), without the 1/h^2
        T pc = p[n.c];
        T s = co.xr(n) * (p[n.xp] - pc) - co.xl(n) * (pc - p[n.xm]);
        s += co.yr(n) * (p[n.yp] - pc) - co.yl(n) * (pc - p[n.ym]);
        if (DIM == 3) s += co.zr(n) * (p[n.zp] - pc) - co.zl(n) * (pc - p[n.zm]);
        return s;
    }
}

// ---------------------------------------------------------------------------
// smoother: one colour of red-black Gauss-Seidel, one thread per cell of the colour.
// ZERO: the red pass of a sweep that starts from p = 0 (p is neither filled nor
// read: every neighbour term is +0, the value the filled array gives, so the
// result is the same bit for bit; the black pass then reads only red cells)
template <typename T, int DIM, bool ZERO = false>
__global__ void k_rbgs(T* __restrict__ p, const T* __restrict__ b, const T* __restrict__ b0,
                       const T* __restrict__ b1, const T* __restrict__ b2, Dims d, T h2, int color) {
    long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    int hx = d.nx >> 1;
    long half = d.cells() >> 1;
    if (t >= half) return;
    int i2 = (int)(t % hx);
    long r = t / hx;
    int j = (int)(r % d.ny);
    int k = (int)(r / d.ny);
    int i = 2 * i2 + ((j + k + color) & 1);
    Nb n = neighbours(d, i, j, k, DIM);
    T br = b0[n.xp], bl = b0[n.c];
    T num = ZERO ? T(0) : br * p[n.xp] + bl * p[n.xm];
    T diag = br + bl;
    br = b1[n.yp];
    bl = b1[n.c];
    if (!ZERO) num += br * p[n.yp] + bl * p[n.ym];
    diag += br + bl;
    if (DIM == 3) {
        br = b2[n.zp];
        bl = b2[n.c];
        if (!ZERO) num += br * p[n.zp] + bl * p[n.zm];
        diag += br + bl;
    }
    p[n.c] = (num - h2 * b[n.c]) / diag;
}

// One full red-black sweep in a single pass (3D levels with nx % 32 == 0,
// ny % 8 == 0, nz even). A workgroup owns a 32 x 8 column tile and an even
// z-range [z0, z1) and marches upward; at plane step k it updates the red
// cells of plane k on the tile plus a one-cell ring, then the black cells of
// plane k - 1 on the tile, then writes plane k - 1. Red values on the ring are
// recomputed (the neighbour tile computes the same numbers from the same
// inputs), and p is double-buffered (read pin, write pout), so workgroups
// never read what another one writes during the sweep. It performs the same
// arithmetic as the two-colour sweep: red reads only old black values, black
// reads only new red values. Lanes are dealt cells of the colour being
// updated only. The planes of a step are loaded into registers two steps
// ahead (two alternating stages) and staged in LDS at the step. Halo rows
// and columns are re-read by the neighbouring tiles; consecutive workgroups
// of one XCD get neighbouring tiles so that part of those reads hit its L2.
constexpr int kFTX = 32, kFTY = 8;
constexpr int kFRX = kFTX + 4, kFRY = kFTY + 4, kFRN = kFRX * kFRY;   // p: tile + 2-cell halo
// coefficient planes are staged on the smaller regions the updates read:
// beta_x on x in [1, RX), y in [1, RY-1); beta_y on x in [1, RX-1), y in [1, RY);
// beta_z and b on the one-cell ring x in [1, RX-1), y in [1, RY-1)
constexpr int kFXW = kFRX - 1, kFXN = kFXW * (kFRY - 2);
constexpr int kFYW = kFRX - 2, kFYN = kFYW * (kFRY - 1);
constexpr int kFZW = kFRX - 2, kFZN = kFZW * (kFRY - 2);
// red updates cover the one-cell ring region (kFRX - 2) x (kFRY - 2), black
// updates the tile; each row holds half its cells of either colour
constexpr int kFRedRow = (kFRX - 2) / 2, kFRedN = kFRedRow * (kFRY - 2);
constexpr int kFBlackRow = kFTX / 2, kFBlackN = kFBlackRow * kFTY;
constexpr int kFLoads = (kFRN + kBlock - 1) / kBlock;
constexpr int kFXLoads = (kFXN + kBlock - 1) / kBlock;
constexpr int kFYLoads = (kFYN + kBlock - 1) / kBlock;
constexpr int kFZLoads = (kFZN + kBlock - 1) / kBlock;

// two adjacent values of T in one memory operation
template <typename T>
using Vec2 = typename std::conditional<sizeof(T) == 8, double2, float2>::type;

// barrier for LDS traffic only: global loads issued before it stay in flight
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

__device__ __forceinline__ int mod3(int k) { return ((k % 3) + 3) % 3; }

template <typename T, bool ZERO>
__global__ __launch_bounds__(kBlock) void k_rbgs_fused(const T* __restrict__ pin, T* __restrict__ pout,
                                                       const T* __restrict__ bb, const T* __restrict__ bx,
                                                       const T* __restrict__ by, const T* __restrict__ bz,
                                                       Dims d, T h2, int TZ, int ntx, int nty, int nzc) {
    __shared__ T P[4][kFRN];
    __shared__ T BX[2][kFXN];
    __shared__ T BY[2][kFYN];
    __shared__ T BZ[3][kFZN];
    __shared__ T B[2][kFZN];
    const int nw = ntx * nty * nzc;
    const int bid = blockIdx.x;
    // blocks are dealt round-robin to the 8 XCDs: give each XCD a contiguous
    // range of tiles so that halo rows are shared in its L2
    const int w = (nw % 8 == 0) ? (bid % 8) * (nw / 8) + bid / 8 : bid;
    const int tx = w % ntx;
    const int r0 = w / ntx;
    const int ty = r0 % nty;
    const int zc = r0 / nty;
    const int i0 = tx * kFTX - 2, j0 = ty * kFTY - 2;
    const int z0 = zc * TZ, z1 = z0 + TZ;
    const long plane = (long)d.nx * d.ny;
    using V2 = Vec2<T>;
    const int t = threadIdx.x;
    // tile origins are at least -2 and regions end within one period
    auto gofs = [&](int x, int y) { return wrap_near(j0 + y, d.ny) * d.nx + wrap_near(i0 + x, d.nx); };
    // every lane issues every load (slots past a region re-read its first
    // cell and are not stored): unconditional loads give exact wait counts
    int gp[kFLoads], gx[kFXLoads], gy[kFYLoads], gz[kFZLoads];
    bool vp[kFLoads], vx[kFXLoads], vy[kFYLoads], vz[kFZLoads];
#pragma unroll
    for (int s = 0; s < kFLoads; ++s) {
        int q = t + s * kBlock;
        vp[s] = q < kFRN;
        gp[s] = vp[s] ? gofs(q % kFRX, q / kFRX) : gofs(0, 0);
    }
#pragma unroll
    for (int s = 0; s < kFXLoads; ++s) {
        int q = t + s * kBlock;
        vx[s] = q < kFXN;
        gx[s] = vx[s] ? gofs(1 + q % kFXW, 1 + q / kFXW) : gofs(1, 1);
    }
#pragma unroll
    for (int s = 0; s < kFYLoads; ++s) {
        int q = t + s * kBlock;
        vy[s] = q < kFYN;
        gy[s] = vy[s] ? gofs(1 + q % kFYW, 1 + q / kFYW) : gofs(1, 1);
    }
#pragma unroll
    for (int s = 0; s < kFZLoads; ++s) {
        int q = t + s * kBlock;
        vz[s] = q < kFZN;
        gz[s] = vz[s] ? gofs(1 + q % kFZW, 1 + q / kFZW) : gofs(1, 1);
    }
    // planes z0 - 2 .. z1 + 2 lie within one period of the box
    auto pl = [&](int k) { return (long)wrap_near(k, d.nz) * plane; };
    // two register stages, alternating, each holding the planes of one step:
    // p(k+1), beta_x/y(k), b(k), beta_z(k+1), loaded two steps ahead
    struct Stage {
        T p[kFLoads], x[kFXLoads], y[kFYLoads], b[kFZLoads], z[kFZLoads];
    };
    Stage SA, SB;
    auto fetch = [&](Stage& S, int k) {
        long bp = pl(k + 1), bk = pl(k);
#pragma unroll
        for (int s = 0; s < kFLoads; ++s) S.p[s] = ZERO ? T(0) : pin[bp + gp[s]];
#pragma unroll
        for (int s = 0; s < kFXLoads; ++s) S.x[s] = bx[bk + gx[s]];
#pragma unroll
        for (int s = 0; s < kFYLoads; ++s) S.y[s] = by[bk + gy[s]];
#pragma unroll
        for (int s = 0; s < kFZLoads; ++s) {
            S.b[s] = bb[bk + gz[s]];
            S.z[s] = bz[bp + gz[s]];
        }
    };
    auto commit = [&](const Stage& S, int k) {
#pragma unroll
        for (int s = 0; s < kFLoads; ++s)
            if (s * kBlock + kBlock <= kFRN || vp[s]) P[(k + 1) & 3][t + s * kBlock] = S.p[s];
#pragma unroll
        for (int s = 0; s < kFXLoads; ++s)
            if (s * kBlock + kBlock <= kFXN || vx[s]) BX[k & 1][t + s * kBlock] = S.x[s];
#pragma unroll
        for (int s = 0; s < kFYLoads; ++s)
            if (s * kBlock + kBlock <= kFYN || vy[s]) BY[k & 1][t + s * kBlock] = S.y[s];
#pragma unroll
        for (int s = 0; s < kFZLoads; ++s)
            if (s * kBlock + kBlock <= kFZN || vz[s]) {
                B[k & 1][t + s * kBlock] = S.b[s];
                BZ[mod3(k + 1)][t + s * kBlock] = S.z[s];
            }
    };
    {
        long a = pl(z0 - 2), a1 = pl(z0 - 1);
#pragma unroll
        for (int s = 0; s < kFLoads; ++s)
            if (vp[s]) {
                P[(z0 - 2) & 3][t + s * kBlock] = ZERO ? T(0) : pin[a + gp[s]];
                P[(z0 - 1) & 3][t + s * kBlock] = ZERO ? T(0) : pin[a1 + gp[s]];
            }
#pragma unroll
        for (int s = 0; s < kFZLoads; ++s)
            if (vz[s]) BZ[mod3(z0 - 1)][t + s * kBlock] = bz[a1 + gz[s]];
    }
    fetch(SA, z0 - 1);
    // keep stage A's loads ahead of stage B's (the wait counts assume that order)
    __builtin_amdgcn_sched_barrier(0);
    fetch(SB, z0);
    // one cell update at region position (x, y) of plane kk
    auto update = [&](int x, int y, int kk) {
        const int c = y * kFRX + x;
        const int ix = (y - 1) * kFXW + (x - 1);
        const int iz = (y - 1) * kFZW + (x - 1);
        const T* Pc = P[kk & 3];
        const T* Pd = P[(kk - 1) & 3];
        const T* Pu = P[(kk + 1) & 3];
        const T* X = BX[kk & 1];
        const T* Y = BY[kk & 1];
        T br = X[ix + 1], bl = X[ix];
        T num = br * Pc[c + 1] + bl * Pc[c - 1];
        T diag = br + bl;
        br = Y[iz + kFYW];
        bl = Y[iz];
        num += br * Pc[c + kFRX] + bl * Pc[c - kFRX];
        diag += br + bl;
        br = BZ[mod3(kk + 1)][iz];
        bl = BZ[mod3(kk)][iz];
        num += br * Pu[c] + bl * Pd[c];
        diag += br + bl;
        return (num - h2 * B[kk & 1][iz]) / diag;
    };
    auto step = [&](Stage& S, int k) {
        commit(S, k);
        // in flight for two steps; past the range it re-reads plane z1 (not
        // committed), which keeps the loads unconditional
        fetch(S, k + 2 <= z1 ? k + 2 : z1);
        lds_barrier();
        // red cells of plane k on the tile and its one-cell ring (only
        // those: every lane has a cell of the colour)
        for (int q = t; q < kFRedN; q += kBlock) {
            int y = 1 + q / kFRedRow;
            int x = 1 + ((i0 + 1 + j0 + y + k) & 1) + 2 * (q % kFRedRow);
            P[k & 3][y * kFRX + x] = update(x, y, k);
        }
        lds_barrier();
        const int kb = k - 1;
        if (kb >= z0 && kb < z1) {
            // black cells of plane k - 1 on the tile; plane k - 1 is then
            // final: each lane writes its black cell and the red cell beside
            // it (computed a step earlier), and no one reads black values of
            // this plane from LDS again
            const long base = pl(kb) + (long)(j0 + 2) * d.nx + (i0 + 2);
            for (int q = t; q < kFBlackN; q += kBlock) {
                int y = 2 + q / kFBlackRow, m = q % kFBlackRow;
                int par = (i0 + 3 + j0 + y + kb) & 1;
                T v = update(2 + par + 2 * m, y, kb);
                T r = P[kb & 3][y * kFRX + 3 - par + 2 * m];
                // the black cell and the red one beside it in one 2-wide store
                // (the pair starts at an even x: 16-byte aligned in float64)
                V2 w2;
                w2.x = par ? r : v;
                w2.y = par ? v : r;
                *reinterpret_cast<V2*>(pout + base + (long)(y - 2) * d.nx + 2 * m) = w2;
            }
        }
        // the next commit overwrites the plane below k - 1
        lds_barrier();
    };
    // steps z0 - 1 .. z1 in pairs (stage A, stage B); TZ is even
    for (int k = z0 - 1; k <= z1; k += 2) {
        step(SA, k);
        step(SB, k + 1);
    }
}

// One fine cell's share of the cell-centred linear prolongation from its
// eight coarse neighbours (3/4 and 1/4 per axis), every product and sum
// rounded on its own as in k_prolong_add_blk: e111 is the coarse parent,
// e11x its neighbour along x, e1y1 along y, ez11 along z, and so on.
template <typename T>
__device__ __forceinline__ T prolong_cell(T e111, T e11x, T e1y1, T e1yx, T ez11, T ez1x, T ezy1, T ezyx) {
#pragma clang fp contract(off)
    const T a = T(0.75), q = T(0.25);
    const T r00 = a * e111 + q * e11x;
    const T r01 = a * e1y1 + q * e1yx;
    const T r10 = a * ez11 + q * ez1x;
    const T r11 = a * ezy1 + q * ezyx;
    return a * (a * r00 + q * r01) + q * (a * r10 + q * r11);
}

// The same single-pass sweep on a finest level given by cell densities: the
// workgroup stages p and rho on the tile plus the two-cell halo in LDS and
// forms each face coefficient 2 / (rho_hi + rho_lo) where it is used (in T:
// float64, or float32 from the float32 densities of the mixed-precision
// cycle). b is read once per update straight into the registers of the lane
// that makes it (two steps ahead, like p and rho), so LDS holds p and rho
// only: 58 KB for a 32 x 16 float64 tile, two workgroups per CU. That is 32
// bytes of memory traffic per cell (p read and written, b, rho) instead of 48
// with three stored face arrays; the update is the one above, operand for
// operand, so the results are bitwise those of the stored-face sweep.
// DOTS (1 or 2): the sweep also leaves per-workgroup partial sums of
// (b, p_new) and, for DOTS = 2, (qv, p_new) in part[bid] and part[nwg + bid]
// (the flexible-CG inner products of the preconditioned residual, taken from
// the values the black lanes write); qv is read in pairs two steps ahead,
// like b. The float32 sweep of the mixed cycle takes them in float64 against
// the float64 residual rv instead of its fl32(b), also read in pairs.
// PRO: the sweep starts from p + P ec, the coarse correction ec (on the grid
// of half the cells along each axis) prolongated as each plane is staged, in
// the order and rounding of k_prolong_add_blk, so the result is bitwise that
// of prolongating first; p + P ec is never stored.
template <typename T, int TX, int TY, int NT, bool ZERO, int DOTS = 0, bool PRO = false>
__global__ __launch_bounds__(NT) void k_rbgs_fused_rho(const T* __restrict__ pin,
                                                       T* __restrict__ pout,
                                                       const T* __restrict__ bb,
                                                       const T* __restrict__ rho, Dims d,
                                                       T h2, int TZ, int ntx, int nty,
                                                       int nzc, const double* __restrict__ qv = nullptr,
                                                       double* __restrict__ part = nullptr,
                                                       const T* __restrict__ ec = nullptr,
                                                       const double* __restrict__ rv = nullptr) {
    // region of p and rho: the tile and a two-cell halo
    constexpr int RX = TX + 4, RY = TY + 4, RN = RX * RY;
    // p and rho move in pairs of cells along x (the region starts at an even x
    // and RX is even, so pair q is cells 2q, 2q + 1 of the region and a pair
    // never straddles the periodic seam)
    constexpr int RN2 = RN / 2;
    static_assert(RX % 2 == 0 && TX % 2 == 0, "the region must split into pairs along x");
    constexpr int NL = (RN2 + NT - 1) / NT;
    // red updates: the one-cell ring region, half of each row; black updates:
    // the tile, one lane per pair of cells (its black cell and the red one
    // beside it, which it also writes)
    constexpr int RedRow = (RX - 2) / 2, RedN = RedRow * (RY - 2);
    constexpr int BlackRow = TX / 2, BlackN = BlackRow * TY;
    constexpr int NR = (RedN + NT - 1) / NT, NB = (BlackN + NT - 1) / NT;
    static_assert(!PRO || (!ZERO && DOTS == 0), "the prolongation starts a plain sweep");
    constexpr int NQ = DOTS == 2 ? NB : 0;
    // float32 inner products: the float64 residual's pairs of the black lanes
    constexpr int NRV = (DOTS > 0 && sizeof(T) == 4) ? NB : 0;
    // PRO: the coarse cells under the region and one more on each side (the
    // region starts at an even x and y, so it covers whole coarse cells), in a
    // ring of three coarse planes; NC loads per lane fill one coarse plane
    constexpr int CX = RX / 2 + 2, CY = RY / 2 + 2, CN = CX * CY;
    constexpr int NC = PRO ? (CN + NT - 1) / NT : 0;
    __shared__ T EC[PRO ? 3 : 1][PRO ? CN : 1];
    // rings of five planes: the black update of plane k - 1 reads planes
    // k - 2 .. k while the next step already stages plane k + 2, so no
    // barrier separates them
    __shared__ __align__(16) T P[5][RN];
    __shared__ __align__(16) T R[5][RN];
    __shared__ double red[DOTS ? 2 * (NT / 64) : 1];
    double acc_b = 0.0, acc_q = 0.0;
    const int nw = ntx * nty * nzc;
    const int bid = blockIdx.x;
    const int w = (nw % 8 == 0) ? (bid % 8) * (nw / 8) + bid / 8 : bid;
    const int tx = w % ntx;
    const int r0 = w / ntx;
    const int ty = r0 % nty;
    const int zc = r0 / nty;
    const int i0 = tx * TX - 2, j0 = ty * TY - 2;
    const int z0 = zc * TZ, z1 = z0 + TZ;
    const long plane = (long)d.nx * d.ny;
    using V2 = Vec2<T>;
    const int t = threadIdx.x;
    // tile origins are at least -2 and regions end within one period
    auto gofs = [&](int x, int y) { return wrap_near(j0 + y, d.ny) * d.nx + wrap_near(i0 + x, d.nx); };
    // every lane issues every load (slots past a region re-read its first
    // cell or pair and are not used), so the loads are unconditional and the
    // compiler's wait counts are exact: a step waits for its own plane only,
    // not for the loads and stores issued after it
    int gp[NL];
    bool vp[NL];
#pragma unroll
    for (int s = 0; s < NL; ++s) {
        int q = t + s * NT;
        vp[s] = q < RN2;
        gp[s] = vp[s] ? gofs(2 * (q % (RX / 2)), q / (RX / 2)) : gofs(0, 0);
    }
    // b of a lane's red cell (row ry, x = 1 + e + 2 c with e the parity of the
    // plane's first red cell in that row) and of its black pair (tile cells,
    // never across the seam)
    int gr[NR][2], er[NR], gb[NB];
#pragma unroll
    for (int s = 0; s < NR; ++s) {
        int q = t + s * NT;
        q = q < RedN ? q : 0;
        const int y = 1 + q / RedRow, c = q % RedRow;
        er[s] = (i0 + 1 + j0 + y) & 1;
        gr[s][0] = gofs(1 + 2 * c, y);
        gr[s][1] = gofs(2 + 2 * c, y);
    }
#pragma unroll
    for (int s = 0; s < NB; ++s) {
        int q = t + s * NT;
        q = q < BlackN ? q : 0;
        gb[s] = (j0 + 2 + q / BlackRow) * d.nx + (i0 + 2) + 2 * (q % BlackRow);
    }
    // planes z0 - 2 .. z1 + 2 lie within one period of the box
    auto pl = [&](int k) { return (long)wrap_near(k, d.nz) * plane; };
    // coarse cell q of the ring's planes (origin (i0 / 2 - 1, j0 / 2 - 1), at
    // least -2 and within one coarse period); coarse planes z0 / 2 - 2 ..
    // z1 / 2 + 3 likewise
    const int cnx = d.nx >> 1, cny = d.ny >> 1, cnz = d.nz >> 1;
    int gc[NC > 0 ? NC : 1];
#pragma unroll
    for (int s = 0; s < NC; ++s) {
        int q = t + s * NT;
        q = q < CN ? q : 0;
        gc[s] = wrap_near(j0 / 2 - 1 + q / CX, cny) * cnx + wrap_near(i0 / 2 - 1 + q % CX, cnx);
    }
    auto cpl = [&](int c) { return (long)wrap_near(c, cnz) * cny * cnx; };
    auto s3 = [](int c) { return (c + 300) % 3; };
    // P ec at region cells 2u, 2u + 1 of row y on plane kk: the even cell's
    // second coarse neighbour along x is the one below, the odd cell's the one
    // above; along y and z the parity of the row and plane decides the same way
    auto prolong2 = [&](int y, int u, int kk, T& v0, T& v1) {
        const int K = kk >> 1;
        const T* E1 = EC[s3(K)];
        const T* E2 = EC[s3((kk & 1) ? K + 1 : K - 1)];
        const int cy = (y >> 1) + 1, cy2 = (y & 1) ? cy + 1 : cy - 1;
        const int o1 = cy * CX + u + 1, o2 = cy2 * CX + u + 1;
        v0 = prolong_cell<T>(E1[o1], E1[o1 - 1], E1[o2], E1[o2 - 1], E2[o1], E2[o1 - 1], E2[o2], E2[o2 - 1]);
        v1 = prolong_cell<T>(E1[o1], E1[o1 + 1], E1[o2], E1[o2 + 1], E2[o1], E2[o1 + 1], E2[o2], E2[o2 + 1]);
    };
    // two register stages, alternating. A stage holds what step k reads from
    // memory: p and rho of plane k + 1 (committed to LDS at the step's start,
    // loaded two steps ahead), b of its red cells on plane k and the b (and
    // qv) pairs of its black cells on plane k - 1 (used after the step's
    // barriers, loaded at the end of step k - 2). Every value is consumed
    // before the stage is loaded again, so no loaded register is copied and
    // no wait drains the loads issued after it.
    // PRO: stage A (the odd steps 2m + 1) also carries coarse plane m + 2,
    // loaded at the end of step 2m - 1 and staged after the first barrier
    struct Stage {
        V2 p[NL], r[NL];
        T br[NR];
        V2 bk[NB];
        double2 qk[NQ > 0 ? NQ : 1];
        double2 rk[NRV > 0 ? NRV : 1];
        T ce[NC > 0 ? NC : 1];
    };
    Stage SA, SB;
    auto ld2 = [](const T* a) { return *reinterpret_cast<const V2*>(a); };
    auto fetch_pr = [&](Stage& S, int k) {
        const long bp = pl(k + 1);
#pragma unroll
        for (int s = 0; s < NL; ++s) {
            if constexpr (ZERO) {
                S.p[s].x = T(0);
                S.p[s].y = T(0);
            } else {
                S.p[s] = ld2(pin + bp + gp[s]);
            }
            S.r[s] = ld2(rho + bp + gp[s]);
        }
    };
    auto fetch_b = [&](Stage& S, int k) {
        const long bk = pl(k), bq = pl(k - 1);
#pragma unroll
        for (int s = 0; s < NR; ++s) S.br[s] = bb[bk + gr[s][(er[s] + k) & 1]];
#pragma unroll
        for (int s = 0; s < NB; ++s) S.bk[s] = ld2(bb + bq + gb[s]);
#pragma unroll
        for (int s = 0; s < NQ; ++s) S.qk[s] = *reinterpret_cast<const double2*>(qv + bq + gb[s]);
#pragma unroll
        for (int s = 0; s < NRV; ++s) S.rk[s] = *reinterpret_cast<const double2*>(rv + bq + gb[s]);
    };
    auto fetch_c = [&](Stage& S, int c) {
#pragma unroll
        for (int s = 0; s < NC; ++s) S.ce[s] = ec[cpl(c) + gc[s]];
    };
    auto stage_c = [&](const Stage& S, int c) {
#pragma unroll
        for (int s = 0; s < NC; ++s)
            if (s * NT + NT <= CN || t + s * NT < CN) EC[s3(c)][t + s * NT] = S.ce[s];
    };
    // ring slots; planes k >= z0 - 2 >= -2
    auto s5 = [](int k) { return (k + 10) % 5; };
    auto commit = [&](const Stage& S, int k) {
        T* Pn = P[s5(k + 1)];
        T* Rn = R[s5(k + 1)];
#pragma unroll
        for (int s = 0; s < NL; ++s)
            if (s * NT + NT <= RN2 || vp[s]) {
                V2 pv = S.p[s];
                if constexpr (PRO) {
                    const int q = t + s * NT;
                    T v0, v1;
                    prolong2(q / (RX / 2), q % (RX / 2), k + 1, v0, v1);
                    pv.x = pv.x + v0;
                    pv.y = pv.y + v1;
                }
                *reinterpret_cast<V2*>(Pn + 2 * (t + s * NT)) = pv;
                *reinterpret_cast<V2*>(Rn + 2 * (t + s * NT)) = S.r[s];
            }
    };
    if constexpr (PRO) {
        // coarse planes z0 / 2 - 2 .. z0 / 2 serve the first three fine planes
        for (int c = z0 / 2 - 2; c <= z0 / 2; ++c) {
            fetch_c(SA, c);
            stage_c(SA, c);
        }
        __syncthreads();
    }
    {
        long a = pl(z0 - 2), a1 = pl(z0 - 1);
#pragma unroll
        for (int s = 0; s < NL; ++s)
            if (vp[s]) {
                const int q = t + s * NT, c2 = 2 * q;
                T v[2][2] = {{T(0), T(0)}, {T(0), T(0)}};
                if constexpr (PRO) {
                    prolong2(q / (RX / 2), q % (RX / 2), z0 - 2, v[0][0], v[0][1]);
                    prolong2(q / (RX / 2), q % (RX / 2), z0 - 1, v[1][0], v[1][1]);
                }
                for (int e = 0; e < 2; ++e) {
                    T pa = ZERO ? T(0) : pin[a + gp[s] + e];
                    T pb = ZERO ? T(0) : pin[a1 + gp[s] + e];
                    if constexpr (PRO) {
                        pa = pa + v[0][e];
                        pb = pb + v[1][e];
                    }
                    P[s5(z0 - 2)][c2 + e] = pa;
                    P[s5(z0 - 1)][c2 + e] = pb;
                    R[s5(z0 - 2)][c2 + e] = rho[a + gp[s] + e];
                    R[s5(z0 - 1)][c2 + e] = rho[a1 + gp[s] + e];
                }
            }
    }
    fetch_pr(SA, z0 - 1);
    fetch_b(SA, z0 - 1);
    if constexpr (PRO) fetch_c(SA, z0 / 2 + 1);
    // keep stage A's loads ahead of stage B's (the wait counts assume that order)
    __builtin_amdgcn_sched_barrier(0);
    fetch_pr(SB, z0);
    fetch_b(SB, z0);
    // plane slots of kk - 1, kk, kk + 1
    struct Slots {
        int d, c, u;
    };
    auto slots = [&](int kk) { return Slots{s5(kk - 1), s5(kk), s5(kk + 1)}; };
    auto update = [&](int x, int y, const Slots& sl, T bv) {
        const int c = y * RX + x;
        const T* Pc = P[sl.c];
        const T* Pd = P[sl.d];
        const T* Pu = P[sl.u];
        const T* Rc = R[sl.c];
        const T rc = Rc[c];
        const T rxp = Rc[c + 1], rxm = Rc[c - 1], ryp = Rc[c + RX], rym = Rc[c - RX];
        const T rzp = R[sl.u][c], rzm = R[sl.d][c];
        if (rxp == rc && rxm == rc && ryp == rc && rym == rc && rzp == rc && rzm == rc) {
            // away from the interface every face is 1 / rc and the update is
            // (sum of the six neighbours - h^2 b rc) / 6: no division
            const T sn = ((Pc[c + 1] + Pc[c - 1]) + (Pc[c + RX] + Pc[c - RX])) + (Pu[c] + Pd[c]);
            return (sn - h2 * bv * rc) * T(1.0 / 6.0);
        }
        const T bxp = T(2) / (rxp + rc);
        const T bxm = T(2) / (rc + rxm);
        const T byp = T(2) / (ryp + rc);
        const T bym = T(2) / (rc + rym);
        const T bzp = T(2) / (rzp + rc);
        const T bzm = T(2) / (rc + rzm);
        T num = bxp * Pc[c + 1] + bxm * Pc[c - 1];
        T diag = bxp + bxm;
        num += byp * Pc[c + RX] + bym * Pc[c - RX];
        diag += byp + bym;
        num += bzp * Pu[c] + bzm * Pd[c];
        diag += bzp + bzm;
        return (num - h2 * bv) / diag;
    };
    // ODD: stage A's steps k = 2m + 1 (z0 is even)
    auto step = [&](Stage& S, int k, auto odd) {
        commit(S, k);
        // past the range the loads re-read plane z1 (not used), which keeps
        // them unconditional
        const int kn = k + 2 <= z1 ? k + 2 : z1;
        fetch_pr(S, kn);
        lds_barrier();
        if constexpr (PRO && decltype(odd)::value) {
            // coarse plane m + 2 replaces m - 1, last read by the commit of
            // fine plane 2m at step 2m - 1; first read at step 2m + 2, after
            // this step's second barrier
            stage_c(S, (k - 1) / 2 + 2);
        }
        const Slots sr = slots(k);
#pragma unroll
        for (int s = 0; s < NR; ++s) {
            const int q = t + s * NT;
            if (q < RedN) {
                int y = 1 + q / RedRow;
                int x = 1 + ((i0 + 1 + j0 + y + k) & 1) + 2 * (q % RedRow);
                P[sr.c][y * RX + x] = update(x, y, sr, S.br[s]);
            }
        }
        lds_barrier();
        const int kb = k - 1;
        if (kb >= z0 && kb < z1) {
            const Slots sb = slots(kb);
            const long base = pl(kb) + (long)(j0 + 2) * d.nx + (i0 + 2);
#pragma unroll
            for (int s = 0; s < NB; ++s) {
                const int q = t + s * NT;
                if (q < BlackN) {
                    int y = 2 + q / BlackRow, m = q % BlackRow;
                    int par = (i0 + 3 + j0 + y + kb) & 1;
                    const T bv = par ? S.bk[s].y : S.bk[s].x;
                    T v = update(2 + par + 2 * m, y, sb, bv);
                    T r = P[sb.c][y * RX + 3 - par + 2 * m];
                    // the black cell and the red one beside it in one 2-wide store
                    // (the pair starts at an even x: 16-byte aligned in float64)
                    V2 w2;
                    w2.x = par ? r : v;
                    w2.y = par ? v : r;
                    *reinterpret_cast<V2*>(pout + base + (long)(y - 2) * d.nx + 2 * m) = w2;
                    if constexpr (DOTS > 0 && sizeof(T) == 8) {
                        const T br2 = par ? S.bk[s].x : S.bk[s].y;
                        acc_b += bv * v + br2 * r;
                    } else if constexpr (DOTS > 0) {
                        const double rb = par ? S.rk[s].y : S.rk[s].x;
                        const double rr = par ? S.rk[s].x : S.rk[s].y;
                        acc_b += rb * (double)v + rr * (double)r;
                    }
                    if constexpr (DOTS == 2) {
                        const double qb = par ? S.qk[s].y : S.qk[s].x;
                        const double qr = par ? S.qk[s].x : S.qk[s].y;
                        acc_q += qb * (double)v + qr * (double)r;
                    }
                }
            }
        }
        fetch_b(S, kn);
        if constexpr (PRO && decltype(odd)::value) fetch_c(S, (k - 1) / 2 + 3);
        // no barrier here: the next step's commit writes the slots of plane
        // k - 3, which this black update does not read, and its first barrier
        // orders everything after
    };
    // steps z0 - 1 .. z1 in pairs (stage A, stage B); TZ is even
    for (int k = z0 - 1; k <= z1; k += 2) {
        step(SA, k, std::true_type{});
        step(SB, k + 1, std::false_type{});
    }
    if constexpr (DOTS > 0) {
        // fixed-order workgroup sums
        for (int off = 32; off > 0; off >>= 1) {
            acc_b += __shfl_xor(acc_b, off);
            acc_q += __shfl_xor(acc_q, off);
        }
        if ((t & 63) == 0) {
            red[t >> 6] = acc_b;
            red[NT / 64 + (t >> 6)] = acc_q;
        }
        __syncthreads();
        if (t == 0) {
            double sb = 0.0, sq = 0.0;
            for (int i = 0; i < NT / 64; ++i) {
                sb += red[i];
                sq += red[NT / 64 + i];
            }
            part[bid] = sb;
            part[nw + bid] = sq;
        }
    }
}

// residual of the fine level restricted to the coarse right side
template <typename T, int DIM>
__global__ void k_residual_restrict(const T* __restrict__ p, const T* __restrict__ b,
                                    CoefArrays<T> co, Dims f, T inv_h2, T* __restrict__ bc) {
    long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    int cx = f.nx >> 1, cy = f.ny >> 1, cz = DIM == 3 ? (f.nz >> 1) : 1;
    long ncells = (long)cx * cy * cz;
    if (t >= ncells) return;
    int I = (int)(t % cx);
    long r = t / cx;
    int J = (int)(r % cy);
    int K = (int)(r / cy);
    T acc = 0;
    for (int dz = 0; dz < (DIM == 3 ? 2 : 1); ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                Nb n = neighbours(f, 2 * I + dx, 2 * J + dy, DIM == 3 ? 2 * K + dz : 0, DIM);
                acc += b[n.c] - apply_row<T, DIM>(p, co, n) * inv_h2;
            }
    bc[t] = acc * (DIM == 3 ? T(0.125) : T(0.25));
}

// Same restriction for 3D levels with nx % 64 == 0: one thread per fine cell
// (block = 64 x 2 x 2 fine cells = 32 coarse cells), the residual of each fine
// cell computed once; the two x-children meet by a lane exchange, the y and
// z pairs through LDS, summed in a fixed order.
template <typename T, class K>
__global__ __launch_bounds__(kBlock) void k_residual_restrict64(const T* __restrict__ p,
                                                                const T* __restrict__ b, K co,
                                                                Dims f, T inv_h2,
                                                                T* __restrict__ bc) {
    __shared__ T part[4][32];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + lane;
    const int j = blockIdx.y * 2 + (wave & 1);
    const int k = blockIdx.z * 2 + (wave >> 1);
    Nb n = neighbours(f, i, j, k, 3);
    T r = b[n.c] - apply_row<T, 3>(p, co, n) * inv_h2;
    T rx = r + __shfl_xor(r, 1);
    if ((lane & 1) == 0) part[wave][lane >> 1] = rx;
    __syncthreads();
    if (threadIdx.x < 32) {
        const int I = blockIdx.x * 32 + threadIdx.x;
        const int cx = f.nx >> 1, cy = f.ny >> 1;
        T v = (part[0][threadIdx.x] + part[1][threadIdx.x]) + (part[2][threadIdx.x] + part[3][threadIdx.x]);
        bc[((long)blockIdx.z * cy + blockIdx.y) * cx + I] = v * T(0.125);
    }
}

// p_fine += P e_coarse (cell-centred linear, 3/4 and 1/4 per axis)
template <typename T, int DIM>
__global__ void k_prolong_add(T* __restrict__ p, const T* __restrict__ e, Dims f) {
    // every product and sum rounded on its own (no fused multiply-add), so that
    // the blocked and the persistent forms give the same bits
#pragma clang fp contract(off)
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= f.nx) return;
    const int j = blockIdx.y, k = blockIdx.z;
    const int cx = f.nx >> 1, cy = f.ny >> 1, cz = DIM == 3 ? (f.nz >> 1) : 1;
    const int I = i >> 1, J = j >> 1, K = k >> 1;
    const int I2 = (i & 1) ? (I + 1 == cx ? 0 : I + 1) : (I == 0 ? cx - 1 : I - 1);
    const int J2 = (j & 1) ? (J + 1 == cy ? 0 : J + 1) : (J == 0 ? cy - 1 : J - 1);
    const T a = T(0.75), q = T(0.25);
    T v;
    if (DIM == 2) {
        T r0 = a * e[J * cx + I] + q * e[J * cx + I2];
        T r1 = a * e[J2 * cx + I] + q * e[J2 * cx + I2];
        v = a * r0 + q * r1;
    } else {
        const int K2 = (k & 1) ? (K + 1 == cz ? 0 : K + 1) : (K == 0 ? cz - 1 : K - 1);
        const int pl = cx * cy;
        const T* e0 = e + K * pl;
        const T* e1 = e + K2 * pl;
        T r00 = a * e0[J * cx + I] + q * e0[J * cx + I2];
        T r01 = a * e0[J2 * cx + I] + q * e0[J2 * cx + I2];
        T r10 = a * e1[J * cx + I] + q * e1[J * cx + I2];
        T r11 = a * e1[J2 * cx + I] + q * e1[J2 * cx + I2];
        v = a * (a * r00 + q * r01) + q * (a * r10 + q * r11);
    }
    p[((long)k * f.ny + j) * f.nx + i] += v;
}

// The same prolongation in 3D with one thread per coarse cell: it loads the
// 27 coarse values around it once and adds the corrections of its 8 children
// (each formed exactly as in k_prolong_add), so consecutive threads update
// consecutive pairs of fine cells along x.
template <typename T>
__global__ void k_prolong_add_blk(T* __restrict__ p, const T* __restrict__ e, Dims f) {
#pragma clang fp contract(off)
    const int cx = f.nx >> 1, cy = f.ny >> 1, cz = f.nz >> 1;
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= cx) return;
    const int J = blockIdx.y, K = blockIdx.z;
    const int Im = I == 0 ? cx - 1 : I - 1, Ip = I + 1 == cx ? 0 : I + 1;
    const int Jm = J == 0 ? cy - 1 : J - 1, Jp = J + 1 == cy ? 0 : J + 1;
    const int Km = K == 0 ? cz - 1 : K - 1, Kp = K + 1 == cz ? 0 : K + 1;
    const long pl = (long)cx * cy;
    // E[z][y][x] with offsets -1, 0, +1
    T E[3][3][3];
    const int ks[3] = {Km, K, Kp}, js[3] = {Jm, J, Jp}, is[3] = {Im, I, Ip};
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int c = 0; c < 3; ++c) E[a][b][c] = e[ks[a] * pl + (long)js[b] * cx + is[c]];
    const T a = T(0.75), q = T(0.25);
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
        for (int dy = 0; dy < 2; ++dy) {
            // the second coarse cell along each axis: below for the even child, above for the odd
            const int z2 = dz ? 2 : 0, y2 = dy ? 2 : 0;
            T* row = p + ((long)(2 * K + dz) * f.ny + (2 * J + dy)) * f.nx + 2 * I;
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {
                const int x2 = dx ? 2 : 0;
                const T r00 = a * E[1][1][1] + q * E[1][1][x2];
                const T r01 = a * E[1][y2][1] + q * E[1][y2][x2];
                const T r10 = a * E[z2][1][1] + q * E[z2][1][x2];
                const T r11 = a * E[z2][y2][1] + q * E[z2][y2][x2];
                row[dx] += a * (a * r00 + q * r01) + q * (a * r10 + q * r11);
            }
        }
}

template <typename T>
__global__ void k_fill(T* __restrict__ x, long n, T v) {
    long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) x[c] = v;
}

__global__ void k_cast_f32(const double* __restrict__ x, float* __restrict__ y, long n) {
    long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) y[c] = (float)x[c];
}

// coarse face coefficient = mean of the fine faces on it
template <int DIM, class K>
__global__ void k_coarsen_beta(K co, Dims f, double* __restrict__ c0, double* __restrict__ c1,
                               double* __restrict__ c2) {
    long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    int cx = f.nx >> 1, cy = f.ny >> 1, cz = DIM == 3 ? (f.nz >> 1) : 1;
    long ncells = (long)cx * cy * cz;
    if (t >= ncells) return;
    int I = (int)(t % cx);
    long r = t / cx;
    int J = (int)(r % cy);
    int K3 = (int)(r / cy);
    auto nb = [&](int i, int j, int k) { return neighbours(f, i, j, k, DIM); };
    if (DIM == 2) {
        c0[t] = 0.5 * (co.xl(nb(2 * I, 2 * J, 0)) + co.xl(nb(2 * I, 2 * J + 1, 0)));
        c1[t] = 0.5 * (co.yl(nb(2 * I, 2 * J, 0)) + co.yl(nb(2 * I + 1, 2 * J, 0)));
    } else {
        const int i = 2 * I, j = 2 * J, k = 2 * K3;
        c0[t] = 0.25 * ((co.xl(nb(i, j, k)) + co.xl(nb(i, j + 1, k))) +
                        (co.xl(nb(i, j, k + 1)) + co.xl(nb(i, j + 1, k + 1))));
        c1[t] = 0.25 * ((co.yl(nb(i, j, k)) + co.yl(nb(i + 1, j, k))) +
                        (co.yl(nb(i, j, k + 1)) + co.yl(nb(i + 1, j, k + 1))));
        c2[t] = 0.25 * ((co.zl(nb(i, j, k)) + co.zl(nb(i + 1, j, k))) +
                        (co.zl(nb(i, j + 1, k)) + co.zl(nb(i + 1, j + 1, k))));
    }
}

// the face arrays of a level from its cell densities (float32 for the mixed
// V-cycle, float64 where the kernels read stored faces)
template <int DIM, typename TO>
__global__ void k_beta_from_rho(CoefRho co, Dims d, TO* __restrict__ b0, TO* __restrict__ b1,
                                TO* __restrict__ b2) {
    long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.cells()) return;
    int i = (int)(c % d.nx);
    long r = c / d.nx;
    int j = (int)(r % d.ny);
    int k = (int)(r / d.ny);
    Nb n = neighbours(d, i, j, k, DIM);
    b0[c] = (TO)co.xl(n);
    b1[c] = (TO)co.yl(n);
    if (DIM == 3) b2[c] = (TO)co.zl(n);
}

// ---------------------------------------------------------------------------
// coarsest level: exact zero-mean solve.
// A is symmetric negative semidefinite with the constants as its null space,
// so M = -A + c 1 1^T (c > 0) is symmetric positive definite, and for a
// right side with zero sum the unique solution of (A - c 1 1^T) x = b has
// sum(x) = 0 and A x = b: it is the zero-mean solution of the singular
// system. M is inverted once per coefficient update (Gauss-Jordan without
// pivoting, stable for SPD matrices) and each cycle applies x = -M^{-1} b.
// c = trace(-A) / nc^2 gives the constant mode an eigenvalue equal to the
// mean eigenvalue of -A.
constexpr int kMaxCoarse = 64;

template <int DIM>
__global__ void k_build_coarse(const double* __restrict__ b0, const double* __restrict__ b1,
                               const double* __restrict__ b2, Dims d, double* __restrict__ M) {
    __shared__ double diag[kMaxCoarse];
    int nc = (int)d.cells();
    int r = threadIdx.x;
    double inv = 1.0 / (d.h * d.h);
    if (r < nc) {
        for (int c = 0; c < nc; ++c) M[(long)r * nc + c] = 0.0;
        int i = r % d.nx, j = (r / d.nx) % d.ny, k = r / (d.nx * d.ny);
        Nb n = neighbours(d, i, j, k, DIM);
        // rows of -A
        auto add = [&](long col, double v) { M[(long)r * nc + col] += v * inv; };
        add(n.xp, -b0[n.xp]); add(n.c, b0[n.xp]);
        add(n.xm, -b0[n.c]);  add(n.c, b0[n.c]);
        add(n.yp, -b1[n.yp]); add(n.c, b1[n.yp]);
        add(n.ym, -b1[n.c]);  add(n.c, b1[n.c]);
        if (DIM == 3) {
            add(n.zp, -b2[n.zp]); add(n.c, b2[n.zp]);
            add(n.zm, -b2[n.c]);  add(n.c, b2[n.c]);
        }
        diag[r] = M[(long)r * nc + r];
    }
    __syncthreads();
    if (r < nc) {
        double tr = 0.0;
        for (int q = 0; q < nc; ++q) tr += diag[q];
        double c = tr / ((double)nc * (double)nc);
        for (int q = 0; q < nc; ++q) M[(long)r * nc + q] += c;
    }
}

// one workgroup, in-place inverse in LDS
__global__ void k_spd_inverse(const double* __restrict__ M, int m, double* __restrict__ Minv) {
    __shared__ double a[kMaxCoarse][kMaxCoarse + 1];
    __shared__ double f[kMaxCoarse];
    int t = threadIdx.x, nt = blockDim.x;
    for (int q = t; q < m * m; q += nt) a[q / m][q % m] = M[q];
    __syncthreads();
    for (int k = 0; k < m; ++k) {
        double piv = a[k][k];
        __syncthreads();
        for (int j = t; j < m; j += nt) a[k][j] = (j == k ? 1.0 : a[k][j]) / piv;
        for (int i = t; i < m; i += nt)
            if (i != k) {
                f[i] = a[i][k];
                a[i][k] = 0.0;
            }
        __syncthreads();
        for (int q = t; q < m * m; q += nt) {
            int i = q / m, j = q % m;
            if (i != k) a[i][j] -= f[i] * a[k][j];
        }
        __syncthreads();
    }
    for (int q = t; q < m * m; q += nt) Minv[q] = -a[q / m][q % m];
}

// x = (-M^{-1}) b on the coarsest level, input/output in T
template <typename T>
__global__ void k_coarse_apply(const double* __restrict__ Minv, int nc, const T* __restrict__ b,
                               T* __restrict__ x) {
    __shared__ double sb[kMaxCoarse];
    int t = threadIdx.x;
    for (int q = t; q < nc; q += blockDim.x) sb[q] = (double)b[q];
    __syncthreads();
    for (int r = t; r < nc; r += blockDim.x) {
        double s = 0.0;
        for (int c = 0; c < nc; ++c) s += Minv[(long)r * nc + c] * sb[c];
        x[r] = (T)s;
    }
}

// ---------------------------------------------------------------------------
// The small coarse levels in one persistent workgroup: the sub-V-cycle from
// level `first` (at most kPersistCells cells) down to the coarsest and back,
// with a workgroup barrier between dependent phases instead of a launch per
// phase. Per cell it performs the arithmetic of the separate kernels
// (k_rbgs, k_residual_restrict, k_prolong_add, k_coarse_apply) in the same
// order, so results are bitwise those of the launch-per-phase cycle.
constexpr int kPersistMaxLevels = 8;
constexpr long kPersistCells = 4096;
constexpr int kPersistThreads = 1024;

template <typename T>
struct PersistLevels {
    int n;  // levels first .. coarsest
    int nu1, nu2;
    int nc;  // coarsest cells
    int zero;  // the first level starts from p = 0 (its p is not read)
    const double* minv;
    Dims d[kPersistMaxLevels];
    T* p[kPersistMaxLevels];
    T* b[kPersistMaxLevels];
    const T* b0[kPersistMaxLevels];
    const T* b1[kPersistMaxLevels];
    const T* b2[kPersistMaxLevels];
};

// ZERO: the red pass from p = 0, which reads no p (as k_rbgs<..., true>)
template <typename T, int DIM, bool ZERO = false>
__device__ void pv_rbgs(const PersistLevels<T>& L, int l, int color) {
    const Dims d = L.d[l];
    T* __restrict__ p = L.p[l];
    const T* __restrict__ b = L.b[l];
    const T* __restrict__ b0 = L.b0[l];
    const T* __restrict__ b1 = L.b1[l];
    const T* __restrict__ b2 = L.b2[l];
    const T h2 = (T)(d.h * d.h);
    const int hx = d.nx >> 1;
    const long half = d.cells() >> 1;
    for (long t = threadIdx.x; t < half; t += blockDim.x) {
        int i2 = (int)(t % hx);
        long r = t / hx;
        int j = (int)(r % d.ny);
        int k = (int)(r / d.ny);
        int i = 2 * i2 + ((j + k + color) & 1);
        Nb n = neighbours(d, i, j, k, DIM);
        T br = b0[n.xp], bl = b0[n.c];
        T num = ZERO ? T(0) : br * p[n.xp] + bl * p[n.xm];
        T diag = br + bl;
        br = b1[n.yp];
        bl = b1[n.c];
        if (!ZERO) num += br * p[n.yp] + bl * p[n.ym];
        diag += br + bl;
        if (DIM == 3) {
            br = b2[n.zp];
            bl = b2[n.c];
            if (!ZERO) num += br * p[n.zp] + bl * p[n.zm];
            diag += br + bl;
        }
        p[n.c] = (num - h2 * b[n.c]) / diag;
    }
}

template <typename T, int DIM>
__device__ void pv_restrict(const PersistLevels<T>& L, int l) {
    const Dims f = L.d[l];
    const CoefArrays<T> co{L.b0[l], L.b1[l], L.b2[l]};
    const T inv_h2 = (T)(1.0 / (f.h * f.h));
    const T* __restrict__ p = L.p[l];
    const T* __restrict__ b = L.b[l];
    T* __restrict__ bc = L.b[l + 1];
    T* __restrict__ pc = L.p[l + 1];
    const bool fill = l + 1 != L.n - 1;
    int cx = f.nx >> 1, cy = f.ny >> 1, cz = DIM == 3 ? (f.nz >> 1) : 1;
    long ncells = (long)cx * cy * cz;
    for (long t = threadIdx.x; t < ncells; t += blockDim.x) {
        int I = (int)(t % cx);
        long r = t / cx;
        int J = (int)(r % cy);
        int K = (int)(r / cy);
        T acc = 0;
        for (int dz = 0; dz < (DIM == 3 ? 2 : 1); ++dz)
            for (int dy = 0; dy < 2; ++dy)
                for (int dx = 0; dx < 2; ++dx) {
                    Nb n = neighbours(f, 2 * I + dx, 2 * J + dy, DIM == 3 ? 2 * K + dz : 0, DIM);
                    acc += b[n.c] - apply_row<T, DIM>(p, co, n) * inv_h2;
                }
        bc[t] = acc * (DIM == 3 ? T(0.125) : T(0.25));
        if (fill) pc[t] = (T)0;
    }
}

template <typename T, int DIM>
__device__ void pv_prolong(const PersistLevels<T>& L, int l) {
    // products and sums rounded one by one, as in k_prolong_add(_blk)
#pragma clang fp contract(off)
    const Dims f = L.d[l];
    T* __restrict__ p = L.p[l];
    const T* __restrict__ e = L.p[l + 1];
    const int cx = f.nx >> 1, cy = f.ny >> 1, cz = DIM == 3 ? (f.nz >> 1) : 1;
    const T a = T(0.75), q = T(0.25);
    for (long t = threadIdx.x; t < f.cells(); t += blockDim.x) {
        const int i = (int)(t % f.nx);
        const long r = t / f.nx;
        const int j = (int)(r % f.ny), k = (int)(r / f.ny);
        const int I = i >> 1, J = j >> 1, K = k >> 1;
        const int I2 = (i & 1) ? (I + 1 == cx ? 0 : I + 1) : (I == 0 ? cx - 1 : I - 1);
        const int J2 = (j & 1) ? (J + 1 == cy ? 0 : J + 1) : (J == 0 ? cy - 1 : J - 1);
        T v;
        if (DIM == 2) {
            T r0 = a * e[J * cx + I] + q * e[J * cx + I2];
            T r1 = a * e[J2 * cx + I] + q * e[J2 * cx + I2];
            v = a * r0 + q * r1;
        } else {
            const int K2 = (k & 1) ? (K + 1 == cz ? 0 : K + 1) : (K == 0 ? cz - 1 : K - 1);
            const int pl = cx * cy;
            const T* e0 = e + K * pl;
            const T* e1 = e + K2 * pl;
            T r00 = a * e0[J * cx + I] + q * e0[J * cx + I2];
            T r01 = a * e0[J2 * cx + I] + q * e0[J2 * cx + I2];
            T r10 = a * e1[J * cx + I] + q * e1[J * cx + I2];
            T r11 = a * e1[J2 * cx + I] + q * e1[J2 * cx + I2];
            v = a * (a * r00 + q * r01) + q * (a * r10 + q * r11);
        }
        p[t] += v;
    }
}

template <typename T, int DIM>
__global__ __launch_bounds__(kPersistThreads) void k_coarse_vcycle(PersistLevels<T> L) {
    __shared__ double sb[kMaxCoarse];
    const int last = L.n - 1;
    // a first level from p = 0: its first red pass reads no p; without
    // pre-smoothing the restriction reads p, which is cleared here
    if (L.zero && L.nu1 == 0 && last > 0) {
        for (long t = threadIdx.x; t < L.d[0].cells(); t += blockDim.x) L.p[0][t] = T(0);
        __syncthreads();
    }
    for (int l = 0; l < last; ++l) {
        for (int s = 0; s < L.nu1; ++s) {
            if (l == 0 && s == 0 && L.zero)
                pv_rbgs<T, DIM, true>(L, l, 0);
            else
                pv_rbgs<T, DIM>(L, l, 0);
            __syncthreads();
            pv_rbgs<T, DIM>(L, l, 1);
            __syncthreads();
        }
        pv_restrict<T, DIM>(L, l);
        __syncthreads();
    }
    // coarsest: x = (-M^{-1}) b, float64 sums
    for (int q = threadIdx.x; q < L.nc; q += blockDim.x) sb[q] = (double)L.b[last][q];
    __syncthreads();
    for (int r = threadIdx.x; r < L.nc; r += blockDim.x) {
        double s = 0.0;
        for (int c = 0; c < L.nc; ++c) s += L.minv[(long)r * L.nc + c] * sb[c];
        L.p[last][r] = (T)s;
    }
    __syncthreads();
    for (int l = last - 1; l >= 0; --l) {
        pv_prolong<T, DIM>(L, l);
        __syncthreads();
        for (int s = 0; s < L.nu2; ++s) {
            pv_rbgs<T, DIM>(L, l, 0);
            __syncthreads();
            pv_rbgs<T, DIM>(L, l, 1);
            __syncthreads();
        }
    }
}

// The same sub-V-cycle for 3D hierarchies with its data in LDS and
// registers. The first level (at most kPersistCells cells) keeps p, b and the
// residual in LDS, and each thread keeps the six face coefficients of its own
// cells in registers (up to four of each colour); the smaller
// levels keep p, b, the residual and the face
// coefficients in an LDS pool. Global memory is read once per cycle (the
// first level's p, b and coefficients, the smaller levels' coefficients, the
// coarsest inverse) and written once (the first level's p). Each phase forms
// every value with the operands and the order of k_coarse_vcycle (the
// residual of a fine cell is formed once and the restriction sums the eight
// children in the same order), so the cycle is bitwise the same.
constexpr int kLdsPool = 512 + 64 + 8 + 1;  // levels below the first: an eighth of the one above each
constexpr int kLdsThreads = 512;

template <typename T>
__global__ __launch_bounds__(kLdsThreads) void k_coarse_vcycle_lds(PersistLevels<T> L) {
    constexpr int NT = kLdsThreads;
    constexpr int NS = (kPersistCells / 2 + NT - 1) / NT;  // cells of each colour per thread
    __shared__ T P0[kPersistCells], B0[kPersistCells], R0[kPersistCells];
    __shared__ T PP[kLdsPool], BB[kLdsPool], RR[kLdsPool], X0[kLdsPool], X1[kLdsPool], X2[kLdsPool];
    __shared__ double sb[kMaxCoarse];
    __shared__ int OFF[kPersistMaxLevels];
    const int t = threadIdx.x;
    const int last = L.n - 1;
    if (t == 0) {
        int o = 0;
        for (int l = 1; l < L.n; ++l) {
            OFF[l] = o;
            o += (int)L.d[l].cells();
        }
    }
    // first level: the cells of colour c dealt t, t + NT (as k_rbgs deals them)
    const Dims d0 = L.d[0];
    const int n0 = (int)d0.cells(), half0 = n0 >> 1, hx0 = d0.nx >> 1;
    // the periodic neighbours of cell (i, j, k) as 32-bit offsets
    struct Nb32 {
        int c, xm, xp, ym, yp, zm, zp;
    };
    auto nb32 = [](const Dims& d, int i, int j, int k) {
        Nb32 n;
        const int pl = d.nx * d.ny;
        n.c = (k * d.ny + j) * d.nx + i;
        n.xm = i == 0 ? n.c + d.nx - 1 : n.c - 1;
        n.xp = i == d.nx - 1 ? n.c - (d.nx - 1) : n.c + 1;
        n.ym = j == 0 ? n.c + (d.ny - 1) * d.nx : n.c - d.nx;
        n.yp = j == d.ny - 1 ? n.c - (d.ny - 1) * d.nx : n.c + d.nx;
        n.zm = k == 0 ? n.c + (d.nz - 1) * pl : n.c - pl;
        n.zp = k == d.nz - 1 ? n.c - (d.nz - 1) * pl : n.c + pl;
        return n;
    };
    int cl[2][NS];
    T bxl[2][NS], bxr[2][NS], byl[2][NS], byr[2][NS], bzl[2][NS], bzr[2][NS];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int t2 = t + s * NT;
            cl[c][s] = -1;
            bxl[c][s] = bxr[c][s] = byl[c][s] = byr[c][s] = bzl[c][s] = bzr[c][s] = T(0);
            if (t2 < half0) {
                const int i2 = t2 % hx0, r = t2 / hx0;
                const int j = r % d0.ny, k = r / d0.ny;
                const int i = 2 * i2 + ((j + k + c) & 1);
                const Nb32 n = nb32(d0, i, j, k);
                cl[c][s] = n.c;
                bxr[c][s] = L.b0[0][n.xp];
                bxl[c][s] = L.b0[0][n.c];
                byr[c][s] = L.b1[0][n.yp];
                byl[c][s] = L.b1[0][n.c];
                bzr[c][s] = L.b2[0][n.zp];
                bzl[c][s] = L.b2[0][n.c];
                B0[n.c] = L.b[0][n.c];
                P0[n.c] = L.zero ? T(0) : L.p[0][n.c];
            }
        }
    __syncthreads();
    // coefficients of the smaller levels (the coarsest is solved directly)
    for (int l = 1; l < last; ++l) {
        const int nl = (int)L.d[l].cells(), o = OFF[l];
        for (int u = t; u < nl; u += NT) {
            X0[o + u] = L.b0[l][u];
            X1[o + u] = L.b1[l][u];
            X2[o + u] = L.b2[l][u];
        }
    }
    const T h20 = (T)(d0.h * d0.h);
    auto cell_nb = [&](const Dims& d, int u) {
        const int i = u % d.nx, r = u / d.nx;
        return nb32(d, i, r % d.ny, r / d.ny);
    };
    auto sweep0 = [&](int c) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (cl[c][s] < 0) continue;
            const Nb32 n = cell_nb(d0, cl[c][s]);
            T br = bxr[c][s], bl = bxl[c][s];
            T num = br * P0[n.xp] + bl * P0[n.xm];
            T diag = br + bl;
            br = byr[c][s];
            bl = byl[c][s];
            num += br * P0[n.yp] + bl * P0[n.ym];
            diag += br + bl;
            br = bzr[c][s];
            bl = bzl[c][s];
            num += br * P0[n.zp] + bl * P0[n.zm];
            diag += br + bl;
            P0[n.c] = (num - h20 * B0[n.c]) / diag;
        }
    };
    auto resid0 = [&]() {
        const T inv_h2 = (T)(1.0 / (d0.h * d0.h));
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                if (cl[c][s] < 0) continue;
                const Nb32 n = cell_nb(d0, cl[c][s]);
                const T pc = P0[n.c];
                T sv = bxr[c][s] * (P0[n.xp] - pc) - bxl[c][s] * (pc - P0[n.xm]);
                sv += byr[c][s] * (P0[n.yp] - pc) - byl[c][s] * (pc - P0[n.ym]);
                sv += bzr[c][s] * (P0[n.zp] - pc) - bzl[c][s] * (pc - P0[n.zm]);
                R0[n.c] = B0[n.c] - sv * inv_h2;
            }
    };
    auto sweepl = [&](int l, int c) {
        const Dims d = L.d[l];
        const int o = OFF[l], hx = d.nx >> 1, half = (int)(d.cells() >> 1);
        const T h2 = (T)(d.h * d.h);
        for (int t2 = t; t2 < half; t2 += NT) {
            const int i2 = t2 % hx, r = t2 / hx;
            const int j = r % d.ny, k = r / d.ny;
            const Nb32 n = nb32(d, 2 * i2 + ((j + k + c) & 1), j, k);
            T br = X0[o + n.xp], bl = X0[o + n.c];
            T num = br * PP[o + n.xp] + bl * PP[o + n.xm];
            T diag = br + bl;
            br = X1[o + n.yp];
            bl = X1[o + n.c];
            num += br * PP[o + n.yp] + bl * PP[o + n.ym];
            diag += br + bl;
            br = X2[o + n.zp];
            bl = X2[o + n.c];
            num += br * PP[o + n.zp] + bl * PP[o + n.zm];
            diag += br + bl;
            PP[o + n.c] = (num - h2 * BB[o + n.c]) / diag;
        }
    };
    auto residl = [&](int l) {
        const Dims d = L.d[l];
        const int o = OFF[l], nl = (int)d.cells();
        const T inv_h2 = (T)(1.0 / (d.h * d.h));
        for (int u = t; u < nl; u += NT) {
            const Nb32 n = cell_nb(d, u);
            const T pc = PP[o + n.c];
            T sv = X0[o + n.xp] * (PP[o + n.xp] - pc) - X0[o + n.c] * (pc - PP[o + n.xm]);
            sv += X1[o + n.yp] * (PP[o + n.yp] - pc) - X1[o + n.c] * (pc - PP[o + n.ym]);
            sv += X2[o + n.zp] * (PP[o + n.zp] - pc) - X2[o + n.c] * (pc - PP[o + n.zm]);
            RR[o + u] = BB[o + u] - sv * inv_h2;
        }
    };
    // coarse right side of level l + 1 from the residuals of level l (children
    // summed in the order dz, dy, dx, from zero), and p of level l + 1 zeroed
    // unless it is the coarsest
    auto restrictl = [&](int l) {
        const Dims f = L.d[l];
        const T* R = l == 0 ? R0 : RR + OFF[l];
        const int oc = OFF[l + 1];
        const int cx = f.nx >> 1, cy = f.ny >> 1, cz = f.nz >> 1;
        const bool fill = l + 1 != last;
        for (int u = t; u < cx * cy * cz; u += NT) {
            const int I = u % cx, r = u / cx;
            const int J = r % cy, K = r / cy;
            T acc = 0;
            for (int dz = 0; dz < 2; ++dz)
                for (int dy = 0; dy < 2; ++dy)
                    for (int dx = 0; dx < 2; ++dx)
                        acc += R[((2 * K + dz) * f.ny + (2 * J + dy)) * f.nx + 2 * I + dx];
            BB[oc + u] = acc * T(0.125);
            if (fill) PP[oc + u] = T(0);
        }
    };
    // p of level l += P e, e = p of level l + 1
    auto prolongl = [&](int l) {
        const Dims f = L.d[l];
        const T* e = PP + OFF[l + 1];
        T* p = l == 0 ? P0 : PP + OFF[l];
        const int cx = f.nx >> 1, cy = f.ny >> 1, cz = f.nz >> 1;
        for (int u = t; u < (int)f.cells(); u += NT) {
            const int i = u % f.nx, r = u / f.nx;
            const int j = r % f.ny, k = r / f.ny;
            const int I = i >> 1, J = j >> 1, K = k >> 1;
            const int I2 = (i & 1) ? (I + 1 == cx ? 0 : I + 1) : (I == 0 ? cx - 1 : I - 1);
            const int J2 = (j & 1) ? (J + 1 == cy ? 0 : J + 1) : (J == 0 ? cy - 1 : J - 1);
            const int K2 = (k & 1) ? (K + 1 == cz ? 0 : K + 1) : (K == 0 ? cz - 1 : K - 1);
            const int pl = cx * cy;
            const T* e0 = e + K * pl;
            const T* e1 = e + K2 * pl;
            const T v = prolong_cell<T>(e0[J * cx + I], e0[J * cx + I2], e0[J2 * cx + I], e0[J2 * cx + I2],
                                        e1[J * cx + I], e1[J * cx + I2], e1[J2 * cx + I], e1[J2 * cx + I2]);
            p[u] = p[u] + v;
        }
    };
    __syncthreads();
    for (int l = 0; l < last; ++l) {
        for (int s = 0; s < L.nu1; ++s)
            for (int c = 0; c < 2; ++c) {
                if (l == 0)
                    sweep0(c);
                else
                    sweepl(l, c);
                __syncthreads();
            }
        if (l == 0)
            resid0();
        else
            residl(l);
        __syncthreads();
        restrictl(l);
        __syncthreads();
    }
    // coarsest: x = (-M^{-1}) b, float64 sums
    const int oc = OFF[last];
    for (int q = t; q < L.nc; q += NT) sb[q] = (double)BB[oc + q];
    __syncthreads();
    for (int r = t; r < L.nc; r += NT) {
        double s = 0.0;
        for (int c = 0; c < L.nc; ++c) s += L.minv[(long)r * L.nc + c] * sb[c];
        PP[oc + r] = (T)s;
    }
    __syncthreads();
    for (int l = last - 1; l >= 0; --l) {
        prolongl(l);
        __syncthreads();
        for (int s = 0; s < L.nu2; ++s)
            for (int c = 0; c < 2; ++c) {
                if (l == 0)
                    sweep0(c);
                else
                    sweepl(l, c);
                __syncthreads();
            }
    }
    for (int u = t; u < n0; u += NT) L.p[0][u] = P0[u];
}

// ---------------------------------------------------------------------------
// norms: partial sums of r^2 (and of p) per block
template <int DIM, class K>
__global__ void k_resid_norm(const double* __restrict__ p, const double* __restrict__ b, K co,
                             Dims d, double inv_h2, double* __restrict__ partial_r2,
                             double* __restrict__ partial_b2) {
    __shared__ double sh[kBlock];
    double ar = 0.0, ab = 0.0;
    const int N = (int)d.cells(), nx = d.nx, ny = d.ny;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < N; c += gridDim.x * blockDim.x) {
        int i = c % nx;
        int r = c / nx;
        int j = r % ny;
        int k = r / ny;
        Nb n = neighbours(d, i, j, k, DIM);
        double bv = b[c];
        double rv = bv - apply_row<double, DIM>(p, co, n) * inv_h2;
        ar += rv * rv;
        ab += bv * bv;
    }
    double s = block_reduce_sum(ar, sh);
    if (threadIdx.x == 0) partial_r2[blockIdx.x] = s;
    if (partial_b2) {
        s = block_reduce_sum(ab, sh);
        if (threadIdx.x == 0) partial_b2[blockIdx.x] = s;
    }
}

// mixed precision: r32 = fl32(b - A p) with partial sums of r^2 and b^2
template <int DIM, class K>
__global__ void k_defect_f32(const double* __restrict__ p, const double* __restrict__ b, K co,
                             Dims d, double inv_h2, float* __restrict__ r32,
                             double* __restrict__ partial_r2, double* __restrict__ partial_b2) {
    __shared__ double sh[kBlock];
    double ar = 0.0, ab = 0.0;
    const int N = (int)d.cells(), nx = d.nx, ny = d.ny;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < N; c += gridDim.x * blockDim.x) {
        int i = c % nx;
        int r = c / nx;
        int j = r % ny;
        int k = r / ny;
        Nb n = neighbours(d, i, j, k, DIM);
        double bv = b[c];
        double rv = bv - apply_row<double, DIM>(p, co, n) * inv_h2;
        r32[c] = (float)rv;
        ar += rv * rv;
        ab += bv * bv;
    }
    double s = block_reduce_sum(ar, sh);
    if (threadIdx.x == 0) partial_r2[blockIdx.x] = s;
    if (partial_b2) {
        s = block_reduce_sum(ab, sh);
        if (threadIdx.x == 0) partial_b2[blockIdx.x] = s;
    }
}

// p += e (float32 correction) with partial sums of the new p
__global__ void k_correct_f32(double* __restrict__ p, const float* __restrict__ e, long N,
                              double* __restrict__ partial) {
    __shared__ double sh[kBlock];
    double acc = 0.0;
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (long)gridDim.x * blockDim.x) {
        double v = p[c] + (double)e[c];
        p[c] = v;
        acc += v;
    }
    double s = block_reduce_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void k_sum_cells(const double* __restrict__ p, long N, double* __restrict__ partial) {
    __shared__ double sh[kBlock];
    double acc = 0.0;
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (long)gridDim.x * blockDim.x)
        acc += p[c];
    double s = block_reduce_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void k_sub_scalar_mean(double* __restrict__ p, long N, const double* __restrict__ sum) {
    long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < N) p[c] -= *sum / (double)N;
}

// ---------------------------------------------------------------------------
// flexible CG. Scalars live on the device (ks) and each kernel forms alpha
// and beta from them, so an iteration needs no host round trip.
enum { KS_RZ0 = 0, KS_RZ1 = 1, KS_DQ = 2, KS_QZ = 3, KS_RR = 4, KS_BB = 5 };

// r = b - A x with partial sums of r^2 and b^2
template <int DIM, class K>
__global__ void k_residual_vec(const double* __restrict__ x, const double* __restrict__ b, K co,
                               Dims d, double inv_h2, double* __restrict__ r,
                               double* __restrict__ partial_r2, double* __restrict__ partial_b2) {
    __shared__ double sh[kBlock];
    double ar = 0.0, ab = 0.0;
    const int N = (int)d.cells(), nx = d.nx, ny = d.ny;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < N; c += gridDim.x * blockDim.x) {
        int i = c % nx;
        int rr = c / nx;
        int j = rr % ny;
        int k = rr / ny;
        Nb n = neighbours(d, i, j, k, DIM);
        double bv = b[c];
        double rv = bv - apply_row<double, DIM>(x, co, n) * inv_h2;
        r[c] = rv;
        ar += rv * rv;
        ab += bv * bv;
    }
    double s = block_reduce_sum(ar, sh);
    if (threadIdx.x == 0) partial_r2[blockIdx.x] = s;
    s = block_reduce_sum(ab, sh);
    if (threadIdx.x == 0) partial_b2[blockIdx.x] = s;
}

// r = b for a zero guess (b - A 0 is b exactly), with the partial sums of
// k_residual_vec in its order (r^2 and b^2 are then the same sum)
__global__ void k_residual_zero(const double* __restrict__ b, int N, double* __restrict__ r,
                                double* __restrict__ partial_r2, double* __restrict__ partial_b2) {
    __shared__ double sh[kBlock];
    double ab = 0.0;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < N; c += gridDim.x * blockDim.x) {
        const double bv = b[c];
        if (r) r[c] = bv;
        ab += bv * bv;
    }
    const double s = block_reduce_sum(ab, sh);
    if (threadIdx.x == 0) {
        partial_r2[blockIdx.x] = s;
        if (partial_b2) partial_b2[blockIdx.x] = s;
    }
}

// q = A d with partial sums of d q
template <int DIM, class K>
__global__ void k_apply_dot(const double* __restrict__ dv, K co, Dims d, double inv_h2,
                            double* __restrict__ q, double* __restrict__ partial) {
    __shared__ double sh[kBlock];
    double acc = 0.0;
    const int N = (int)d.cells(), nx = d.nx, ny = d.ny;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < N; c += gridDim.x * blockDim.x) {
        int i = c % nx;
        int rr = c / nx;
        int j = rr % ny;
        int k = rr / ny;
        Nb n = neighbours(d, i, j, k, DIM);
        double qv = apply_row<double, DIM>(dv, co, n) * inv_h2;
        q[c] = qv;
        acc += dv[c] * qv;
    }
    double s = block_reduce_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// alpha = (r,z) / (d,q); x += alpha d; r -= alpha q; partial sums of r^2;
// r32 (when not null) = fl32(r), the next float32 preconditioner's right side
__global__ void k_pcg_xr(double* __restrict__ x, double* __restrict__ r,
                         const double* __restrict__ dv, const double* __restrict__ q, long N,
                         const double* __restrict__ ks, int rz_slot,
                         double* __restrict__ partial, float* __restrict__ r32) {
    __shared__ double sh[kBlock];
    const double alpha = ks[rz_slot] / ks[KS_DQ];
    double acc = 0.0;
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (long)gridDim.x * blockDim.x) {
        x[c] += alpha * dv[c];
        double rv = r[c] - alpha * q[c];
        r[c] = rv;
        if (r32) r32[c] = (float)rv;
        acc += rv * rv;
    }
    double s = block_reduce_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// The x/r update with the x part left to the next direction pass (which
// makes it as k_cg_dir_apply_rho<..., XUPD>): r -= alpha q, fl32(r) when r32
// is given, partial sums of r^2; alpha formed as k_pcg_xr forms it.
__global__ void k_pcg_r(double* __restrict__ r, const double* __restrict__ q, long N,
                        const double* __restrict__ ks, int rz_slot, double* __restrict__ partial,
                        float* __restrict__ r32) {
    __shared__ double sh[kBlock];
    const double alpha = ks[rz_slot] / ks[KS_DQ];
    double acc = 0.0;
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (long)gridDim.x * blockDim.x) {
        double rv = r[c] - alpha * q[c];
        r[c] = rv;
        if (r32) r32[c] = (float)rv;
        acc += rv * rv;
    }
    double s = block_reduce_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// the x part of k_pcg_xr on its own (a deferred update made before x is read)
__global__ void k_pcg_x(double* __restrict__ x, const double* __restrict__ dv, long N,
                        const double* __restrict__ ks, int rz_slot) {
    const double alpha = ks[rz_slot] / ks[KS_DQ];
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (long)gridDim.x * blockDim.x)
        x[c] += alpha * dv[c];
}

// partial sums of r z and (when q is given) q z; z is the float64 V-cycle
// output or the float32 one
template <typename TZ>
__global__ void k_pcg_dots(const double* __restrict__ r, const double* __restrict__ q,
                           const TZ* __restrict__ z, long N, double* __restrict__ partial_rz,
                           double* __restrict__ partial_qz) {
    __shared__ double sh[kBlock];
    double a = 0.0, b = 0.0;
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (long)gridDim.x * blockDim.x) {
        double zv = (double)z[c];
        a += r[c] * zv;
        if (q) b += q[c] * zv;
    }
    double s = block_reduce_sum(a, sh);
    if (threadIdx.x == 0) partial_rz[blockIdx.x] = s;
    if (q) {
        s = block_reduce_sum(b, sh);
        if (threadIdx.x == 0) partial_qz[blockIdx.x] = s;
    }
}

// d = z + beta d, beta = -alpha (q,z) / (r,z)_old with alpha = (r,z)_old / (d,q);
// on the first iteration d = z
template <typename TZ>
__global__ void k_pcg_dir(double* __restrict__ dv, const TZ* __restrict__ z, long N,
                          const double* __restrict__ ks, int rz_old_slot, int first) {
    long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= N) return;
    if (first) {
        dv[c] = (double)z[c];
        return;
    }
    const double rz = ks[rz_old_slot];
    const double alpha = rz / ks[KS_DQ];
    const double beta = -alpha * ks[KS_QZ] / rz;
    dv[c] = (double)z[c] + beta * dv[c];
}

// One flexible-CG direction update fused with the product and its inner
// product, on a finest level given by densities (3D): dnew = z + beta d
// (dnew = z on the first iteration), q = A dnew, partial sums of dnew q per
// workgroup. d and dnew are distinct buffers: neighbouring workgroups read the
// old direction in their halos while this one writes the new one. Same
// z-march as the sweep: a workgroup owns a CG_TX x CG_TY tile and a z-range,
// stages the new d and rho of each plane on the tile plus a one-cell ring in
// LDS (three-plane rings), and loads the planes two steps ahead. The
// arithmetic of each q is that of apply_row_rho, operand for operand. FIRST
// (the first iteration, dnew = z) is a template argument, so that every step
// issues the same loads and the waits for a staged plane never drain the
// loads issued after it. XUPD: the pass also makes the previous iteration's
// x += alpha d on its tile (alpha = rz_old / dq from the device scalars, as
// the x/r update forms it; d the old direction, which the pass reads anyway),
// so that update need not read d and write x again.
constexpr int CG_TX = 64, CG_TY = 8, CG_NT = 512;
constexpr int CG_RX = CG_TX + 2, CG_RY = CG_TY + 2, CG_RN = CG_RX * CG_RY;
constexpr int CG_NL = (CG_RN + CG_NT - 1) / CG_NT;

template <typename TZ, bool FIRST, bool XUPD = false>
__global__ __launch_bounds__(CG_NT) void k_cg_dir_apply_rho(const TZ* __restrict__ z,
                                                            const double* __restrict__ d,
                                                            double* __restrict__ dnew,
                                                            const double* __restrict__ rho,
                                                            double* __restrict__ q, Dims dm,
                                                            double inv_h2, const double* __restrict__ ks,
                                                            int rz_old_slot, int TZr,
                                                            int ntx, int nty, int nzc,
                                                            double* __restrict__ partial,
                                                            double* __restrict__ x = nullptr) {
    static_assert(!(FIRST && XUPD), "the first iteration has no previous update");
    __shared__ double DN[3][CG_RN];
    __shared__ double RR[3][CG_RN];
    __shared__ double red[CG_NT / 64];
    const int nw = ntx * nty * nzc;
    const int bid = blockIdx.x;
    const int w = (nw % 8 == 0) ? (bid % 8) * (nw / 8) + bid / 8 : bid;
    const int tx = w % ntx;
    const int r0 = w / ntx;
    const int ty = r0 % nty;
    const int zc = r0 / nty;
    const int i0 = tx * CG_TX - 1, j0 = ty * CG_TY - 1;
    const int z0 = zc * TZr, z1 = z0 + TZr;
    const long plane = (long)dm.nx * dm.ny;
    const int t = threadIdx.x;
    // beta of the direction update from the device scalars
    double beta = 0.0, alpha = 0.0;
    if (!FIRST) {
        const double rz = ks[rz_old_slot];
        alpha = rz / ks[KS_DQ];
        beta = -alpha * ks[KS_QZ] / rz;
    }
    const int lx = t % CG_TX, ly = t / CG_TX;  // one cell of the tile per thread
    const long own = (long)(j0 + 1 + ly) * dm.nx + (i0 + 1 + lx);
    auto gofs = [&](int x, int y) {
        return (long)wrap_near(j0 + y, dm.ny) * dm.nx + wrap_near(i0 + x, dm.nx);
    };
    long gp[CG_NL];
    bool vp[CG_NL];
#pragma unroll
    for (int s = 0; s < CG_NL; ++s) {
        int qq = t + s * CG_NT;
        vp[s] = qq < CG_RN;
        gp[s] = vp[s] ? gofs(qq % CG_RX, qq / CG_RX) : gofs(0, 0);
    }
    auto pl = [&](int k) { return (long)wrap_near(k, dm.nz) * plane; };
    // a stage holds z, the old d and rho of a plane as loaded; the new
    // direction is formed when the plane is committed to LDS (XUPD: with x and
    // the old d of the lane's own cell, updated at the same commit)
    struct Stage {
        TZ z[CG_NL];
        double d[FIRST ? 1 : CG_NL], r[CG_NL];
        double xo, dv;
    };
    Stage SA, SB;
    auto fetch = [&](Stage& S, int k) {
        const long b = pl(k);
#pragma unroll
        for (int s = 0; s < CG_NL; ++s) {
            S.z[s] = z[b + gp[s]];
            if constexpr (!FIRST) S.d[s] = d[b + gp[s]];
            S.r[s] = rho[b + gp[s]];
        }
        if constexpr (XUPD) {
            S.xo = x[b + own];
            S.dv = d[b + own];
        }
    };
    auto commit = [&](const Stage& S, int k) {
        // the x update of plane k on this workgroup's tile (planes z0 .. z1 - 1
        // are committed once each; z0 - 1 and z1 belong to the neighbours)
        if constexpr (XUPD)
            if (k >= z0 && k < z1) x[pl(k) + own] = S.xo + alpha * S.dv;
#pragma unroll
        for (int s = 0; s < CG_NL; ++s)
            if (s * CG_NT + CG_NT <= CG_RN || vp[s]) {
                const double zv = (double)S.z[s];
                double dv;
                if constexpr (FIRST)
                    dv = zv;
                else
                    dv = zv + beta * S.d[s];
                DN[(k + 3) % 3][t + s * CG_NT] = dv;
                RR[(k + 3) % 3][t + s * CG_NT] = S.r[s];
            }
    };
    // planes z0 - 1 and z0 staged before the march; the march step k computes
    // plane k and stages plane k + 1
    {
        Stage S0;
        fetch(S0, z0 - 1);
        commit(S0, z0 - 1);
        fetch(S0, z0);
        commit(S0, z0);
    }
    fetch(SA, z0 + 1);
    __builtin_amdgcn_sched_barrier(0);
    fetch(SB, z0 + 2);
    const int c = (ly + 1) * CG_RX + lx + 1;
    double acc = 0.0;
    auto step = [&](Stage& S, int k) {
        commit(S, k + 1);
        fetch(S, k + 3 <= z1 ? k + 3 : z1);
        lds_barrier();
        const double* Dc = DN[(k + 3) % 3];
        const double* Rc = RR[(k + 3) % 3];
        const double pc = Dc[c], rc = Rc[c];
        const double rxp = Rc[c + 1], rxm = Rc[c - 1], ryp = Rc[c + CG_RX], rym = Rc[c - CG_RX];
        const double rzp = RR[(k + 4) % 3][c], rzm = RR[(k + 2) % 3][c];
        double bxp, bxm, byp, bym, bzp, bzm;
        if (rxp == rc && rxm == rc && ryp == rc && rym == rc && rzp == rc && rzm == rc) {
            bxp = bxm = byp = bym = bzp = bzm = 1.0 / rc;
        } else {
            bxp = 2.0 / (rxp + rc);
            bxm = 2.0 / (rc + rxm);
            byp = 2.0 / (ryp + rc);
            bym = 2.0 / (rc + rym);
            bzp = 2.0 / (rzp + rc);
            bzm = 2.0 / (rc + rzm);
        }
        double sv = bxp * (Dc[c + 1] - pc) - bxm * (pc - Dc[c - 1]);
        sv += byp * (Dc[c + CG_RX] - pc) - bym * (pc - Dc[c - CG_RX]);
        sv += bzp * (DN[(k + 4) % 3][c] - pc) - bzm * (pc - DN[(k + 2) % 3][c]);
        const double qv = sv * inv_h2;
        const long o = pl(k) + (long)(j0 + 1 + ly) * dm.nx + (i0 + 1 + lx);
        dnew[o] = pc;
        q[o] = qv;
        acc += pc * qv;
        // the next commit overwrites plane k - 1's slot
        lds_barrier();
    };
    // steps z0 .. z1 - 1 in pairs; TZr is even
    for (int k = z0; k < z1; k += 2) {
        step(SA, k);
        step(SB, k + 1);
    }
    // fixed-order workgroup sum
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if ((t & 63) == 0) red[t >> 6] = acc;
    __syncthreads();
    if (t == 0) {
        double sacc = 0.0;
        for (int i = 0; i < CG_NT / 64; ++i) sacc += red[i];
        partial[bid] = sacc;
    }
}

// Residual of a finest level given by densities, restricted to the coarse
// right side, as a z-march with the tiling of k_cg_dir_apply_rho: p and rho of
// each plane staged on the tile plus a one-cell ring (three-plane rings,
// loaded two steps ahead), b read per cell. Each fine residual is formed
// operand for operand as apply_row_rho does, and the 2 x 2 x 2 children are
// summed in the order of k_residual_restrict64 (x pairs by a lane exchange;
// then the y pair of the lower plane plus the y pair of the upper), so the
// coarse right side is bitwise that kernel's. Reads p and rho 1.29 times (the
// ring) and b once, instead of re-reading the neighbour rows and planes of
// small blocks through the cache. T = float: the float32 finest level of the
// mixed cycle, its faces formed from the float32 densities as CoefRhoF forms
// them (2 / (rho + rho') is 1 / rho exactly where the densities agree), so the
// coarse right side is bitwise that of k_residual_restrict64<float, CoefRhoF>.
template <typename T>
__global__ __launch_bounds__(CG_NT) void k_resrestrict_rho(const T* __restrict__ p,
                                                           const T* __restrict__ bb,
                                                           const T* __restrict__ rho, Dims dm,
                                                           T inv_h2, int TZr, int ntx, int nty,
                                                           int nzc, T* __restrict__ bc) {
    __shared__ T PP[3][CG_RN];
    __shared__ T RR[3][CG_RN];
    __shared__ T XS[2][CG_TY][CG_TX / 2];
    const int nw = ntx * nty * nzc;
    const int bid = blockIdx.x;
    const int w = (nw % 8 == 0) ? (bid % 8) * (nw / 8) + bid / 8 : bid;
    const int tx = w % ntx;
    const int r0 = w / ntx;
    const int ty = r0 % nty;
    const int zc = r0 / nty;
    const int i0 = tx * CG_TX - 1, j0 = ty * CG_TY - 1;
    const int z0 = zc * TZr, z1 = z0 + TZr;
    const long plane = (long)dm.nx * dm.ny;
    const int t = threadIdx.x;
    auto gofs = [&](int x, int y) {
        return (long)wrap_near(j0 + y, dm.ny) * dm.nx + wrap_near(i0 + x, dm.nx);
    };
    long gp[CG_NL];
    bool vp[CG_NL];
#pragma unroll
    for (int s = 0; s < CG_NL; ++s) {
        int qq = t + s * CG_NT;
        vp[s] = qq < CG_RN;
        gp[s] = vp[s] ? gofs(qq % CG_RX, qq / CG_RX) : gofs(0, 0);
    }
    const int lx = t % CG_TX, ly = t / CG_TX;  // one cell of the tile per thread
    const int c = (ly + 1) * CG_RX + lx + 1;
    const long own = (long)(j0 + 1 + ly) * dm.nx + (i0 + 1 + lx);
    auto pl = [&](int k) { return (long)wrap_near(k, dm.nz) * plane; };
    struct Stage {
        T p[CG_NL], r[CG_NL], b;
    };
    Stage SA, SB;
    // a stage carries p and rho of plane k + 1 (committed at the start of step
    // k, loaded two steps ahead) and b of plane k (used after the step's
    // barrier, loaded at the end of step k - 2): each value is consumed before
    // the stage is loaded again, so no loaded register is copied and no wait
    // drains the loads issued after it
    auto fetch_pr = [&](Stage& S, int k) {
        const long bp = pl(k + 1);
#pragma unroll
        for (int s = 0; s < CG_NL; ++s) {
            S.p[s] = p[bp + gp[s]];
            S.r[s] = rho[bp + gp[s]];
        }
    };
    auto fetch_b = [&](Stage& S, int k) { S.b = bb[pl(k) + own]; };
    auto commit = [&](const Stage& S, int k) {
#pragma unroll
        for (int s = 0; s < CG_NL; ++s)
            if (s * CG_NT + CG_NT <= CG_RN || vp[s]) {
                PP[(k + 4) % 3][t + s * CG_NT] = S.p[s];
                RR[(k + 4) % 3][t + s * CG_NT] = S.r[s];
            }
    };
    {
        const long a = pl(z0 - 1), a0 = pl(z0);
#pragma unroll
        for (int s = 0; s < CG_NL; ++s)
            if (vp[s]) {
                PP[(z0 + 2) % 3][t + s * CG_NT] = p[a + gp[s]];
                RR[(z0 + 2) % 3][t + s * CG_NT] = rho[a + gp[s]];
                PP[z0 % 3][t + s * CG_NT] = p[a0 + gp[s]];
                RR[z0 % 3][t + s * CG_NT] = rho[a0 + gp[s]];
            }
    }
    fetch_pr(SA, z0);
    fetch_b(SA, z0);
    __builtin_amdgcn_sched_barrier(0);
    fetch_pr(SB, z0 + 1);
    fetch_b(SB, z0 + 1);
    auto step = [&](Stage& S, int k) {
        commit(S, k);
        // past the range the loads re-read plane z1 - 1 (its stage is not used)
        const int kn = k + 2 < z1 ? k + 2 : z1 - 1;
        fetch_pr(S, kn);
        lds_barrier();
        const T* Pc = PP[k % 3];
        const T* Rc = RR[k % 3];
        const T rc = Rc[c];
        const T rxp = Rc[c + 1], rxm = Rc[c - 1], ryp = Rc[c + CG_RX], rym = Rc[c - CG_RX];
        const T rzp = RR[(k + 1) % 3][c], rzm = RR[(k + 2) % 3][c];
        T bxp, bxm, byp, bym, bzp, bzm;
        if (rxp == rc && rxm == rc && ryp == rc && rym == rc && rzp == rc && rzm == rc) {
            bxp = bxm = byp = bym = bzp = bzm = T(1) / rc;
        } else {
            bxp = T(2) / (rxp + rc);
            bxm = T(2) / (rc + rxm);
            byp = T(2) / (ryp + rc);
            bym = T(2) / (rc + rym);
            bzp = T(2) / (rzp + rc);
            bzm = T(2) / (rc + rzm);
        }
        const T pc = Pc[c];
        T sv = bxp * (Pc[c + 1] - pc) - bxm * (pc - Pc[c - 1]);
        sv += byp * (Pc[c + CG_RX] - pc) - bym * (pc - Pc[c - CG_RX]);
        sv += bzp * (PP[(k + 1) % 3][c] - pc) - bzm * (pc - PP[(k + 2) % 3][c]);
        const T r = S.b - sv * inv_h2;
        __builtin_amdgcn_sched_barrier(0);
        fetch_b(S, kn);
        const T rx = r + __shfl_xor(r, 1);
        if ((lx & 1) == 0) XS[k & 1][ly][lx >> 1] = rx;
        lds_barrier();
        if ((k & 1) && t < (CG_TX / 2) * (CG_TY / 2)) {
            const int cx = t % (CG_TX / 2), cy = t / (CG_TX / 2);
            const T v = (XS[0][2 * cy][cx] + XS[0][2 * cy + 1][cx]) +
                             (XS[1][2 * cy][cx] + XS[1][2 * cy + 1][cx]);
            const int cnx = dm.nx >> 1, cny = dm.ny >> 1;
            const long o = ((long)(k >> 1) * cny + (ty * (CG_TY / 2) + cy)) * cnx + (tx * (CG_TX / 2) + cx);
            bc[o] = v * T(0.125);
        }
        // the next commit overwrites plane k - 1's slot and the next plane's sums
        lds_barrier();
    };
    // steps z0 .. z1 - 1 in pairs (stage A: even planes, B: odd); z0 and TZr are even
    for (int k = z0; k < z1; k += 2) {
        step(SA, k);
        step(SB, k + 1);
    }
}

// Residual r = b - A x of a finest level given by densities, with its
// partial norms, as a z-march with the tiling of k_cg_dir_apply_rho: x and rho
// of each plane staged on the tile plus a one-cell ring (three-plane rings,
// loaded two steps ahead), b read per cell. Each residual is formed operand
// for operand as apply_row_rho does; it is stored in r as TR when r is not null
// (float64: the CG residual; float32: the mixed-precision defect), and each
// workgroup leaves the sums of r^2 and b^2 over its cells in a fixed order in
// partial_r2[bid] and partial_b2[bid] (when not null). Reads x and rho 1.29
// times (the ring) and b once.
template <typename TR, bool STORE>
__global__ __launch_bounds__(CG_NT) void k_residual_rho(const double* __restrict__ x,
                                                        const double* __restrict__ bb,
                                                        const double* __restrict__ rho, Dims dm,
                                                        double inv_h2, int TZr, int ntx, int nty,
                                                        int nzc, TR* __restrict__ r,
                                                        double* __restrict__ partial_r2,
                                                        double* __restrict__ partial_b2) {
    __shared__ double PP[3][CG_RN];
    __shared__ double RR[3][CG_RN];
    __shared__ double red[2][CG_NT / 64];
    const int nw = ntx * nty * nzc;
    const int bid = blockIdx.x;
    const int w = (nw % 8 == 0) ? (bid % 8) * (nw / 8) + bid / 8 : bid;
    const int tx = w % ntx;
    const int r0 = w / ntx;
    const int ty = r0 % nty;
    const int zc = r0 / nty;
    const int i0 = tx * CG_TX - 1, j0 = ty * CG_TY - 1;
    const int z0 = zc * TZr, z1 = z0 + TZr;
    const long plane = (long)dm.nx * dm.ny;
    const int t = threadIdx.x;
    auto gofs = [&](int xx, int yy) {
        return (long)wrap_near(j0 + yy, dm.ny) * dm.nx + wrap_near(i0 + xx, dm.nx);
    };
    long gp[CG_NL];
    bool vp[CG_NL];
#pragma unroll
    for (int s = 0; s < CG_NL; ++s) {
        int qq = t + s * CG_NT;
        vp[s] = qq < CG_RN;
        gp[s] = vp[s] ? gofs(qq % CG_RX, qq / CG_RX) : gofs(0, 0);
    }
    const int lx = t % CG_TX, ly = t / CG_TX;  // one cell of the tile per thread
    const int c = (ly + 1) * CG_RX + lx + 1;
    const long own = (long)(j0 + 1 + ly) * dm.nx + (i0 + 1 + lx);
    auto pl = [&](int k) { return (long)wrap_near(k, dm.nz) * plane; };
    struct Stage {
        double p[CG_NL], r[CG_NL], b;
    };
    Stage SA, SB;
    // a stage carries x and rho of plane k + 1 (committed at the start of step
    // k, loaded two steps ahead) and b of plane k (used after the step's
    // barrier, loaded at the end of step k - 2): each value is consumed before
    // the stage is loaded again, so no loaded register is copied and no wait
    // drains the loads issued after it
    auto fetch_pr = [&](Stage& S, int k) {
        const long bp = pl(k + 1);
#pragma unroll
        for (int s = 0; s < CG_NL; ++s) {
            S.p[s] = x[bp + gp[s]];
            S.r[s] = rho[bp + gp[s]];
        }
    };
    auto fetch_b = [&](Stage& S, int k) { S.b = bb[pl(k) + own]; };
    auto commit = [&](const Stage& S, int k) {
#pragma unroll
        for (int s = 0; s < CG_NL; ++s)
            if (s * CG_NT + CG_NT <= CG_RN || vp[s]) {
                PP[(k + 4) % 3][t + s * CG_NT] = S.p[s];
                RR[(k + 4) % 3][t + s * CG_NT] = S.r[s];
            }
    };
    {
        const long a = pl(z0 - 1), a0 = pl(z0);
#pragma unroll
        for (int s = 0; s < CG_NL; ++s)
            if (vp[s]) {
                PP[(z0 + 2) % 3][t + s * CG_NT] = x[a + gp[s]];
                RR[(z0 + 2) % 3][t + s * CG_NT] = rho[a + gp[s]];
                PP[z0 % 3][t + s * CG_NT] = x[a0 + gp[s]];
                RR[z0 % 3][t + s * CG_NT] = rho[a0 + gp[s]];
            }
    }
    fetch_pr(SA, z0);
    fetch_b(SA, z0);
    __builtin_amdgcn_sched_barrier(0);
    fetch_pr(SB, z0 + 1);
    fetch_b(SB, z0 + 1);
    double ar = 0.0, ab = 0.0;
    auto step = [&](Stage& S, int k) {
        commit(S, k);
        // past the range the loads re-read plane z1 - 1 (its stage is not used)
        const int kn = k + 2 < z1 ? k + 2 : z1 - 1;
        fetch_pr(S, kn);
        lds_barrier();
        const double* Pc = PP[k % 3];
        const double* Rc = RR[k % 3];
        const double rc = Rc[c];
        const double rxp = Rc[c + 1], rxm = Rc[c - 1], ryp = Rc[c + CG_RX], rym = Rc[c - CG_RX];
        const double rzp = RR[(k + 1) % 3][c], rzm = RR[(k + 2) % 3][c];
        double bxp, bxm, byp, bym, bzp, bzm;
        if (rxp == rc && rxm == rc && ryp == rc && rym == rc && rzp == rc && rzm == rc) {
            bxp = bxm = byp = bym = bzp = bzm = 1.0 / rc;
        } else {
            bxp = 2.0 / (rxp + rc);
            bxm = 2.0 / (rc + rxm);
            byp = 2.0 / (ryp + rc);
            bym = 2.0 / (rc + rym);
            bzp = 2.0 / (rzp + rc);
            bzm = 2.0 / (rc + rzm);
        }
        const double pc = Pc[c];
        double sv = bxp * (Pc[c + 1] - pc) - bxm * (pc - Pc[c - 1]);
        sv += byp * (Pc[c + CG_RX] - pc) - bym * (pc - Pc[c - CG_RX]);
        sv += bzp * (PP[(k + 1) % 3][c] - pc) - bzm * (pc - PP[(k + 2) % 3][c]);
        const double bv = S.b;
        const double rv = bv - sv * inv_h2;
        if constexpr (STORE) r[pl(k) + own] = (TR)rv;
        ar += rv * rv;
        ab += bv * bv;
        // b is used up before its stage is loaded again (keeps the compiler
        // from holding two copies of it across the load)
        __builtin_amdgcn_sched_barrier(0);
        fetch_b(S, kn);
        // the next commit overwrites plane k - 1's slot
        lds_barrier();
    };
    // steps z0 .. z1 - 1 in pairs (stage A: even planes, B: odd); z0 and TZr are even
    for (int k = z0; k < z1; k += 2) {
        step(SA, k);
        step(SB, k + 1);
    }
    // fixed-order workgroup sums
    for (int off = 32; off > 0; off >>= 1) {
        ar += __shfl_xor(ar, off);
        ab += __shfl_xor(ab, off);
    }
    if ((t & 63) == 0) {
        red[0][t >> 6] = ar;
        red[1][t >> 6] = ab;
    }
    __syncthreads();
    if (t == 0) {
        double sr = 0.0, sb = 0.0;
        for (int i = 0; i < CG_NT / 64; ++i) {
            sr += red[0][i];
            sb += red[1][i];
        }
        partial_r2[bid] = sr;
        if (partial_b2) partial_b2[bid] = sb;
    }
}

// For the learned guess's judge: r = b - A x with partial sums of r^2, b^2 and
// x (b + r) per block
template <int DIM, class K>
__global__ void k_energy(const double* __restrict__ x, const double* __restrict__ b, K co, Dims d,
                         double inv_h2, double* __restrict__ partial_r2, double* __restrict__ partial_b2,
                         double* __restrict__ partial_e) {
    __shared__ double sh[kBlock];
    double ar = 0.0, ab = 0.0, ae = 0.0;
    const int N = (int)d.cells(), nx = d.nx, ny = d.ny;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < N; c += gridDim.x * blockDim.x) {
        const int i = c % nx;
        const int rr = c / nx;
        const Nb n = neighbours(d, i, rr % ny, rr / ny, DIM);
        const double bv = b[c];
        const double rv = bv - apply_row<double, DIM>(x, co, n) * inv_h2;
        ar += rv * rv;
        ab += bv * bv;
        ae += x[c] * (bv + rv);
    }
    double v = block_reduce_sum(ar, sh);
    if (threadIdx.x == 0) partial_r2[blockIdx.x] = v;
    v = block_reduce_sum(ab, sh);
    if (threadIdx.x == 0) partial_b2[blockIdx.x] = v;
    v = block_reduce_sum(ae, sh);
    if (threadIdx.x == 0) partial_e[blockIdx.x] = v;
}

// ---------------------------------------------------------------------------
// host side
// tile of the density sweep: 32 x 16 cells, 512 threads (2 workgroups per
// CU); its halo region holds 1.41 cells per tile cell against 1.59 for 64 x 8
constexpr int kRTX = 32, kRTY = 16, kRNT = 512;

template <typename T> LevelT<T>& lvl(Level& L);
template <> LevelT<double>& lvl<double>(Level& L) { return L.f64; }
template <> LevelT<float>& lvl<float>(Level& L) { return L.f32; }

// zero: the red pass of a sweep from p = 0 (p is not read)
template <typename T>
static void launch_rbgs(Level& L, int color, hipStream_t st, bool finest, bool zero = false) {
    ProfScope ps(sizeof(T) == 8 ? IB_PROF_SMOOTH64 : IB_PROF_SMOOTH32, st, finest);
    LevelT<T>& A = lvl<T>(L);
    T h2 = (T)(L.d.h * L.d.h);
    long half = L.d.cells() / 2;
    const dim3 g(grid_for(half)), blk(kBlock);
    const T* b2 = L.d.dim == 2 ? A.beta[1] : A.beta[2];
    if (L.d.dim == 2 && zero)
        hipLaunchKernelGGL((k_rbgs<T, 2, true>), g, blk, 0, st, A.p, A.b, A.beta[0], A.beta[1], b2, L.d, h2, 0);
    else if (L.d.dim == 2)
        hipLaunchKernelGGL((k_rbgs<T, 2>), g, blk, 0, st, A.p, A.b, A.beta[0], A.beta[1], b2, L.d, h2, color);
    else if (zero)
        hipLaunchKernelGGL((k_rbgs<T, 3, true>), g, blk, 0, st, A.p, A.b, A.beta[0], A.beta[1], b2, L.d, h2, 0);
    else
        hipLaunchKernelGGL((k_rbgs<T, 3>), g, blk, 0, st, A.p, A.b, A.beta[0], A.beta[1], b2, L.d, h2, color);
}

// zero: the sweep starts from p = 0 (pin is not read); pe (density levels
// only): the sweep starts from pin + P pe, pe the correction on the coarse
// level below (the prolongation folded into the sweep)
template <typename T>
static void launch_fused(Level& L, T* pin, T* pout, hipStream_t st, bool finest, bool zero,
                         bool dots = false, const T* pe = nullptr) {
    // sweeps from p = 0 read less and are timed under their own kind
    ProfScope ps(zero ? IB_PROF_SWEEP_ZERO
                      : dots ? IB_PROF_SWEEP_DOTS
                             : pe ? IB_PROF_SWEEP_PRO
                                  : (sizeof(T) == 8 ? (L.rho ? IB_PROF_SWEEP64_RHO : IB_PROF_SWEEP64)
                                                    : IB_PROF_SWEEP32),
                 st, finest);
    LevelT<T>& A = lvl<T>(L);
    T h2 = (T)(L.d.h * L.d.h);
    int ntx = L.d.nx / kFTX, nty = L.d.ny / kFTY, nzc = L.d.nz / L.tz;
    if constexpr (sizeof(T) == 8) {
        if (L.rho) {
            const int rx = L.d.nx / kRTX, ry = L.d.ny / kRTY, rz = L.d.nz / L.rtz;
            if (dots && L.dots_q)
                hipLaunchKernelGGL((k_rbgs_fused_rho<double, kRTX, kRTY, kRNT, false, 2>), dim3(rx * ry * rz),
                                   dim3(kRNT), 0, st, pin, pout, A.b, L.rho, L.d, h2, L.rtz, rx, ry, rz,
                                   L.dots_q, L.dots_part);
            else if (dots)
                hipLaunchKernelGGL((k_rbgs_fused_rho<double, kRTX, kRTY, kRNT, false, 1>), dim3(rx * ry * rz),
                                   dim3(kRNT), 0, st, pin, pout, A.b, L.rho, L.d, h2, L.rtz, rx, ry, rz,
                                   nullptr, L.dots_part);
            else if (zero)
                hipLaunchKernelGGL((k_rbgs_fused_rho<double, kRTX, kRTY, kRNT, true>), dim3(rx * ry * rz),
                                   dim3(kRNT), 0, st, pin, pout, A.b, L.rho, L.d, h2, L.rtz, rx, ry, rz);
            else if (pe)
                hipLaunchKernelGGL((k_rbgs_fused_rho<double, kRTX, kRTY, kRNT, false, 0, true>),
                                   dim3(rx * ry * rz), dim3(kRNT), 0, st, pin, pout, A.b, L.rho, L.d, h2, L.rtz,
                                   rx, ry, rz, nullptr, nullptr, pe);
            else
                hipLaunchKernelGGL((k_rbgs_fused_rho<double, kRTX, kRTY, kRNT, false>), dim3(rx * ry * rz),
                                   dim3(kRNT), 0, st, pin, pout, A.b, L.rho, L.d, h2, L.rtz, rx, ry, rz);
            return;
        }
    } else {
        if (L.rho32) {
            // the float32 cycle's finest level from the float32 densities
            const int rx = L.d.nx / kRTX, ry = L.d.ny / kRTY, rz = L.d.nz / L.rtz;
            if (dots && L.dots_q)
                hipLaunchKernelGGL((k_rbgs_fused_rho<float, kRTX, kRTY, kRNT, false, 2>), dim3(rx * ry * rz),
                                   dim3(kRNT), 0, st, pin, pout, A.b, L.rho32, L.d, h2, L.rtz, rx, ry, rz,
                                   L.dots_q, L.dots_part, nullptr, L.dots_r);
            else if (dots)
                hipLaunchKernelGGL((k_rbgs_fused_rho<float, kRTX, kRTY, kRNT, false, 1>), dim3(rx * ry * rz),
                                   dim3(kRNT), 0, st, pin, pout, A.b, L.rho32, L.d, h2, L.rtz, rx, ry, rz,
                                   nullptr, L.dots_part, nullptr, L.dots_r);
            else if (zero)
                hipLaunchKernelGGL((k_rbgs_fused_rho<float, kRTX, kRTY, kRNT, true>), dim3(rx * ry * rz),
                                   dim3(kRNT), 0, st, pin, pout, A.b, L.rho32, L.d, h2, L.rtz, rx, ry, rz);
            else if (pe)
                hipLaunchKernelGGL((k_rbgs_fused_rho<float, kRTX, kRTY, kRNT, false, 0, true>),
                                   dim3(rx * ry * rz), dim3(kRNT), 0, st, pin, pout, A.b, L.rho32, L.d, h2,
                                   L.rtz, rx, ry, rz, nullptr, nullptr, pe);
            else
                hipLaunchKernelGGL((k_rbgs_fused_rho<float, kRTX, kRTY, kRNT, false>), dim3(rx * ry * rz),
                                   dim3(kRNT), 0, st, pin, pout, A.b, L.rho32, L.d, h2, L.rtz, rx, ry, rz);
            return;
        }
    }
    if (zero)
        hipLaunchKernelGGL((k_rbgs_fused<T, true>), dim3(ntx * nty * nzc), dim3(kBlock), 0, st, pin, pout,
                           A.b, A.beta[0], A.beta[1], A.beta[2], L.d, h2, L.tz, ntx, nty, nzc);
    else
        hipLaunchKernelGGL((k_rbgs_fused<T, false>), dim3(ntx * nty * nzc), dim3(kBlock), 0, st, pin, pout,
                           A.b, A.beta[0], A.beta[1], A.beta[2], L.d, h2, L.tz, ntx, nty, nzc);
}

// nu red-black sweeps on level L; returns the buffer holding the result.
// zero_first: the level starts from p = 0, which the first sweep takes
// without reading p (p need not be filled)
// dots_last: the last sweep leaves the inner products of Level::dots_*
template <typename T>
static T* smooth(Level& L, T* cur, int nu, hipStream_t st, bool finest, bool zero_first,
                 bool dots_last = false, const T* pe = nullptr) {
    LevelT<T>& A = lvl<T>(L);
    for (int s = 0; s < nu; ++s) {
        if (L.fused) {
            T* other = cur == A.p ? A.alt : A.p;
            launch_fused<T>(L, cur, other, st, finest, zero_first && s == 0,
                            dots_last && s == nu - 1 && !(zero_first && s == 0), s == 0 ? pe : nullptr);
            cur = other;
        } else {
            T* save = A.p;
            A.p = cur;
            launch_rbgs<T>(L, 0, st, finest, zero_first && s == 0);
            launch_rbgs<T>(L, 1, st, finest);
            A.p = save;
        }
    }
    return cur;
}

// the coarse right side B.b = R (A.b - A_L cur) of level L (mean of the 2^dim
// children of the fine residual)
template <typename T>
static void restrict_residual(Level& L, Level& C, const T* cur, hipStream_t st, bool fin) {
    LevelT<T>& A = lvl<T>(L);
    LevelT<T>& B = lvl<T>(C);
    T inv_h2 = (T)(1.0 / (L.d.h * L.d.h));
    long nc = C.d.cells();
    {
        ProfScope ps(sizeof(T) == 8 ? IB_PROF_RESTRICT64 : IB_PROF_RESTRICT32, st, fin);
        const CoefArrays<T> co{A.beta[0], A.beta[1], L.d.dim == 3 ? A.beta[2] : A.beta[1]};
        const dim3 g64(L.d.nx / 64, L.d.ny / 2, L.d.nz / 2);
        bool done = false;
        if constexpr (sizeof(T) == 8) {
            if (L.rho && L.d.ny % CG_TY == 0 && L.rtz > 0 && L.rtz % 2 == 0) {
                // tiled z-march (nx % 64 == 0 where rho is set)
                const int tx = L.d.nx / CG_TX, ty = L.d.ny / CG_TY, tz = L.d.nz / L.rtz;
                hipLaunchKernelGGL(k_resrestrict_rho<double>, dim3(tx * ty * tz), dim3(CG_NT), 0, st, cur, A.b,
                                   L.rho, L.d, inv_h2, L.rtz, tx, ty, tz, B.b);
                done = true;
            } else if (L.rho) {  // set only where nx % 64 == 0 in 3D
                hipLaunchKernelGGL((k_residual_restrict64<double, CoefRho>), g64, dim3(kBlock), 0, st,
                                   cur, A.b, CoefRho{L.rho}, L.d, inv_h2, B.b);
                done = true;
            }
        } else {
            if (L.rho32 && L.d.ny % CG_TY == 0 && L.rtz > 0 && L.rtz % 2 == 0 && L.d.nx % CG_TX == 0) {
                // the same tiled z-march on the float32 densities
                const int tx = L.d.nx / CG_TX, ty = L.d.ny / CG_TY, tz = L.d.nz / L.rtz;
                hipLaunchKernelGGL(k_resrestrict_rho<float>, dim3(tx * ty * tz), dim3(CG_NT), 0, st, cur, A.b,
                                   L.rho32, L.d, inv_h2, L.rtz, tx, ty, tz, B.b);
                done = true;
            } else if (L.rho32 && L.d.nx % 64 == 0) {
                hipLaunchKernelGGL((k_residual_restrict64<float, CoefRhoF>), g64, dim3(kBlock), 0, st, cur, A.b,
                                   CoefRhoF{L.rho32}, L.d, inv_h2, B.b);
                done = true;
            }
        }
        if (done) {
        } else if (L.d.dim == 2)
            hipLaunchKernelGGL((k_residual_restrict<T, 2>), dim3(grid_for(nc)), dim3(kBlock), 0, st,
                               cur, A.b, co, L.d, inv_h2, B.b);
        else if (L.d.nx % 64 == 0)
            hipLaunchKernelGGL((k_residual_restrict64<T, CoefArrays<T>>), g64, dim3(kBlock), 0, st,
                               cur, A.b, co, L.d, inv_h2, B.b);
        else
            hipLaunchKernelGGL((k_residual_restrict<T, 3>), dim3(grid_for(nc)), dim3(kBlock), 0, st,
                               cur, A.b, co, L.d, inv_h2, B.b);
    }
}

// zero_start: level l starts from p = 0; on levels with the single-pass
// smoother p is then neither filled nor read, elsewhere the caller filled it
template <typename T>
static void vcycle(mg_handle* m, int l, hipStream_t st, bool zero_start) {
    Level& L = m->lv[l];
    LevelT<T>& A = lvl<T>(L);
    int last = (int)m->lv.size() - 1;
    if (l == m->persist) {
        // this level and all below in one workgroup
        PersistLevels<T> P;
        P.n = last - l + 1;
        P.nu1 = m->o.nu1;
        P.nu2 = m->o.nu2;
        P.nc = m->nc;
        P.zero = zero_start ? 1 : 0;
        P.minv = m->cinv;
        for (int i = 0; i < P.n; ++i) {
            Level& Li = m->lv[l + i];
            LevelT<T>& Ai = lvl<T>(Li);
            P.d[i] = Li.d;
            P.p[i] = Ai.p;
            P.b[i] = Ai.b;
            P.b0[i] = Ai.beta[0];
            P.b1[i] = Ai.beta[1];
            P.b2[i] = Li.d.dim == 3 ? Ai.beta[2] : Ai.beta[1];
        }
        // 3D: the LDS-resident form when the levels below the first fit its pool
        long pool = 0;
        for (int i = 1; i < P.n; ++i) pool += P.d[i].cells();
        if (L.d.dim == 3 && L.d.cells() <= kPersistCells && pool <= kLdsPool && P.nc <= kMaxCoarse)
            hipLaunchKernelGGL((k_coarse_vcycle_lds<T>), dim3(1), dim3(kLdsThreads), 0, st, P);
        else if (L.d.dim == 3)
            hipLaunchKernelGGL((k_coarse_vcycle<T, 3>), dim3(1), dim3(kPersistThreads), 0, st, P);
        else
            hipLaunchKernelGGL((k_coarse_vcycle<T, 2>), dim3(1), dim3(kPersistThreads), 0, st, P);
        return;
    }
    if (l == last) {
        hipLaunchKernelGGL((k_coarse_apply<T>), dim3(1), dim3(64), 0, st, m->cinv, m->nc, A.b, A.p);
        return;
    }
    Level& C = m->lv[l + 1];
    LevelT<T>& B = lvl<T>(C);
    bool fin = l == 0;
    // from p = 0 the first sweep reads no p; without pre-smoothing the
    // restriction reads it, so it is cleared
    if (zero_start && m->o.nu1 == 0)
        hipLaunchKernelGGL((k_fill<T>), dim3(grid_for(L.d.cells())), dim3(kBlock), 0, st, A.p, L.d.cells(),
                           (T)0);
    T* cur = smooth<T>(L, A.p, m->o.nu1, st, fin, zero_start);
    restrict_residual<T>(L, C, cur, st, fin);
    // every coarser level starts from p = 0 without a fill
    vcycle<T>(m, l + 1, st, true);
    // on a 3D density level with at least two post-smoothing sweeps the first
    // (a plain sweep) adds the prolongated correction as it stages p
    const bool fold = L.fused && L.d.dim == 3 && m->o.nu2 >= 2 && !m->o.split_coarse &&
                      (sizeof(T) == 8 ? L.rho != nullptr : L.rho32 != nullptr);
    if (!fold) {
        ProfScope ps(sizeof(T) == 8 ? IB_PROF_PROLONG64 : IB_PROF_PROLONG32, st, fin);
        int bx = std::min(L.d.nx, kBlock);
        dim3 pg((L.d.nx + bx - 1) / bx, L.d.ny, L.d.nz);
        if (L.d.dim == 2) {
            hipLaunchKernelGGL((k_prolong_add<T, 2>), pg, dim3(bx), 0, st, cur, B.p, L.d);
        } else {
            const int cxn = L.d.nx / 2, cb = std::min(cxn, 128);
            hipLaunchKernelGGL((k_prolong_add_blk<T>), dim3((cxn + cb - 1) / cb, L.d.ny / 2, L.d.nz / 2),
                               dim3(cb), 0, st, cur, B.p, L.d);
        }
    }
    cur = smooth<T>(L, cur, m->o.nu2, st, fin, false, L.dots_on, fold ? B.p : nullptr);
    if (cur != A.p)
        (void)hipMemcpyAsync(A.p, cur, sizeof(T) * L.d.cells(), hipMemcpyDeviceToDevice, st);
}

static int red_blocks(long N) { return (int)std::min<long>(kRed, (long)grid_for(N)); }


// z-range per workgroup of the density kernels (the sweep's 32 x 16 tiles
// and the 64 x 8 tiles of the CG and residual kernels, as many of either) on a
// 3D level the single-pass smoother takes, or 0 where they do not apply
static int density_rtz(const Dims& d) {
    if (d.dim != 3 || d.nx % kFTX != 0 || d.ny % kFTY != 0 || d.nz < 32 || d.nz % 2 != 0 ||
        d.cells() < 128L * 128 * 128 || d.nx % kRTX != 0 || d.ny % kRTY != 0)
        return 0;
    long rtiles = (long)(d.nx / kRTX) * (d.ny / kRTY);
    int rtz = d.nz;
    // 1024 workgroups on 256^3 (z-range 32): two rounds of the 512
    // resident ones keep the z-marches short and the XCDs balanced
    while (rtz % 4 == 0 && rtz > 16 && rtiles * (d.nz / rtz) < 1024) rtz /= 2;
    return rtz;
}

// the finest level is given by densities on a grid the CG z-march tiles
// (64 x 8 columns, an even z-range per workgroup)
static bool tiled_rho(const Level& L) {
    return L.rho != nullptr && L.d.dim == 3 && L.d.nx % CG_TX == 0 && L.d.ny % CG_TY == 0 && L.rtz > 0 &&
           L.rtz % 2 == 0 && (long)(L.d.nx / CG_TX) * (L.d.ny / CG_TY) * (L.d.nz / L.rtz) <= kRed;
}

// r = b - A x on a tiled density level (r stored as TR when not null) with
// per-workgroup partial sums of r^2 in pr and b^2 in pb (when not null);
// returns the number of partials
template <typename TR>
static int launch_residual_rho(const Level& L, const double* x, const double* b, TR* r, double* pr,
                               double* pb, hipStream_t st) {
    const int tx = L.d.nx / CG_TX, ty = L.d.ny / CG_TY, tz = L.d.nz / L.rtz;
    // whether r is stored is fixed at compile time: a store on one path only
    // would make the loop's waits drain every load in flight
    if (r)
        hipLaunchKernelGGL((k_residual_rho<TR, true>), dim3(tx * ty * tz), dim3(CG_NT), 0, st, x, b, L.rho,
                           L.d, 1.0 / (L.d.h * L.d.h), L.rtz, tx, ty, tz, r, pr, pb);
    else
        hipLaunchKernelGGL((k_residual_rho<TR, false>), dim3(tx * ty * tz), dim3(CG_NT), 0, st, x, b, L.rho,
                           L.d, 1.0 / (L.d.h * L.d.h), L.rtz, tx, ty, tz, r, pr, pb);
    return tx * ty * tz;
}

// ||b - A p||^2 (and ||b||^2 when want_b) into m->host[0], m->host[1]; syncs
// (zero: p is known to be zero, so r = b)
static int fp64_norms(mg_handle* m, bool want_b, hipStream_t st, bool zero = false) {
    Level& L = m->lv[0];
    long N = L.d.cells();
    int nb = red_blocks(N);
    double inv_h2 = 1.0 / (L.d.h * L.d.h);
    double* pr = m->red;
    double* pb = want_b ? m->red + kRed : nullptr;
    {
    ProfScope ps(IB_PROF_RESID, st, true);
    const CoefArrays<double> co{L.f64.beta[0], L.f64.beta[1],
                                L.d.dim == 3 ? L.f64.beta[2] : L.f64.beta[1]};
    if (zero)
        hipLaunchKernelGGL(k_residual_zero, dim3(nb), dim3(kBlock), 0, st, L.f64.b, (int)N, nullptr, pr, pb);
    else if (tiled_rho(L))
        nb = launch_residual_rho<double>(L, L.f64.p, L.f64.b, nullptr, pr, pb, st);
    else if (L.rho)
        hipLaunchKernelGGL((k_resid_norm<3, CoefRho>), dim3(nb), dim3(kBlock), 0, st, L.f64.p,
                           L.f64.b, CoefRho{L.rho}, L.d, inv_h2, pr, pb);
    else if (L.d.dim == 2)
        hipLaunchKernelGGL((k_resid_norm<2, CoefArrays<double>>), dim3(nb), dim3(kBlock), 0, st,
                           L.f64.p, L.f64.b, co, L.d, inv_h2, pr, pb);
    else
        hipLaunchKernelGGL((k_resid_norm<3, CoefArrays<double>>), dim3(nb), dim3(kBlock), 0, st,
                           L.f64.p, L.f64.b, co, L.d, inv_h2, pr, pb);
    }
    if (want_b)
        IB_TRY(device_sum2(pr, pb, nb, m->red + 3 * kRed, m->red + 3 * kRed + 1, st));
    else
        IB_TRY(device_sum(pr, nb, m->red + 3 * kRed, st));
    IB_HIP(hipMemcpyAsync(m->host, m->red + 3 * kRed, sizeof(double) * 2, hipMemcpyDeviceToHost, st));
    IB_HIP(hipStreamSynchronize(st));
    prof_drain();
    return IB_OK;
}

static int mixed_defect(mg_handle* m, bool want_b, hipStream_t st, bool sync = true) {
    Level& L = m->lv[0];
    long N = L.d.cells();
    int nb = red_blocks(N);
    double inv_h2 = 1.0 / (L.d.h * L.d.h);
    double* pr = m->red;
    double* pb = want_b ? m->red + kRed : nullptr;
    {
    ProfScope ps(IB_PROF_RESID, st, true);
    const CoefArrays<double> co{L.f64.beta[0], L.f64.beta[1],
                                L.d.dim == 3 ? L.f64.beta[2] : L.f64.beta[1]};
    if (tiled_rho(L))
        nb = launch_residual_rho<float>(L, L.f64.p, L.f64.b, L.f32.b, pr, pb, st);
    else if (L.rho)
        hipLaunchKernelGGL((k_defect_f32<3, CoefRho>), dim3(nb), dim3(kBlock), 0, st, L.f64.p,
                           L.f64.b, CoefRho{L.rho}, L.d, inv_h2, L.f32.b, pr, pb);
    else if (L.d.dim == 2)
        hipLaunchKernelGGL((k_defect_f32<2, CoefArrays<double>>), dim3(nb), dim3(kBlock), 0, st,
                           L.f64.p, L.f64.b, co, L.d, inv_h2, L.f32.b, pr, pb);
    else
        hipLaunchKernelGGL((k_defect_f32<3, CoefArrays<double>>), dim3(nb), dim3(kBlock), 0, st,
                           L.f64.p, L.f64.b, co, L.d, inv_h2, L.f32.b, pr, pb);
    }
    if (!sync) return IB_OK;
    if (want_b)
        IB_TRY(device_sum2(pr, pb, nb, m->red + 3 * kRed, m->red + 3 * kRed + 1, st));
    else
        IB_TRY(device_sum(pr, nb, m->red + 3 * kRed, st));
    IB_HIP(hipMemcpyAsync(m->host, m->red + 3 * kRed, sizeof(double) * 2, hipMemcpyDeviceToHost, st));
    IB_HIP(hipStreamSynchronize(st));
    prof_drain();
    return IB_OK;
}

static int remove_mean(mg_handle* m, bool sums_ready, hipStream_t st) {
    Level& L = m->lv[0];
    long N = L.d.cells();
    int nb = red_blocks(N);
    if (!sums_ready)
        hipLaunchKernelGGL(k_sum_cells, dim3(nb), dim3(kBlock), 0, st, L.f64.p, N, m->red + 2 * kRed);
    IB_TRY(device_sum(m->red + 2 * kRed, nb, m->red + 3 * kRed + 2, st));
    hipLaunchKernelGGL(k_sub_scalar_mean, dim3(grid_for(N)), dim3(kBlock), 0, st, L.f64.p, N,
                       m->red + 3 * kRed + 2);
    IB_HIP(hipGetLastError());
    return IB_OK;
}

}  // namespace ib

using namespace ib;

extern "C" void ib_profile_enable(int on) { g_prof.on = on != 0; }

extern "C" void ib_profile_reset(void) {
    for (int k = 0; k < IB_PROF_KINDS; ++k) {
        g_prof.count[k] = 0;
        g_prof.ms[k] = 0.0;
    }
}

extern "C" int ib_profile_read(int kind, long long* launches, double* total_ms) {
    IB_CHECK(kind >= 0 && kind < IB_PROF_KINDS && launches && total_ms, IB_EINVAL,
             "ib_profile_read: bad argument");
    *launches = g_prof.count[kind];
    *total_ms = g_prof.ms[kind];
    return IB_OK;
}

extern "C" int mg_setup(const ib_grid* g, const mg_opts* o, mg_handle** out) {
    IB_CHECK(g && o && out, IB_EINVAL, "mg_setup: null argument");
    IB_CHECK(g->dim == 2 || g->dim == 3, IB_EINVAL, "mg_setup: dim must be 2 or 3");
    IB_CHECK(o->precision == MG_FP64 || o->precision == MG_MIXED, IB_EINVAL, "mg_setup: precision");
    IB_CHECK(o->nu1 >= 0 && o->nu2 >= 0 && o->nu1 + o->nu2 > 0, IB_EINVAL, "mg_setup: sweeps");
    IB_CHECK(o->n_coarsest >= 2, IB_EINVAL, "mg_setup: n_coarsest");
    IB_CHECK(o->krylov == 0 || o->krylov == 1, IB_EINVAL, "mg_setup: krylov must be 0 or 1");
    IB_CHECK(o->split_coarse == 0 || o->split_coarse == 1, IB_EINVAL, "mg_setup: split_coarse must be 0 or 1");
    IB_CHECK(g->h > 0, IB_EINVAL, "mg_setup: h");
    int nmin = g->n[0];
    for (int e = 0; e < g->dim; ++e) {
        IB_CHECK(g->n[e] >= 2, IB_EINVAL, "mg_setup: grid size");
        nmin = std::min(nmin, g->n[e]);
    }
    int L = 0;
    while ((nmin >> L) > o->n_coarsest) ++L;
    IB_CHECK((nmin >> L) == o->n_coarsest && ((nmin >> L) << L) == nmin, IB_EINVAL,
             "mg_setup: the smallest axis must be n_coarsest * 2^L");
    long ncoarse = 1;
    for (int e = 0; e < g->dim; ++e) {
        IB_CHECK(((g->n[e] >> L) << L) == g->n[e], IB_EINVAL,
                 "mg_setup: every axis must be divisible by 2^levels");
        ncoarse *= (g->n[e] >> L);
    }
    IB_CHECK(ncoarse <= kMaxCoarse, IB_EINVAL, "mg_setup: coarsest grid larger than 64 cells");
    mg_handle* m = new mg_handle();
    m->g = *g;
    m->o = *o;
    m->nc = (int)ncoarse;
    bool mixed = o->precision == MG_MIXED;
    auto cleanup = [&](int code, const char* msg) {
        mg_destroy(m);
        return fail(code, msg);
    };
    for (int l = 0; l <= L; ++l) {
        Level lv;
        lv.d = make_dims(*g);
        lv.d.nx = g->n[0] >> l;
        lv.d.ny = g->n[1] >> l;
        lv.d.nz = g->dim == 3 ? (g->n[2] >> l) : 1;
        lv.d.h = g->h * (double)(1 << l);
        long N = lv.d.cells();
        lv.own_pb = l > 0;
        if (g->dim == 3 && lv.d.nx % kFTX == 0 && lv.d.ny % kFTY == 0 && lv.d.nz >= 32 &&
            lv.d.nz % 2 == 0 && N >= 128L * 128 * 128) {
            // z-range per workgroup: an even divisor of nz (the sweep runs its
            // steps in pairs), halved while the grid has under 1024 workgroups
            lv.fused = true;
            long tiles = (long)(lv.d.nx / kFTX) * (lv.d.ny / kFTY);
            int tz = lv.d.nz;
            while (tz % 4 == 0 && tz > 16 && tiles * (lv.d.nz / tz) < 1024) tz /= 2;
            lv.tz = tz;
            lv.rtz = density_rtz(lv.d);
        }
        if (l > 0) {
            if (hipMalloc(&lv.f64.p, N * sizeof(double)) != hipSuccess ||
                hipMalloc(&lv.f64.b, N * sizeof(double)) != hipSuccess)
                return cleanup(IB_ENOMEM, "mg_setup: out of device memory");
            for (int e = 0; e < g->dim; ++e)
                if (hipMalloc(&lv.f64.beta[e], N * sizeof(double)) != hipSuccess)
                    return cleanup(IB_ENOMEM, "mg_setup: out of device memory");
        }
        if (lv.fused && hipMalloc(&lv.f64.alt, N * sizeof(double)) != hipSuccess)
            return cleanup(IB_ENOMEM, "mg_setup: out of device memory");
        if (lv.fused && mixed && hipMalloc(&lv.f32.alt, N * sizeof(float)) != hipSuccess)
            return cleanup(IB_ENOMEM, "mg_setup: out of device memory");
        if (mixed) {
            if (hipMalloc(&lv.f32.p, N * sizeof(float)) != hipSuccess ||
                hipMalloc(&lv.f32.b, N * sizeof(float)) != hipSuccess)
                return cleanup(IB_ENOMEM, "mg_setup: out of device memory");
            for (int e = 0; e < g->dim; ++e)
                if (hipMalloc(&lv.f32.beta[e], N * sizeof(float)) != hipSuccess)
                    return cleanup(IB_ENOMEM, "mg_setup: out of device memory");
        }
        m->lv.push_back(lv);
    }
    // the persistent coarse kernel takes the first level of at most
    // kPersistCells cells (with at least one level below it) whose
    // restriction is the generic one (2D, or x not a multiple of 64)
    if (!o->split_coarse) {
        const int nl = (int)m->lv.size();
        for (int l = 1; l < nl - 1; ++l) {
            const Level& lv = m->lv[l];
            if (lv.d.cells() <= kPersistCells && !lv.fused && (g->dim == 2 || lv.d.nx % 64 != 0) &&
                nl - l <= kPersistMaxLevels) {
                m->persist = l;
                break;
            }
        }
    }
    int m1 = m->nc;
    if (hipMalloc(&m->cmat, sizeof(double) * m1 * m1) != hipSuccess ||
        hipMalloc(&m->cinv, sizeof(double) * m1 * m1) != hipSuccess ||
        hipMalloc(&m->red, sizeof(double) * (3 * kRed + 8)) != hipSuccess ||
        hipHostMalloc(&m->host, sizeof(double) * 8) != hipSuccess)
        return cleanup(IB_ENOMEM, "mg_setup: out of memory");
    if (o->krylov) {
        const long N = m->lv[0].d.cells();
        if (hipMalloc(&m->kr, N * sizeof(double)) != hipSuccess ||
            hipMalloc(&m->kd, N * sizeof(double)) != hipSuccess ||
            hipMalloc(&m->kd2, N * sizeof(double)) != hipSuccess ||
            hipMalloc(&m->kq, N * sizeof(double)) != hipSuccess ||
            (!mixed && hipMalloc(&m->kz, N * sizeof(double)) != hipSuccess) ||
            hipMalloc(&m->ks, 16 * sizeof(double)) != hipSuccess)
            return cleanup(IB_ENOMEM, "mg_setup: out of device memory");
    }
    *out = m;
    return IB_OK;
}

extern "C" void mg_destroy(mg_handle* m) {
    if (!m) return;
    for (auto& lv : m->lv) {
        if (lv.own_pb) {
            hipFree(lv.f64.p);
            hipFree(lv.f64.b);
            for (int e = 0; e < 3; ++e) hipFree(lv.f64.beta[e]);
        }
        hipFree(lv.f64.alt);
        hipFree(lv.f32.alt);
        hipFree(lv.f32.p);
        hipFree(lv.f32.b);
        for (int e = 0; e < 3; ++e) hipFree(lv.f32.beta[e]);
    }
    for (int e = 0; e < 3; ++e) hipFree(m->beta0[e]);
    hipFree(m->kr);
    hipFree(m->kz);
    hipFree(m->kd);
    hipFree(m->kd2);
    hipFree(m->kq);
    hipFree(m->ks);
    hipFree(m->cmat);
    hipFree(m->cinv);
    hipFree(m->red);
    if (m->host) hipHostFree(m->host);
    delete m;
}

// finest level from stored faces (beta) or from cell densities (rho)
static int update_hierarchy(mg_handle* m, const double* const beta[3], const double* rho,
                            hipStream_t st) {
    int dim = m->g.dim;
    Level& L0 = m->lv[0];
    L0.rho = rho;
    for (int e = 0; e < 3; ++e) L0.f64.beta[e] = (!rho && e < dim) ? const_cast<double*>(beta[e]) : nullptr;
    for (size_t l = 1; l < m->lv.size(); ++l) {
        Level& F = m->lv[l - 1];
        Level& C = m->lv[l];
        long nc = C.d.cells();
        const CoefArrays<double> co{F.f64.beta[0], F.f64.beta[1], dim == 3 ? F.f64.beta[2] : F.f64.beta[1]};
        if (F.rho)
            hipLaunchKernelGGL((k_coarsen_beta<3, CoefRho>), dim3(grid_for(nc)), dim3(kBlock), 0, st,
                               CoefRho{F.rho}, F.d, C.f64.beta[0], C.f64.beta[1], C.f64.beta[2]);
        else if (dim == 2)
            hipLaunchKernelGGL((k_coarsen_beta<2, CoefArrays<double>>), dim3(grid_for(nc)), dim3(kBlock),
                               0, st, co, F.d, C.f64.beta[0], C.f64.beta[1], C.f64.beta[1]);
        else
            hipLaunchKernelGGL((k_coarsen_beta<3, CoefArrays<double>>), dim3(grid_for(nc)), dim3(kBlock),
                               0, st, co, F.d, C.f64.beta[0], C.f64.beta[1], C.f64.beta[2]);
    }
    if (m->o.precision == MG_MIXED)
        for (auto& L : m->lv) {
            L.rho32 = nullptr;
            if (L.rho) {
                hipLaunchKernelGGL(k_cast_f32, dim3(grid_for(L.d.cells())), dim3(kBlock), 0, st, L.rho,
                                   L.f32.beta[0], L.d.cells());
                L.rho32 = L.f32.beta[0];
                continue;
            }
            for (int e = 0; e < dim; ++e)
                hipLaunchKernelGGL(k_cast_f32, dim3(grid_for(L.d.cells())), dim3(kBlock), 0, st,
                                   L.f64.beta[e], L.f32.beta[e], L.d.cells());
        }
    Level& Cl = m->lv.back();
    if (dim == 2)
        hipLaunchKernelGGL(k_build_coarse<2>, dim3(1), dim3(kMaxCoarse), 0, st, Cl.f64.beta[0],
                           Cl.f64.beta[1], Cl.f64.beta[1], Cl.d, m->cmat);
    else
        hipLaunchKernelGGL(k_build_coarse<3>, dim3(1), dim3(kMaxCoarse), 0, st, Cl.f64.beta[0],
                           Cl.f64.beta[1], Cl.f64.beta[2], Cl.d, m->cmat);
    hipLaunchKernelGGL(k_spd_inverse, dim3(1), dim3(1024), 0, st, m->cmat, m->nc, m->cinv);
    IB_HIP(hipGetLastError());
    m->coeffs_ready = true;
    return IB_OK;
}

// the finest-level kernels read densities directly on 3D grids with the
// single-pass smoother, the 64-wide restriction and at least one coarse level
static bool density_direct(const mg_handle* m) {
    const Level& L0 = m->lv[0];
    return m->g.dim == 3 && L0.fused && L0.rtz > 0 && L0.d.nx % 64 == 0 && m->lv.size() >= 2;
}

int mg_takes_density(const mg_handle* m) { return m && density_direct(m) ? 1 : 0; }

void mg_hint_zero_guess(mg_handle* m) {
    if (m) m->x_zero = true;
}

// For a start x (NULL: zero): ||b - A x|| / ||b|| and the energy functional
// E(x) = x . (b + r(x)), r = b - A x. With K = -A (positive definite on
// zero-mean vectors) and K p = -b, E(x) = ||x - p||_K^2 - ||p||_K^2: of two
// starts, the smaller E has the smaller error in the energy norm, the norm in
// which conjugate gradients and multigrid converge. E(0) = 0; constants do
// not change E (b has zero sum). Syncs.
int mg_energy(mg_handle* m, const double* b, const double* x, double* rel, double* E, hipStream_t st) {
    IB_CHECK(m && b && rel && E, IB_EINVAL, "mg_energy: null argument");
    IB_CHECK(m->coeffs_ready, IB_EINVAL, "mg_energy: no coefficients yet");
    if (!x) {
        *rel = 1.0;
        *E = 0.0;
        return IB_OK;
    }
    Level& L = m->lv[0];
    const long N = L.d.cells();
    const int nb = red_blocks(N);
    const double inv_h2 = 1.0 / (L.d.h * L.d.h);
    double* pr = m->red;
    double* pb = m->red + kRed;
    double* pe = m->red + 2 * kRed;
    const CoefArrays<double> co{L.f64.beta[0], L.f64.beta[1], L.d.dim == 3 ? L.f64.beta[2] : L.f64.beta[1]};
    if (L.rho)
        hipLaunchKernelGGL((k_energy<3, CoefRho>), dim3(nb), dim3(kBlock), 0, st, x, b, CoefRho{L.rho}, L.d,
                           inv_h2, pr, pb, pe);
    else if (L.d.dim == 2)
        hipLaunchKernelGGL((k_energy<2, CoefArrays<double>>), dim3(nb), dim3(kBlock), 0, st, x, b, co, L.d,
                           inv_h2, pr, pb, pe);
    else
        hipLaunchKernelGGL((k_energy<3, CoefArrays<double>>), dim3(nb), dim3(kBlock), 0, st, x, b, co, L.d,
                           inv_h2, pr, pb, pe);
    double* fin = m->red + 3 * kRed + 4;
    IB_TRY(device_sum(pr, nb, fin, st));
    IB_TRY(device_sum(pb, nb, fin + 1, st));
    IB_TRY(device_sum(pe, nb, fin + 2, st));
    IB_HIP(hipMemcpyAsync(m->host + 4, fin, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
    IB_HIP(hipStreamSynchronize(st));
    prof_drain();
    const double bn = std::sqrt(m->host[5]);
    *rel = bn > 0.0 ? std::sqrt(m->host[4]) / bn : 0.0;
    *E = m->host[6];
    IB_HIP(hipGetLastError());
    return IB_OK;
}

extern "C" int mg_update_coeffs(mg_handle* m, const double* const beta[3], void* stream) {
    IB_CHECK(m && beta, IB_EINVAL, "mg_update_coeffs: null argument");
    for (int e = 0; e < m->g.dim; ++e)
        IB_CHECK(beta[e], IB_EINVAL, "mg_update_coeffs: null coefficient array");
    return update_hierarchy(m, beta, nullptr, (hipStream_t)stream);
}

extern "C" int mg_update_density(mg_handle* m, const double* rho, void* stream) {
    IB_CHECK(m && rho, IB_EINVAL, "mg_update_density: null argument");
    hipStream_t st = (hipStream_t)stream;
    if (density_direct(m)) return update_hierarchy(m, nullptr, rho, st);
    // other grids: form the finest face arrays once, into storage of the handle
    Level& L0 = m->lv[0];
    long N = L0.d.cells();
    int dim = m->g.dim;
    for (int e = 0; e < dim; ++e)
        if (!m->beta0[e] && hipMalloc(&m->beta0[e], N * sizeof(double)) != hipSuccess)
            return fail(IB_ENOMEM, "mg_update_density: out of device memory");
    if (dim == 2)
        hipLaunchKernelGGL((k_beta_from_rho<2, double>), dim3(grid_for(N)), dim3(kBlock), 0, st,
                           CoefRho{rho}, L0.d, m->beta0[0], m->beta0[1], m->beta0[1]);
    else
        hipLaunchKernelGGL((k_beta_from_rho<3, double>), dim3(grid_for(N)), dim3(kBlock), 0, st,
                           CoefRho{rho}, L0.d, m->beta0[0], m->beta0[1], m->beta0[2]);
    const double* b[3] = {m->beta0[0], m->beta0[1], m->beta0[2]};
    return update_hierarchy(m, b, nullptr, st);
}

extern "C" int mg_residual_norm(mg_handle* m, const double* b, const double* p, double* rel,
                                void* stream) {
    IB_CHECK(m && b && p && rel, IB_EINVAL, "mg_residual_norm: null argument");
    IB_CHECK(m->coeffs_ready, IB_EINVAL, "mg_residual_norm: no coefficients yet (mg_update_coeffs or mg_update_density)");
    Level& L0 = m->lv[0];
    double* sp = L0.f64.p;
    double* sb = L0.f64.b;
    L0.f64.p = const_cast<double*>(p);
    L0.f64.b = const_cast<double*>(b);
    int rc = fp64_norms(m, true, (hipStream_t)stream);
    L0.f64.p = sp;
    L0.f64.b = sb;
    IB_TRY(rc);
    double bn = std::sqrt(m->host[1]);
    *rel = bn > 0.0 ? std::sqrt(m->host[0]) / bn : 0.0;
    return IB_OK;
}

// flexible CG preconditioned by one V-cycle (float64, or a float32 V-cycle
// under MG_MIXED); same stopping logic and residual-check skipping as the
// plain cycles, on the recursive residual
static int solve_krylov(mg_handle* m, const double* b, double* x, double rtol, int max_it,
                        int fixed, mg_stats* S, hipStream_t st, bool zero) {
    Level& L0 = m->lv[0];
    const long N = L0.d.cells();
    const int nb = red_blocks(N);
    const int dim = L0.d.dim;
    const double inv_h2 = 1.0 / (L0.d.h * L0.d.h);
    const bool mixed = m->o.precision == MG_MIXED;
    double* pa = m->red;
    double* pb = m->red + kRed;
    const CoefArrays<double> co{L0.f64.beta[0], L0.f64.beta[1],
                                dim == 3 ? L0.f64.beta[2] : L0.f64.beta[1]};
    const dim3 g1(grid_for(N)), gr(nb), blk(kBlock);
    // r = b - A x into m->kr with the sums of r^2 and b^2 in the device scalars
    auto residual = [&](bool from_zero) {
        int parts = nb;
        ProfScope ps(IB_PROF_RESID, st, true);
        if (from_zero)
            hipLaunchKernelGGL(k_residual_zero, gr, blk, 0, st, b, (int)N, m->kr, pa, pb);
        else if (tiled_rho(L0))
            parts = launch_residual_rho<double>(L0, x, b, m->kr, pa, pb, st);
        else if (L0.rho)
            hipLaunchKernelGGL((k_residual_vec<3, CoefRho>), gr, blk, 0, st, x, b, CoefRho{L0.rho}, L0.d,
                               inv_h2, m->kr, pa, pb);
        else if (dim == 2)
            hipLaunchKernelGGL((k_residual_vec<2, CoefArrays<double>>), gr, blk, 0, st, x, b, co, L0.d,
                               inv_h2, m->kr, pa, pb);
        else
            hipLaunchKernelGGL((k_residual_vec<3, CoefArrays<double>>), gr, blk, 0, st, x, b, co, L0.d,
                               inv_h2, m->kr, pa, pb);
        return device_sum2(pa, pb, parts, m->ks + KS_RR, m->ks + KS_BB, st);
    };
    IB_TRY(residual(zero));
    IB_HIP(hipMemcpyAsync(m->host, m->ks + KS_RR, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    IB_HIP(hipStreamSynchronize(st));
    prof_drain();
    const double bnorm = std::sqrt(m->host[1]);
    if (!(bnorm > 0.0)) {
        hipLaunchKernelGGL((k_fill<double>), g1, blk, 0, st, x, N, 0.0);
        S->rel_res0 = S->rel_res = 0.0;
        IB_HIP(hipGetLastError());
        return bnorm == 0.0 ? IB_OK : fail(IB_ENAN, "mg_solve: right side is not finite");
    }
    double rel = std::sqrt(m->host[0]) / bnorm;
    S->rel_res0 = S->rel_res = rel;
    // z = V(r) from zero; fl32(r) is left by the r update of the previous
    // iteration unless r was formed anew (the first iteration, a true residual)
    bool r32_ready = false;
    auto precond = [&]() {
        if (mixed) {
            if (!r32_ready) hipLaunchKernelGGL(k_cast_f32, g1, blk, 0, st, m->kr, L0.f32.b, N);
            r32_ready = false;
            vcycle<float>(m, 0, st, true);
        } else {
            L0.f64.b = m->kr;
            L0.f64.p = m->kz;
            vcycle<double>(m, 0, st, true);
        }
    };
    // the preconditioner points the finest level at (r, z); the mean
    // removal works on the level's p, which must be the solution again
    auto restore = [&]() {
        L0.f64.p = x;
        L0.f64.b = const_cast<double*>(b);
    };
    auto dots = [&](const double* q, int rz_slot) {
        if (mixed)
            hipLaunchKernelGGL((k_pcg_dots<float>), gr, blk, 0, st, m->kr, q, L0.f32.p, N, pa, pb);
        else
            hipLaunchKernelGGL((k_pcg_dots<double>), gr, blk, 0, st, m->kr, q, m->kz, N, pa, pb);
        if (q) return device_sum2(pa, pb, nb, m->ks + rz_slot, m->ks + KS_QZ, st);
        return device_sum(pa, nb, m->ks + rz_slot, st);
    };
    auto direction = [&](int rz_old_slot, int first) {
        if (mixed)
            hipLaunchKernelGGL((k_pcg_dir<float>), g1, blk, 0, st, m->kd, L0.f32.p, N, m->ks,
                               rz_old_slot, first);
        else
            hipLaunchKernelGGL((k_pcg_dir<double>), g1, blk, 0, st, m->kd, m->kz, N, m->ks,
                               rz_old_slot, first);
    };
    // the fused tiled update on the density path (64 x 8 tiles, the sweep's z-range)
    const bool fused = L0.rho != nullptr && L0.d.nx % CG_TX == 0 && L0.d.ny % CG_TY == 0 &&
                       L0.rtz > 0 && L0.rtz % 2 == 0;
    const int cg_tx = L0.d.nx / CG_TX, cg_ty = L0.d.ny / CG_TY;
    const int cg_tz = fused ? L0.d.nz / L0.rtz : 0;
    const int cg_wgs = cg_tx * cg_ty * cg_tz;
    IB_CHECK(!fused || cg_wgs <= kRed, IB_EINVAL, "mg_solve: too many workgroups for the partial sums");
    // the inner products of z = V(r) come from the last post-smoothing sweep
    // of the finest level (sweep_wgs partial sums of each; the float32 sweep
    // of the mixed cycle takes them against the float64 r)
    const bool fold = fused && L0.fused && m->o.nu2 >= 1 && (!mixed || L0.rho32 != nullptr);
    const int sweep_wgs = fold ? (L0.d.nx / kRTX) * (L0.d.ny / kRTY) * (L0.d.nz / L0.rtz) : 0;
    IB_CHECK(sweep_wgs <= kRed, IB_EINVAL, "mg_solve: too many sweep workgroups for the partial sums");
    int it = 0, slot = KS_RZ0;
    int skip = 0, last_check = 0, checks = 0;
    double rel_check = rel;
    // on the tiled path x += alpha d rides on the next direction pass; x lags
    // by that update (pending) until it is made before x is read
    bool pending = false;
    auto flush = [&]() {
        if (pending) hipLaunchKernelGGL(k_pcg_x, g1, blk, 0, st, x, m->kd, N, m->ks, slot);
        pending = false;
    };
    while (true) {
        if (!std::isfinite(rel)) return fail(IB_ENAN, "mg_solve: residual is not finite");
        if (fixed > 0 ? it >= fixed : rel <= rtol) break;
        if (fixed == 0 && it >= max_it) {
            S->cycles = it;
            flush();
            restore();
            IB_TRY(remove_mean(m, false, st));
            return fail(IB_ENOTCONV, "mg_solve: no convergence within max_cycles");
        }
        const bool check = fixed > 0 || skip == 0 || it + 1 >= max_it;
        if (fold) {
            L0.dots_on = true;
            L0.dots_q = it == 0 ? nullptr : m->kq;
            L0.dots_part = pa;
            L0.dots_r = m->kr;
        }
        precond();
        L0.dots_on = false;
        const int rz_old = slot;
        if (fold) {
            const int next = it == 0 ? slot : (slot == KS_RZ0 ? KS_RZ1 : KS_RZ0);
            if (it > 0)
                IB_TRY(device_sum2(pa, pa + sweep_wgs, sweep_wgs, m->ks + next, m->ks + KS_QZ, st));
            else
                IB_TRY(device_sum(pa, sweep_wgs, m->ks + next, st));
            slot = next;
        } else if (it == 0) {
            IB_TRY(dots(nullptr, slot));
        } else {
            const int next = slot == KS_RZ0 ? KS_RZ1 : KS_RZ0;
            IB_TRY(dots(m->kq, next));
            slot = next;
        }
        if (fused) {
            // d = z + beta d, q = A d and (d, q) in one tiled pass
            if (mixed && it == 0)
                hipLaunchKernelGGL((k_cg_dir_apply_rho<float, true>), dim3(cg_wgs), dim3(CG_NT), 0, st,
                                   L0.f32.p, m->kd, m->kd2, L0.rho, m->kq, L0.d, inv_h2, m->ks, rz_old,
                                   L0.rtz, cg_tx, cg_ty, cg_tz, pa);
            else if (mixed && pending)
                hipLaunchKernelGGL((k_cg_dir_apply_rho<float, false, true>), dim3(cg_wgs), dim3(CG_NT), 0, st,
                                   L0.f32.p, m->kd, m->kd2, L0.rho, m->kq, L0.d, inv_h2, m->ks, rz_old,
                                   L0.rtz, cg_tx, cg_ty, cg_tz, pa, x);
            else if (mixed)
                hipLaunchKernelGGL((k_cg_dir_apply_rho<float, false>), dim3(cg_wgs), dim3(CG_NT), 0, st,
                                   L0.f32.p, m->kd, m->kd2, L0.rho, m->kq, L0.d, inv_h2, m->ks, rz_old,
                                   L0.rtz, cg_tx, cg_ty, cg_tz, pa);
            else if (it == 0)
                hipLaunchKernelGGL((k_cg_dir_apply_rho<double, true>), dim3(cg_wgs), dim3(CG_NT), 0, st,
                                   m->kz, m->kd, m->kd2, L0.rho, m->kq, L0.d, inv_h2, m->ks, rz_old,
                                   L0.rtz, cg_tx, cg_ty, cg_tz, pa);
            else if (pending)
                hipLaunchKernelGGL((k_cg_dir_apply_rho<double, false, true>), dim3(cg_wgs), dim3(CG_NT), 0,
                                   st, m->kz, m->kd, m->kd2, L0.rho, m->kq, L0.d, inv_h2, m->ks, rz_old,
                                   L0.rtz, cg_tx, cg_ty, cg_tz, pa, x);
            else
                hipLaunchKernelGGL((k_cg_dir_apply_rho<double, false>), dim3(cg_wgs), dim3(CG_NT), 0, st,
                                   m->kz, m->kd, m->kd2, L0.rho, m->kq, L0.d, inv_h2, m->ks, rz_old,
                                   L0.rtz, cg_tx, cg_ty, cg_tz, pa);
            std::swap(m->kd, m->kd2);
            IB_TRY(device_sum(pa, cg_wgs, m->ks + KS_DQ, st));
        } else {
            direction(rz_old, it == 0 ? 1 : 0);
            if (L0.rho)
                hipLaunchKernelGGL((k_apply_dot<3, CoefRho>), gr, blk, 0, st, m->kd, CoefRho{L0.rho},
                                   L0.d, inv_h2, m->kq, pa);
            else if (dim == 2)
                hipLaunchKernelGGL((k_apply_dot<2, CoefArrays<double>>), gr, blk, 0, st, m->kd, co, L0.d,
                                   inv_h2, m->kq, pa);
            else
                hipLaunchKernelGGL((k_apply_dot<3, CoefArrays<double>>), gr, blk, 0, st, m->kd, co, L0.d,
                                   inv_h2, m->kq, pa);
            IB_TRY(device_sum(pa, nb, m->ks + KS_DQ, st));
        }
        // the pending update was made by the direction pass above
        pending = false;
        if (fused) {
            hipLaunchKernelGGL(k_pcg_r, gr, blk, 0, st, m->kr, m->kq, N, m->ks, slot, pa,
                               mixed ? L0.f32.b : nullptr);
            pending = true;
        } else {
            hipLaunchKernelGGL(k_pcg_xr, gr, blk, 0, st, x, m->kr, m->kd, m->kq, N, m->ks, slot, pa,
                               mixed ? L0.f32.b : nullptr);
        }
        r32_ready = mixed;
        // (r, r) is read only by the host's checks
        if (check) IB_TRY(device_sum(pa, nb, m->ks + KS_RR, st));
        ++it;
        S->cycles = it;
        if (!check) {
            --skip;
            if (it <= 128) S->res_hist[it - 1] = -1.0;
            continue;
        }
        IB_HIP(hipMemcpyAsync(m->host, m->ks + KS_RR, sizeof(double), hipMemcpyDeviceToHost, st));
        IB_HIP(hipStreamSynchronize(st));
        prof_drain();
        rel = std::sqrt(m->host[0]) / bnorm;
        if (fixed == 0 && rel <= rtol) {
            // the recursive residual drifts from b - A x by rounding: the stop
            // is decided on the true residual, which replaces r (and the
            // recursion goes on from it) when it has not reached rtol yet
            flush();
            IB_TRY(residual(false));
            r32_ready = false;
            IB_HIP(hipMemcpyAsync(m->host, m->ks + KS_RR, sizeof(double), hipMemcpyDeviceToHost, st));
            IB_HIP(hipStreamSynchronize(st));
            prof_drain();
            rel = std::sqrt(m->host[0]) / bnorm;
            ++S->true_checks;
        }
        if (it <= 128) S->res_hist[it - 1] = rel;
        S->rel_res = rel;
        ++checks;
        if (fixed == 0 && checks >= 3 && rel > rtol && rel < rel_check) {
            double rho = std::pow(rel / rel_check, 1.0 / (double)(it - last_check));
            if (rho < 0.9) {
                int need = (int)std::ceil(std::log(rtol / rel) / std::log(rho));
                skip = std::min(std::max(0, need - 2), kMaxSkip);
            }
        }
        rel_check = rel;
        last_check = it;
    }
    flush();
    restore();
    if (it > 0) IB_TRY(remove_mean(m, false, st));
    IB_HIP(hipGetLastError());
    return IB_OK;
}

extern "C" int mg_solve(mg_handle* m, const double* b, double* p, double rtol, int max_cycles,
                        int fixed_cycles, mg_stats* stats, void* stream) {
    IB_CHECK(m && b && p, IB_EINVAL, "mg_solve: null argument");
    const bool zero = m->x_zero;   // a hint holds for this call only
    m->x_zero = false;
    IB_CHECK(m->coeffs_ready, IB_EINVAL, "mg_solve: no coefficients yet (mg_update_coeffs or mg_update_density)");
    IB_CHECK(max_cycles >= 0 && fixed_cycles >= 0, IB_EINVAL, "mg_solve: cycle counts");
    hipStream_t st = (hipStream_t)stream;
    Level& L0 = m->lv[0];
    L0.f64.p = p;
    L0.f64.b = const_cast<double*>(b);
    long N = L0.d.cells();
    bool mixed = m->o.precision == MG_MIXED;
    mg_stats loc;
    mg_stats* S = stats ? stats : &loc;
    S->cycles = 0;
    S->true_checks = 0;
    if (m->o.krylov) return solve_krylov(m, b, p, rtol, max_cycles, fixed_cycles, S, st, zero);
    if (mixed) IB_TRY(mixed_defect(m, true, st));
    else IB_TRY(fp64_norms(m, true, st, zero));
    double bnorm = std::sqrt(m->host[1]);
    if (!(bnorm > 0.0)) {
        hipLaunchKernelGGL((k_fill<double>), dim3(grid_for(N)), dim3(kBlock), 0, st, p, N, 0.0);
        S->rel_res0 = S->rel_res = 0.0;
        IB_HIP(hipGetLastError());
        return bnorm == 0.0 ? IB_OK : fail(IB_ENAN, "mg_solve: right side is not finite");
    }
    double rel = std::sqrt(m->host[0]) / bnorm;
    S->rel_res0 = rel;
    S->rel_res = rel;
    int cycles = 0;
    // residual checks: after two measured contraction factors the solver
    // predicts how many cycles remain and skips the norm (and its host sync)
    // until two cycles before the predicted end; it always checks before
    // stopping, so the stopping test is unchanged
    int skip = 0, last_check = 0, checks = 0;
    double rel_check = rel;
    while (true) {
        if (!std::isfinite(rel)) return fail(IB_ENAN, "mg_solve: residual is not finite");
        if (fixed_cycles > 0 ? cycles >= fixed_cycles : rel <= rtol) break;
        if (fixed_cycles == 0 && cycles >= max_cycles) {
            S->cycles = cycles;
            IB_TRY(remove_mean(m, false, st));
            return fail(IB_ENOTCONV, "mg_solve: no convergence within max_cycles");
        }
        const bool check = fixed_cycles > 0 || skip == 0 || cycles + 1 >= max_cycles;
        // A annihilates constants and every step of a cycle commutes with adding
        // one, so the mean is removed once, after the last cycle
        if (mixed) {
            vcycle<float>(m, 0, st, true);
            int nb = red_blocks(N);
            hipLaunchKernelGGL(k_correct_f32, dim3(nb), dim3(kBlock), 0, st, p, L0.f32.p, N,
                               m->red + 2 * kRed);
            IB_TRY(mixed_defect(m, false, st, check));
        } else {
            vcycle<double>(m, 0, st, false);
            if (check) IB_TRY(fp64_norms(m, false, st));
        }
        ++cycles;
        S->cycles = cycles;
        if (!check) {
            --skip;
            if (cycles <= 128) S->res_hist[cycles - 1] = -1.0;
            continue;
        }
        rel = std::sqrt(m->host[0]) / bnorm;
        if (cycles <= 128) S->res_hist[cycles - 1] = rel;
        S->rel_res = rel;
        ++checks;
        if (fixed_cycles == 0 && checks >= 3 && rel > rtol && rel < rel_check) {
            double rho = std::pow(rel / rel_check, 1.0 / (double)(cycles - last_check));
            if (rho < 0.9) {
                int need = (int)std::ceil(std::log(rtol / rel) / std::log(rho));
                skip = std::min(std::max(0, need - 2), kMaxSkip);
            }
        }
        rel_check = rel;
        last_check = cycles;
    }
    if (cycles > 0) IB_TRY(remove_mean(m, false, st));
    IB_HIP(hipGetLastError());
    return IB_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free residual norm: the partial sums of mg_residual_norm live in
// a file-scope device array instead of the handle's workspace. Each GPU the
// library runs on holds its own copy until the process ends; the host finds
// its address once per device (hipGetSymbolAddress) and passes that address
// to the kernels. Calls on one GPU share the array: overlapping calls race.
namespace ib {

constexpr int kScratchDoubles = 2 * kRed + 8;   // r^2 and b^2 partials, the two sums
constexpr long kNoallocMaxCells = (1L << 31) - 1;  // the residual kernels index cells with int
constexpr int kScratchDevices = 64;
static __device__ __align__(256) double scratch[kScratchDoubles];

static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kScratchDevices] = {};

// the current device's copy of `scratch` (looked up on its first use)
static int scratch_on_device(double** out) {
    int dev = -1;
    IB_HIP(hipGetDevice(&dev));
    IB_CHECK(dev >= 0 && dev < kScratchDevices, IB_EINVAL, "mg_residual_norm_noalloc: device ordinal");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(IB_EHIP, std::string("mg_residual_norm_noalloc: hipGetSymbolAddress failed: ") +
                                     hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<double*>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return IB_OK;
}

__global__ void k_rel_from_sums(const double* __restrict__ sums, double* __restrict__ rel) {
    const double bb = sums[1];
    *rel = bb > 0.0 ? sqrt(sums[0]) / sqrt(bb) : 0.0;
}

}  // namespace ib

extern "C" int mg_residual_norm_noalloc(const ib_grid* g, const double* rho, const double* b,
                                        const double* p, double* rel, void* stream) {
    IB_CHECK(g && rho && b && p && rel, IB_EINVAL, "mg_residual_norm_noalloc: null argument");
    IB_CHECK(g->dim == 2 || g->dim == 3, IB_EINVAL, "mg_residual_norm_noalloc: dim must be 2 or 3");
    IB_CHECK(g->h > 0.0, IB_EINVAL, "mg_residual_norm_noalloc: h must be positive");
    long cells = 1;
    for (int e = 0; e < g->dim; ++e) {
        IB_CHECK(g->n[e] >= 2, IB_EINVAL, "mg_residual_norm_noalloc: cells per axis must be >= 2");
        cells *= g->n[e];
        IB_CHECK(cells <= kNoallocMaxCells, IB_EINVAL,
                 "mg_residual_norm_noalloc: grid larger than the maximum of 2^31 - 1 cells");
    }
    hipStream_t st = (hipStream_t)stream;
    double* sc = nullptr;
    IB_TRY(scratch_on_device(&sc));
    Level L;
    L.d = make_dims(*g);
    L.rho = rho;
    L.rtz = density_rtz(L.d);
    double* pr = sc;
    double* pb = sc + kRed;
    int parts = red_blocks(cells);
    if (tiled_rho(L)) {
        parts = launch_residual_rho<double>(L, p, b, nullptr, pr, pb, st);
    } else {
        const double inv_h2 = 1.0 / (L.d.h * L.d.h);
        if (L.d.dim == 2)
            hipLaunchKernelGGL((k_resid_norm<2, CoefRho>), dim3(parts), dim3(kBlock), 0, st, p, b,
                               CoefRho{rho}, L.d, inv_h2, pr, pb);
        else
            hipLaunchKernelGGL((k_resid_norm<3, CoefRho>), dim3(parts), dim3(kBlock), 0, st, p, b,
                               CoefRho{rho}, L.d, inv_h2, pr, pb);
    }
    IB_TRY(device_sum2(pr, pb, parts, sc + 2 * kRed, sc + 2 * kRed + 1, st));
    hipLaunchKernelGGL(k_rel_from_sums, dim3(1), dim3(1), 0, st, sc + 2 * kRed, rel);
    IB_HIP(hipGetLastError());
    return IB_OK;
}
