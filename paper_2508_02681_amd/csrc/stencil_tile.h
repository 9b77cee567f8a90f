// LDS-tiled matrix-free operator apply (Sec. 3.1: the stiffness matrix of the
// periodic linear FE discretization, applied without assembly).
//
// A workgroup of 256 threads owns a TX x TY x TZ tile of nodes (TY = 256 /
// TZ).  It stages the vector on the tile plus a one-node halo and the
// conductivities of the (TX+1) x (TY+1) x (TZ+1) voxels touching the tile in
// LDS (periodic wrap on each coordinate), then each thread walks one (y, z)
// column of the tile along x, keeping the 3 x 3 neighbourhood of three node
// planes and the 2 x 2 voxel conductivities of two voxel planes in
// registers: 9 + 4 LDS reads per node.
//
// Node-centred form of the assembled operator: node i touches the 8 voxels
// i + sigma, sigma in {-1,0}^3, and
//   (A u)_i = sum_{delta in {-1,0,1}^3} w[m(delta)] * ksum(i, delta) * u_{i+delta},
// m(delta) flagging the axes where delta != 0, ksum adding the voxels that
// contain both nodes (axis b: delta_b = -1 -> sigma_b = -1, +1 -> 0,
// 0 -> both); w[m] is the brick element's corner coupling.
//
// CG variant (fused into Algorithm 1's direction update and matvec): the
// staged vector is d = s + beta d_old, the tile's own d is written to d_new,
// p = A d, and per-workgroup partials of d.p are written.
#pragma once

#include "unocg_internal.h"
#include "reduce.h"
#include "cg_ctl.h"

namespace unocg {

struct TileGeom {
    int tiles_y, tiles_z;
};

__device__ __forceinline__ int wrap_mod(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

// periodic wrap of v in [-n, 2n) without a division
__device__ __forceinline__ int wrap_near(int v, int n)
{
    v = v < 0 ? v + n : v;
    return v >= n ? v - n : v;
}

template <typename T>
__device__ __forceinline__ T stencil_node(const GridDev& g, const T dm[3][3], const T d0[3][3], const T dp[3][3],
                                          const T km[2][2], const T kp[2][2])
{
    // conductivity sums over compatible voxels, per offset (a, b, c) in {-1,0,1}^3
    T S[3][2][2];  // along x: [0] sigma0=-1, [1] both, [2] sigma0=0
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            S[0][b][c] = km[b][c];
            S[1][b][c] = km[b][c] + kp[b][c];
            S[2][b][c] = kp[b][c];
        }
    T acc = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        T K3[3][3];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            T lo = (b == 2) ? (T)0 : S[a][0][0];
            T hi = (b == 0) ? (T)0 : S[a][1][0];
            T lo1 = (b == 2) ? (T)0 : S[a][0][1];
            T hi1 = (b == 0) ? (T)0 : S[a][1][1];
            T c0 = lo + hi;     // sigma2 = -1 column
            T c1 = lo1 + hi1;   // sigma2 = 0 column
            K3[b][0] = c0;
            K3[b][1] = c0 + c1;
            K3[b][2] = c1;
        }
        const T(*D)[3] = (a == 0) ? dm : (a == 1 ? d0 : dp);
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int m = ((a != 1) << 2) | ((b != 1) << 1) | (c != 1);
                acc += (T)g.w[m] * K3[b][c] * D[b][c];
            }
    }
    return acc;
}

// Mean removal of the search direction (FP32 operator mode): partial sums of
// s (count np_s, same producer as r.s) and of the previous d_new (count =
// this grid), and where to write the partial sums of the new d.
struct MeanFree {
    const double* part_s;
    const double* part_dold;
    double* part_dnew;
};

// NEAR: every tile dimension fits in the grid, so staging coordinates lie in
// [-n, 2n) and wrap without a division (decided on the host per launch).
template <typename T, int TX, int TZ, bool CG, bool HEAD, bool NEAR>
__global__ void __launch_bounds__(256) k_stencil_tile(GridDev g, TileGeom tg, const T* __restrict__ kappa,
                                                      const T* __restrict__ s, const T* __restrict__ dold,
                                                      T* __restrict__ dnew, T* __restrict__ p,
                                                      double* __restrict__ part_dp, CgIter it,
                                                      const double* __restrict__ part_rs, int np_rs, double* gam,
                                                      MeanFree mf)
{
    // In FP32 the direction is kept mean-free: A 1 = 0 and sum(A d) = 0, so
    // shifting d by a constant leaves p, d.p, alpha, r and beta unchanged and
    // moves u by a constant (removed at the end); it avoids the cancellation
    // a large constant component causes in the FP32 stencil sums.
    constexpr bool MF = CG && sizeof(T) == 4;
    constexpr int TY = 256 / TZ;
    constexpr int DX = TX + 2, DY = TY + 2, DZ = TZ + 2;
    constexpr int KX = TX + 1, KY = TY + 1, KZ = TZ + 1;
    __shared__ T Dl[DX * DY * DZ];
    __shared__ T Kl[KX * KY * KZ];
    __shared__ double slots[4];

    int b = blockIdx.x;
    const int tzi = b % tg.tiles_z;
    b /= tg.tiles_z;
    const int tyi = b % tg.tiles_y;
    const int txi = b / tg.tiles_y;
    const int x0 = txi * TX, y0 = tyi * TY, z0 = tzi * TZ;
    if (CG && blockIdx.y > 0) {  // right-hand side blockIdx.y of a batch
        const int64_t vo = (int64_t)blockIdx.y * it.vs, po = (int64_t)blockIdx.y * it.ps;
        kappa += (int64_t)blockIdx.y * it.ks;
        s += vo;
        dold += vo;
        dnew += vo;
        p += vo;
        part_dp += po;
        part_rs += po;
        gam += (int64_t)blockIdx.y * it.hs;
        if (MF) {
            mf.part_s += po;
            mf.part_dold += po;
            mf.part_dnew += po;
        }
        it = rhs_iter(it);
    }

    // every global load is issued before the first decision, so the loop
    // state, the partials, the previous gamma and the staged data overlap
    StateLoad sl;
    double head_share = 0.0, rs_share = 0.0, gprev = 1.0, ssum_share = 0.0, dsum_share = 0.0;
    if (CG) {
        sl = load_state(it.st);
        if (HEAD) head_share = load_share<OpMax>(it.part_rmax, it.np_rmax);
        rs_share = load_share<OpSum>(part_rs, np_rs);
        if (it.k > it.k0) gprev = gam[it.k - 1];
        if (MF) {
            ssum_share = load_share<OpSum>(mf.part_s, np_rs);
            if (it.k > it.k0) dsum_share = load_share<OpSum>(mf.part_dold, gridDim.x);
        }
    }
    constexpr int ND = DX * DY * DZ, NK = KX * KY * KZ;
    constexpr int PD = (ND + 255) / 256, PK = (NK + 255) / 256;
    // staging coordinates lie in [-1, n - 1 + T]; a single conditional wrap
    // covers [-n, 2n) unless the tile is wider than the grid (small grids)
    auto wrapc = [](int v, int n) {
        if constexpr (NEAR) return wrap_near(v, n);
        else return wrap_mod(v, n);
    };
    T sv[PD], dv[PD], kv[PK];
#pragma unroll
    for (int j = 0; j < PD; ++j) {
        const int q = threadIdx.x + 256 * j;
        sv[j] = dv[j] = (T)0;
        if (q < ND) {
            const int zl = q % DZ, t = q / DZ;  // constant divisors
            const int yl = t % DY, xl = t / DY;
            const int x = wrapc(x0 - 1 + xl, g.n0), y = wrapc(y0 - 1 + yl, g.n1), z = wrapc(z0 - 1 + zl, g.n2);
            const int64_t idx = ((int64_t)x * g.n1 + y) * g.n2 + z;
            sv[j] = s[idx];
            if (CG && it.k > it.k0) dv[j] = dold[idx];
        }
    }
#pragma unroll
    for (int j = 0; j < PK; ++j) {
        const int q = threadIdx.x + 256 * j;
        kv[j] = (T)0;
        if (q < NK) {
            const int zl = q % KZ, t = q / KZ;
            const int yl = t % KY, xl = t / KY;
            const int x = wrapc(x0 - 1 + xl, g.n0), y = wrapc(y0 - 1 + yl, g.n1), z = wrapc(z0 - 1 + zl, g.n2);
            kv[j] = kappa[((int64_t)x * g.n1 + y) * g.n2 + z];
        }
    }
    T beta = 0;
    bool first = true;
    if (CG) {
        if (HEAD) {
            if (head_decide(it, sl, head_share, slots)) return;
        } else if (ended(sl, it.k)) {
            return;
        }
        const int k = it.k;
        const double gk = combine_share<OpSum>(rs_share, slots);
        const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
        if (lead) gam[k] = gk;
        if (!(gk > 0.0) || !isfinite(gk)) {
            if (lead) { it.st->status = 1; it.st->fail_iter = k; }
            return;
        }
        first = (k == it.k0);  // d = s on the first pass of a cycle (Algorithm 1: d_0 = 0)
        beta = first ? (T)0 : (T)(gk / gprev);
    }
    T shift = (T)0;
    if (MF) {
        const double ssum = combine_share<OpSum>(ssum_share, slots);
        const double dsum = first ? 0.0 : combine_share<OpSum>(dsum_share, slots);
        shift = (T)((ssum + (double)beta * dsum) / (double)g.n);
    }
#pragma unroll
    for (int j = 0; j < PD; ++j) {
        const int q = threadIdx.x + 256 * j;
        if (q < ND) Dl[q] = ((CG && !first) ? sv[j] + beta * dv[j] : sv[j]) - shift;
    }
#pragma unroll
    for (int j = 0; j < PK; ++j) {
        const int q = threadIdx.x + 256 * j;
        if (q < NK) Kl[q] = kv[j];
    }
    __syncthreads();

    const int tz = threadIdx.x % TZ, ty = threadIdx.x / TZ;
    const int y = y0 + ty, z = z0 + tz;
    const bool yz_ok = (y < g.n1) && (z < g.n2);
    T dm[3][3], d0[3][3], dq[3][3], km[2][2], kp[2][2];
#pragma unroll
    for (int bb = 0; bb < 3; ++bb)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            dm[bb][c] = Dl[(0 * DY + ty + bb) * DZ + tz + c];
            d0[bb][c] = Dl[(1 * DY + ty + bb) * DZ + tz + c];
        }
#pragma unroll
    for (int bb = 0; bb < 2; ++bb)
#pragma unroll
        for (int c = 0; c < 2; ++c) km[bb][c] = Kl[(0 * KY + ty + bb) * KZ + tz + c];
    double dot = 0.0, dsum_own = 0.0;
#pragma unroll
    for (int xi = 0; xi < TX; ++xi) {
#pragma unroll
        for (int bb = 0; bb < 3; ++bb)
#pragma unroll
            for (int c = 0; c < 3; ++c) dq[bb][c] = Dl[((xi + 2) * DY + ty + bb) * DZ + tz + c];
#pragma unroll
        for (int bb = 0; bb < 2; ++bb)
#pragma unroll
            for (int c = 0; c < 2; ++c) kp[bb][c] = Kl[((xi + 1) * KY + ty + bb) * KZ + tz + c];
        const int x = x0 + xi;
        if (yz_ok && x < g.n0) {
            const T acc = stencil_node<T>(g, dm, d0, dq, km, kp);
            const int64_t i = ((int64_t)x * g.n1 + y) * g.n2 + z;
            p[i] = acc;
            if (CG) {
                dnew[i] = d0[1][1];
                dot += (double)d0[1][1] * (double)acc;
                if (MF) dsum_own += (double)d0[1][1];
            }
        }
#pragma unroll
        for (int bb = 0; bb < 3; ++bb)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                dm[bb][c] = d0[bb][c];
                d0[bb][c] = dq[bb][c];
            }
#pragma unroll
        for (int bb = 0; bb < 2; ++bb)
#pragma unroll
            for (int c = 0; c < 2; ++c) km[bb][c] = kp[bb][c];
    }
    if (CG) {
        const double bd = block_reduce<OpSum>(dot, slots);
        if (threadIdx.x == 0) part_dp[blockIdx.x] = bd;
        if (MF) {
            const double bs = block_reduce<OpSum>(dsum_own, slots);
            if (threadIdx.x == 0) mf.part_dnew[blockIdx.x] = bs;
        }
    }
}

// Tile shape for a grid: TZ covers the contiguous axis, TX = 1 for a single
// voxel layer (2D problems), otherwise 4 (2 on small grids, for parallelism).
struct TileChoice {
    int tx, tz;
    TileGeom geom;
    int blocks;
};

inline TileChoice choose_tile(const Grid& g)
{
    // measured on MI355X (FP64 apply): 32-wide z tiles beat 64-wide ones at
    // 64^3 .. 192^3; 4-deep x tiles once there are >= 1024 of them
    TileChoice c;
    c.tz = g.n[2] >= 24 ? 32 : 16;
    const int ty = 256 / c.tz;
    const int tiles_y = (g.n[1] + ty - 1) / ty, tiles_z = (g.n[2] + c.tz - 1) / c.tz;
    if (g.n[0] < 3) c.tx = 1;
    else {
        const int64_t t4 = (int64_t)((g.n[0] + 3) / 4) * tiles_y * tiles_z;
        c.tx = (t4 >= 1024 && g.n[0] >= 4) ? 4 : 2;
    }
    c.geom.tiles_y = tiles_y;
    c.geom.tiles_z = tiles_z;
    c.blocks = ((g.n[0] + c.tx - 1) / c.tx) * tiles_y * tiles_z;
    return c;
}

template <typename T, bool CG, bool HEAD, int TX, bool NEAR>
inline void launch_tile_near(const TileChoice& c, const GridDev& g, const T* kappa, const T* s, const T* dold, T* dnew,
                             T* p, double* part_dp, const CgIter& it, const double* part_rs, int np_rs, double* gam,
                             hipStream_t st, const MeanFree& mf, int nrhs)
{
    const dim3 grid(c.blocks, nrhs);
    const int fam = CG ? UNO_KT_MATVEC : UNO_KT_APPLY;  // timing family
    switch (c.tz) {
        case 64:
            uno_launch(fam, k_stencil_tile<T, TX, 64, CG, HEAD, NEAR>, grid, dim3(256), 0, st, g, c.geom, kappa, s,
                       dold, dnew, p, part_dp, it, part_rs, np_rs, gam, mf);
            break;
        case 32:
            uno_launch(fam, k_stencil_tile<T, TX, 32, CG, HEAD, NEAR>, grid, dim3(256), 0, st, g, c.geom, kappa, s,
                       dold, dnew, p, part_dp, it, part_rs, np_rs, gam, mf);
            break;
        default:
            uno_launch(fam, k_stencil_tile<T, TX, 16, CG, HEAD, NEAR>, grid, dim3(256), 0, st, g, c.geom, kappa, s,
                       dold, dnew, p, part_dp, it, part_rs, np_rs, gam, mf);
            break;
    }
}

// tile dimensions within the grid (single conditional wrap)
inline bool tile_near(const TileChoice& c, const GridDev& g)
{
    return c.tx <= g.n0 && 256 / c.tz <= g.n1 && c.tz <= g.n2;
}

template <typename T, bool CG, bool HEAD, int TX>
inline void launch_tile_tx(const TileChoice& c, const GridDev& g, const T* kappa, const T* s, const T* dold, T* dnew,
                           T* p, double* part_dp, const CgIter& it, const double* part_rs, int np_rs, double* gam,
                           hipStream_t st, const MeanFree& mf, int nrhs)
{
    if (tile_near(c, g))
        launch_tile_near<T, CG, HEAD, TX, true>(c, g, kappa, s, dold, dnew, p, part_dp, it, part_rs, np_rs, gam, st, mf,
                                                nrhs);
    else
        launch_tile_near<T, CG, HEAD, TX, false>(c, g, kappa, s, dold, dnew, p, part_dp, it, part_rs, np_rs, gam, st,
                                                 mf, nrhs);
}

// Launches the tiled operator (nrhs right-hand sides along grid y); returns
// the number of workgroups per right-hand side (= d.p partials).
template <typename T, bool CG, bool HEAD>
inline int launch_tile(const Grid& g, const T* kappa, const T* s, const T* dold, T* dnew, T* p, double* part_dp,
                       const CgIter& it, const double* part_rs, int np_rs, double* gam, hipStream_t st,
                       const MeanFree& mf = MeanFree{nullptr, nullptr, nullptr}, int nrhs = 1)
{
    const TileChoice c = choose_tile(g);
    if (c.tx == 1)
        launch_tile_tx<T, CG, HEAD, 1>(c, g.dev, kappa, s, dold, dnew, p, part_dp, it, part_rs, np_rs, gam, st, mf,
                                       nrhs);
    else if (c.tx == 2)
        launch_tile_tx<T, CG, HEAD, 2>(c, g.dev, kappa, s, dold, dnew, p, part_dp, it, part_rs, np_rs, gam, st, mf,
                                       nrhs);
    else
        launch_tile_tx<T, CG, HEAD, 4>(c, g.dev, kappa, s, dold, dnew, p, part_dp, it, part_rs, np_rs, gam, st, mf,
                                       nrhs);
    return c.blocks;
}

}  // namespace unocg
