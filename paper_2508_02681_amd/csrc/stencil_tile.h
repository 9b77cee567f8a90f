// Matrix-free operator apply (Sec. 3.1: the stiffness matrix of the periodic
// linear FE discretization, applied without assembly).
//
// A workgroup of 256 threads owns a TY x TZ footprint of nodes (TY = RY 256
// / TZ: each thread takes RY consecutive rows) and marches along x over xb
// node planes.  Planes of the vector (with a one-node halo in y and z) and
// of the conductivities of the voxels touching them stream through a small
// ring of LDS planes (periodic wrap on each coordinate); each thread keeps
// the (RY + 2) x 3 neighbourhood of its rows in three node planes and the
// (RY + 1) x 2 voxel conductivities of two voxel planes in registers and
// rolls them along x: (3 (RY + 2) + 2 (RY + 1)) / RY LDS reads per node.
//
// Node-centred form of the assembled operator: node i touches the 8 voxels
// i + sigma, sigma in {-1,0}^3, and
//   (A u)_i = sum_{delta in {-1,0,1}^3} w[m(delta)] * ksum(i, delta) * u_{i+delta},
// m(delta) flagging the axes where delta != 0, ksum adding the voxels that
// contain both nodes (axis b: delta_b = -1 -> sigma_b = -1, +1 -> 0,
// 0 -> both); w[m] is the brick element's corner coupling.
//
// CG variant (fused into Algorithm 1's direction update and matvec): the
// staged vector is d = s + beta d_old, the workgroup's own d is written to
// d_new, p = A d, and per-workgroup partials of d.p are written.
#pragma once

#include "unocg_internal.h"
#include "reduce.h"
#include "cg_ctl.h"

namespace unocg {

// A value the whole wavefront holds alike, moved to scalar registers.
__device__ __forceinline__ double wave_uniform(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffLL));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float wave_uniform(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

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

// The kernel: a workgroup owns a TY x TZ footprint (TY = RY 256 / TZ) and xb
// consecutive node planes along x, and sweeps the input planes x0 - 1 ..
// x0 + xb.  Input node plane xi (with a one-node halo in y and z) and voxel
// plane xi stream through two LDS buffers, the loads of planes xi + 1 and
// xi + 2 in flight while plane xi is used (a workgroup's sweep is a chain of
// dependent steps, and a few workgroups per CU hold the chip's memory
// parallelism), one barrier per plane.  Each thread keeps
// three partial sums: input plane xi contributes to the outputs at xi + 1
// (started), xi and xi - 1 (complete after it), so only the 3 x 3
// neighbourhood of one plane and the 2 x 2 conductivities of two voxel
// planes are live per row (rows of one thread share the staged rows
// between them).  Through voxel face
// (sy, sz) in the y-z plane, plane xi contributes
//   sum over the face's 4 nodes (b, c) of w[m] d[b][c] =: E[sy][sz],
// with the weights of the neighbour-plane class (output xi -/+ 1) or the
// same-plane class (output xi), times the conductivity of the voxel
// (voxel plane xi - 1 for output xi - 1, xi for xi + 1, both for xi).
// Per node plane the halo costs (TY+2)(TZ+2)/(TY TZ) of the plane; along x
// only the two end planes of the sweep are extra.  Right-hand side
// blockIdx.y of a batch reads its vectors at + blockIdx.y n (conductivities
// at + blockIdx.y ks).
//
// In FP32 the direction is kept mean-free: A 1 = 0 and sum(A d) = 0, so
// shifting d by a constant leaves p, d.p, alpha, r and beta unchanged and
// moves u by a constant (removed at the end); it avoids the cancellation a
// large constant component causes in the FP32 stencil sums.
//
// NEAR: the footprint fits in the grid, so staging coordinates lie in
// [-n, 2n) and wrap without a division (decided on the host per launch).
struct MarchGeom {
    int tiles_y, tiles_z, xb, tiles_x;
};

template <typename T, int TZ, int RY, bool CG, bool HEAD, bool NEAR>
__global__ void __launch_bounds__(256) k_stencil_march(GridDev g, MarchGeom mg, const T* __restrict__ kappa,
                                                       const T* __restrict__ s, const T* __restrict__ dold,
                                                       T* __restrict__ dnew, T* __restrict__ p,
                                                       double* __restrict__ part_dp, CgIter it,
                                                       const double* __restrict__ part_rs, int np_rs, double* gam,
                                                       MeanFree mf)
{
    resolve_pass(it);
    constexpr bool MF = CG && sizeof(T) == 4;
    constexpr int TY = 256 / TZ * RY;  // footprint rows: RY rows per thread
    constexpr int DY = TY + 2, DZ = TZ + 2, KY = TY + 1, KZ = TZ + 1;
    constexpr int ND = DY * DZ, NK = KY * KZ;
    constexpr int PD = (ND + 255) / 256, PK = (NK + 255) / 256;
    __shared__ T Dr[2][ND];
    __shared__ T Kr[2][NK];
    __shared__ double slots[4];

    int b = xcd_tile(blockIdx.x, gridDim.x);
    const int tzi = b % mg.tiles_z;
    b /= mg.tiles_z;
    const int tyi = b % mg.tiles_y;
    const int txi = b / mg.tiles_y;
    const int x0 = txi * mg.xb, y0 = tyi * TY, z0 = tzi * TZ;
    const int xe = min(g.n0, x0 + mg.xb);
    if (!CG && blockIdx.y > 0) {  // plain applies of a batch: u, y at + it.vs, kappa at + it.ks
        kappa += (int64_t)blockIdx.y * it.ks;
        s += (int64_t)blockIdx.y * it.vs;
        p += (int64_t)blockIdx.y * it.vs;
    }
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
    auto wrapc = [](int v, int n) {
        if constexpr (NEAR) return wrap_near(v, n);
        else return wrap_mod(v, n);
    };
    // this thread's staging offsets within a plane (y, z wrapped once);
    // slots past the staged plane read its first node and are not stored,
    // so that every load is unconditional (no branch between the loads of
    // a plane and their use, which lets the next plane's loads stay in
    // flight across the wait for this one's)
    int doff[PD], koff[PK];
#pragma unroll
    for (int j = 0; j < PD; ++j) {
        const int q = threadIdx.x + 256 * j;
        doff[j] = 0;
        if (q < ND) {
            const int zl = q % DZ, yl = q / DZ;
            doff[j] = wrapc(y0 - 1 + yl, g.n1) * g.n2 + wrapc(z0 - 1 + zl, g.n2);
        }
    }
#pragma unroll
    for (int j = 0; j < PK; ++j) {
        const int q = threadIdx.x + 256 * j;
        koff[j] = 0;
        if (q < NK) {
            const int zl = q % KZ, yl = q / KZ;
            koff[j] = wrapc(y0 - 1 + yl, g.n1) * g.n2 + wrapc(z0 - 1 + zl, g.n2);
        }
    }
    // d = s + beta d_old; on the first pass of a cycle beta = 0 and d_old is
    // not yet written, so s stands in for it (s + 0 s = s exactly)
    const T* __restrict__ dsrc = (CG && it.k > it.k0) ? dold : s;
    const int64_t pl = (int64_t)g.n1 * g.n2;
    // a plane's values in registers between its load and its LDS store; two
    // sets, so that the loads of two planes are in flight during each step
    struct Stage {
        T s[PD], d[PD], k[PK];
    };
    Stage ra, rb;
    // node plane xp and voxel plane xp (voxel xp lies between node planes xp and xp + 1)
    auto load = [&](Stage& R, int xp) {
        const int64_t base = (int64_t)wrapc(xp, g.n0) * pl;
#pragma unroll
        for (int j = 0; j < PD; ++j) {
            R.s[j] = s[base + doff[j]];
            if (CG) R.d[j] = dsrc[base + doff[j]];
        }
#pragma unroll
        for (int j = 0; j < PK; ++j) R.k[j] = kappa[base + koff[j]];
    };

    // loads first: loop state, partials, previous gamma and the first plane
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
    load(ra, x0 - 1);
    load(rb, x0);  // the sweep has at least three input planes (xe > x0)
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
    // the same in every lane: held in scalar registers
    beta = wave_uniform(beta);
    shift = wave_uniform(shift);
    auto put = [&](const Stage& R, int slot) {
#pragma unroll
        for (int j = 0; j < PD; ++j) {
            const int q = threadIdx.x + 256 * j;
            if (q < ND) Dr[slot][q] = (CG ? R.s[j] + beta * R.d[j] : R.s[j]) - shift;
        }
#pragma unroll
        for (int j = 0; j < PK; ++j) {
            const int q = threadIdx.x + 256 * j;
            if (q < NK) Kr[slot][q] = R.k[j];
        }
    };
    put(ra, 0);
    __syncthreads();

    const int tz = threadIdx.x % TZ, ty = threadIdx.x / TZ * RY;  // first of the thread's RY rows
    const int z = z0 + tz;
    bool yz_ok[RY];
#pragma unroll
    for (int j = 0; j < RY; ++j) yz_ok[j] = (y0 + ty + j < g.n1) && (z < g.n2);
    T km[RY + 1][2];
    T acc_prev[RY], acc_cur[RY], dc_prev[RY];
#pragma unroll
    for (int bb = 0; bb <= RY; ++bb) km[bb][0] = km[bb][1] = (T)0;
#pragma unroll
    for (int j = 0; j < RY; ++j) acc_prev[j] = acc_cur[j] = dc_prev[j] = (T)0;
    double dot = 0.0, dsum_own = 0.0;
    const int nsteps = xe - x0 + 2;
    // steps in pairs, so that the two register sets swap roles statically:
    // at step t, `next` holds plane xi + 1 (stored to LDS after the step's
    // arithmetic) and `ahead` receives plane xi + 2
    for (int t0 = 0; t0 < nsteps; t0 += 2) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int t = t0 + h;
            if (t >= nsteps) break;
            Stage& next = h ? ra : rb;
            Stage& ahead = h ? rb : ra;
            const int xi = x0 - 1 + t;
            const int slot = t & 1;
            const bool more = t + 1 < nsteps;
            // (the last two steps reload plane xe, recently read: no branch)
            load(ahead, min(xi + 2, xe));
            T D[RY + 2][3], kp[RY + 1][2];
#pragma unroll
            for (int bb = 0; bb < RY + 2; ++bb)
#pragma unroll
                for (int c = 0; c < 3; ++c) D[bb][c] = Dr[slot][(ty + bb) * DZ + tz + c];
            const bool has_kp = xi < xe;  // voxel planes x0 - 1 .. xe - 1
#pragma unroll
            for (int bb = 0; bb < RY + 1; ++bb)
#pragma unroll
                for (int c = 0; c < 2; ++c) kp[bb][c] = has_kp ? Kr[slot][(ty + bb) * KZ + tz + c] : (T)0;
#pragma unroll
            for (int j = 0; j < RY; ++j) {
                // row sums of w d along z per voxel column over rows j .. j + 2
                // of the staged plane (j + 1 the output's own row), neighbour-
                // plane (rh) and same-plane (rl) weights; face (sy, sz) adds rows
                // sy and sy + 1.  Outputs xi - 1 (through voxel plane xi - 1), xi
                // (both) and xi + 1 (xi)
                T rh[3][2], rl[3][2];
#pragma unroll
                for (int bb = 0; bb < 3; ++bb)
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        const int m0 = ((bb != 1) << 1) | (c != 1), m1 = ((bb != 1) << 1) | (c + 1 != 1);
                        rh[bb][c] = (T)g.w[4 | m0] * D[j + bb][c] + (T)g.w[4 | m1] * D[j + bb][c + 1];
                        rl[bb][c] = (T)g.w[m0] * D[j + bb][c] + (T)g.w[m1] * D[j + bb][c + 1];
                    }
                T accA = acc_prev[j], accB = acc_cur[j], accC = 0;
#pragma unroll
                for (int sy = 0; sy < 2; ++sy)
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        const T eh = rh[sy][c] + rh[sy + 1][c], el = rl[sy][c] + rl[sy + 1][c];
                        accA += km[j + sy][c] * eh;
                        accB += (km[j + sy][c] + kp[j + sy][c]) * el;
                        accC += kp[j + sy][c] * eh;
                    }
                if (t >= 2 && yz_ok[j]) {  // output xi - 1 is complete
                    const int64_t i = (int64_t)(xi - 1) * pl + (int64_t)(y0 + ty + j) * g.n2 + z;
                    p[i] = accA;
                    if (CG) {
                        dnew[i] = dc_prev[j];
                        dot += (double)dc_prev[j] * (double)accA;
                        if (MF) dsum_own += (double)dc_prev[j];
                    }
                }
                acc_prev[j] = accB;  // (meaningful from t = 1 while xi < xe)
                dc_prev[j] = D[j + 1][1];
                acc_cur[j] = accC;   // (meaningful while xi + 1 < xe)
            }
#pragma unroll
            for (int bb = 0; bb < RY + 1; ++bb)
#pragma unroll
                for (int c = 0; c < 2; ++c) km[bb][c] = kp[bb][c];
            if (more) put(next, slot ^ 1);
            __syncthreads();
        }
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

// tile dimensions within the grid (single conditional wrap)
inline bool tile_near(const TileChoice& c, const GridDev& g)
{
    return c.tx <= g.n0 && 256 / c.tz <= g.n1 && c.tz <= g.n2;
}

// Operator march shape of a (grid, right-hand sides, vector precision,
// conductivity field per right-hand side or shared): the
// footprint width tz (16, 32 or 64), the rows per thread ry (1, or 2 with
// tz of 32 or 64: fewer halo rows per node) and the planes per workgroup xb (>= 2,
// or the whole axis when it is shorter).  uno_autotune_operator measures the
// candidates and records the fastest (autotune.hip); without a record the
// rules below apply.
struct MarchShape {
    int tz, ry, xb;
};
bool march_tuned(const Grid& g, int nrhs, int tsize, bool kappa_per_rhs, MarchShape* out);

// Footprint width by rule: whole 64-node rows where the contiguous axis
// allows (measured: 64 x 4 footprints beat 32 x 8 by 3 % at 64^3 x 48 and by
// 1 % at 192^3 x 3), else 32 or 16.
inline int march_tz_rule(const Grid& g) { return g.n[2] >= 64 ? 64 : (g.n[2] >= 24 ? 32 : 16); }

// Upper bound of the marching kernel's workgroups per right-hand side over
// every footprint width (xb >= 2).
inline int march_max_blocks(const Grid& g)
{
    const int tx = g.n[0] < 2 ? 1 : (g.n[0] + 1) / 2;
    int most = 0;
    for (int tz = 16; tz <= 64; tz *= 2) {
        const int ty = 256 / tz;
        const int b = tx * ((g.n[1] + ty - 1) / ty) * ((g.n[2] + tz - 1) / tz);
        if (b > most) most = b;
    }
    return most;
}

// Marching geometry for footprint width tz, ry rows per thread and planes
// per workgroup xb0: the planes split evenly into chunks of at most xb0.
inline MarchGeom march_geom_of(const Grid& g, int tz, int ry, int64_t xb0)
{
    const int ty = 256 / tz * ry;
    MarchGeom m;
    m.tiles_y = (g.n[1] + ty - 1) / ty;
    m.tiles_z = (g.n[2] + tz - 1) / tz;
    int64_t xb = xb0;
    if (xb < 2) xb = 2;
    if (xb > g.n[0]) xb = g.n[0];
    m.tiles_x = (int)((g.n[0] + xb - 1) / xb);
    m.xb = (g.n[0] + m.tiles_x - 1) / m.tiles_x;  // even split
    return m;
}

// Marching geometry of a launch: the recorded shape, else TY x TZ footprints
// and the planes split evenly into chunks of xb >= 2 so that a launch has
// about 2048 workgroups or more (measured at 64^3 x 48: 2304 workgroups of
// 22 planes 111 us, 6144 of 8 planes 111 us, 4608 of 12 and 3072 of 16
// planes 118-119 us, 1536 of 32 planes 127 us; 192^3 x 3: 199-204 us from
// 1728 to 6912 workgroups).
inline MarchGeom march_geom(const Grid& g, int nrhs, int tsize, bool kappa_per_rhs, int* tz_out, int* ry_out)
{
    MarchShape sh;
    if (march_tuned(g, nrhs, tsize, kappa_per_rhs, &sh)) {
        *tz_out = sh.tz;
        *ry_out = sh.ry;
        return march_geom_of(g, sh.tz, sh.ry, sh.xb);
    }
    const int tz = march_tz_rule(g), ty = 256 / tz;
    *tz_out = tz;
    *ry_out = 1;
    const int64_t yz = (int64_t)((g.n[1] + ty - 1) / ty) * ((g.n[2] + tz - 1) / tz) * nrhs;
    return march_geom_of(g, tz, 1, (g.n[0] * yz + 2047) / 2048);
}

// the footprints built: (tz, ry) in {(64, 1), (32, 1), (16, 1), (64, 2), (32, 2)}
inline bool march_shape_built(int tz, int ry) { return ry == 1 ? (tz == 16 || tz == 32 || tz == 64) : (ry == 2 && tz >= 32 && tz <= 64); }

template <typename T, bool CG, bool HEAD, bool NEAR>
inline void launch_march_near(const MarchGeom& m, int tz, int ry, const GridDev& g, const T* kappa, const T* s,
                              const T* dold, T* dnew, T* p, double* part_dp, const CgIter& it,
                              const double* part_rs, int np_rs, double* gam, hipStream_t st, const MeanFree& mf,
                              int nrhs)
{
    const dim3 grid(m.tiles_x * m.tiles_y * m.tiles_z, nrhs);
    const int fam = CG ? UNO_KT_MATVEC : UNO_KT_APPLY;  // timing family
    switch (ry * 100 + tz) {
        case 164:
            uno_launch(fam, k_stencil_march<T, 64, 1, CG, HEAD, NEAR>, grid, dim3(256), 0, st, g, m, kappa, s, dold,
                       dnew, p, part_dp, it, part_rs, np_rs, gam, mf);
            break;
        case 132:
            uno_launch(fam, k_stencil_march<T, 32, 1, CG, HEAD, NEAR>, grid, dim3(256), 0, st, g, m, kappa, s, dold,
                       dnew, p, part_dp, it, part_rs, np_rs, gam, mf);
            break;
        case 264:
            uno_launch(fam, k_stencil_march<T, 64, 2, CG, HEAD, NEAR>, grid, dim3(256), 0, st, g, m, kappa, s, dold,
                       dnew, p, part_dp, it, part_rs, np_rs, gam, mf);
            break;
        case 232:
            uno_launch(fam, k_stencil_march<T, 32, 2, CG, HEAD, NEAR>, grid, dim3(256), 0, st, g, m, kappa, s, dold,
                       dnew, p, part_dp, it, part_rs, np_rs, gam, mf);
            break;
        default:
            uno_launch(fam, k_stencil_march<T, 16, 1, CG, HEAD, NEAR>, grid, dim3(256), 0, st, g, m, kappa, s, dold,
                       dnew, p, part_dp, it, part_rs, np_rs, gam, mf);
            break;
    }
}

// Launches the operator apply (nrhs right-hand sides along grid y); returns
// the number of workgroups per right-hand side (= d.p partials).
template <typename T, bool CG, bool HEAD>
inline int launch_tile(const Grid& g, const T* kappa, const T* s, const T* dold, T* dnew, T* p, double* part_dp,
                       const CgIter& it, const double* part_rs, int np_rs, double* gam, hipStream_t st,
                       const MeanFree& mf = MeanFree{nullptr, nullptr, nullptr}, int nrhs = 1)
{
    int tz = 0, ry = 1;
    const MarchGeom m = march_geom(g, nrhs, (int)sizeof(T), it.ks != 0, &tz, &ry);
    const bool near = 256 / tz * ry <= g.n[1] && tz <= g.n[2];
    if (near)
        launch_march_near<T, CG, HEAD, true>(m, tz, ry, g.dev, kappa, s, dold, dnew, p, part_dp, it, part_rs, np_rs,
                                             gam, st, mf, nrhs);
    else
        launch_march_near<T, CG, HEAD, false>(m, tz, ry, g.dev, kappa, s, dold, dnew, p, part_dp, it, part_rs, np_rs,
                                              gam, st, mf, nrhs);
    return m.tiles_x * m.tiles_y * m.tiles_z;
}

}  // namespace unocg
