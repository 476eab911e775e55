// kernels.hip -- gfx950 kernels of the staggered-grid acoustic stepper (Sec. 2.1, eq. 3-4),
// CPML (Sec. 2.1), source injection / receiver sampling (Alg. 2), boundary save/restore and
// reconstruction (Sec. 4.2), adjoint propagation and gradient / image accumulation (eq. 7,
// 8, 10), misfit (eq. 6) and the shot reduction.
//
// Two families of half-step kernels cover one time step of every shot of the batch per
// launch, each shot restricted to its computing box:
//   * sweep kernels (k_step_*, k_recon_*): one lane per cell, 64 consecutive z cells per
//     wavefront (a 256-byte coalesced row), 4 x-columns per 256-lane workgroup, neighbours
//     from the L1/L2 caches -- the plain stepper and an option;
//   * register-blocked kernels (k_march_*, the default): a lane updates a short run of cells
//     along the slowest axis from one register window of the stencil along that axis, with
//     every load issued before the arithmetic, in an XCD-contiguous tile order in 2D.
// The register-blocked launches also carry small side work on extra workgroups (receiver
// sampling of the previous step, band cells of saved levels), and the 2D reverse step of small
// batches runs its reconstruction and adjoint half steps on one shared grid (k_rev_*).  The
// free surface (image method), the density face sums, the tangent-linear source and the
// small data kernels (bands, receivers, adjoint sources, misfit, reductions) close the file.
#include <type_traits>
#include <algorithm>
#include <cmath>

#include <hip/hip_ext.h>

#include "smi_internal.hpp"
#include "device.hpp"
#include "side.hpp"

namespace smi {

namespace {

constexpr int BZ = 64, BX = 4;


struct Cell {
    int s, z, x, y;
    long long k;
    bool ok;
};

// Grid: x = z-block, y = x-block, z = y-plane + ny * shot (shot slowest: neighbouring tiles
// of one shot run together and share halos in L2).
// With nxc > 0 the tiles are handed to the 8 XCDs in contiguous x ranges: workgroups are
// dispatched round-robin over the XCDs in launch order, so blockIdx.x & 7 names the XCD and
// XCD k takes x-blocks [k nxc, (k + 1) nxc) (tiles that share x halos share one L2).
struct LG {
    int ny;             // y-planes of the launch (1 in 2D)
    int nxc;            // x-blocks per XCD (0: plain order, blockIdx.y = x-block)
};

__device__ __forceinline__ Cell cell_of(const Geom &g, const int *__restrict__ box, int shot0,
                                        LG lg) {
    Cell c;
    const int zb = lg.nxc ? (int)blockIdx.x >> 3 : (int)blockIdx.x;
    const int xb = lg.nxc ? ((int)blockIdx.x & 7) * lg.nxc + (int)blockIdx.y : (int)blockIdx.y;
    const int sy = lg.ny == 1 ? 0 : (int)blockIdx.z / lg.ny;
    const int yo = lg.ny == 1 ? 0 : (int)blockIdx.z - sy * lg.ny;
    c.s = shot0 + (lg.ny == 1 ? (int)blockIdx.z : sy);
    const int *b = box + 6 * c.s;
    // z tiles start on a 128-byte boundary of the storage (the ghost frame shifts z = 0)
    c.z = zalign(b[0]) + zb * BZ + threadIdx.x;
    c.x = b[2] + xb * BX + threadIdx.y;
    c.y = b[4] + yo;
    c.ok = c.z >= b[0] && c.z < b[1] && c.x < b[3] && c.y < b[5];
    c.k = g.org + c.z + (long long)g.ld1 * c.x + g.ld2 * c.y;
    return c;
}

__device__ __forceinline__ long long stride_of(const Geom &g, int a) {
    return a == 0 ? 1 : (a == 1 ? (long long)g.ld1 : g.ld2);
}

__device__ __forceinline__ int coord(const Cell &c, int a) { return a == 0 ? c.z : (a == 1 ? c.x : c.y); }

// slab offset of the memory variable of axis a at cell c (or -1 outside the slabs)
__device__ __forceinline__ long long slab_off(const Geom &g, const Cell &c, int a) {
    if (a == 0) {
        int zc = slab_index(c.z, g.M[0], g.nb);
        return zc < 0 ? -1 : zc + (long long)g.W * (c.x + (long long)g.M[1] * c.y);
    } else if (a == 1) {
        int xc = slab_index(c.x, g.M[1], g.nb);
        return xc < 0 ? -1 : c.z + (long long)g.ld1 * (xc + (long long)g.W * c.y);
    } else {
        int yc = slab_index(c.y, g.M[2], g.nb);
        return yc < 0 ? -1 : c.z + (long long)g.ld1 * (c.x + (long long)g.M[1] * yc);
    }
}

// (D+_a p)(i + 1/2) * d_a = sum_l a_l (p[i+l] - p[i-l+1])          eq. (4), second row
template <int N>
__device__ __forceinline__ float dplus(const Geom &g, const float *__restrict__ p, const Cell &c, int a) {
    long long st = stride_of(g, a);
    float e = 0.f;
#pragma unroll
    for (int l = 1; l <= N; ++l) e += g.c[a][l - 1] * (p[c.k + l * st] - p[c.k - (l - 1) * st]);
    return e;
}

// (D-_a v)(i) * d_a = sum_l a_l (v[i+l-1] - v[i-l])                  eq. (4), first row
template <int N>
__device__ __forceinline__ float dminus(const Geom &g, const float *__restrict__ v, const Cell &c, int a) {
    long long st = stride_of(g, a);
    float e = 0.f;
#pragma unroll
    for (int l = 1; l <= N; ++l) e += g.c[a][l - 1] * (v[c.k + (l - 1) * st] - v[c.k - l * st]);
    return e;
}

// ---------------------------------------------------------------- model preparation

// Extend vp, rho into the absorbing layers by edge replication; kdt = dt rho vp^2 (eq. 1),
// bdt_a = 2 dt / (rho_i + rho_{i+1}) along a (rho beyond the last node repeats it).
__global__ __launch_bounds__(256) void k_model_prep(Geom g, Model m, const float *__restrict__ vp,
                                                     const float *__restrict__ rho,
                                                     unsigned *status, float vlo, float vhi) {
    long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t >= g.P) return;
    // storage index -> node of the padded grid (ghost nodes get zeros)
    int z = (int)(t % g.ld1) - GH;
    long long r = t / g.ld1;
    const int ex = g.M[1] + 2 * GH;
    int x = (int)(r % ex) - GH;
    int y = g.nd == 3 ? (int)(r / ex) - GH : 0;
    if (z < 0 || z >= g.M[0] || x < 0 || x >= g.M[1] || y < 0 || y >= g.M[2]) {
        m.kdt[t] = 0.f;
        for (int a = 0; a < g.nd; ++a) m.bdt[a][t] = 0.f;
        return;
    }
    int i[3] = {z - g.nb, x - g.nb, g.nd == 3 ? y - g.nb : 0};
    int j[3];
    for (int a = 0; a < 3; ++a) j[a] = min(max(i[a], 0), g.n[a] - 1);
    long long s = j[0] + (long long)g.n[0] * (j[1] + (long long)g.n[1] * j[2]);
    float v = vp[s], rh = rho[s];
    bool own = i[0] == j[0] && i[1] == j[1] && i[2] == j[2];
    if (own && (!(v > 0.f) || !(rh > 0.f) || !isfinite(v) || !isfinite(rh) ||
                v < vlo || v > vhi))
        atomicOr(status, 1u);
    m.kdt[t] = g.dt * rh * v * v;
    for (int a = 0; a < g.nd; ++a) {
        int jn[3] = {j[0], j[1], j[2]};
        jn[a] = min(max(i[a] + 1, 0), g.n[a] - 1);
        long long sn = jn[0] + (long long)g.n[0] * (jn[1] + (long long)g.n[1] * jn[2]);
        m.bdt[a][t] = 2.f * g.dt / (rh + rho[sn]);
    }
}

// positive finite floats order like their bit patterns
__global__ __launch_bounds__(256) void k_minmax(const float *__restrict__ v, long long n, unsigned *out) {
    unsigned lo = 0x7f7fffffu, hi = 0u;
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n;
         t += (long long)gridDim.x * blockDim.x) {
        float x = v[t];
        unsigned u = x > 0.f && isfinite(x) ? __float_as_uint(x) : 0u;
        if (u) { lo = min(lo, u); hi = max(hi, u); } else { lo = 0u; }
    }
    atomicMin(out, lo);
    atomicMax(out + 1, hi);
}

// ---------------------------------------------------------------- leap-frog step (eq. 3 + CPML)

template <int ND, int N>
__global__ __launch_bounds__(256) void k_step_v(Geom g, Fields f, Model m, Cpml cp,
                                                const int *__restrict__ box, int shot0, LG lg) {
    Cell c = cell_of(g, box, shot0, lg);
    if (!c.ok) return;
    const float *p = f.p + c.s * g.P;
#pragma unroll
    for (int a = 0; a < ND; ++a) {
        float e = dplus<N>(g, p, c, a);
        long long so = slab_off(g, c, a);
        if (so >= 0) {
            int i = coord(c, a);
            float *ps = f.psp[a] + c.s * g.psz[a] + so;
            float psi = cp.b_h[a][i] * *ps + cp.a_h[a][i] * e;
            *ps = psi;
            e += psi;
        }
        f.v[a][c.s * g.P + c.k] -= m.bdt[a][c.k] * e;
    }
}

// p update; SRC: add dt stf[it]/dV at the shot's source; IMG: accumulate the image of the
// interior with the (already reconstructed) source field pf.
template <int ND, int N, bool SRC, bool IMG>
__global__ __launch_bounds__(256) void k_step_p(Geom g, Fields f, Model m, Cpml cp,
                                                const int *__restrict__ box, int shot0, LG lg,
                                                const long long *__restrict__ src_cell,
                                                const float *__restrict__ stf, int nt, int it,
                                                const float *__restrict__ pf, float *acc_i) {
    Cell c = cell_of(g, box, shot0, lg);
    if (!c.ok) return;
    float sdiv = 0.f;
#pragma unroll
    for (int a = 0; a < ND; ++a) {
        float e = dminus<N>(g, f.v[a] + c.s * g.P, c, a);
        long long so = slab_off(g, c, a);
        if (so >= 0) {
            int i = coord(c, a);
            float *ps = f.psv[a] + c.s * g.psz[a] + so;
            float psi = cp.b_i[a][i] * *ps + cp.a_i[a][i] * e;
            *ps = psi;
            e += psi;
        }
        sdiv += e;
    }
    float *pp = f.p + c.s * g.P + c.k;
    float pn = *pp - m.kdt[c.k] * sdiv;
    if (SRC && it < nt && c.k == src_cell[c.s]) pn += src_amp(g.src_scale, stf[(long long)c.s * nt + it]);
    *pp = pn;
    if (IMG) {
        int iz = c.z - g.nb, ix = c.x - g.nb, iy = ND == 3 ? c.y - g.nb : 0;
        if ((unsigned)iz < (unsigned)g.n[0] && (unsigned)ix < (unsigned)g.n[1] &&
            (unsigned)iy < (unsigned)g.n[2]) {
            long long ii = c.s * g.I + iz + (long long)g.n[0] * (ix + (long long)g.n[1] * iy);
            acc_i[ii] += g.dt * pn * pf[c.s * g.P + c.k];
        }
    }
}

// ---------------------------------------------------------------- marching sweep kernels
//
// The same two half steps, with each lane marching along the slowest axis (x in 2D, y in 3D)
// over CM consecutive cells.  The values of the differentiated field along the march axis
// stay in a register window that slides by one cell per step, so each is loaded once per
// march instead of 2N times, and the halo of the tile along that axis shrinks to 2N - 1 cells
// per CM.  Lanes run along z (one 256-byte row per wavefront, rows aligned to 128 bytes of
// storage); in 2D the four wavefronts of a workgroup take four consecutive z tiles, in 3D
// four consecutive x columns (whose x-stencil reads then share the L1).  Every lane updates
// only its own cells, so the updates stay in place.

struct MG {
    int nmarch;         // march strips per shot along the march axis (3D: grid z = strip + nmarch shot)
    int nxc;            // > 0: XCD-contiguous order, blockIdx.x & 7 = XCD, which takes nxc
                        // consecutive blocks of x (2D: march strips, 3D: 4-column groups)
    // 3D XCD-contiguous order (ymap = 1, one-dimensional grid): the tiles (shot, y-strip,
    // x-group, z-block), z-block fastest, are cut into 8 contiguous ranges of `per` tiles, one
    // per XCD (blockIdx.x & 7), so that the workgroups resident on one XCD at a time cover a
    // block of neighbouring columns of one strip, whose halo columns and planes they read from
    // the same L2.
    // 2D shot-inner order (ymap = 2; every shot of the launch has the same box): XCD k still
    // takes the strips [k nxc, (k + 1) nxc), but its consecutive workgroups run one tile of
    // every shot (`per` shots, then gz z-blocks, then the strips), so the model under a tile
    // is read once from HBM for all shots.  3D shot-inner order (ymap = 3): grid plane z holds
    // y-strip z / per of shot z % per, so one strip of every shot runs before the next strip
    int gz, gx, per, ntile, ymap;
    int sb = 0;         // first shot of the launch: the shot indices of the tile map count from it
};

// the band cells of every shot over the blocks from grid plane z0 on (one lane per cell)
__device__ __forceinline__ void band_part(const Geom &g, const Fields &f, const BandArg &ba,
                                          int z0, int dir, int which) {
    const long long lin = ((long long)((int)blockIdx.z - z0) * gridDim.y + blockIdx.y) *
                              gridDim.x + blockIdx.x;
    band_lin(g, f, ba, lin, (int)threadIdx.y * 64 + (int)threadIdx.x, dir, which);
}

struct MCell {
    int s, z, x, y;     // y unused in 2D
    int lo, hi;         // march range [lo, hi) along the march axis
    int zb0, zb1;       // the box along z
    long long k;        // storage offset of the first cell
    bool ok;            // this lane updates cells
    bool run;           // the wavefront has work (uniform over the wavefront)
    bool need;          // this lane's row is within 4 of the box along z (z-neighbour of a cell)
};

// SI: the kernel may be launched in a shot-inner order (2D: ymap 2, 3D: ymap 3; compiled out
// of the forward p update, whose launches never use it)
template <int ND, int CM, bool SI = true>
__device__ __forceinline__ MCell mcell_of(const int *__restrict__ box, int shot0, MG mg) {
    MCell c;
    const int wv = threadIdx.y, lane = threadIdx.x;
    const int bz = mg.nxc ? (int)blockIdx.x >> 3 : (int)blockIdx.x;
    const int bx = mg.nxc ? ((int)blockIdx.x & 7) * mg.nxc + (int)blockIdx.y : (int)blockIdx.y;
    if (ND == 2 && SI && mg.ymap == 2) {
        // planes in front of the shots (receiver sampling, or another part of a shared grid)
        // are counted by shot0 < 0; the workgroup's rank among the shots' workgroups keeps
        // the hardware XCD in its low 3 bits
        const int front = shot0 < 0 ? -shot0 : 0;
        const long long rk = (long long)blockIdx.x +
                             (long long)gridDim.x * ((long long)blockIdx.y +
                                                     (long long)gridDim.y * ((int)blockIdx.z - front));
        const long long slot = rk >> 3;
        const long long r = slot / mg.per;
        const int sx = (int)(r / mg.gz);
        c.s = mg.sb + shot0 + front + (int)(slot % mg.per);
        const int *b = box + 6 * c.s;
        c.z = zalign(b[0]) + ((int)(r % mg.gz) * 4 + wv) * 64 + lane;
        c.lo = b[2] + ((int)(rk & 7) * mg.nxc + sx) * CM;
        c.hi = min(c.lo + CM, b[3]);
        c.x = c.lo;
        c.y = 0;
        c.zb0 = b[0];
        c.zb1 = b[1];
        c.run = sx < mg.nxc && c.lo < c.hi && c.z - lane < b[1];
    } else if (ND == 2) {
        c.s = mg.sb + shot0 + (int)blockIdx.z;
        const int *b = box + 6 * c.s;
        c.z = zalign(b[0]) + (bz * 4 + wv) * 64 + lane;
        c.lo = b[2] + bx * CM;
        c.hi = min(c.lo + CM, b[3]);
        c.x = c.lo;
        c.y = 0;
        c.zb0 = b[0];
        c.zb1 = b[1];
        c.run = c.lo < c.hi && c.z - lane < b[1];
    } else {
        int strip = (int)blockIdx.z % mg.nmarch;
        c.s = mg.sb + shot0 + (int)blockIdx.z / mg.nmarch;
        if (SI && mg.ymap == 3) {       // shot-inner: consecutive planes take one strip of every shot
            c.s = mg.sb + shot0 + (int)blockIdx.z % mg.per;
            strip = (int)blockIdx.z / mg.per;
        }
        int zb3 = bz, xg3 = bx;
        bool live = true;
        if (mg.ymap == 1) {
            const int t = ((int)blockIdx.x & 7) * mg.per + ((int)blockIdx.x >> 3);
            live = t < mg.ntile;
            const int tt = live ? t : 0;
            zb3 = tt % mg.gz;
            int r = tt / mg.gz;
            xg3 = r % mg.gx;
            r /= mg.gx;
            strip = r % mg.nmarch;
            c.s = mg.sb + shot0 + r / mg.nmarch;
        }
        const int *b = box + 6 * c.s;
        c.z = zalign(b[0]) + zb3 * 64 + lane;
        c.x = b[2] + xg3 * 4 + wv;
        c.lo = b[4] + strip * CM;
        c.hi = min(c.lo + CM, b[5]);
        c.y = c.lo;
        c.zb0 = b[0];
        c.zb1 = b[1];
        c.run = live && c.lo < c.hi && c.x < b[3] && c.z - lane < b[1];
    }
    // in a grid shared with another half step, blocks past this one's x-blocks per XCD would
    // repeat the next XCD's blocks
    if (mg.nxc && mg.ymap != 2 && (int)blockIdx.y >= mg.nxc) c.run = false;
    c.ok = c.run && c.z >= c.zb0 && c.z < c.zb1;
    c.need = c.run && c.z >= c.zb0 - 4 && c.z < c.zb1 + 4;
    return c;
}

// z-neighbours through LDS: each wavefront stages, per cell of its lanes' runs, the 64 rows it
// owns plus 4 rows each side in its own slice (rows z0 - 4 .. z0 + 67 at index 0 .. 71);
// lanes 0-7 load the 8 outside rows.  Rows more than 4 away from the box are never read and
// are staged as 0.  No workgroup barrier: a wavefront reads only its own slice.
constexpr int ZS = 72;

template <int CM>
__device__ __forceinline__ void zstage(float (*zs)[ZS], const float (&cv)[CM], const float (&hv)[CM]) {
    const int lane = threadIdx.x;
#pragma unroll
    for (int t = 0; t < CM; ++t) zs[t][4 + lane] = cv[t];
    if (lane < 8) {
#pragma unroll
        for (int t = 0; t < CM; ++t) zs[t][lane < 4 ? lane : 64 + lane] = hv[t];
    }
    __builtin_amdgcn_wave_barrier();
}

// the outside row lane (< 8) stages: z0 - 4 + lane (lane < 4) or z0 + 60 + lane (lane >= 4),
// as an offset from the lane's own row z0 + lane; `ok` when that row is within 4 of the box
__device__ __forceinline__ int zhalo(const MCell &mc, bool &ok) {
    const int lane = threadIdx.x;
    const int z0 = mc.z - lane;
    const int r = lane < 4 ? z0 - 4 + lane : z0 + 60 + lane;
    ok = mc.run && lane < 8 && r >= mc.zb0 - 4 && r < mc.zb1 + 4;
    return r - mc.z;
}

template <int ND>
__device__ __forceinline__ Cell as_cell(const Geom &g, const MCell &m, int t) {
    Cell c;
    c.s = m.s;
    c.z = m.z;
    c.x = ND == 2 ? t : m.x;
    c.y = ND == 2 ? 0 : t;
    c.k = g.org + c.z + (long long)g.ld1 * c.x + g.ld2 * c.y;
    c.ok = true;
    return c;
}

// v_a -= dt beta_a (D+_a p + psi_a), psi updated in the slabs (eq. 3 first row, CPML).
// All loads of the lane's CM cells are issued before any arithmetic (the loads are
// independent, so a wavefront keeps CM times more requests in flight); cells past the end of
// the march range re-read the last cell and store nothing.  ZL: the z-neighbours come from
// the wavefront's LDS slice instead of seven unaligned global loads per cell.  FS: the grid
// has a free surface (the lanes near it write the image rows of v_z).
template <int ND, int N, int CM, bool ZL, bool FS = false>
__device__ __forceinline__ void march_v_body(Geom g, Fields f, Model m, Cpml cp,
                                                 const int *__restrict__ box, int shot0, MG mg,
                                                 Ext ex, BandArg sv, int sv_z0) {
    // the p band cells of this level (the v update leaves p alone), on the planes from sv_z0
    if (sv.buf && (int)blockIdx.z >= sv_z0) {
        band_part(g, f, sv, sv_z0, 0, 0);
        return;
    }
    if (ex.it >= 0 && (int)blockIdx.z < mg.nmarch) {   // receivers of the previous step
        const int nthr = (int)(gridDim.x * gridDim.y) * mg.nmarch * 256;
        const int t0 = (((int)blockIdx.z * (int)gridDim.y + (int)blockIdx.y) * (int)gridDim.x +
                        (int)blockIdx.x) * 256 + (int)threadIdx.y * 64 + (int)threadIdx.x;
        for (int r = t0; r < ex.rv.R; r += nthr)
            sample_receiver(g, f.p, ex.rv, ex.dcal, ex.it, ex.status, r);
        return;
    }
    constexpr int MA = ND - 1;              // march axis
    constexpr int NW = CM + 2 * N - 1;      // window: march offsets -(N-1) .. CM-1+N
    constexpr int A0 = ZL ? 1 : 0;          // first axis read through global stencil loads
    __shared__ float zsh[ZL ? 4 : 1][ZL ? CM : 1][ZS];
    MCell mc = mcell_of<ND, CM>(box, shot0, mg);
    if (ZL ? !mc.run : !mc.ok) return;
    const bool ld = ZL ? mc.need : true;
    const int cnt = mc.hi - mc.lo;
    const long long ms = MA == 1 ? (long long)g.ld1 : g.ld2;
    const float *__restrict__ p = f.p + mc.s * g.P;
    const long long k0 = as_cell<ND>(g, mc, mc.lo).k;
    float w[NW];
#pragma unroll
    for (int j = 0; j < NW; ++j) w[j] = ld ? p[k0 + min(j - (N - 1), cnt - 1 + N) * ms] : 0.f;
    // axes other than the march axis (and z when ZL): p at offsets d = -(N-1) .. N, d != 0
    float st[CM][ND - 1 > A0 ? ND - 1 - A0 : 1][2 * N - 1];
    float vo[CM][ND], bd[CM][ND], hv[CM];
    bool hok = false;
    const int hoff = ZL ? zhalo(mc, hok) : 0;
#pragma unroll
    for (int t = 0; t < CM; ++t) {
        const long long k = k0 + min(t, cnt - 1) * ms;
#pragma unroll
        for (int a = A0; a < ND - 1; ++a) {
            const long long sa = stride_of(g, a);
#pragma unroll
            for (int j = 0; j < 2 * N - 1; ++j) {
                const int d = j < N - 1 ? j - (N - 1) : j - (N - 1) + 1;
                st[t][a - A0][j] = mc.ok ? p[k + d * sa] : 0.f;
            }
        }
#pragma unroll
        for (int a = 0; a < ND; ++a) {
            vo[t][a] = mc.ok ? f.v[a][mc.s * g.P + k] : 0.f;
            bd[t][a] = mc.ok ? m.bdt[a][k] : 0.f;
        }
        if (ZL) hv[t] = hok ? p[k + hoff] : 0.f;
    }
    if (ZL) {
        float cv[CM];
#pragma unroll
        for (int t = 0; t < CM; ++t) cv[t] = w[t + N - 1];
        zstage<CM>(zsh[threadIdx.y], cv, hv);
    }
    if (!mc.ok) return;
    const int zl = 4 + (int)threadIdx.x;
#pragma unroll
    for (int t = 0; t < CM; ++t) {
        if (t >= cnt) break;
        Cell c = as_cell<ND>(g, mc, mc.lo + t);
        const float pc = w[t + N - 1];
#pragma unroll
        for (int a = 0; a < ND; ++a) {
            float e = 0.f;
            if (a == MA) {
#pragma unroll
                for (int l = 1; l <= N; ++l) e += g.c[a][l - 1] * (w[t + N - 1 + l] - w[t + N - l]);
            } else if (ZL && a == 0) {
#pragma unroll
                for (int l = 1; l <= N; ++l)
                    e += g.c[0][l - 1] * (zsh[threadIdx.y][t][zl + l] - zsh[threadIdx.y][t][zl - l + 1]);
            } else {
                // st index of offset d: d < 0 -> d + N - 1, d > 0 -> d + N - 2
#pragma unroll
                for (int l = 1; l <= N; ++l) {
                    const float hi = st[t][a - A0][l + N - 2];
                    const float lo = l == 1 ? pc : st[t][a - A0][-(l - 1) + N - 1];
                    e += g.c[a][l - 1] * (hi - lo);
                }
            }
            long long so = slab_off(g, c, a);
            if (so >= 0) {
                int i = coord(c, a);
                float *ps = f.psp[a] + c.s * g.psz[a] + so;
                float psi = cp.b_h[a][i] * *ps + cp.a_h[a][i] * e;
                *ps = psi;
                e += psi;
            }
            const float nv = vo[t][a] - bd[t][a] * e;
            float *vd = f.v[a] + c.s * g.P + c.k;
            if (FS && a == 0) {
                // free surface (image method): v_z on the rows nb - N .. nb - 1 mirrors the rows
                // nb + N - 1 .. nb, written by the lanes of those rows
                const int zr = c.z - g.nb;
                if (zr >= 0 || zr < -N) *vd = nv;
                if (zr >= 0 && zr < N) vd[-1 - 2 * zr] = nv;
            } else {
                *vd = nv;
            }
        }
    }
}

template <int ND, int N, int CM, bool ZL, bool FS>
__global__ __launch_bounds__(256) void k_march_v(Geom g, Fields f, Model m, Cpml cp,
                                                 const int *__restrict__ box, int shot0, MG mg,
                                                 Ext ex, BandArg sv, int sv_z0) {
    march_v_body<ND, N, CM, ZL, FS>(g, f, m, cp, box, shot0, mg, ex, sv, sv_z0);
}

// Adjoint sources of node u at level it (eq. 8, the transpose of the receiver sampling): the
// weighted sum of its receivers' samples in the plan's fixed order, and its addition to p~.
// Both the gather kernel and the adjoint p update that adds the injection itself use these
// two, so either way gives the same bits.
__device__ __forceinline__ float inj_sum(const int *__restrict__ off, const int *__restrict__ rec,
                                         const float *__restrict__ w,
                                         const long long *__restrict__ obase,
                                         const int *__restrict__ stride,
                                         const float *__restrict__ G, int it, int u) {
    float acc = 0.f;
    for (int t = off[u]; t < off[u + 1]; ++t) {
        const int r = rec[t];
        acc = __builtin_fmaf(w[t], G[obase[r] + (long long)it * stride[r]], acc);
    }
    return acc;
}

__device__ __forceinline__ float inj_add(float p, float kdt, float inv_dt, float acc) {
    return __builtin_fmaf(kdt * inv_dt, acc, p);
}

// the injection of level it that an adjoint p update adds on the lanes owning the nodes (2D)
struct InjArg {
    const int *map;         // [nshot][nrow][m1] node of (shot, z - zlo, x), or -1
    int zlo, nrow, m1;
    const int *off, *rec;   // the gather (Inj)
    const float *w;
    const long long *obase; // the receivers (Recv)
    const int *stride;
    const float *G;
    int it;
    float inv_dt;
};

// p -= dt kappa sum_a (D-_a v_a + psi_a) [+ source] [image] (eq. 3 second row, CPML); loads
// first, as in k_march_v.  INJ (2D adjoint update): p~ then takes the adjoint sources of the
// next reverse level at the nodes, after the image has read it (a pass of its own after the
// update, so that the update keeps its registers and schedule).  FS: free surface (the lanes
// near it write the surface row and the image rows of p).
template <int ND, int N, int CM, bool ZL, bool SRC, bool IMG, bool INJ = false, bool FS = false>
__device__ __forceinline__ void march_p_body(Geom g, Fields f, Model m, Cpml cp,
                                                 const int *__restrict__ box, int shot0, MG mg,
                                                 const long long *__restrict__ src_cell,
                                                 const float *__restrict__ stf, int nt, int it,
                                                 const float *__restrict__ pf, float *acc_i, BandArg sv, int sv_z0,
                                                 InjArg ia = InjArg{}) {
    // the v band cells of the next level (the p update leaves v alone), on the planes from sv_z0
    if (sv.buf && (int)blockIdx.z >= sv_z0) {
        band_part(g, f, sv, sv_z0, 0, 1);
        return;
    }
    constexpr int MA = ND - 1;
    constexpr int NW = CM + 2 * N - 1;      // window: march offsets -N .. CM-1+N-1
    constexpr int A0 = ZL ? 1 : 0;
    __shared__ float zsh[ZL ? 4 : 1][ZL ? CM : 1][ZS];
    MCell mc = mcell_of<ND, CM, !SRC>(box, shot0, mg);
    if (ZL ? !mc.run : !mc.ok) return;
    const int cnt = mc.hi - mc.lo;
    const long long ms = MA == 1 ? (long long)g.ld1 : g.ld2;
    const long long so0 = mc.s * g.P;
    const float *__restrict__ vm = f.v[MA] + so0;
    const long long k0 = as_cell<ND>(g, mc, mc.lo).k;
    float w[NW];
#pragma unroll
    for (int j = 0; j < NW; ++j) w[j] = mc.ok ? vm[k0 + min(j - N, cnt - 1 + N - 1) * ms] : 0.f;
    // other axes (x in 3D, and z unless ZL): v_a at offsets -N .. N-1 per cell
    float st[CM][ND - 1 > A0 ? ND - 1 - A0 : 1][2 * N];
    float po[CM], kd[CM], zc[CM], hv[CM];
    bool hok = false;
    const int hoff = ZL ? zhalo(mc, hok) : 0;
    const float *__restrict__ vz = f.v[0] + so0;
#pragma unroll
    for (int t = 0; t < CM; ++t) {
        const long long k = k0 + min(t, cnt - 1) * ms;
#pragma unroll
        for (int a = A0; a < ND - 1; ++a) {
            const long long sa = stride_of(g, a);
            const float *__restrict__ va = f.v[a] + so0;
#pragma unroll
            for (int j = 0; j < 2 * N; ++j) st[t][a - A0][j] = mc.ok ? va[k + (j - N) * sa] : 0.f;
        }
        po[t] = mc.ok ? f.p[so0 + k] : 0.f;
        kd[t] = mc.ok ? m.kdt[k] : 0.f;
        if (ZL) {
            zc[t] = mc.need ? vz[k] : 0.f;
            hv[t] = hok ? vz[k + hoff] : 0.f;
        }
    }
    if (ZL) zstage<CM>(zsh[threadIdx.y], zc, hv);
    if (!mc.ok) return;
    const int zl = 4 + (int)threadIdx.x;
    const long long sc = SRC ? src_cell[mc.s] : -1;
#pragma unroll
    for (int t = 0; t < CM; ++t) {
        if (t >= cnt) break;
        Cell c = as_cell<ND>(g, mc, mc.lo + t);
        float sdiv = 0.f;
#pragma unroll
        for (int a = 0; a < ND; ++a) {
            float e = 0.f;
            if (a == MA) {
#pragma unroll
                for (int l = 1; l <= N; ++l) e += g.c[a][l - 1] * (w[t + N + l - 1] - w[t + N - l]);
            } else if (ZL && a == 0) {
#pragma unroll
                for (int l = 1; l <= N; ++l)
                    e += g.c[0][l - 1] * (zsh[threadIdx.y][t][zl + l - 1] - zsh[threadIdx.y][t][zl - l]);
            } else {
#pragma unroll
                for (int l = 1; l <= N; ++l)
                    e += g.c[a][l - 1] * (st[t][a - A0][N + l - 1] - st[t][a - A0][N - l]);
            }
            long long so = slab_off(g, c, a);
            if (so >= 0) {
                int i = coord(c, a);
                float *ps = f.psv[a] + c.s * g.psz[a] + so;
                float psi = cp.b_i[a][i] * *ps + cp.a_i[a][i] * e;
                *ps = psi;
                e += psi;
            }
            sdiv += e;
        }
        float pn = po[t] - kd[t] * sdiv;
        if (SRC && it < nt && c.k == sc) pn += src_amp(g.src_scale, stf[(long long)c.s * nt + it]);
        float *pd = f.p + so0 + c.k;
        if (FS) {
            // free surface (image method): p = 0 on row nb and odd about it, the rows nb - N ..
            // nb - 1 written by the lanes of rows nb + N .. nb + 1 (the image below still takes
            // the updated value)
            const int zr = c.z - g.nb;
            if (zr > 0 || zr < -N) *pd = pn;
            else if (zr == 0) *pd = 0.f;
            if (zr > 0 && zr <= N) pd[-2 * zr] = -pn;
        } else {
            *pd = pn;
        }
        if (IMG) {
            int iz = c.z - g.nb, ix = c.x - g.nb, iy = ND == 3 ? c.y - g.nb : 0;
            if ((unsigned)iz < (unsigned)g.n[0] && (unsigned)ix < (unsigned)g.n[1] &&
                (unsigned)iy < (unsigned)g.n[2]) {
                long long ii = c.s * g.I + iz + (long long)g.n[0] * (ix + (long long)g.n[1] * iy);
                acc_i[ii] += g.dt * pn * pf[so0 + c.k];
            }
        }
    }
    // the next level's adjoint sources on this lane's nodes (2D: the lane's cells are one row),
    // added to the stored p~ after the update above, as the gather launch would add them
    if (INJ && ND == 2 && (unsigned)(mc.z - ia.zlo) < (unsigned)ia.nrow) {
        const int *__restrict__ row = ia.map + ((long long)mc.s * ia.nrow + (mc.z - ia.zlo)) * ia.m1;
#pragma unroll
        for (int t = 0; t < CM; ++t) {
            if (t >= cnt) break;
            const int u = row[mc.lo + t];
            const int zr = mc.z - g.nb;
            // with a free surface, the surface row stays 0 and the image rows follow row nb + k
            if (u >= 0 && !(FS && zr <= 0 && zr >= -N)) {
                const long long k = as_cell<ND>(g, mc, mc.lo + t).k;
                float *q = f.p + so0 + k;
                const float pv = inj_add(*q, m.kdt[k], ia.inv_dt,
                                         inj_sum(ia.off, ia.rec, ia.w, ia.obase, ia.stride, ia.G, ia.it, u));
                *q = pv;
                if (FS && zr > 0 && zr <= N) q[-2 * zr] = -pv;
            }
        }
    }
}

template <int ND, int N, int CM, bool ZL, bool SRC, bool IMG, bool FS>
__global__ __launch_bounds__(256) void k_march_p(Geom g, Fields f, Model m, Cpml cp,
                                                 const int *__restrict__ box, int shot0, MG mg,
                                                 const long long *__restrict__ src_cell,
                                                 const float *__restrict__ stf, int nt, int it,
                                                 const float *__restrict__ pf, float *acc_i, BandArg sv, int sv_z0) {
    march_p_body<ND, N, CM, ZL, SRC, IMG, false, FS>(g, f, m, cp, box, shot0, mg, src_cell, stf, nt,
                                                     it, pf, acc_i, sv, sv_z0);
}

// ---------------------------------------------------------------- reconstruction (Sec. 4.2)

// p^it = p^{it+1} - dt stf[it]/dV [at the source] + dt kappa div v^{it+1/2}  on the interior;
// GRAD: acc_g += p~ div v^{it+1/2}  (p~: adjoint pressure after this step's injection);
// ILL:  acc_l += dt (p^it)^2  (source illumination).
template <int ND, int N, bool GRAD, bool ILL>
__global__ __launch_bounds__(256) void k_recon_p(Geom g, Fields f, Model m,
                                                 const int *__restrict__ rbox, int shot0, LG lg,
                                                 const long long *__restrict__ src_cell,
                                                 const float *__restrict__ stf, int nt, int it,
                                                 const float *__restrict__ qp, float *acc_g,
                                                 float *acc_l) {
    Cell c = cell_of(g, rbox, shot0, lg);
    if (!c.ok) return;
    float div = 0.f;
#pragma unroll
    for (int a = 0; a < ND; ++a) div += dminus<N>(g, f.v[a] + c.s * g.P, c, a);
    float *pp = f.p + c.s * g.P + c.k;
    float pv = *pp;
    if (c.k == src_cell[c.s]) pv -= src_amp(g.src_scale, stf[(long long)c.s * nt + it]);
    // p^it vanishes on a free surface (the update gives the value before its image)
    float pn = g.fs && c.z == g.nb ? 0.f : pv + m.kdt[c.k] * div;
    *pp = pn;
    long long ii = c.s * g.I + (c.z - g.nb) +
                   (long long)g.n[0] * ((c.x - g.nb) + (long long)g.n[1] * (ND == 3 ? c.y - g.nb : 0));
    if (GRAD) acc_g[ii] += qp[c.s * g.P + c.k] * div;
    if (ILL) acc_l[ii] += g.dt * pn * pn;
}

// v_a^{it-1/2} = v_a^{it+1/2} + dt beta_a D+_a p^it  at v_a points strictly between interior
// p nodes along a (interior along the other axes).
template <int ND, int N>
__global__ __launch_bounds__(256) void k_recon_v(Geom g, Fields f, Model m,
                                                 const int *__restrict__ rbox, int shot0, LG lg) {
    Cell c = cell_of(g, rbox, shot0, lg);
    if (!c.ok) return;
    const float *p = f.p + c.s * g.P;
#pragma unroll
    for (int a = 0; a < ND; ++a) {
        if (coord(c, a) >= g.nb + g.n[a] - 1) continue;
        float e = dplus<N>(g, p, c, a);
        f.v[a][c.s * g.P + c.k] += m.bdt[a][c.k] * e;
    }
}

// Register-blocked forms of the two reconstruction kernels (cells per lane along the slowest
// axis, loads first, z-neighbours through LDS when ZL), as k_march_v / k_march_p.
template <int ND, int N, int CM, bool ZL, bool GRAD, bool ILL>
__device__ __forceinline__ void march_recon_p_body(Geom g, Fields f, Model m,
                                                       const int *__restrict__ rbox, int shot0,
                                                       MG mg, const long long *__restrict__ src_cell,
                                                       const float *__restrict__ stf, int nt, int it,
                                                       const float *__restrict__ qp, float *acc_g,
                                                       float *acc_l) {
    constexpr int MA = ND - 1;
    constexpr int NW = CM + 2 * N - 1;
    constexpr int A0 = ZL ? 1 : 0;
    __shared__ float zsh[ZL ? 4 : 1][ZL ? CM : 1][ZS];
    MCell mc = mcell_of<ND, CM>(rbox, shot0, mg);
    if (ZL ? !mc.run : !mc.ok) return;
    const int cnt = mc.hi - mc.lo;
    const long long ms = MA == 1 ? (long long)g.ld1 : g.ld2;
    const long long so0 = mc.s * g.P;
    const float *__restrict__ vm = f.v[MA] + so0;
    const long long k0 = as_cell<ND>(g, mc, mc.lo).k;
    // interior index of the first cell and its step along the march axis
    const long long ii0 = mc.s * g.I + (mc.z - g.nb) +
                          (long long)g.n[0] * ((ND == 2 ? mc.lo : mc.x) - g.nb +
                                               (long long)g.n[1] * (ND == 3 ? mc.lo - g.nb : 0));
    const long long iis = ND == 2 ? (long long)g.n[0] : (long long)g.n[0] * g.n[1];
    const bool ok = mc.ok;
    float w[NW];
#pragma unroll
    for (int j = 0; j < NW; ++j) w[j] = ok ? vm[k0 + min(j - N, cnt - 1 + N - 1) * ms] : 0.f;
    float st[CM][ND - 1 > A0 ? ND - 1 - A0 : 1][2 * N];
    float po[CM], kd[CM], qv[CM], ag[CM], al[CM], zc[CM], hv[CM];
    bool hok = false;
    const int hoff = ZL ? zhalo(mc, hok) : 0;
    const float *__restrict__ vz = f.v[0] + so0;
#pragma unroll
    for (int t = 0; t < CM; ++t) {
        const int tc = min(t, cnt - 1);
        const long long k = k0 + tc * ms;
#pragma unroll
        for (int a = A0; a < ND - 1; ++a) {
            const long long sa = stride_of(g, a);
            const float *__restrict__ va = f.v[a] + so0;
#pragma unroll
            for (int j = 0; j < 2 * N; ++j) st[t][a - A0][j] = ok ? va[k + (j - N) * sa] : 0.f;
        }
        po[t] = ok ? f.p[so0 + k] : 0.f;
        kd[t] = ok ? m.kdt[k] : 0.f;
        if (GRAD) {
            qv[t] = ok ? qp[so0 + k] : 0.f;
            ag[t] = ok ? acc_g[ii0 + tc * iis] : 0.f;
        }
        if (ILL) al[t] = ok ? acc_l[ii0 + tc * iis] : 0.f;
        if (ZL) {
            zc[t] = mc.need ? vz[k] : 0.f;
            hv[t] = hok ? vz[k + hoff] : 0.f;
        }
    }
    if (ZL) zstage<CM>(zsh[threadIdx.y], zc, hv);
    if (!ok) return;
    const int zl = 4 + (int)threadIdx.x;
    const long long sc = src_cell[mc.s];
#pragma unroll
    for (int t = 0; t < CM; ++t) {
        if (t >= cnt) break;
        const long long k = k0 + t * ms;
        float div = 0.f;
#pragma unroll
        for (int a = 0; a < ND; ++a) {
            float e = 0.f;
            if (a == MA) {
#pragma unroll
                for (int l = 1; l <= N; ++l) e += g.c[a][l - 1] * (w[t + N + l - 1] - w[t + N - l]);
            } else if (ZL && a == 0) {
#pragma unroll
                for (int l = 1; l <= N; ++l)
                    e += g.c[0][l - 1] * (zsh[threadIdx.y][t][zl + l - 1] - zsh[threadIdx.y][t][zl - l]);
            } else {
#pragma unroll
                for (int l = 1; l <= N; ++l)
                    e += g.c[a][l - 1] * (st[t][a - A0][N + l - 1] - st[t][a - A0][N - l]);
            }
            div += e;
        }
        float pv = po[t];
        if (k == sc) pv -= src_amp(g.src_scale, stf[(long long)mc.s * nt + it]);
        // p^it vanishes on a free surface (the update gives the value before its image)
        const float pn = g.fs && mc.z == g.nb ? 0.f : pv + kd[t] * div;
        f.p[so0 + k] = pn;
        if (GRAD) acc_g[ii0 + t * iis] = ag[t] + qv[t] * div;
        if (ILL) acc_l[ii0 + t * iis] = al[t] + g.dt * pn * pn;
    }
}

template <int ND, int N, int CM, bool ZL, bool GRAD, bool ILL>
__global__ __launch_bounds__(256) void k_march_recon_p(Geom g, Fields f, Model m,
                                                       const int *__restrict__ rbox, int shot0,
                                                       MG mg, const long long *__restrict__ src_cell,
                                                       const float *__restrict__ stf, int nt, int it,
                                                       const float *__restrict__ qp, float *acc_g,
                                                       float *acc_l) {
    march_recon_p_body<ND, N, CM, ZL, GRAD, ILL>(g, f, m, rbox, shot0, mg, src_cell, stf, nt, it, qp, acc_g, acc_l);
}

template <int ND, int N, int CM, bool ZL>
__device__ __forceinline__ void march_recon_v_body(Geom g, Fields f, Model m,
                                                       const int *__restrict__ rbox, int shot0,
                                                       MG mg) {
    constexpr int MA = ND - 1;
    constexpr int NW = CM + 2 * N - 1;
    constexpr int A0 = ZL ? 1 : 0;
    __shared__ float zsh[ZL ? 4 : 1][ZL ? CM : 1][ZS];
    MCell mc = mcell_of<ND, CM>(rbox, shot0, mg);
    if (ZL ? !mc.run : !mc.ok) return;
    const bool ld = ZL ? mc.need : true;
    const bool ok = mc.ok;
    const int cnt = mc.hi - mc.lo;
    const long long ms = MA == 1 ? (long long)g.ld1 : g.ld2;
    const float *__restrict__ p = f.p + mc.s * g.P;
    const long long k0 = as_cell<ND>(g, mc, mc.lo).k;
    float w[NW];
#pragma unroll
    for (int j = 0; j < NW; ++j) w[j] = ld ? p[k0 + min(j - (N - 1), cnt - 1 + N) * ms] : 0.f;
    float st[CM][ND - 1 > A0 ? ND - 1 - A0 : 1][2 * N - 1];
    float vo[CM][ND], bd[CM][ND], hv[CM];
    bool hok = false;
    const int hoff = ZL ? zhalo(mc, hok) : 0;
#pragma unroll
    for (int t = 0; t < CM; ++t) {
        const long long k = k0 + min(t, cnt - 1) * ms;
#pragma unroll
        for (int a = A0; a < ND - 1; ++a) {
            const long long sa = stride_of(g, a);
#pragma unroll
            for (int j = 0; j < 2 * N - 1; ++j) {
                const int d = j < N - 1 ? j - (N - 1) : j - (N - 1) + 1;
                st[t][a - A0][j] = ok ? p[k + d * sa] : 0.f;
            }
        }
#pragma unroll
        for (int a = 0; a < ND; ++a) {
            vo[t][a] = ok ? f.v[a][mc.s * g.P + k] : 0.f;
            bd[t][a] = ok ? m.bdt[a][k] : 0.f;
        }
        if (ZL) hv[t] = hok ? p[k + hoff] : 0.f;
    }
    if (ZL) {
        float cv[CM];
#pragma unroll
        for (int t = 0; t < CM; ++t) cv[t] = w[t + N - 1];
        zstage<CM>(zsh[threadIdx.y], cv, hv);
    }
    if (!ok) return;
    const int zl = 4 + (int)threadIdx.x;
    // v_a points strictly between interior p nodes along a
    const int lastz = g.nb + g.n[0] - 1, lastx = g.nb + g.n[1] - 1, lasty = g.nb + g.n[2] - 1;
#pragma unroll
    for (int t = 0; t < CM; ++t) {
        if (t >= cnt) break;
        const int tt = mc.lo + t;
        const long long k = k0 + t * ms;
        const float pc = w[t + N - 1];
#pragma unroll
        for (int a = 0; a < ND; ++a) {
            const int ca = a == 0 ? mc.z : (a == MA ? tt : mc.x);
            if (ca >= (a == 0 ? lastz : (a == 1 ? lastx : lasty))) continue;
            float e = 0.f;
            if (a == MA) {
#pragma unroll
                for (int l = 1; l <= N; ++l) e += g.c[a][l - 1] * (w[t + N - 1 + l] - w[t + N - l]);
            } else if (ZL && a == 0) {
#pragma unroll
                for (int l = 1; l <= N; ++l)
                    e += g.c[0][l - 1] * (zsh[threadIdx.y][t][zl + l] - zsh[threadIdx.y][t][zl - l + 1]);
            } else {
#pragma unroll
                for (int l = 1; l <= N; ++l) {
                    const float hi = st[t][a - A0][l + N - 2];
                    const float lo = l == 1 ? pc : st[t][a - A0][-(l - 1) + N - 1];
                    e += g.c[a][l - 1] * (hi - lo);
                }
            }
            f.v[a][mc.s * g.P + k] = vo[t][a] + bd[t][a] * e;
        }
    }
}

template <int ND, int N, int CM, bool ZL>
__global__ __launch_bounds__(256) void k_march_recon_v(Geom g, Fields f, Model m,
                                                       const int *__restrict__ rbox, int shot0,
                                                       MG mg) {
    march_recon_v_body<ND, N, CM, ZL>(g, f, m, rbox, shot0, mg);
}

// ---------------------------------------------------------------- saved boundaries (Sec. 4.2)

// one lane per band cell; shot shot0 + blockIdx.y
__global__ __launch_bounds__(256) void k_band(Geom g, Fields f, BandDesc bd, float *buf,
                                              const float *buf2, long long shot_stride, int shot0,
                                              int dir, int which, float wt) {
    band_cell(g, f, bd, buf, buf2, shot_stride, shot0 + (int)blockIdx.y,
              blockIdx.x * (long long)blockDim.x + threadIdx.x, dir, which, wt);
}

// The reverse step of the 2D default path in two launches.  Launch 1 runs, on disjoint
// blocks of one grid, the reconstruction of p^it with the gradient and illumination sums
// (blockIdx.z < nshot), the adjoint v update (the next nshot planes) and, with bands saved
// at every step, the restore of the p band cells of level it (the planes after); launch 2 runs
// the reconstruction of v^{it-1/2}, the adjoint p update with the image, and the restore of
// the v band cells.  The parts of a launch touch disjoint data: the bands lie outside the
// interior that the reconstruction writes, the adjoint fields are separate, and the v bands are
// restored only after the gradient has read v^{it+1/2} next to the interior.
template <int N, int CM, bool GRAD, bool ILL, bool BAND, bool FS>
__global__ __launch_bounds__(256) void k_rev_pv(Geom g, Fields f, Fields q, Model m, Cpml cp,
                                                const int *__restrict__ rb,
                                                const int *__restrict__ ab, MG mgr, MG mga,
                                                int nshot, const long long *__restrict__ src_cell,
                                                const float *__restrict__ stf, int nt, int it,
                                                float *acc_g, float *acc_l, BandArg ba) {
    const int bz = (int)blockIdx.z;
    if (bz < nshot)
        march_recon_p_body<2, N, CM, false, GRAD, ILL>(g, f, m, rb, 0, mgr, src_cell, stf, nt, it,
                                                       q.p, acc_g, acc_l);
    else if (bz < 2 * nshot)
        march_v_body<2, N, CM, false, FS>(g, q, m, cp, ab, -nshot, mga,
                                          Ext{Recv{}, nullptr, -1, nullptr}, BandArg{}, 0);
    else if (BAND)
        band_part(g, f, ba, 2 * nshot, 1, 0);
}

// INJ: the adjoint p update also adds the adjoint sources of level it - 1 (ia), which the next
// reverse step would otherwise inject with a launch of its own.  The injection's arguments
// would take the kernel to 102 scalar registers and seven wavefronts per SIMD (13 % slower);
// asked for eight, the compiler fits 78 without spilling.
template <int N, int CM, bool IMG, bool BAND, bool INJ, bool FS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_rev_vp(Geom g, Fields f, Fields q, Model m, Cpml cp,
                                                const int *__restrict__ rb,
                                                const int *__restrict__ ab, MG mgr, MG mga,
                                                int nshot, const long long *__restrict__ src_cell,
                                                const float *__restrict__ stf, int nt, int it,
                                                float *acc_i, BandArg ba, InjArg ia) {
    const int bz = (int)blockIdx.z;
    if (bz < nshot)
        march_recon_v_body<2, N, CM, false>(g, f, m, rb, 0, mgr);
    else if (bz < 2 * nshot)
        march_p_body<2, N, CM, false, false, IMG, INJ, FS>(g, q, m, cp, ab, -nshot, mga, src_cell,
                                                           stf, nt, it, f.p, acc_i, BandArg{}, 0, ia);
    else if (BAND)
        band_part(g, f, ba, 2 * nshot, 1, 1);
}

// Band cells at level it = sum_j w[j] * saved level slot[j] (decimated bands, dr > 1).
struct Taps {
    int n;
    int slot[2 * kTaps];
    float w[2 * kTaps];
};

__global__ __launch_bounds__(256) void k_band_mix(Geom g, Fields f, BandDesc bd, const float *buf,
                                                  long long shot_stride, int shot0, Taps tp,
                                                  int which) {
    long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (q >= bd.B) return;
    int s = shot0 + (int)blockIdx.y;
    int b = 0;
#pragma unroll 1
    while (b + 1 < bd.nblk && q >= bd.blk[b + 1].off) ++b;
    const BandBlock &bl = bd.blk[b];
    if (which != 2 && bl.field != which) return;
    // 32-bit unsigned index arithmetic (a shot's band holds fewer than 2^31 cells; 64-bit
    // division is emulated and dominated these kernels)
    const unsigned r0 = (unsigned)(q - bl.off), e0 = (unsigned)bl.ext[0], e1 = (unsigned)bl.ext[1];
    const unsigned r1 = r0 / e0;
    int z = bl.org[0] + (int)(r0 - r1 * e0);
    int x = bl.org[1] + (int)(r1 % e1);
    int y = bl.org[2] + (int)(r1 / e1);
    long long k = g.org + z + (long long)g.ld1 * x + g.ld2 * y;
    float acc = 0.f;
    for (int j = 0; j < tp.n; ++j) acc += tp.w[j] * buf[s * shot_stride + (long long)tp.slot[j] * bd.B + q];
    (bl.field == 0 ? f.p : f.v[bl.axis])[s * g.P + k] = acc;
}

// ---------------------------------------------------------------- receivers

// dcal[it][r] = p^{it+1} sampled by receiver r's operator  (Alg. 2 extract_wavefield)
__global__ __launch_bounds__(256) void k_extract(Geom g, const float *__restrict__ p, Recv rv,
                                                 float *dcal, int it, unsigned *status) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rv.R) return;
    sample_receiver(g, p, rv, dcal, it, status, r);
}

// p += sign (dt / dV) stf[s][it] w_t on the nodes of the operators of the sources that spread
// over several nodes (shot shot0 + blockIdx.y; one-tap sources have src_cell >= 0 and are injected
// inside the p kernels)
__global__ __launch_bounds__(256) void k_src_taps(Geom g, float *p, const long long *__restrict__ src_cell,
                                                  const int *__restrict__ toff,
                                                  const long long *__restrict__ tcell,
                                                  const float *__restrict__ tw,
                                                  const float *__restrict__ stf, int nt, int it,
                                                  float sign, int shot0) {
    const int s = shot0 + (int)blockIdx.y;
    if (src_cell[s] >= 0) return;
    const int t = toff[s] + blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= toff[s + 1]) return;
    p[s * g.P + tcell[t]] += sign * src_amp(src_amp(g.src_scale, tw[t]), stf[(long long)s * nt + it]);
}

__global__ __launch_bounds__(256) void k_scale(const float *__restrict__ in, float *out, long long n,
                                               float a) {
    long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t < n) out[t] = a * in[t];
}

// p~ += kappa sum_r w_r G[it][r] on every node that receiver operators touch (eq. 8 source in
// the scaled adjoint variable; the transpose of the sampling).  One lane per distinct node sums
// its contributions in the plan's fixed order (ascending receiver), so overlapping operators and
// co-located receivers give the same bits on every run.  Nodes of shots outside [s0, s1) are
// left to the reverse loop of their own shot group.
__global__ __launch_bounds__(256) void k_inject(Geom g, float *qp, const float *__restrict__ kdt,
                                                Recv rv, Inj in, const float *__restrict__ G,
                                                int it, float inv_dt, int s0, int s1) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= in.U || in.shot[u] < s0 || in.shot[u] >= s1) return;
    const float acc = inj_sum(in.off, in.rec, in.w, rv.obase, rv.stride, G, it, u);
    const long long c = in.cell[u];
    float *q = qp + in.shot[u] * g.P + c;
    *q = inj_add(*q, kdt[c], inv_dt, acc);
}

// ---------------------------------------------------------------- misfit (eq. 6)

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// r = dcal - dobs, G = dt r, partial[b] = sum over this block's grid-stride share of r^2
__global__ __launch_bounds__(256) void k_residual(const float *__restrict__ dcal,
                                                  const float *__restrict__ dobs, float *G,
                                                  long long n, float dt, double *partial) {
    __shared__ double red[4];
    double acc = 0.0;
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n;
         t += (long long)gridDim.x * blockDim.x) {
        float r = dcal[t] - dobs[t];
        G[t] = dt * r;
        acc += (double)r * (double)r;
    }
    acc = wave_sum(acc);
    int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) red[wv] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// out = scale * sum(partial[0..n)) in a fixed order (one workgroup)
__global__ __launch_bounds__(256) void k_sum_partial(const double *__restrict__ partial, int n,
                                                     double *out, double scale) {
    __shared__ double red[4];
    double acc = 0.0;
    for (int t = threadIdx.x; t < n; t += blockDim.x) acc += partial[t];
    acc = wave_sum(acc);
    int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) red[wv] = acc;
    __syncthreads();
    if (threadIdx.x == 0) *out = scale * (red[0] + red[1] + red[2] + red[3]);
}

// ---------------------------------------------------------------- shot reduction + chain rule

// grad = -(2 dt / vp) sum_s acc_g[s]  (dJ/dVp = 2 rho Vp dJ/dkappa, dJ/dkappa = -(dt/kappa) sum p~ div v)
__global__ __launch_bounds__(256) void k_finalize_grad(const float *__restrict__ acc, int nshot,
                                                       long long I, const float *__restrict__ vp,
                                                       float dt, float *grad) {
    long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= I) return;
    float s = 0.f;
    for (int k = 0; k < nshot; ++k) s += acc[k * I + i];
    grad[i] = -2.f * dt / vp[i] * s;
}

__global__ __launch_bounds__(256) void k_finalize_sum(const float *__restrict__ acc, int nshot,
                                                      long long I, float *out) {
    long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= I) return;
    float s = 0.f;
    for (int k = 0; k < nshot; ++k) s += acc[k * I + i];
    out[i] = s;
}

// Per-shot peak of the illumination (non-negative floats order like their bit patterns).
__global__ __launch_bounds__(256) void k_shot_max(const float *__restrict__ acc, long long I,
                                                  unsigned *mx) {
    const int s = blockIdx.y;
    unsigned hi = 0u;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < I;
         i += (long long)gridDim.x * blockDim.x)
        hi = max(hi, __float_as_uint(fmaxf(acc[s * I + i], 0.f)));
    for (int o = 32; o > 0; o >>= 1) hi = max(hi, (unsigned)__shfl_down((int)hi, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(mx + s, hi);
}

__global__ void k_fill_u32(unsigned *p, int n, unsigned v) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Normalised imaging condition (Sec. 2.3): sum_s image_s / (illum_s + eps max(illum_s)).
__global__ __launch_bounds__(256) void k_finalize_norm(const float *__restrict__ img,
                                                       const float *__restrict__ ill, int nshot,
                                                       long long I, const unsigned *__restrict__ mx,
                                                       float eps, float *out) {
    long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= I) return;
    float s = 0.f;
    for (int k = 0; k < nshot; ++k) {
        const float st = eps * __uint_as_float(mx[k]);
        const float den = ill[k * I + i] + st;
        s += den > 0.f ? img[k * I + i] / den : 0.f;
    }
    out[i] = s;
}

// Laplace filter of an image (Sec. 2.3): second-order central differences along each axis,
// divided by the squared spacing, zero outside the image.
__global__ __launch_bounds__(256) void k_laplacian(const float *__restrict__ f, float *out,
                                                   int n1, int n2, int n3, float w1, float w2,
                                                   float w3) {
    long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long tot = (long long)n1 * n2 * n3;
    if (i >= tot) return;
    const int z = (int)(i % n1);
    const long long r = i / n1;
    const int x = (int)(r % n2);
    const int y = (int)(r / n2);
    const long long s2 = n1, s3 = (long long)n1 * n2;
    const float c = f[i];
    float acc = w1 * ((z + 1 < n1 ? f[i + 1] : 0.f) - 2.f * c + (z > 0 ? f[i - 1] : 0.f));
    acc += w2 * ((x + 1 < n2 ? f[i + s2] : 0.f) - 2.f * c + (x > 0 ? f[i - s2] : 0.f));
    if (n3 > 1 || w3 != 0.f)
        acc += w3 * ((y + 1 < n3 ? f[i + s3] : 0.f) - 2.f * c + (y > 0 ? f[i - s3] : 0.f));
    out[i] = acc;
}

// Density part of eq. (7): per face of axis a, acc_r[a] += v~_a D+_a p with v~^{it+1/2} the
// adjoint velocity and p^it the rebuilt source field, on the faces from the one below the
// first interior node to the one above the last (interior along the other axes), inside the
// shot's reconstruction region widened by one face downwards.  Lanes cover the region
// [lo - 1, hi) per axis; blockIdx.z = shot * ny + y-plane.
template <int ND, int N>
__global__ __launch_bounds__(256) void k_rho_faces(Geom g, Fields f, Fields q, float *acc0,
                                                   float *acc1, float *acc2,
                                                   const int *__restrict__ rbox, int ny,
                                                   int shot0) {
    const int s = shot0 + (int)blockIdx.z / ny;
    const int *b = rbox + 6 * s;
    Cell c;
    c.s = s;
    c.z = b[0] - 1 + (int)blockIdx.x * 64 + (int)threadIdx.x;
    c.x = b[2] - 1 + (int)blockIdx.y * 4 + (int)threadIdx.y;
    c.y = ND == 3 ? b[4] - 1 + (int)blockIdx.z % ny : 0;
    const int lo[3] = {b[0], b[2], b[4]}, hi[3] = {b[1], b[3], b[5]};
    const int co[3] = {c.z, c.x, c.y};
    c.k = g.org + c.z + (long long)g.ld1 * c.x + g.ld2 * c.y;
    c.ok = true;
    const float *p = f.p + s * g.P;
    float *acc[3] = {acc0, acc1, acc2};
#pragma unroll
    for (int a = 0; a < ND; ++a) {
        bool ok = co[a] >= max(lo[a] - 1, g.nb - 1) && co[a] < min(hi[a], g.nb + g.n[a]);
#pragma unroll
        for (int o = 0; o < ND; ++o)
            if (o != a) ok = ok && co[o] >= lo[o] && co[o] < hi[o];
        if (!ok) continue;
        const float e = dplus<N>(g, p, c, a);
        acc[a][s * g.P + c.k] += q.v[a][s * g.P + c.k] * e;
    }
}

// Secondary source of the tangent-linear step: dp -= dt dkappa div v^{it+1/2} (background v)
// on the interior cells of the forward box.
template <int ND, int N>
__global__ __launch_bounds__(256) void k_born_src(Geom g, Fields f, Fields q,
                                                  const int *__restrict__ box, int shot0, LG lg,
                                                  const float *__restrict__ dkap) {
    Cell c = cell_of(g, box, shot0, lg);
    if (!c.ok) return;
    const int iz = c.z - g.nb, ix = c.x - g.nb, iy = ND == 3 ? c.y - g.nb : 0;
    if ((unsigned)iz >= (unsigned)g.n[0] || (unsigned)ix >= (unsigned)g.n[1] ||
        (unsigned)iy >= (unsigned)g.n[2])
        return;
    const float dk = dkap[iz + (long long)g.n[0] * (ix + (long long)g.n[1] * iy)];
    float div = 0.f;
#pragma unroll
    for (int a = 0; a < ND; ++a) div += dminus<N>(g, f.v[a] + c.s * g.P, c, a);
    q.p[c.s * g.P + c.k] -= g.dt * dk * div;
}

// Gradients of a parametrisation family from A = sum_s acc_g (g_kappa = -(dt/kappa) A) and
// the face sums (g_rho at fixed kappa = -1/2 sum_a sum_s (dt beta S)_{face below} +
// (dt beta S)_{face above}): family 1 (Vp, rho): g1 = 2 rho Vp g_kappa, g2 = Vp^2 g_kappa +
// g_rho; family 2 (Vp, Ip = rho Vp): g1 = rho Vp g_kappa - (rho/Vp) g_rho,
// g2 = Vp g_kappa + g_rho / Vp.  Shots are summed in order.
__global__ __launch_bounds__(256) void k_finalize_family(Geom g, const float *__restrict__ acc_g,
                                                         const float *__restrict__ r0,
                                                         const float *__restrict__ r1,
                                                         const float *__restrict__ r2, Model m,
                                                         int nshot, const float *__restrict__ vp,
                                                         const float *__restrict__ rho,
                                                         int family, float *g1, float *g2) {
    long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= g.I) return;
    const int iz = (int)(i % g.n[0]);
    const long long r = i / g.n[0];
    const int ix = (int)(r % g.n[1]);
    const int iy = (int)(r / g.n[1]);
    const long long k = g.org + (iz + g.nb) + (long long)g.ld1 * (ix + g.nb) +
                        g.ld2 * (g.nd == 3 ? iy + g.nb : 0);
    const float *ra[3] = {r0, r1, r2};
    float A = 0.f, S = 0.f;
    for (int sh = 0; sh < nshot; ++sh) {
        A += acc_g[sh * g.I + i];
        for (int a = 0; a < g.nd; ++a) {
            const long long st = a == 0 ? 1 : (a == 1 ? (long long)g.ld1 : g.ld2);
            S += m.bdt[a][k] * ra[a][sh * g.P + k] + m.bdt[a][k - st] * ra[a][sh * g.P + k - st];
        }
    }
    const float v = vp[i], rh = rho[i];
    const float gk = -g.dt / (rh * v * v) * A;
    const float grk = -0.5f * S;
    if (family == 2) {
        if (g1) g1[i] = rh * v * gk - rh / v * grk;
        if (g2) g2[i] = v * gk + grk / v;
    } else {
        if (g1) g1[i] = 2.f * rh * v * gk;
        if (g2) g2[i] = v * v * gk + grk;
    }
}

// Free surface by the image method (Sec. 2.1): the surface is the first interior row z = nb,
// and the rows above it hold mirror images.  mode 0 (v_z, at half rows): even, row nb-1-k =
// row nb+k for k < N; mode 1 (p): odd, row nb = 0 and row nb-k = -(row nb+k) for k = 1..N;
// mode 2: row nb of p = 0 only.  One lane per column (x, y) of the padded plane, blockIdx.y =
// shot - shot0.  nb >= N keeps every row inside the padded grid.
__global__ __launch_bounds__(256) void k_free_surface(Geom g, float *f, int shot0, int mode) {
    const long long col = (long long)blockIdx.x * 256 + threadIdx.x;
    if (col >= (long long)g.M[1] * g.M[2]) return;
    const int x = (int)(col % g.M[1]), y = (int)(col / g.M[1]);
    float *c = f + (long long)(shot0 + (int)blockIdx.y) * g.P + g.org + g.nb +
               (long long)g.ld1 * x + g.ld2 * y;
    if (mode == 0) {
        for (int k = 0; k < g.N; ++k) c[-1 - k] = c[k];
        return;
    }
    c[0] = 0.f;
    if (mode == 1)
        for (int k = 1; k <= g.N; ++k) c[-k] = -c[k];
}

// interior p of shot shot0 + blockIdx.y -> snaps[s][k][...]
__global__ __launch_bounds__(256) void k_snap(Geom g, const float *__restrict__ p, float *snaps,
                                              int k, int nsnap, int shot0) {
    long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= g.I) return;
    int s = shot0 + (int)blockIdx.y;
    int iz = (int)(i % g.n[0]);
    long long r = i / g.n[0];
    int ix = (int)(r % g.n[1]);
    int iy = (int)(r / g.n[1]);
    long long c = g.org + (iz + g.nb) + (long long)g.ld1 * (ix + g.nb) + g.ld2 * (g.nd == 3 ? iy + g.nb : 0);
    snaps[((long long)s * nsnap + k) * g.I + i] = p[s * g.P + c];
}

unsigned blocks(long long n, int b = 256) { return (unsigned)((n + b - 1) / b); }

#define SMI_TRY(x)                                                                        \
    do {                                                                                  \
        hipError_t e_ = (x);                                                              \
        if (e_ != hipSuccess) return e_;                                                  \
    } while (0)

// mirror images of a free surface over the shots [s0, s1) (nothing without one)
hipError_t fs_launch(const Plan &pl, hipStream_t st, float *f, int mode, int s0, int s1) {
    if (!pl.g.freesurf || s1 <= s0) return hipSuccess;
    hipLaunchKernelGGL(k_free_surface, dim3(blocks((long long)pl.M[1] * pl.M[2]), s1 - s0),
                       dim3(256), 0, st, pl.geom, f, s0, mode);
    return hipGetLastError();
}

// the receivers of the context's shots: a view of the flattened receiver table, in which the
// receivers of a shot are consecutive and follow those of the shot before
Recv group_recv(const StepCtx &c) {
    Recv r = c.w->recv;
    const Plan &pl = *c.pl;
    const int r0 = pl.rec_off[c.s0], r1 = pl.rec_off[shot_end(c)];
    r.R = r1 - r0;
    r.shot += r0;
    r.obase += r0;
    r.stride += r0;
    r.toff += r0;
    return r;
}

// launch geometry of one step over a box table row: max extents over the shots [s0, s1)
struct Launch {
    dim3 grid, block;
    LG ey;
    bool empty;
};

Launch box_launch(const Plan &pl, const std::vector<int> &tab, int it, int s0, int s1,
                  bool xcd) {
    int ez = 0, ex = 0, ey = 0;
    for (int s = s0; s < s1; ++s) {
        const int *b = &tab[((size_t)it * pl.nshot + s) * 6];
        ez = std::max(ez, b[1] - zalign(b[0]));
        ex = std::max(ex, b[3] - b[2]);
        ey = std::max(ey, b[5] - b[4]);
    }
    Launch L;
    L.empty = ez <= 0 || ex <= 0 || ey <= 0;
    const int nzb = std::max(1, (ez + BZ - 1) / BZ), nxb = std::max(1, (ex + BX - 1) / BX);
    const int nxc = xcd ? (nxb + 7) / 8 : 0;
    L.ey = LG{std::max(ey, 1), nxc};
    L.block = dim3(BZ, BX, 1);
    L.grid = dim3((unsigned)(xcd ? 8 * nzb : nzb), (unsigned)(xcd ? nxc : nxb),
                  (unsigned)((s1 - s0) * std::max(ey, 1)));
    return L;
}

// launch geometry of a marching half step over a box table row (max extents over the shots)
struct MLaunch {
    dim3 grid, block;
    MG mg;
    bool empty;
};

MLaunch march_launch(const Plan &pl, const std::vector<int> &tab, int it, int s0, int s1,
                     int cm, bool xcd, bool ymap = false, bool inner = true) {
    int ez = 0, ex = 0, ey = 0;
    for (int s = s0; s < s1; ++s) {
        const int *b = &tab[((size_t)it * pl.nshot + s) * 6];
        ez = std::max(ez, b[1] - zalign(b[0]));
        ex = std::max(ex, b[3] - b[2]);
        ey = std::max(ey, b[5] - b[4]);
    }
    MLaunch L;
    L.empty = ez <= 0 || ex <= 0 || ey <= 0;
    L.block = dim3(64, 4, 1);
    int gz, gx, nm = 1;
    if (pl.nd == 2) {
        gz = std::max(1, (ez + 255) / 256);
        gx = std::max(1, (ex + cm - 1) / cm);
    } else {
        nm = std::max(1, (ey + cm - 1) / cm);
        gz = std::max(1, (ez + 63) / 64);
        gx = std::max(1, (ex + 3) / 4);
    }
    if (pl.nd == 3 && ymap) {
        const int ntile = (s1 - s0) * gz * gx * nm;
        const int per = (ntile + 7) / 8;
        L.mg = MG{nm, 0, gz, gx, per, ntile, 1};
        L.mg.sb = s0;
        L.grid = dim3((unsigned)(8 * per), 1u, 1u);
        return L;
    }
    const int nxc = xcd ? (gx + 7) / 8 : 0;
    L.mg = MG{nm, nxc, 0, 0, 0, 0, 0};
    // several shots with one box (the adjoint pass under a common receiver spread, or the box
    // off): the shot-inner order shares the model of each tile across the shots
    bool same = inner && (pl.nd == 3 || xcd) && s1 - s0 > 1;
    const int *b0 = &tab[((size_t)it * pl.nshot + s0) * 6];
    for (int s = s0 + 1; same && s < s1; ++s)
        same = std::equal(b0, b0 + 6, &tab[((size_t)it * pl.nshot + s) * 6]);
    if (same) L.mg = pl.nd == 2 ? MG{nm, nxc, gz, 0, s1 - s0, 0, 2} : MG{nm, nxc, 0, 0, s1 - s0, 0, 3};
    L.mg.sb = s0;
    L.grid = dim3((unsigned)(xcd ? 8 * gz : gz), (unsigned)(xcd ? nxc : gx), (unsigned)((s1 - s0) * nm));
    return L;
}

}  // namespace

// ---------------------------------------------------------------- host launchers

hipError_t launch_model_prep(const Plan &pl, const Views &w, const float *vp, const float *rho,
                             hipStream_t st) {
    long long tot = pl.P;
    float lo = (float)(pl.vmin * (1.0 - 1e-6)), hi = (float)(pl.vmax * (1.0 + 1e-6));
    hipLaunchKernelGGL(k_model_prep, dim3(blocks(tot)), dim3(256), 0, st, pl.geom, w.model, vp,
                       rho, w.status, lo, hi);
    return hipGetLastError();
}

hipError_t launch_minmax(const float *vp, long long n, unsigned *out2, hipStream_t st) {
    unsigned nb = std::min<unsigned>(blocks(n), 2048u);
    hipLaunchKernelGGL(k_minmax, dim3(nb), dim3(256), 0, st, vp, n, out2);
    return hipGetLastError();
}

namespace {

template <int ND, int N, int CM, bool ZL>
hipError_t fwd_march_t(const StepCtx &c, int it) {
    const Plan &pl = *c.pl;
    const Views &w = *c.w;
    const int *box = w.fbox + (size_t)it * pl.nshot * 6;
    // the forward half steps keep the shot-outer order (the shots' boxes differ while the
    // source fields grow, and the p update is compiled without the shot-inner order)
    const int g0 = c.s0, g1 = shot_end(c), gn = g1 - g0;
    MLaunch L = march_launch(pl, pl.fbox, it, g0, g1, CM, c.xcd, c.ymap, false);
    const Recv rv = group_recv(c);
    const bool ext = c.ext_it >= 0 && rv.R > 0;
    if (L.empty) {
        // nothing to update: the carried work runs on its own
        if (c.save_p_slot >= 0) SMI_TRY(band_save_part(c, w.f, c.save_p_slot, 0));
        if (c.save_v_slot >= 0) SMI_TRY(band_save_part(c, w.f, c.save_v_slot, 1));
        return ext ? extract(c, c.ext_it, c.ext_dcal) : hipSuccess;
    }
    const Ext ex{rv, c.ext_dcal, ext ? c.ext_it : -1, w.status};
    dim3 gv = L.grid;
    if (ext) gv.z += L.mg.nmarch;
    const int s0 = ext ? -1 : 0;
    // bands of the saved levels ride on the half steps: the p cells of level it on the v launch,
    // the v cells of level it + 1 on the p launch (planes after the shots)
    const int nqb = (int)((pl.band.B + 255) / 256);
    auto band_planes = [&](const dim3 &gr) {
        const long long per = (long long)gr.x * gr.y;
        return (unsigned)(((long long)gn * nqb + per - 1) / per);
    };
    const long long sstride = (long long)pl.nsave * pl.band.B;
    BandArg svp{}, svv{};
    int zp = 0, zv = 0;
    if (c.save_p_slot >= 0) {
        svp = BandArg{w.bdesc, w.bands + (size_t)c.save_p_slot * pl.band.B, sstride, nqb, gn, g0};
        zp = (int)gv.z;
        gv.z += band_planes(gv);
    }
    dim3 gp = L.grid;
    if (c.save_v_slot >= 0) {
        svv = BandArg{w.bdesc, w.bands + (size_t)c.save_v_slot * pl.band.B, sstride, nqb, gn, g0};
        zv = (int)gp.z;
        gp.z += band_planes(gp);
    }
    // F: a free surface, whose image rows the kernels write themselves
    auto launch = [&](auto fs) -> hipError_t {
        constexpr bool F = decltype(fs)::value;
        if (c.ev) {
            hipExtLaunchKernelGGL((k_march_v<ND, N, CM, ZL, F>), gv, L.block, 0, c.st, c.ev[0],
                                  c.ev[1], 0, pl.geom, w.f, w.model, w.cpml, box, s0, L.mg, ex, svp,
                                  zp);
            hipExtLaunchKernelGGL((k_march_p<ND, N, CM, ZL, true, false, F>), gp, L.block, 0, c.st,
                                  c.ev[2], c.ev[3], 0, pl.geom, w.f, w.model, w.cpml, box, 0, L.mg,
                                  (const long long *)w.src_cell, c.stf, pl.g.nt, it,
                                  (const float *)nullptr, (float *)nullptr, svv, zv);
            return hipGetLastError();
        }
        hipLaunchKernelGGL((k_march_v<ND, N, CM, ZL, F>), gv, L.block, 0, c.st, pl.geom, w.f,
                           w.model, w.cpml, box, s0, L.mg, ex, svp, zp);
        hipLaunchKernelGGL((k_march_p<ND, N, CM, ZL, true, false, F>), gp, L.block, 0, c.st,
                           pl.geom, w.f, w.model, w.cpml, box, 0, L.mg,
                           (const long long *)w.src_cell, c.stf, pl.g.nt, it,
                           (const float *)nullptr, (float *)nullptr, svv, zv);
        return hipGetLastError();
    };
    return pl.g.freesurf ? launch(std::true_type{}) : launch(std::false_type{});
}

// adjoint half steps with the marching kernels (image with the source field when asked)
template <int ND, int N, int CM, bool ZL>
hipError_t adj_march_t(const StepCtx &c, int it, bool image) {
    const Plan &pl = *c.pl;
    const Views &w = *c.w;
    const int *ab = w.abox + (size_t)it * pl.nshot * 6;
    const int s0 = c.s0, s1 = shot_end(c);
    MLaunch L = march_launch(pl, pl.abox, it, s0, s1, CM, c.xcd, c.ymap);
    if (L.empty) return hipSuccess;
    auto launch = [&](auto fs) -> hipError_t {
        constexpr bool F = decltype(fs)::value;
        hipLaunchKernelGGL((k_march_v<ND, N, CM, ZL, F>), L.grid, L.block, 0, c.st, pl.geom, w.q,
                           w.model, w.cpml, ab, 0, L.mg, Ext{w.recv, nullptr, -1, nullptr},
                           BandArg{}, 0);
        if (image)
            hipLaunchKernelGGL((k_march_p<ND, N, CM, ZL, false, true, F>), L.grid, L.block, 0, c.st,
                               pl.geom, w.q, w.model, w.cpml, ab, 0, L.mg,
                               (const long long *)w.src_cell, c.stf, pl.g.nt, it,
                               (const float *)w.f.p, w.acc_i, BandArg{}, 0);
        else
            hipLaunchKernelGGL((k_march_p<ND, N, CM, ZL, false, false, F>), L.grid, L.block, 0,
                               c.st, pl.geom, w.q, w.model, w.cpml, ab, 0, L.mg,
                               (const long long *)w.src_cell, c.stf, pl.g.nt, it,
                               (const float *)w.f.p, w.acc_i, BandArg{}, 0);
        return hipGetLastError();
    };
    return pl.g.freesurf ? launch(std::true_type{}) : launch(std::false_type{});
}

template <int ND, int N>
hipError_t fwd_step_t(const StepCtx &c, int it) {
    const Plan &pl = *c.pl;
    const Views &w = *c.w;
#define SMI_MARCH(fn, ...)                                                                      \
    do {                                                                                        \
        if (c.march == 2) return c.zl ? fn<ND, N, 2, true>(__VA_ARGS__) : fn<ND, N, 2, false>(__VA_ARGS__); \
        if (c.march == 8) return c.zl ? fn<ND, N, 8, true>(__VA_ARGS__) : fn<ND, N, 8, false>(__VA_ARGS__); \
        return c.zl ? fn<ND, N, 4, true>(__VA_ARGS__) : fn<ND, N, 4, false>(__VA_ARGS__);          \
    } while (0)
    if (!c.plain && c.yp && ND == 3) return fwd_step_yp(c, it);
    if (!c.plain && c.y3 && ND == 3) return fwd_step_y3(c, it);
    if (!c.plain && c.march) SMI_MARCH(fwd_march_t, c, it);
    const int *box = w.fbox + (size_t)it * pl.nshot * 6;
    int step = c.plain ? 1 : pl.nshot;
    for (int s0 = 0; s0 < pl.nshot; s0 += step) {
        int s1 = std::min(pl.nshot, s0 + step);
        Launch L = box_launch(pl, pl.fbox, it, s0, s1, c.xcd);
        if (L.empty) continue;
        if (c.ev && step == pl.nshot) {
            // timed step: the device stamps the events at each kernel's start and end
            hipExtLaunchKernelGGL((k_step_v<ND, N>), L.grid, L.block, 0, c.st, c.ev[0], c.ev[1],
                                  0, pl.geom, w.f, w.model, w.cpml, box, s0, L.ey);
            SMI_TRY(fs_launch(pl, c.st, w.f.v[0], 0, s0, s1));
            hipExtLaunchKernelGGL((k_step_p<ND, N, true, false>), L.grid, L.block, 0, c.st,
                                  c.ev[2], c.ev[3], 0, pl.geom, w.f, w.model, w.cpml, box, s0,
                                  L.ey, (const long long *)w.src_cell, c.stf, pl.g.nt, it,
                                  (const float *)nullptr, (float *)nullptr);
            SMI_TRY(fs_launch(pl, c.st, w.f.p, 1, s0, s1));
            continue;
        }
        hipLaunchKernelGGL((k_step_v<ND, N>), L.grid, L.block, 0, c.st, pl.geom, w.f, w.model,
                           w.cpml, box, s0, L.ey);
        SMI_TRY(fs_launch(pl, c.st, w.f.v[0], 0, s0, s1));
        hipLaunchKernelGGL((k_step_p<ND, N, true, false>), L.grid, L.block, 0, c.st, pl.geom,
                           w.f, w.model, w.cpml, box, s0, L.ey, (const long long *)w.src_cell,
                           c.stf, pl.g.nt, it, (const float *)nullptr, (float *)nullptr);
        SMI_TRY(fs_launch(pl, c.st, w.f.p, 1, s0, s1));
    }
    return hipGetLastError();
}

// reconstruction half steps with the register-blocked kernels (region: rbox row it)
template <int ND, int N, int CM, bool ZL>
hipError_t recon_march_t(const StepCtx &c, int it, bool grad, bool image) {
    const Plan &pl = *c.pl;
    const Views &w = *c.w;
    const int *rb = w.rbox + (size_t)it * pl.nshot * 6;
    MLaunch L = march_launch(pl, pl.rbox, it, c.s0, shot_end(c), CM, c.xcd, c.ymap);
    if (!L.empty) {
#define SMI_MRECON_P(G_, L_)                                                                   \
    hipLaunchKernelGGL((k_march_recon_p<ND, N, CM, ZL, G_, L_>), L.grid, L.block, 0, c.st, pl.geom, \
                       w.f, w.model, rb, 0, L.mg, (const long long *)w.src_cell, c.stf,         \
                       pl.g.nt, it, (const float *)w.q.p, w.acc_g, w.acc_l)
        if (grad && image) SMI_MRECON_P(true, true);
        else if (grad) SMI_MRECON_P(true, false);
        else if (image) SMI_MRECON_P(false, true);
        else SMI_MRECON_P(false, false);
#undef SMI_MRECON_P
    }
    // p and v bands of level it in one launch: the v reconstruction reads the p bands and
    // neither reads nor writes the v band cells (they lie outside the interior)
    hipError_t e = band_restore(c, it, 2);
    if (e != hipSuccess) return e;
    if (!L.empty)
        hipLaunchKernelGGL((k_march_recon_v<ND, N, CM, ZL>), L.grid, L.block, 0, c.st, pl.geom, w.f,
                           w.model, rb, 0, L.mg);
    return hipGetLastError();
}

// the two-launch reverse step of the 2D default path (see k_rev_pv); G: the adjoint sources
// of level it - 1 join the second launch (k_rev_vp with INJ), or null
template <int N>
hipError_t rev_pair_t(const StepCtx &c, int it, bool grad, bool image, const float *G) {
    constexpr int CM = 4;
    const Plan &pl = *c.pl;
    const Views &w = *c.w;
    const int *rb = w.rbox + (size_t)it * pl.nshot * 6;
    const int *ab = w.abox + (size_t)it * pl.nshot * 6;
    const int s0 = c.s0, s1 = shot_end(c), ns = s1 - s0;
    const MLaunch LR = march_launch(pl, pl.rbox, it, s0, s1, CM, c.xcd);
    const MLaunch LA = march_launch(pl, pl.abox, it, s0, s1, CM, c.xcd);
    const bool band = pl.g.dr == 1;
    const BandArg ba{w.bdesc, w.bands + (size_t)it * pl.band.B, (long long)pl.nsave * pl.band.B,
                     (int)((pl.band.B + 255) / 256), ns, s0};
    dim3 grid(std::max(LR.grid.x, LA.grid.x), std::max(LR.grid.y, LA.grid.y), 2u * ns);
    if (band) {
        const long long per = (long long)grid.x * grid.y;
        grid.z += (unsigned)(((long long)ns * ba.nqb + per - 1) / per);
    }
    const dim3 block(64, 4, 1);
    // F: a free surface, whose image rows the adjoint half steps write themselves
    auto first = [&](auto fs) {
        constexpr bool F = decltype(fs)::value;
#define SMI_RPV(G_, L_, B_)                                                                    \
    hipLaunchKernelGGL((k_rev_pv<N, CM, G_, L_, B_, F>), grid, block, 0, c.st, pl.geom, w.f, w.q, \
                       w.model, w.cpml, rb, ab, LR.mg, LA.mg, ns,                               \
                       (const long long *)w.src_cell, c.stf, pl.g.nt, it, w.acc_g, w.acc_l, ba)
#define SMI_RPV_B(G_, L_) do { if (band) SMI_RPV(G_, L_, true); else SMI_RPV(G_, L_, false); } while (0)
        if (grad && image) SMI_RPV_B(true, true);
        else if (grad) SMI_RPV_B(true, false);
        else if (image) SMI_RPV_B(false, true);
        else SMI_RPV_B(false, false);
#undef SMI_RPV_B
#undef SMI_RPV
    };
    if (pl.g.freesurf) first(std::true_type{});
    else first(std::false_type{});
    if (!band) SMI_TRY(band_restore(c, it, 2));      // interpolated levels: one launch of their own
    InjArg ia{};
    if (G) {
        ia = InjArg{w.injmap, pl.inj_zlo, pl.inj_nrow, pl.M[1], w.inj.off, w.inj.rec, w.inj.w,
                    w.recv.obase, w.recv.stride, G, it - 1, (float)(1.0 / pl.g.dt)};
    }
    auto second = [&](auto fs) {
        constexpr bool F = decltype(fs)::value;
#define SMI_RVP(I_, B_, J_)                                                                    \
    hipLaunchKernelGGL((k_rev_vp<N, CM, I_, B_, J_, F>), grid, block, 0, c.st, pl.geom, w.f, w.q, \
                       w.model, w.cpml, rb, ab, LR.mg, LA.mg, ns,                               \
                       (const long long *)w.src_cell, c.stf, pl.g.nt, it, w.acc_i, ba, ia)
#define SMI_RVP_J(I_, B_) do { if (G) SMI_RVP(I_, B_, true); else SMI_RVP(I_, B_, false); } while (0)
        if (image) { if (band) SMI_RVP_J(true, true); else SMI_RVP_J(true, false); }
        else { if (band) SMI_RVP_J(false, true); else SMI_RVP_J(false, false); }
#undef SMI_RVP_J
#undef SMI_RVP
    };
    if (pl.g.freesurf) second(std::true_type{});
    else second(std::false_type{});
    return hipGetLastError();
}

template <int ND, int N>
hipError_t rev_step_t(const StepCtx &c, int it, bool grad, bool image, const float *Gn,
                      bool *fused) {
    const Plan &pl = *c.pl;
    const Views &w = *c.w;
    // Launches over up to 8 M padded cells (the shots of the reverse loop's group) take the
    // two-launch step (10 % faster on 8 shots of 300 x 900, 30 % less host time on one);
    // above, where the host keeps ahead and the two orders measure the same, the five-launch
    // order keeps consecutive kernels on one field.
    constexpr double kPairCells = 8.0e6;
    const int sa = c.s0, se = shot_end(c);
    if constexpr (ND == 2) {
        const bool small = (double)(se - sa) * (double)pl.P <= kPairCells;
        if (!c.plain && c.march == 4 && !c.zl && (c.rev == 1 || (c.rev == 0 && small))) {
            const bool inj = Gn && it > 0 && pl.inj_fused;
            if (fused) *fused = inj;
            return rev_pair_t<N>(c, it, grad, image, inj ? Gn : nullptr);
        }
    }
    if (!c.plain && c.march) {
        auto recon = [&]() -> hipError_t { SMI_MARCH(recon_march_t, c, it, grad, image); };
        hipError_t e = recon();
        if (e != hipSuccess) return e;
        if (c.yp && ND == 3) return adj_step_yp(c, it, image);
        if (c.y3 && ND == 3) return adj_step_y3(c, it, image);
        SMI_MARCH(adj_march_t, c, it, image);
    }
    const int *rb = w.rbox + (size_t)it * pl.nshot * 6;
    const int *ab = w.abox + (size_t)it * pl.nshot * 6;
    const int step = c.plain ? 1 : se - sa;
    // source field: p^{it} (with the gradient read of p~ before the adjoint step)
    for (int s0 = sa; s0 < se; s0 += step) {
        int s1 = std::min(se, s0 + step);
        Launch L = box_launch(pl, pl.rbox, it, s0, s1, c.xcd);
        if (L.empty) continue;
#define SMI_RECON_P(G_, L_)                                                                    \
    hipLaunchKernelGGL((k_recon_p<ND, N, G_, L_>), L.grid, L.block, 0, c.st, pl.geom, w.f,      \
                       w.model, rb, s0, L.ey, (const long long *)w.src_cell, c.stf, pl.g.nt, it, \
                       (const float *)w.q.p, w.acc_g, w.acc_l)
        if (grad && image) SMI_RECON_P(true, true);
        else if (grad) SMI_RECON_P(true, false);
        else if (image) SMI_RECON_P(false, true);
        else SMI_RECON_P(false, false);
#undef SMI_RECON_P
    }
    hipError_t e = band_restore(c, it, 0);
    if (e != hipSuccess) return e;
    for (int s0 = sa; s0 < se; s0 += step) {
        int s1 = std::min(se, s0 + step);
        Launch L = box_launch(pl, pl.rbox, it, s0, s1, c.xcd);
        if (L.empty) continue;
        hipLaunchKernelGGL((k_recon_v<ND, N>), L.grid, L.block, 0, c.st, pl.geom, w.f, w.model,
                           rb, s0, L.ey);
    }
    e = band_restore(c, it, 1);
    if (e != hipSuccess) return e;
    // adjoint field: one step of the same solver (eq. 8), image with p^{it}
    for (int s0 = sa; s0 < se; s0 += step) {
        int s1 = std::min(se, s0 + step);
        Launch L = box_launch(pl, pl.abox, it, s0, s1, c.xcd);
        if (L.empty) continue;
        hipLaunchKernelGGL((k_step_v<ND, N>), L.grid, L.block, 0, c.st, pl.geom, w.q, w.model,
                           w.cpml, ab, s0, L.ey);
        SMI_TRY(fs_launch(pl, c.st, w.q.v[0], 0, s0, s1));
        if (image)
            hipLaunchKernelGGL((k_step_p<ND, N, false, true>), L.grid, L.block, 0, c.st, pl.geom,
                               w.q, w.model, w.cpml, ab, s0, L.ey, (const long long *)w.src_cell,
                               c.stf, pl.g.nt, it, (const float *)w.f.p, w.acc_i);
        else
            hipLaunchKernelGGL((k_step_p<ND, N, false, false>), L.grid, L.block, 0, c.st,
                               pl.geom, w.q, w.model, w.cpml, ab, s0, L.ey,
                               (const long long *)w.src_cell, c.stf, pl.g.nt, it,
                               (const float *)w.f.p, w.acc_i);
        SMI_TRY(fs_launch(pl, c.st, w.q.p, 1, s0, s1));
    }
    return hipGetLastError();
}

}  // namespace

#define SMI_DISPATCH(fn, ...)                                                    \
    do {                                                                         \
        const Plan &pl_ = *c.pl;                                                 \
        if (pl_.nd == 2 && pl_.N == 2) return fn<2, 2>(__VA_ARGS__);             \
        if (pl_.nd == 2 && pl_.N == 4) return fn<2, 4>(__VA_ARGS__);             \
        if (pl_.nd == 3 && pl_.N == 2) return fn<3, 2>(__VA_ARGS__);             \
        if (pl_.nd == 3 && pl_.N == 4) return fn<3, 4>(__VA_ARGS__);             \
        return hipErrorInvalidValue;                                             \
    } while (0)

hipError_t fwd_step(const StepCtx &c, int it) { SMI_DISPATCH(fwd_step_t, c, it); }

bool march_forward(const StepCtx &c) {
    // (the XCD-contiguous 3D order uses a one-dimensional grid: no planes to carry other work)
    return !c.plain && c.march && !((c.y3 || c.yp) && c.pl->nd == 3) && !c.ymap;
}

hipError_t rev_step(const StepCtx &c, int it, bool grad, bool image, const float *Gn,
                    bool *fused) {
    if (fused) *fused = false;
    SMI_DISPATCH(rev_step_t, c, it, grad, image, Gn, fused);
}

hipError_t extract(const StepCtx &c, int it, float *dcal, const float *p) {
    const Views &w = *c.w;
    const Recv rv = group_recv(c);
    if (rv.R == 0) return hipSuccess;
    hipLaunchKernelGGL(k_extract, dim3(blocks(rv.R)), dim3(256), 0, c.st, c.pl->geom,
                       p ? p : (const float *)w.f.p, rv, dcal, it, w.status);
    return hipGetLastError();
}

hipError_t src_taps(const StepCtx &c, int it, float *p, float sign) {
    const Plan &pl = *c.pl;
    if (!pl.src_multi) return hipSuccess;
    const Views &w = *c.w;
    const int s0 = c.s0, s1 = shot_end(c);
    int most = 0;
    for (int s = s0; s < s1; ++s) most = std::max(most, pl.src_toff[s + 1] - pl.src_toff[s]);
    if (most == 0) return hipSuccess;
    hipLaunchKernelGGL(k_src_taps, dim3(blocks(most), s1 - s0), dim3(256), 0, c.st, pl.geom, p,
                       (const long long *)w.src_cell, (const int *)w.src_toff,
                       (const long long *)w.src_tcell, (const float *)w.src_tw, c.stf, pl.g.nt,
                       it, sign, s0);
    // an injection on a free-surface grid is followed by the images of what it added (the
    // removal in the reconstruction is not: the rows above the surface come from the bands)
    if (sign > 0.f) SMI_TRY(fs_launch(pl, c.st, p, 1, s0, s1));
    return hipGetLastError();
}

hipError_t band_save_part(const StepCtx &c, const Fields &f, int slot, int which) {
    const Plan &pl = *c.pl;
    const Views &w = *c.w;
    long long ss = (long long)pl.nsave * pl.band.B;
    hipLaunchKernelGGL(k_band, dim3(blocks(pl.band.B), shot_end(c) - c.s0), dim3(256), 0, c.st,
                       pl.geom, f, pl.band, w.bands + (size_t)slot * pl.band.B,
                       (const float *)nullptr, ss, c.s0, 0, which, 0.f);
    return hipGetLastError();
}

hipError_t band_save(const StepCtx &c, const Fields &f, int slot) {
    const Plan &pl = *c.pl;
    const Views &w = *c.w;
    long long ss = (long long)pl.nsave * pl.band.B;
    hipLaunchKernelGGL(k_band, dim3(blocks(pl.band.B), shot_end(c) - c.s0), dim3(256), 0, c.st,
                       pl.geom, f, pl.band, w.bands + (size_t)slot * pl.band.B,
                       (const float *)nullptr, ss, c.s0, 0, 2, 0.f);
    return hipGetLastError();
}

// Kaiser-windowed sinc of half-width kTaps levels (u in saved levels)
static double ksinc(double u) {
    if (std::fabs(u) >= kTaps) return 0.0;
    auto i0 = [](double x) {
        double s = 1.0, t = 1.0;
        for (int k = 1; k < 60; ++k) {
            t *= (x / (2.0 * k)) * (x / (2.0 * k));
            s += t;
            if (t < 1e-17 * s) break;
        }
        return s;
    };
    double x = u / kTaps;
    double win = i0(kKaiserBeta * std::sqrt(1.0 - x * x)) / i0(kKaiserBeta);
    return (u == 0.0 ? 1.0 : std::sin(M_PI * u) / (M_PI * u)) * win;
}

// Bands at level it (p^it and v^{it-1/2}): the saved level itself when it is one (dr = 1 or
// it % dr == 0); otherwise a Kaiser-windowed sinc in time over the 2 kTaps saved levels
// around it, weights normalised to sum 1, levels before 0 being zero (field at rest).
hipError_t band_restore(const StepCtx &c, int it, int which) {
    const Plan &pl = *c.pl;
    const Views &w = *c.w;
    long long ss = (long long)pl.nsave * pl.band.B;
    const int dr = pl.g.dr;
    const int k0 = it / dr;
    const int s0 = c.s0, ns = shot_end(c) - c.s0;
    if (it % dr == 0) {
        hipLaunchKernelGGL(k_band, dim3(blocks(pl.band.B), ns), dim3(256), 0, c.st,
                           pl.geom, w.f, pl.band, w.bands + (size_t)k0 * pl.band.B,
                           (const float *)nullptr, ss, s0, 1, which, 0.f);
        return hipGetLastError();
    }
    Taps tp{};
    const double u = (double)it / dr;
    double ws = 0.0, wk[2 * kTaps];
    int sl[2 * kTaps], n = 0;
    for (int k = k0 - kTaps + 1; k <= k0 + kTaps; ++k) {
        const double wt = ksinc(u - k);
        ws += wt;
        if (k < 0) continue;
        sl[n] = k;
        wk[n++] = wt;
    }
    tp.n = n;
    for (int j = 0; j < n; ++j) { tp.slot[j] = sl[j]; tp.w[j] = (float)(wk[j] / ws); }
    hipLaunchKernelGGL(k_band_mix, dim3(blocks(pl.band.B), ns), dim3(256), 0, c.st,
                       pl.geom, w.f, pl.band, (const float *)w.bands, ss, s0, tp, which);
    return hipGetLastError();
}

hipError_t scale_copy(const StepCtx &c, const float *in, float *out, float a) {
    const Plan &pl = *c.pl;
    long long n = (long long)pl.g.nt * pl.rec_off[pl.nshot];
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scale, dim3(blocks(n)), dim3(256), 0, c.st, in, out, n, a);
    return hipGetLastError();
}

hipError_t snap(const StepCtx &c, const Fields &f, float *snaps, int k, int nsnap) {
    const Plan &pl = *c.pl;
    hipLaunchKernelGGL(k_snap, dim3(blocks(pl.I), shot_end(c) - c.s0), dim3(256), 0, c.st,
                       pl.geom, (const float *)f.p, snaps, k, nsnap, c.s0);
    return hipGetLastError();
}

hipError_t adj_inject(const StepCtx &c, int it, const float *G) {
    const Views &w = *c.w;
    if (w.inj.U == 0) return hipSuccess;
    const int s0 = c.s0, s1 = shot_end(c);
    hipLaunchKernelGGL(k_inject, dim3(blocks(w.inj.U)), dim3(256), 0, c.st, c.pl->geom, w.q.p,
                       (const float *)w.model.kdt, w.recv, w.inj, G, it, (float)(1.0 / c.pl->g.dt),
                       s0, s1);
    // the injected adjoint sources get their images too (the transpose of the sampling of a
    // mirrored field)
    SMI_TRY(fs_launch(*c.pl, c.st, w.q.p, 1, s0, s1));
    return hipGetLastError();
}

hipError_t residual(const StepCtx &c, const float *dcal, const float *dobs, float *G,
                    double *misfit, int s0, int s1) {
    const Plan &pl = *c.pl;
    const Views &w = *c.w;
    const long long o = (long long)pl.g.nt * pl.rec_off[s0];
    const long long n = (long long)pl.g.nt * pl.rec_off[s1] - o;
    hipLaunchKernelGGL(k_residual, dim3(pl.npartial), dim3(256), 0, c.st, dcal + o, dobs + o,
                       G + o, n, (float)pl.g.dt, w.partial);
    hipLaunchKernelGGL(k_sum_partial, dim3(1), dim3(256), 0, c.st, (const double *)w.partial,
                       pl.npartial, misfit ? misfit : w.misfit_tmp, 0.5 * pl.g.dt);
    return hipGetLastError();
}

template <int ND, int N>
hipError_t rho_faces_t(const StepCtx &c, int it) {
    const Plan &pl = *c.pl;
    const Views &w = *c.w;
    const int s0 = c.s0, s1 = shot_end(c);
    int ez = 0, ex = 0, ey = 0;
    for (int s = s0; s < s1; ++s) {
        const int *b = &pl.rbox[((size_t)it * pl.nshot + s) * 6];
        ez = std::max(ez, b[1] - b[0] + 1);
        ex = std::max(ex, b[3] - b[2] + 1);
        ey = std::max(ey, ND == 3 ? b[5] - b[4] + 1 : 1);
    }
    const int ny = std::max(1, ey);
    dim3 grid((unsigned)((ez + 63) / 64), (unsigned)((ex + 3) / 4), (unsigned)((s1 - s0) * ny));
    hipLaunchKernelGGL((k_rho_faces<ND, N>), grid, dim3(64, 4, 1), 0, c.st, pl.geom, w.f, w.q,
                       w.acc_r[0], w.acc_r[1], w.acc_r[2],
                       (const int *)(w.rbox + (size_t)it * pl.nshot * 6), ny, s0);
    return hipGetLastError();
}

hipError_t rho_faces(const StepCtx &c, int it) { SMI_DISPATCH(rho_faces_t, c, it); }

template <int ND, int N>
hipError_t born_step_t(const StepCtx &c, int it, const float *dkappa) {
    const Plan &pl = *c.pl;
    const Views &w = *c.w;
    const int *box = w.fbox + (size_t)it * pl.nshot * 6;
    Launch L = box_launch(pl, pl.fbox, it, 0, pl.nshot, c.xcd);
    if (L.empty) return hipSuccess;
    hipLaunchKernelGGL((k_step_v<ND, N>), L.grid, L.block, 0, c.st, pl.geom, w.q, w.model,
                       w.cpml, box, 0, L.ey);
    SMI_TRY(fs_launch(pl, c.st, w.q.v[0], 0, 0, pl.nshot));
    hipLaunchKernelGGL((k_step_p<ND, N, false, false>), L.grid, L.block, 0, c.st, pl.geom, w.q,
                       w.model, w.cpml, box, 0, L.ey, (const long long *)w.src_cell, c.stf,
                       pl.g.nt, it, (const float *)nullptr, (float *)nullptr);
    hipLaunchKernelGGL((k_born_src<ND, N>), L.grid, L.block, 0, c.st, pl.geom, w.f, w.q, box, 0,
                       L.ey, dkappa);
    hipError_t e = hipGetLastError();
    return e != hipSuccess ? e : fs_launch(pl, c.st, w.q.p, 1, 0, pl.nshot);
}

hipError_t born_step(const StepCtx &c, int it, const float *dkappa) {
    SMI_DISPATCH(born_step_t, c, it, dkappa);
}

hipError_t finalize_family(const StepCtx &c, const float *vp, const float *rho, int family,
                           float *g1, float *g2, int s0, int s1) {
    const Plan &pl = *c.pl;
    const Views &w = *c.w;
    auto rs = [&](int a) -> const float * { return w.acc_r[a] ? w.acc_r[a] + (size_t)s0 * pl.P : nullptr; };
    hipLaunchKernelGGL(k_finalize_family, dim3(blocks(pl.I)), dim3(256), 0, c.st, pl.geom,
                       (const float *)(w.acc_g + (size_t)s0 * pl.I), rs(0), rs(1), rs(2), w.model,
                       s1 - s0, vp, rho, family, g1, g2);
    return hipGetLastError();
}

hipError_t launch_laplacian(const smi_grid *g, const float *in, float *out, hipStream_t st) {
    const int n3 = g->ndim == 3 ? g->n3 : 1;
    const long long tot = (long long)g->n1 * g->n2 * n3;
    const float w1 = 1.f / (g->d1 * g->d1), w2 = 1.f / (g->d2 * g->d2);
    const float w3 = g->ndim == 3 ? 1.f / (g->d3 * g->d3) : 0.f;
    hipLaunchKernelGGL(k_laplacian, dim3(blocks(tot)), dim3(256), 0, st, in, out, g->n1, g->n2, n3,
                       w1, w2, w3);
    return hipGetLastError();
}

// stabiliser of the normalised image, as a fraction of each shot's peak illumination
constexpr float kNormEps = 1e-3f;

hipError_t finalize(const StepCtx &c, const float *vp, float *grad, float *image, float *illum,
                    float *image_norm, int s0, int s1) {
    const Plan &pl = *c.pl;
    const Views &w = *c.w;
    const int ns = s1 - s0;
    const size_t o = (size_t)s0 * pl.I;
    if (image_norm) {
        unsigned *mx = (unsigned *)w.partial;
        hipLaunchKernelGGL(k_fill_u32, dim3(blocks(ns)), dim3(256), 0, c.st, mx, ns, 0u);
        hipLaunchKernelGGL(k_shot_max, dim3(std::min<unsigned>(blocks(pl.I), 1024u), ns),
                           dim3(256), 0, c.st, (const float *)(w.acc_l + o), pl.I, mx);
        hipLaunchKernelGGL(k_finalize_norm, dim3(blocks(pl.I)), dim3(256), 0, c.st,
                           (const float *)(w.acc_i + o), (const float *)(w.acc_l + o), ns, pl.I,
                           (const unsigned *)mx, kNormEps, image_norm);
    }
    if (grad)
        hipLaunchKernelGGL(k_finalize_grad, dim3(blocks(pl.I)), dim3(256), 0, c.st,
                           (const float *)(w.acc_g + o), ns, pl.I, vp, (float)pl.g.dt, grad);
    if (image)
        hipLaunchKernelGGL(k_finalize_sum, dim3(blocks(pl.I)), dim3(256), 0, c.st,
                           (const float *)(w.acc_i + o), ns, pl.I, image);
    if (illum)
        hipLaunchKernelGGL(k_finalize_sum, dim3(blocks(pl.I)), dim3(256), 0, c.st,
                           (const float *)(w.acc_l + o), ns, pl.I, illum);
    return hipGetLastError();
}

}  // namespace smi
