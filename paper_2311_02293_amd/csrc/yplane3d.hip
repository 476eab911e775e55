// yplane3d.hip -- 3D half steps (eq. 3-4 with CPML, Sec. 2.1) on plane tiles marching along y.
//
// A workgroup of NWX wavefronts owns a tile of 64 z-rows x TX = CX NWX x-columns of one shot
// and walks CY consecutive y-planes.  A lane is one z-row and updates CX consecutive
// x-columns (the wavefront's columns), so per plane and cell:
//   * the y-stencil comes from a register queue of 2N planes per column, one load per plane;
//   * the z- and x-stencils read the plane from LDS, where the workgroup stages it once:
//     the tile's own values (taken from the queue, not loaded again) and a halo of N rows
//     above and below and N columns either side (the corners are never read), loaded by the
//     whole workgroup;
//   * the x-stencil of the lane's CX columns slides over one row of LDS (CX + 2N - 1 reads);
//   * every other operand (the old velocity or pressure, the model, the memory variables
//     of the slabs, the image terms) is one load per cell.
// Every load of plane y + 2 is issued before the arithmetic of plane y, and none sits under a
// branch: a value a lane does not need is read at an offset past the end of its buffer
// resource, which returns 0 without touching memory (the memory variables outside the slabs,
// the halo values a thread does not own), so no load is waited for before the plane that uses
// it.  The LDS plane is double-buffered: one workgroup barrier per plane orders the staging of
// plane y + 1 after every read of plane y - 1.  Addresses are 32-bit byte offsets into one
// buffer resource per array and shot: the plane as the uniform offset, the row and column as
// the lane's offset; rows and columns past the grid's storage are clamped -- their values
// reach only cells that are not stored.  The arithmetic, the order of the terms and the box
// rules (a cell outside the shot's computing box is neither updated nor written) are those of
// the register-blocked half-step kernels; the fields agree with theirs to rounding (the
// compiler contracts the memory-variable update b psi + a e on one product or the other
// depending on where its coefficients come from: differences of 1e-12 of the field's peak).
#include <algorithm>

#include <hip/hip_ext.h>

#include "smi_internal.hpp"
#include "device.hpp"

namespace smi {

namespace {

constexpr int kZB = 16;              // row bias of the lane offsets (rows >= -12 stay >= 0)
constexpr unsigned kOOB = 0x80000000u;   // a lane offset past every resource: reads 0

template <int N, int CX, int NWX>
struct YPT {
    static constexpr int TX = CX * NWX;       // x-columns of a tile
    static constexpr int NT = 64 * NWX;       // threads
    static constexpr int LR = 64 + 2 * N;     // LDS rows per column (z-halo N each side)
    static constexpr int LC = TX + 2 * N;     // LDS columns (x-halo N each side)
    static constexpr int NHZ = 2 * N * TX;    // z-halo values of a plane
    static constexpr int HZT = (NHZ + NT - 1) / NT;   // of them per thread
    static_assert(NWX >= 2 * N, "one wavefront per x-halo column");
};

struct YPMap {
    int nshot, nstrip, nxt, nzt, ntile;
};

struct YPTile {
    int s, z0, x0, ylo, yhi;
    bool live;
};

template <int TX>
__device__ __forceinline__ YPTile yp_tile(const int *__restrict__ box, const YPMap &mp, int cy) {
    YPTile t;
    // tiles in XCD-contiguous ranges, z-tile fastest, then x-tile, y-strip and shot: the
    // workgroups resident on one XCD at a time cover a block of neighbouring tiles of one strip,
    // so the halo rows and columns one reads are the planes its neighbours read as well, from
    // the same L2
    const int L = xcd_remap((int)blockIdx.x, mp.ntile);
    const int zt = L % mp.nzt;
    int r = L / mp.nzt;
    const int xt = r % mp.nxt;
    r /= mp.nxt;
    const int strip = r % mp.nstrip;
    t.s = r / mp.nstrip;
    const int *b = box + 6 * t.s;
    t.z0 = zalign(b[0]) + 64 * zt;
    t.x0 = b[2] + TX * xt;
    t.ylo = b[4] + cy * strip;
    t.yhi = min(t.ylo + cy, b[5]);
    t.live = t.ylo < t.yhi && t.z0 < b[1] && t.x0 < b[3] && b[1] > b[0];
    return t;
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const float *p, long long n) {
    return __builtin_amdgcn_make_buffer_rsrc((void *)p, (short)0, (int)(4 * n), 0x00020000);
}
__device__ __forceinline__ float bl(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
}
__device__ __forceinline__ void bs(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, vo, so, 0);
}

// Addressing of one tile: byte offset of node (z, x, y) of a field or model array =
// lane(z, x) + plane(y), lane(z, x) = 4 (z + kZB) + 4 ld1 (x - xb) with z and x clamped to the
// stored rows and columns, plane(y) = 4 (org - kZB + ld1 xb + ld2 y), xb = x0 - N.  Both parts
// are non-negative for every node a tile touches (z >= -12, x >= xb >= -4, y >= -4, and the
// ghost frame puts org at 8 (1 + ld1 + ld2)).
struct YPAddr {
    int zmax, xmax, xb;
    unsigned c1, c2, p0;
    __device__ __forceinline__ unsigned lane(int z, int x) const {
        return 4u * (unsigned)(min(z, zmax) + kZB) + c1 * (unsigned)(min(x, xmax) - xb);
    }
    __device__ __forceinline__ unsigned plane(int y) const { return p0 + c2 * (unsigned)y; }
};

__device__ __forceinline__ YPAddr yp_addr(const Geom &g, int x0, int N) {
    YPAddr a;
    a.zmax = g.ld1 - GH - 1;
    a.xmax = g.M[1] + GH - 1;
    a.xb = x0 - N;
    a.c1 = 4u * (unsigned)g.ld1;
    a.c2 = 4u * (unsigned)g.ld2;
    a.p0 = (unsigned)(4LL * ((long long)g.org - kZB + (long long)g.ld1 * a.xb));
    return a;
}

// The memory variables of a tile (one slab array per axis and shot): offset of the value of
// node (z, x, y) = lane + plane; lanes outside an axis' slab (or outside the grid) get kOOB.
//   z slab: zc + W (x + M1 y);  x slab: z + ld1 (xc + W y);  y slab: z + ld1 (x + M1 yc)
template <int CX>
struct YPSlab {
    unsigned oz[CX], ox[CX], oy[CX];
    int zsl, xsl[CX];
    unsigned pz, px, py;    // bytes per plane of the z and x slab arrays, per slab plane of y
    __device__ __forceinline__ void init(const Geom &g, int z, int xs) {
        const bool zin = z >= 0 && z < g.M[0];
        zsl = zin ? slab_index(z, g.M[0], g.nb) : -1;
#pragma unroll
        for (int k = 0; k < CX; ++k) {
            const int x = xs + k;
            const bool xin = x < g.M[1];
            const int xk = min(x, g.M[1] - 1);
            xsl[k] = xin ? slab_index(x, g.M[1], g.nb) : -1;
            oz[k] = zsl >= 0 ? 4u * (unsigned)(zsl + g.W * xk) : kOOB;
            ox[k] = zin && xsl[k] >= 0 ? 4u * (unsigned)(z + g.ld1 * xsl[k]) : kOOB;
            oy[k] = zin ? 4u * (unsigned)(z + g.ld1 * xk) : kOOB;
        }
        pz = 4u * (unsigned)(g.W * g.M[1]);
        px = 4u * (unsigned)(g.ld1 * g.W);
        py = 4u * (unsigned)(g.ld1 * g.M[1]);
    }
};

// v_a -= dt beta_a (D+_a p + psi_a), a = z, x, y
template <int N, int CX, int NWX, int CY>
__global__ __launch_bounds__(64 * NWX) void k_yplane_v(Geom g, Fields f, Model m, Cpml cp,
                                                       const int *__restrict__ box, YPMap mp) {
    using K = YPT<N, CX, NWX>;
    constexpr int TX = K::TX, NT = K::NT, LR = K::LR, LC = K::LC, NHZ = K::NHZ, HZT = K::HZT;
    __shared__ float sp[2][LC][LR];
    const YPTile T = yp_tile<TX>(box, mp, CY);
    if (!T.live) return;                                   // uniform over the workgroup
    const int t = (int)threadIdx.x, lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int *b = box + 6 * T.s;
    const int b0 = b[0], b1 = b[1], b3 = b[3];
    const int z = T.z0 + lane, xs = T.x0 + CX * wv;
    const bool zok = z >= b0 && z < b1;
    const long long so = (long long)T.s * g.P;
    const YPAddr A = yp_addr(g, T.x0, N);
    const auto rp = rsrc(f.p + so, g.P);
    const auto rv0 = rsrc(f.v[0] + so, g.P), rv1 = rsrc(f.v[1] + so, g.P), rv2 = rsrc(f.v[2] + so, g.P);
    const auto rb0 = rsrc(m.bdt[0], g.P), rb1 = rsrc(m.bdt[1], g.P), rb2 = rsrc(m.bdt[2], g.P);
    const auto rz = rsrc(f.psp[0] + (long long)T.s * g.psz[0], g.psz[0]);
    const auto rx = rsrc(f.psp[1] + (long long)T.s * g.psz[1], g.psz[1]);
    const auto ry = rsrc(f.psp[2] + (long long)T.s * g.psz[2], g.psz[2]);
    unsigned own[CX];
    bool xok[CX];
#pragma unroll
    for (int k = 0; k < CX; ++k) {
        own[k] = A.lane(z, xs + k);
        xok[k] = xs + k < b3;
    }
    // halo: wavefront w < 2N loads x-halo column w (N left, N right of the tile) at its rows;
    // thread t loads the z-halo values t, t + NT, ... (N rows above and below the tile)
    const bool hxon = wv < 2 * N;
    const int hxq = wv % (2 * N);
    const unsigned ohx = A.lane(z, hxq < N ? T.x0 - N + hxq : T.x0 + TX + hxq - N);
    const int hxl = hxq < N ? hxq : TX + hxq;              // its LDS column
    unsigned ohz[HZT];
    int hzl[HZT];                                          // its LDS index, -1: none
#pragma unroll
    for (int j = 0; j < HZT; ++j) {
        const int i = t + NT * j;
        const int ii = i < NHZ ? i : 0;
        const int hc = ii / (2 * N), hh = ii % (2 * N);
        ohz[j] = A.lane(hh < N ? T.z0 - N + hh : T.z0 + 64 + hh - N, T.x0 + hc);
        hzl[j] = i < NHZ ? (N + hc) * LR + (hh < N ? hh : 64 + hh) : -1;
    }
    YPSlab<CX> S;
    S.init(g, z, xs);
    float azh = 0.f, bzh = 0.f, axh[CX], bxh[CX];
    if (S.zsl >= 0) {
        azh = cp.a_h[0][z];
        bzh = cp.b_h[0][z];
    }
#pragma unroll
    for (int k = 0; k < CX; ++k) {
        axh[k] = S.xsl[k] >= 0 ? cp.a_h[1][xs + k] : 0.f;
        bxh[k] = S.xsl[k] >= 0 ? cp.b_h[1][xs + k] : 0.f;
    }

    // queue of p along y per column: q[k][j] = p(y - (N - 1) + j), j = 0 .. 2N - 1
    float q[CX][2 * N];
#pragma unroll
    for (int k = 0; k < CX; ++k)
#pragma unroll
        for (int j = 0; j < 2 * N - 1; ++j) q[k][j] = bl(rp, own[k], A.plane(T.ylo - (N - 1) + j));
    struct Ld {
        float pn[CX], vo[CX][3], bd[CX][3], ps[CX][3], hx, hz[HZT];
    };
    auto load = [&](int y, Ld &d) {
        const unsigned sy = A.plane(y), syn = A.plane(y + N);
        const int ysl = slab_index(y, g.M[2], g.nb);
        const unsigned syz = S.pz * (unsigned)y, syx = S.px * (unsigned)y;
        const unsigned syy = ysl >= 0 ? S.py * (unsigned)ysl : 0u;
#pragma unroll
        for (int k = 0; k < CX; ++k) {
            d.pn[k] = bl(rp, own[k], syn);
            d.vo[k][0] = bl(rv0, own[k], sy);
            d.vo[k][1] = bl(rv1, own[k], sy);
            d.vo[k][2] = bl(rv2, own[k], sy);
            d.bd[k][0] = bl(rb0, own[k], sy);
            d.bd[k][1] = bl(rb1, own[k], sy);
            d.bd[k][2] = bl(rb2, own[k], sy);
            d.ps[k][0] = bl(rz, S.oz[k], syz);
            d.ps[k][1] = bl(rx, S.ox[k], syx);
            d.ps[k][2] = bl(ry, ysl >= 0 ? S.oy[k] : kOOB, syy);
        }
        d.hx = bl(rp, ohx, sy);
#pragma unroll
        for (int j = 0; j < HZT; ++j) d.hz[j] = bl(rp, ohz[j], sy);
    };
    // planes y + 2 load while plane y is computed: three load buffers rotate over the trips of
    // three planes (the planes past the strip's end only load, at its last plane, and are
    // otherwise skipped)
    auto plane = [&](int y, const Ld &cur, Ld &fill) {
        load(min(y + 2, T.yhi - 1), fill);
        if (y >= T.yhi) return;                            // uniform over the workgroup
        const int bf = (y - T.ylo) & 1;
#pragma unroll
        for (int k = 0; k < CX; ++k) {
            q[k][2 * N - 1] = cur.pn[k];
            sp[bf][N + CX * wv + k][N + lane] = q[k][N - 1];
        }
        if (hxon) sp[bf][hxl][N + lane] = cur.hx;
#pragma unroll
        for (int j = 0; j < HZT; ++j)
            if (hzl[j] >= 0) (&sp[bf][0][0])[hzl[j]] = cur.hz[j];
        __syncthreads();
        const int ysl = slab_index(y, g.M[2], g.nb);
        const float ayh = ysl >= 0 ? cp.a_h[2][y] : 0.f, byh = ysl >= 0 ? cp.b_h[2][y] : 0.f;
        const unsigned sy = A.plane(y);
        const unsigned syz = S.pz * (unsigned)y, syx = S.px * (unsigned)y;
        const unsigned syy = ysl >= 0 ? S.py * (unsigned)ysl : 0u;
        if (zok) {
            float wx[CX + 2 * N - 1];                      // p of this row at x = xs - (N-1) ..
#pragma unroll
            for (int d = 0; d < CX + 2 * N - 1; ++d) wx[d] = sp[bf][CX * wv + 1 + d][N + lane];
#pragma unroll
            for (int k = 0; k < CX; ++k) {
                if (!xok[k]) break;
                const float pc = q[k][N - 1];
                {   // z
                    float e = 0.f;
                    const float *col = &sp[bf][N + CX * wv + k][N + lane];
#pragma unroll
                    for (int l = 1; l <= N; ++l) {
                        const float lo = l == 1 ? pc : col[1 - l];
                        e += g.c[0][l - 1] * (col[l] - lo);
                    }
                    const float psi = bzh * cur.ps[k][0] + azh * e;
                    bs(rz, S.oz[k], syz, psi);
                    e = S.zsl >= 0 ? e + psi : e;
                    bs(rv0, own[k], sy, cur.vo[k][0] - cur.bd[k][0] * e);
                }
                {   // x
                    float e = 0.f;
#pragma unroll
                    for (int l = 1; l <= N; ++l) {
                        const float lo = l == 1 ? pc : wx[k + N - l];
                        e += g.c[1][l - 1] * (wx[k + N - 1 + l] - lo);
                    }
                    if (S.xsl[k] >= 0) {
                        const float psi = bxh[k] * cur.ps[k][1] + axh[k] * e;
                        bs(rx, S.ox[k], syx, psi);
                        e += psi;
                    }
                    bs(rv1, own[k], sy, cur.vo[k][1] - cur.bd[k][1] * e);
                }
                {   // y
                    float e = 0.f;
#pragma unroll
                    for (int l = 1; l <= N; ++l) e += g.c[2][l - 1] * (q[k][N - 1 + l] - q[k][N - l]);
                    if (ysl >= 0) {
                        const float psi = byh * cur.ps[k][2] + ayh * e;
                        bs(ry, S.oy[k], syy, psi);
                        e += psi;
                    }
                    bs(rv2, own[k], sy, cur.vo[k][2] - cur.bd[k][2] * e);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < CX; ++k)
#pragma unroll
            for (int j = 0; j < 2 * N - 1; ++j) q[k][j] = q[k][j + 1];
    };
    Ld L0, L1, L2;
    load(T.ylo, L0);
    load(min(T.ylo + 1, T.yhi - 1), L1);
    for (int y = T.ylo; y < T.yhi; y += 3) {
        plane(y, L0, L2);
        plane(y + 1, L1, L0);
        plane(y + 2, L2, L1);
    }
}

// p -= dt kappa sum_a (D-_a v_a + psi_a) [+ source] [image += dt p p_f]
template <int N, int CX, int NWX, int CY, bool SRC, bool IMG>
__global__ __launch_bounds__(64 * NWX) void k_yplane_p(Geom g, Fields f, Model m, Cpml cp,
                                                       const int *__restrict__ box, YPMap mp,
                                                       const long long *__restrict__ src_cell,
                                                       const float *__restrict__ stf, int nt, int it,
                                                       const float *__restrict__ pf, float *acc_i) {
    using K = YPT<N, CX, NWX>;
    constexpr int TX = K::TX, NT = K::NT, LR = K::LR, LC = K::LC, NHZ = K::NHZ, HZT = K::HZT;
    __shared__ float sz[2][TX][LR];                        // v_z: tile columns, rows with halo
    __shared__ float sx[2][LC][64];                        // v_x: tile rows, columns with halo
    const YPTile T = yp_tile<TX>(box, mp, CY);
    if (!T.live) return;
    const int t = (int)threadIdx.x, lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int *b = box + 6 * T.s;
    const int b0 = b[0], b1 = b[1], b3 = b[3];
    const int z = T.z0 + lane, xs = T.x0 + CX * wv;
    const bool zok = z >= b0 && z < b1;
    const long long so = (long long)T.s * g.P;
    const YPAddr A = yp_addr(g, T.x0, N);
    const auto rp = rsrc(f.p + so, g.P);
    const auto rv0 = rsrc(f.v[0] + so, g.P), rv1 = rsrc(f.v[1] + so, g.P), rv2 = rsrc(f.v[2] + so, g.P);
    const auto rk = rsrc(m.kdt, g.P);
    const auto rz = rsrc(f.psv[0] + (long long)T.s * g.psz[0], g.psz[0]);
    const auto rx = rsrc(f.psv[1] + (long long)T.s * g.psz[1], g.psz[1]);
    const auto ry = rsrc(f.psv[2] + (long long)T.s * g.psz[2], g.psz[2]);
    unsigned own[CX];
    bool xok[CX];
#pragma unroll
    for (int k = 0; k < CX; ++k) {
        own[k] = A.lane(z, xs + k);
        xok[k] = xs + k < b3;
    }
    const bool hxon = wv < 2 * N;
    const int hxq = wv % (2 * N);
    const unsigned ohx = A.lane(z, hxq < N ? T.x0 - N + hxq : T.x0 + TX + hxq - N);
    const int hxl = hxq < N ? hxq : TX + hxq;
    unsigned ohz[HZT];
    int hzl[HZT];
#pragma unroll
    for (int j = 0; j < HZT; ++j) {
        const int i = t + NT * j;
        const int ii = i < NHZ ? i : 0;
        const int hc = ii / (2 * N), hh = ii % (2 * N);
        ohz[j] = A.lane(hh < N ? T.z0 - N + hh : T.z0 + 64 + hh - N, T.x0 + hc);
        hzl[j] = i < NHZ ? hc * LR + (hh < N ? hh : 64 + hh) : -1;
    }
    YPSlab<CX> S;
    S.init(g, z, xs);
    float azi = 0.f, bzi = 0.f, axi[CX], bxi[CX];
    if (S.zsl >= 0) {
        azi = cp.a_i[0][z];
        bzi = cp.b_i[0][z];
    }
#pragma unroll
    for (int k = 0; k < CX; ++k) {
        axi[k] = S.xsl[k] >= 0 ? cp.a_i[1][xs + k] : 0.f;
        bxi[k] = S.xsl[k] >= 0 ? cp.b_i[1][xs + k] : 0.f;
    }
    // the source node (one tap) as (z, x, y), or none
    int sz0 = -(1 << 20), sx0 = 0, sy0 = 0;
    float samp = 0.f;
    if (SRC) {
        const long long sc = src_cell[T.s];
        if (sc >= 0 && it < nt) {
            // a source node lies inside the padded grid: every coordinate is non-negative
            const long long r0 = sc - g.org;
            sy0 = (int)(r0 / g.ld2);
            sx0 = (int)((r0 % g.ld2) / g.ld1);
            sz0 = (int)((r0 % g.ld2) % g.ld1);
            samp = src_amp(g.src_scale, stf[(long long)T.s * nt + it]);
        }
    }
    // image terms: the forward field at the cell, and this shot's interior accumulator
    // (offset iz + n0 (ix + n1 iy); lanes or columns outside the interior get kOOB)
    unsigned oi[CX];
    const auto rpf = rsrc(IMG ? pf + so : f.p, g.P);
    const auto ri = rsrc(IMG ? acc_i + (long long)T.s * g.I : f.p, IMG ? g.I : 1);
#pragma unroll
    for (int k = 0; k < CX; ++k) {
        const int iz = z - g.nb, ix = xs + k - g.nb;
        oi[k] = (unsigned)iz < (unsigned)g.n[0] && (unsigned)ix < (unsigned)g.n[1]
                    ? 4u * (unsigned)(iz + g.n[0] * ix) : kOOB;
    }
    const unsigned pi = 4u * (unsigned)(g.n[0] * g.n[1]);
    // queue of v_y along y per column: q[k][j] = v_y(y - N + j), j = 0 .. 2N - 1
    float q[CX][2 * N];
#pragma unroll
    for (int k = 0; k < CX; ++k)
#pragma unroll
        for (int j = 0; j < 2 * N - 1; ++j) q[k][j] = bl(rv2, own[k], A.plane(T.ylo - N + j));
    struct Ld {
        float yn[CX], vz[CX], vx[CX], po[CX], kd[CX], ps[CX][3], pf[CX], ai[CX], hx, hz[HZT];
    };
    auto load = [&](int y, Ld &d) {
        const unsigned sy = A.plane(y), syn = A.plane(y + N - 1);
        const int ysl = slab_index(y, g.M[2], g.nb);
        const unsigned syz = S.pz * (unsigned)y, syx = S.px * (unsigned)y;
        const unsigned syy = ysl >= 0 ? S.py * (unsigned)ysl : 0u;
        const int iy = y - g.nb;
        const bool yin = (unsigned)iy < (unsigned)g.n[2];
#pragma unroll
        for (int k = 0; k < CX; ++k) {
            d.yn[k] = bl(rv2, own[k], syn);
            d.vz[k] = bl(rv0, own[k], sy);
            d.vx[k] = bl(rv1, own[k], sy);
            d.po[k] = bl(rp, own[k], sy);
            d.kd[k] = bl(rk, own[k], sy);
            d.ps[k][0] = bl(rz, S.oz[k], syz);
            d.ps[k][1] = bl(rx, S.ox[k], syx);
            d.ps[k][2] = bl(ry, ysl >= 0 ? S.oy[k] : kOOB, syy);
            if (IMG) {
                d.pf[k] = bl(rpf, own[k], sy);
                d.ai[k] = bl(ri, yin ? oi[k] : kOOB, yin ? pi * (unsigned)iy : 0u);
            }
        }
        d.hx = bl(rv1, ohx, sy);
#pragma unroll
        for (int j = 0; j < HZT; ++j) d.hz[j] = bl(rv0, ohz[j], sy);
    };
    // planes y + 2 load while plane y is computed: three load buffers rotate over the trips of
    // three planes (the planes past the strip's end only load, at its last plane, and are
    // otherwise skipped)
    auto plane = [&](int y, const Ld &cur, Ld &fill) {
        load(min(y + 2, T.yhi - 1), fill);
        if (y >= T.yhi) return;                            // uniform over the workgroup
        const int bf = (y - T.ylo) & 1;
#pragma unroll
        for (int k = 0; k < CX; ++k) {
            q[k][2 * N - 1] = cur.yn[k];
            sz[bf][CX * wv + k][N + lane] = cur.vz[k];
            sx[bf][N + CX * wv + k][lane] = cur.vx[k];
        }
        if (hxon) sx[bf][hxl][lane] = cur.hx;
#pragma unroll
        for (int j = 0; j < HZT; ++j)
            if (hzl[j] >= 0) (&sz[bf][0][0])[hzl[j]] = cur.hz[j];
        __syncthreads();
        const int ysl = slab_index(y, g.M[2], g.nb);
        const float ayi = ysl >= 0 ? cp.a_i[2][y] : 0.f, byi = ysl >= 0 ? cp.b_i[2][y] : 0.f;
        const unsigned sy = A.plane(y);
        const unsigned syz = S.pz * (unsigned)y, syx = S.px * (unsigned)y;
        const unsigned syy = ysl >= 0 ? S.py * (unsigned)ysl : 0u;
        const int iy = y - g.nb;
        const bool yin = (unsigned)iy < (unsigned)g.n[2];
        if (zok) {
            float wx[CX + 2 * N - 1];                      // v_x of this row at x = xs - N ..
#pragma unroll
            for (int d = 0; d < CX + 2 * N - 1; ++d) wx[d] = sx[bf][CX * wv + d][lane];
#pragma unroll
            for (int k = 0; k < CX; ++k) {
                if (!xok[k]) break;
                const int x = xs + k;
                float sdiv = 0.f;
                {   // z
                    float e = 0.f;
                    const float *col = &sz[bf][CX * wv + k][N + lane];
#pragma unroll
                    for (int l = 1; l <= N; ++l) e += g.c[0][l - 1] * (col[l - 1] - col[-l]);
                    const float psi = bzi * cur.ps[k][0] + azi * e;
                    bs(rz, S.oz[k], syz, psi);
                    e = S.zsl >= 0 ? e + psi : e;
                    sdiv += e;
                }
                {   // x
                    float e = 0.f;
#pragma unroll
                    for (int l = 1; l <= N; ++l) e += g.c[1][l - 1] * (wx[k + N + l - 1] - wx[k + N - l]);
                    if (S.xsl[k] >= 0) {
                        const float psi = bxi[k] * cur.ps[k][1] + axi[k] * e;
                        bs(rx, S.ox[k], syx, psi);
                        e += psi;
                    }
                    sdiv += e;
                }
                {   // y
                    float e = 0.f;
#pragma unroll
                    for (int l = 1; l <= N; ++l) e += g.c[2][l - 1] * (q[k][N + l - 1] - q[k][N - l]);
                    if (ysl >= 0) {
                        const float psi = byi * cur.ps[k][2] + ayi * e;
                        bs(ry, S.oy[k], syy, psi);
                        e += psi;
                    }
                    sdiv += e;
                }
                float pn = cur.po[k] - cur.kd[k] * sdiv;
                if (SRC && z == sz0 && x == sx0 && y == sy0) pn += samp;
                bs(rp, own[k], sy, pn);
                if (IMG) bs(ri, yin ? oi[k] : kOOB, yin ? pi * (unsigned)iy : 0u,
                            cur.ai[k] + g.dt * pn * cur.pf[k]);
            }
        }
#pragma unroll
        for (int k = 0; k < CX; ++k)
#pragma unroll
            for (int j = 0; j < 2 * N - 1; ++j) q[k][j] = q[k][j + 1];
    };
    Ld L0, L1, L2;
    load(T.ylo, L0);
    load(min(T.ylo + 1, T.yhi - 1), L1);
    for (int y = T.ylo; y < T.yhi; y += 3) {
        plane(y, L0, L2);
        plane(y + 1, L1, L0);
        plane(y + 2, L2, L1);
    }
}

struct YPLaunch {
    YPMap mp;
    unsigned grid;
};

YPLaunch yp_launch(const Plan &pl, const std::vector<int> &tab, int it, int cy, int tx) {
    int ez = 0, ex = 0, ey = 0;
    for (int s = 0; s < pl.nshot; ++s) {
        const int *b = &tab[((size_t)it * pl.nshot + s) * 6];
        if (b[1] <= b[0] || b[3] <= b[2] || b[5] <= b[4]) continue;
        ez = std::max(ez, b[1] - zalign(b[0]));
        ex = std::max(ex, b[3] - b[2]);
        ey = std::max(ey, b[5] - b[4]);
    }
    YPLaunch L{};
    if (ez <= 0 || ex <= 0 || ey <= 0) return L;
    L.mp.nshot = pl.nshot;
    L.mp.nstrip = (ey + cy - 1) / cy;
    L.mp.nxt = (ex + tx - 1) / tx;
    L.mp.nzt = (ez + 63) / 64;
    const long long n = (long long)pl.nshot * L.mp.nstrip * L.mp.nxt * L.mp.nzt;
    L.mp.ntile = (int)n;
    L.grid = (unsigned)n;
    return L;
}

template <int N, int CX, int NWX, int CY>
hipError_t fwd_yp_t(const StepCtx &c, int it) {
    const Plan &pl = *c.pl;
    const Views &w = *c.w;
    const int *box = w.fbox + (size_t)it * pl.nshot * 6;
    const YPLaunch L = yp_launch(pl, pl.fbox, it, CY, CX * NWX);
    if (L.grid == 0) return hipSuccess;
    const dim3 blk(64 * NWX);
    if (c.ev) {
        hipExtLaunchKernelGGL((k_yplane_v<N, CX, NWX, CY>), dim3(L.grid), blk, 0, c.st, c.ev[0],
                              c.ev[1], 0, pl.geom, w.f, w.model, w.cpml, box, L.mp);
        hipExtLaunchKernelGGL((k_yplane_p<N, CX, NWX, CY, true, false>), dim3(L.grid), blk, 0, c.st,
                              c.ev[2], c.ev[3], 0, pl.geom, w.f, w.model, w.cpml, box, L.mp,
                              (const long long *)w.src_cell, c.stf, pl.g.nt, it,
                              (const float *)nullptr, (float *)nullptr);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((k_yplane_v<N, CX, NWX, CY>), dim3(L.grid), blk, 0, c.st, pl.geom, w.f,
                       w.model, w.cpml, box, L.mp);
    hipLaunchKernelGGL((k_yplane_p<N, CX, NWX, CY, true, false>), dim3(L.grid), blk, 0, c.st,
                       pl.geom, w.f, w.model, w.cpml, box, L.mp, (const long long *)w.src_cell,
                       c.stf, pl.g.nt, it, (const float *)nullptr, (float *)nullptr);
    return hipGetLastError();
}

template <int N, int CX, int NWX, int CY>
hipError_t adj_yp_t(const StepCtx &c, int it, bool image) {
    const Plan &pl = *c.pl;
    const Views &w = *c.w;
    const int *ab = w.abox + (size_t)it * pl.nshot * 6;
    const YPLaunch L = yp_launch(pl, pl.abox, it, CY, CX * NWX);
    if (L.grid == 0) return hipSuccess;
    const dim3 blk(64 * NWX);
    hipLaunchKernelGGL((k_yplane_v<N, CX, NWX, CY>), dim3(L.grid), blk, 0, c.st, pl.geom, w.q,
                       w.model, w.cpml, ab, L.mp);
    if (image)
        hipLaunchKernelGGL((k_yplane_p<N, CX, NWX, CY, false, true>), dim3(L.grid), blk, 0, c.st,
                           pl.geom, w.q, w.model, w.cpml, ab, L.mp, (const long long *)w.src_cell,
                           c.stf, pl.g.nt, it, (const float *)w.f.p, w.acc_i);
    else
        hipLaunchKernelGGL((k_yplane_p<N, CX, NWX, CY, false, false>), dim3(L.grid), blk, 0, c.st,
                           pl.geom, w.q, w.model, w.cpml, ab, L.mp, (const long long *)w.src_cell,
                           c.stf, pl.g.nt, it, (const float *)w.f.p, w.acc_i);
    return hipGetLastError();
}

// c.yp = CY + 1000 form: CY = 16, 32 or 64 planes per workgroup; form 0: 2 cells per lane x 8
// wavefronts (16-column tiles), 1: 4 x 8 (32 columns), 2: 2 x 16 (32 columns); order 4 has
// form 0 at CY 32 only
#define SMI_YP(fn, ...)                                                                       \
    do {                                                                                      \
        const int cy_ = c.yp % 1000, form_ = c.yp / 1000;                                     \
        if (pl.N == 2) return fn<2, 2, 8, 32>(__VA_ARGS__);                                   \
        if (form_ == 1) return cy_ == 16 ? fn<4, 4, 8, 16>(__VA_ARGS__) : fn<4, 4, 8, 32>(__VA_ARGS__); \
        if (form_ == 2) return cy_ == 16 ? fn<4, 2, 16, 16>(__VA_ARGS__) : fn<4, 2, 16, 32>(__VA_ARGS__); \
        if (cy_ == 16) return fn<4, 2, 8, 16>(__VA_ARGS__);                                   \
        if (cy_ == 64) return fn<4, 2, 8, 64>(__VA_ARGS__);                                   \
        return fn<4, 2, 8, 32>(__VA_ARGS__);                                                  \
    } while (0)

}  // namespace

// 3D, no free surface, and each array of a shot within 2 GiB of byte offsets
bool yp_available(const Plan &pl) {
    const double slab = (double)std::max(pl.geom.psz[0], std::max(pl.geom.psz[1], pl.geom.psz[2]));
    return pl.nd == 3 && !pl.g.freesurf && 4.0 * (double)pl.P < 2147483647.0 &&
           4.0 * slab < 2147483647.0 && 4.0 * (double)pl.geom.I < 2147483647.0;
}

hipError_t fwd_step_yp(const StepCtx &c, int it) {
    const Plan &pl = *c.pl;
    SMI_YP(fwd_yp_t, c, it);
}

hipError_t adj_step_yp(const StepCtx &c, int it, bool image) {
    const Plan &pl = *c.pl;
    SMI_YP(adj_yp_t, c, it, image);
}

}  // namespace smi
