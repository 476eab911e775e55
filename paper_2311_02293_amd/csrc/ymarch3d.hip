// ymarch3d.hip -- 3D half steps (eq. 3-4 with CPML, Sec. 2.1) marching along y.
//
// A workgroup owns a tile of 64 z-rows x BX x-columns of one shot and walks CY consecutive
// y-planes.  Per lane, the differentiated field's values along y at the lane's (z, x) stay in
// a register window that slides by one plane per step (one load per plane instead of 2N); the
// current plane's values of the tile, with N rows / columns of halo in z and x, are staged in
// LDS for the z- and x-stencils (a cross-shaped region: the corners are never read).  Each
// lane updates only its own cell, so the update stays in place, as for the other half-step
// kernels.  Lanes and wavefronts outside the shot's box still load and stage their values:
// they are the halo of the cells inside it.
#include <type_traits>
#include <hip/hip_ext.h>

#include "smi_internal.hpp"
#include "device.hpp"

namespace smi {

namespace {

struct Tile {
    int s, z0, x0, ylo, yhi, z, x;
    bool ok;        // the lane's (z, x) lies in the box (cells of the march are updated)
    bool zin, xin;  // the lane's row / wavefront's column lies in the storage of the grid
};

template <int BX>
__device__ __forceinline__ Tile tile_of(const Geom &g, const int *__restrict__ box, int nstrip,
                                        int cy) {
    Tile t;
    // the grid's blocks in XCD-contiguous ranges (consecutive blocks go to different XCDs),
    // z-tile fastest, then x-tile, y-strip and shot: the workgroups resident on one XCD cover a
    // block of neighbouring tiles of one strip, whose halo planes they read from the same L2
    const int G = (int)(gridDim.x * gridDim.y * gridDim.z);
    const int L = xcd_remap((int)(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)), G);
    const int zt = L % (int)gridDim.x;
    int r = L / (int)gridDim.x;
    const int xt = r % (int)gridDim.y;
    r /= (int)gridDim.y;
    t.s = r / nstrip;
    const int strip = r % nstrip;
    const int *b = box + 6 * t.s;
    t.z0 = zalign(b[0]) + zt * 64;
    t.x0 = b[2] + xt * BX;
    t.ylo = b[4] + strip * cy;
    t.yhi = min(t.ylo + cy, b[5]);
    t.z = t.z0 + (int)threadIdx.x;
    t.x = t.x0 + (int)threadIdx.y;
    t.ok = t.z >= b[0] && t.z < b[1] && t.x < b[3];
    t.zin = t.z < g.M[0] + GH;
    t.xin = t.x < g.M[1] + GH;
    return t;
}

// row of the z-halo value lane (< 2N) stages, and its LDS index
template <int N>
__device__ __forceinline__ int zhalo_row(int z0, int lane) {
    return lane < N ? z0 - N + lane : z0 + 64 + lane - N;
}

template <int N, int BX, int CY, bool FS>
__global__ __launch_bounds__(64 * BX) void k_y3_v(Geom g, Fields f, Model m, Cpml cp,
                                                  const int *__restrict__ box, int nstrip) {
    __shared__ float sp[BX + 2 * N][64 + 2 * N];   // p of the plane: [x - x0 + N][z - z0 + N]
    const Tile t = tile_of<BX>(g, box, nstrip, CY);
    if (t.ylo >= t.yhi) return;                    // uniform over the workgroup
    const int lane = threadIdx.x, wv = threadIdx.y;
    const long long so = t.s * g.P, ld1 = g.ld1, ld2 = g.ld2;
    const float *__restrict__ P0 = f.p + so;
    const bool own = t.zin && t.xin;
    const long long kc = g.org + t.z + ld1 * t.x;
    const int zh = zhalo_row<N>(t.z0, lane);
    const bool hz = lane < 2 * N && t.xin && zh >= -GH && zh < g.M[0] + GH;
    constexpr int NXH = (2 * N + BX - 1) / BX;     // x-halo columns staged per wavefront
    float w[2 * N];                                // p at y + d, d = -(N-1) .. N
#pragma unroll
    for (int j = 0; j < 2 * N - 1; ++j) w[j] = own ? P0[kc + ld2 * (t.ylo + j - (N - 1))] : 0.f;
    // the loads of one plane, issued one plane ahead (software pipelining)
    struct Ld {
        float wn, hz, hx[NXH], vo[3], bd[3];
    };
    auto load = [&](int y, Ld &d) {
        const long long k = kc + ld2 * y;
        d.wn = own ? P0[k + N * ld2] : 0.f;
        d.hz = hz ? P0[g.org + zh + ld1 * t.x + ld2 * y] : 0.f;
#pragma unroll
        for (int q = 0; q < NXH; ++q) {
            const int j = wv + q * BX;
            const int xh = j < N ? t.x0 - N + j : t.x0 + BX + j - N;
            d.hx[q] = j < 2 * N && t.zin && xh < g.M[1] + GH ? P0[g.org + t.z + ld1 * xh + ld2 * y] : 0.f;
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            d.vo[a] = t.ok ? f.v[a][so + k] : 0.f;
            d.bd[a] = t.ok ? m.bdt[a][k] : 0.f;
        }
    };
    Ld cur, nxt;
    load(t.ylo, cur);
    nxt = cur;
    for (int y = t.ylo; y < t.yhi; ++y) {
        const long long k = kc + ld2 * y;
        if (y + 1 < t.yhi) load(y + 1, nxt);
        w[2 * N - 1] = cur.wn;
        __syncthreads();                           // the previous plane's readers are done
        sp[wv + N][lane + N] = w[N - 1];
        if (lane < 2 * N) sp[wv + N][lane < N ? lane : 64 + lane] = cur.hz;
#pragma unroll
        for (int q = 0; q < NXH; ++q) {
            const int j = wv + q * BX;
            if (j < 2 * N) sp[j < N ? j : BX + j][lane + N] = cur.hx[q];
        }
        __syncthreads();
        if (t.ok) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                float e = 0.f;
#pragma unroll
                for (int l = 1; l <= N; ++l) {
                    float hi, lo;
                    if (a == 0) { hi = sp[wv + N][lane + N + l]; lo = sp[wv + N][lane + N - l + 1]; }
                    else if (a == 1) { hi = sp[wv + N + l][lane + N]; lo = sp[wv + N - l + 1][lane + N]; }
                    else { hi = w[N - 1 + l]; lo = w[N - l]; }
                    e += g.c[a][l - 1] * (hi - lo);
                }
                const int i = a == 0 ? t.z : (a == 1 ? t.x : y);
                const int sl = slab_index(i, g.M[a], g.nb);
                if (sl >= 0) {
                    const long long q = a == 0 ? sl + (long long)g.W * (t.x + (long long)g.M[1] * y)
                                      : a == 1 ? t.z + ld1 * (sl + (long long)g.W * y)
                                               : t.z + ld1 * (t.x + (long long)g.M[1] * sl);
                    float *ps = f.psp[a] + t.s * g.psz[a] + q;
                    const float psi = cp.b_h[a][i] * *ps + cp.a_h[a][i] * e;
                    *ps = psi;
                    e += psi;
                }
                const float nv = cur.vo[a] - cur.bd[a] * e;
                float *vd = f.v[a] + so + k;
                if (FS && a == 0) {
                    // free surface (image method): v_z on the rows nb - N .. nb - 1 mirrors the
                    // rows nb + N - 1 .. nb, written by the lanes of those rows
                    const int zr = t.z - g.nb;
                    if (zr >= 0 || zr < -N) *vd = nv;
                    if (zr >= 0 && zr < N) vd[-1 - 2 * zr] = nv;
                } else {
                    *vd = nv;
                }
            }
        }
#pragma unroll
        for (int j = 0; j < 2 * N - 1; ++j) w[j] = w[j + 1];
        cur = nxt;
    }
}

template <int N, int BX, int CY, bool SRC, bool IMG, bool FS>
__global__ __launch_bounds__(64 * BX) void k_y3_p(Geom g, Fields f, Model m, Cpml cp,
                                                  const int *__restrict__ box, int nstrip,
                                                  const long long *__restrict__ src_cell,
                                                  const float *__restrict__ stf, int nt, int it,
                                                  const float *__restrict__ pf, float *acc_i) {
    __shared__ float sz[BX][64 + 2 * N];           // v_z of the plane, own columns + z-halo
    __shared__ float sx[BX + 2 * N][64];           // v_x of the plane, own rows + x-halo
    const Tile t = tile_of<BX>(g, box, nstrip, CY);
    if (t.ylo >= t.yhi) return;
    const int lane = threadIdx.x, wv = threadIdx.y;
    const long long so = t.s * g.P, ld1 = g.ld1, ld2 = g.ld2;
    const float *__restrict__ VZ = f.v[0] + so;
    const float *__restrict__ VX = f.v[1] + so;
    const float *__restrict__ VY = f.v[2] + so;
    const bool own = t.zin && t.xin;
    const long long kc = g.org + t.z + ld1 * t.x;
    const int zh = zhalo_row<N>(t.z0, lane);
    const bool hz = lane < 2 * N && t.xin && zh >= -GH && zh < g.M[0] + GH;
    constexpr int NXH = (2 * N + BX - 1) / BX;
    const long long sc = SRC ? src_cell[t.s] : -1;
    float w[2 * N];                                // v_y at y + d, d = -N .. N-1
#pragma unroll
    for (int j = 0; j < 2 * N - 1; ++j) w[j] = t.ok ? VY[kc + ld2 * (t.ylo + j - N)] : 0.f;
    struct Ld {
        float wn, vz, vx, hz, hx[NXH], po, kd;
    };
    auto load = [&](int y, Ld &d) {
        const long long k = kc + ld2 * y;
        d.wn = t.ok ? VY[k + (N - 1) * ld2] : 0.f;
        d.vz = own ? VZ[k] : 0.f;
        d.vx = own ? VX[k] : 0.f;
        d.hz = hz ? VZ[g.org + zh + ld1 * t.x + ld2 * y] : 0.f;
#pragma unroll
        for (int q = 0; q < NXH; ++q) {
            const int j = wv + q * BX;
            const int xh = j < N ? t.x0 - N + j : t.x0 + BX + j - N;
            d.hx[q] = j < 2 * N && t.zin && xh < g.M[1] + GH ? VX[g.org + t.z + ld1 * xh + ld2 * y] : 0.f;
        }
        d.po = t.ok ? f.p[so + k] : 0.f;
        d.kd = t.ok ? m.kdt[k] : 0.f;
    };
    Ld cur, nxt;
    load(t.ylo, cur);
    nxt = cur;
    for (int y = t.ylo; y < t.yhi; ++y) {
        const long long k = kc + ld2 * y;
        if (y + 1 < t.yhi) load(y + 1, nxt);
        w[2 * N - 1] = cur.wn;
        __syncthreads();
        sz[wv][lane + N] = cur.vz;
        if (lane < 2 * N) sz[wv][lane < N ? lane : 64 + lane] = cur.hz;
        sx[wv + N][lane] = cur.vx;
#pragma unroll
        for (int q = 0; q < NXH; ++q) {
            const int j = wv + q * BX;
            if (j < 2 * N) sx[j < N ? j : BX + j][lane] = cur.hx[q];
        }
        __syncthreads();
        if (t.ok) {
            float sdiv = 0.f;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                float e = 0.f;
#pragma unroll
                for (int l = 1; l <= N; ++l) {
                    float hi, lo;
                    if (a == 0) { hi = sz[wv][lane + N + l - 1]; lo = sz[wv][lane + N - l]; }
                    else if (a == 1) { hi = sx[wv + N + l - 1][lane]; lo = sx[wv + N - l][lane]; }
                    else { hi = w[N + l - 1]; lo = w[N - l]; }
                    e += g.c[a][l - 1] * (hi - lo);
                }
                const int i = a == 0 ? t.z : (a == 1 ? t.x : y);
                const int sl = slab_index(i, g.M[a], g.nb);
                if (sl >= 0) {
                    const long long q = a == 0 ? sl + (long long)g.W * (t.x + (long long)g.M[1] * y)
                                      : a == 1 ? t.z + ld1 * (sl + (long long)g.W * y)
                                               : t.z + ld1 * (t.x + (long long)g.M[1] * sl);
                    float *ps = f.psv[a] + t.s * g.psz[a] + q;
                    const float psi = cp.b_i[a][i] * *ps + cp.a_i[a][i] * e;
                    *ps = psi;
                    e += psi;
                }
                sdiv += e;
            }
            float pn = cur.po - cur.kd * sdiv;
            if (SRC && it < nt && k == sc) pn += src_amp(g.src_scale, stf[(long long)t.s * nt + it]);
            float *pd = f.p + so + k;
            if (FS) {
                // free surface: p = 0 on row nb and odd about it, the rows nb - N .. nb - 1
                // written by the lanes of rows nb + N .. nb + 1 (the image takes the updated value)
                const int zr = t.z - g.nb;
                if (zr > 0 || zr < -N) *pd = pn;
                else if (zr == 0) *pd = 0.f;
                if (zr > 0 && zr <= N) pd[-2 * zr] = -pn;
            } else {
                *pd = pn;
            }
            if (IMG) {
                const int iz = t.z - g.nb, ix = t.x - g.nb, iy = y - g.nb;
                if ((unsigned)iz < (unsigned)g.n[0] && (unsigned)ix < (unsigned)g.n[1] &&
                    (unsigned)iy < (unsigned)g.n[2]) {
                    const long long ii = t.s * g.I + iz + (long long)g.n[0] * (ix + (long long)g.n[1] * iy);
                    acc_i[ii] += g.dt * pn * pf[so + k];
                }
            }
        }
#pragma unroll
        for (int j = 0; j < 2 * N - 1; ++j) w[j] = w[j + 1];
        cur = nxt;
    }
}

struct YLaunch {
    dim3 grid, block;
    int nstrip;
    bool empty;
};

YLaunch y3_launch(const Plan &pl, const std::vector<int> &tab, int it, int bx, int cy) {
    int ez = 0, ex = 0, ey = 0;
    for (int s = 0; s < pl.nshot; ++s) {
        const int *b = &tab[((size_t)it * pl.nshot + s) * 6];
        ez = std::max(ez, b[1] - zalign(b[0]));
        ex = std::max(ex, b[3] - b[2]);
        ey = std::max(ey, b[5] - b[4]);
    }
    YLaunch L;
    L.empty = ez <= 0 || ex <= 0 || ey <= 0;
    L.nstrip = std::max(1, (ey + cy - 1) / cy);
    L.block = dim3(64, bx, 1);
    L.grid = dim3((unsigned)std::max(1, (ez + 63) / 64), (unsigned)std::max(1, (ex + bx - 1) / bx),
                  (unsigned)(pl.nshot * L.nstrip));
    return L;
}

template <int N, int BX, int CY>
hipError_t fwd_y3_t(const StepCtx &c, int it) {
    const Plan &pl = *c.pl;
    const Views &w = *c.w;
    const int *box = w.fbox + (size_t)it * pl.nshot * 6;
    YLaunch L = y3_launch(pl, pl.fbox, it, BX, CY);
    if (L.empty) return hipSuccess;
    // F: a free surface, whose image rows the kernels write themselves
    auto launch = [&](auto fs) -> hipError_t {
        constexpr bool F = decltype(fs)::value;
        if (c.ev) {
            hipExtLaunchKernelGGL((k_y3_v<N, BX, CY, F>), L.grid, L.block, 0, c.st, c.ev[0],
                                  c.ev[1], 0, pl.geom, w.f, w.model, w.cpml, box, L.nstrip);
            hipExtLaunchKernelGGL((k_y3_p<N, BX, CY, true, false, F>), L.grid, L.block, 0, c.st,
                                  c.ev[2], c.ev[3], 0, pl.geom, w.f, w.model, w.cpml, box, L.nstrip,
                                  (const long long *)w.src_cell, c.stf, pl.g.nt, it,
                                  (const float *)nullptr, (float *)nullptr);
            return hipGetLastError();
        }
        hipLaunchKernelGGL((k_y3_v<N, BX, CY, F>), L.grid, L.block, 0, c.st, pl.geom, w.f, w.model,
                           w.cpml, box, L.nstrip);
        hipLaunchKernelGGL((k_y3_p<N, BX, CY, true, false, F>), L.grid, L.block, 0, c.st, pl.geom,
                           w.f, w.model, w.cpml, box, L.nstrip, (const long long *)w.src_cell,
                           c.stf, pl.g.nt, it, (const float *)nullptr, (float *)nullptr);
        return hipGetLastError();
    };
    return pl.g.freesurf ? launch(std::true_type{}) : launch(std::false_type{});
}

template <int N, int BX, int CY>
hipError_t adj_y3_t(const StepCtx &c, int it, bool image) {
    const Plan &pl = *c.pl;
    const Views &w = *c.w;
    const int *ab = w.abox + (size_t)it * pl.nshot * 6;
    YLaunch L = y3_launch(pl, pl.abox, it, BX, CY);
    if (L.empty) return hipSuccess;
    auto launch = [&](auto fs) -> hipError_t {
        constexpr bool F = decltype(fs)::value;
        hipLaunchKernelGGL((k_y3_v<N, BX, CY, F>), L.grid, L.block, 0, c.st, pl.geom, w.q, w.model,
                           w.cpml, ab, L.nstrip);
        if (image)
            hipLaunchKernelGGL((k_y3_p<N, BX, CY, false, true, F>), L.grid, L.block, 0, c.st,
                               pl.geom, w.q, w.model, w.cpml, ab, L.nstrip,
                               (const long long *)w.src_cell, c.stf, pl.g.nt, it,
                               (const float *)w.f.p, w.acc_i);
        else
            hipLaunchKernelGGL((k_y3_p<N, BX, CY, false, false, F>), L.grid, L.block, 0, c.st,
                               pl.geom, w.q, w.model, w.cpml, ab, L.nstrip,
                               (const long long *)w.src_cell, c.stf, pl.g.nt, it,
                               (const float *)w.f.p, w.acc_i);
        return hipGetLastError();
    };
    return pl.g.freesurf ? launch(std::true_type{}) : launch(std::false_type{});
}

// tiles: y3 = 100 BX + CY with BX in {4, 8} and CY in {16, 32, 64}; others fall back to 832
#define SMI_Y3(fn, ...)                                                                       \
    do {                                                                                      \
        const int bx_ = c.y3 / 100, cy_ = c.y3 % 100;                                         \
        if (pl.N == 2) {                                                                      \
            if (bx_ == 4) return fn<2, 4, 32>(__VA_ARGS__);                                   \
            return fn<2, 8, 32>(__VA_ARGS__);                                                 \
        }                                                                                     \
        if (bx_ == 4 && cy_ == 16) return fn<4, 4, 16>(__VA_ARGS__);                          \
        if (bx_ == 4 && cy_ == 32) return fn<4, 4, 32>(__VA_ARGS__);                          \
        if (bx_ == 4 && cy_ == 64) return fn<4, 4, 64>(__VA_ARGS__);                          \
        if (bx_ == 8 && cy_ == 16) return fn<4, 8, 16>(__VA_ARGS__);                          \
        if (bx_ == 8 && cy_ == 64) return fn<4, 8, 64>(__VA_ARGS__);                          \
        return fn<4, 8, 32>(__VA_ARGS__);                                                     \
    } while (0)

}  // namespace

// (not with a free surface, whose mirror images the y-marching kernels do not write)
bool y3_available(const Plan &pl) { return pl.nd == 3; }

hipError_t fwd_step_y3(const StepCtx &c, int it) {
    const Plan &pl = *c.pl;
    SMI_Y3(fwd_y3_t, c, it);
}

hipError_t adj_step_y3(const StepCtx &c, int it, bool image) {
    const Plan &pl = *c.pl;
    SMI_Y3(adj_y3_t, c, it, image);
}

}  // namespace smi
