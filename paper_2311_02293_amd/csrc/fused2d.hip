// fused2d.hip -- one kernel per 2D time step: v update, p update, CPML and source injection
// (eq. 3-4, Sec. 2.1, Alg. 2 forward loop) for every shot of the batch, reading level n from
// one buffer and writing level n + 1 to the other.
//
// Work decomposition (as the register-blocked half-step kernels): a lane owns one z row of a
// run of CM consecutive columns [lo, hi); the four wavefronts of a workgroup take four
// consecutive 64-row tiles; the 8 XCDs take contiguous ranges of column runs.  One step needs
//   * v_x^{n+1/2} on the lane's row at columns lo-N .. hi+N-2 (the p stencil along x): formed
//     in registers from a window of p^n over lo-2N+1 .. hi+2N-2;
//   * v_z^{n+1/2} at rows z-N .. z+N-1 of each owned column: formed from p^n staged in the
//     wavefront's LDS slice (rows z0-2N+1 .. z0+64+2N-2), for the 64 own rows and, by lanes
//     0 .. 2N-2, for the 2N-1 rows just outside; staged again in LDS for the p update.
// Values computed for neighbours' cells (halo columns and rows) are used and not stored, so
// every cell is written by exactly one lane, and every read is of level n: the two levels
// live in different buffers.  Cells outside the shot's computing box keep their old value
// (they are zero), as in the half-step kernels.  All global loads of a lane are issued before
// its arithmetic.
#include <hip/hip_ext.h>

#include "smi_internal.hpp"
#include "device.hpp"

namespace smi {

namespace {

constexpr int kRows = 64 + 2 * (2 * kMaxN - 1);   // staged p rows per column (own + halo)

template <int N, int CM>
__global__ __launch_bounds__(256) void k_fused2d(Geom g, Fields src, Fields dst, Model m, Cpml cp,
                                                 const int *__restrict__ box, int nxc,
                                                 const long long *__restrict__ src_cell,
                                                 const float *__restrict__ stf, int nt, int it) {
    constexpr int H = 2 * N - 1;           // p halo of the fused step
    constexpr int NP = CM + 2 * H;         // p window along x: columns lo-H .. hi-1+H
    constexpr int NV = CM + 2 * N - 1;     // v_x window: columns lo-N .. hi-1+N-1
    __shared__ float sp[4][CM][kRows];     // p^n, rows z0-H .. z0+63+H
    __shared__ float sv[4][CM][64 + 2 * N]; // v_z^{n+1/2}, rows z0-N .. z0+63+N

    const int lane = threadIdx.x, wv = threadIdx.y;
    const int xcd = (int)blockIdx.x & 7;
    const int bz = (int)blockIdx.x >> 3;
    const int s = (int)blockIdx.z;
    const int *b = box + 6 * s;
    const int z0 = zalign(b[0]) + (bz * 4 + wv) * 64;
    const int z = z0 + lane;
    const int lo = b[2] + (xcd * nxc + (int)blockIdx.y) * CM;
    const int hi = min(lo + CM, b[3]);
    if (lo >= hi || z0 >= b[1]) return;                 // uniform over the wavefront
    const int cnt = hi - lo;
    const bool ok = z >= b[0] && z < b[1];              // owns cells
    const bool needp = z >= b[0] - H && z < b[1] + H;  // p row read by some owned cell's stencil
    const bool needv = z >= b[0] - N && z < b[1] + N;  // v_z row read by some owned cell
    const long long so = (long long)s * g.P;
    const long long kz = g.org + z;                     // offset of (z, 0)
    const int ld1 = g.ld1;
    const float *__restrict__ P0 = src.p + so;
    const float *__restrict__ VZ0 = src.v[0] + so;
    const float *__restrict__ VX0 = src.v[1] + so;

    // ---- loads (level n, and the model)
    float pw[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const int x = lo - H + min(j, cnt - 1 + 2 * H);
        pw[j] = (ok || (needp && j >= H && j < H + CM)) ? P0[kz + (long long)ld1 * x] : 0.f;
    }
    float vxo[NV], bx[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        const int x = lo - N + min(j, cnt - 1 + 2 * N - 1);
        vxo[j] = ok ? VX0[kz + (long long)ld1 * x] : 0.f;
        bx[j] = ok ? m.bdt[1][kz + (long long)ld1 * x] : 0.f;
    }
    float vzo[CM], bzz[CM], kd[CM];
#pragma unroll
    for (int t = 0; t < CM; ++t) {
        const long long k = kz + (long long)ld1 * (lo + min(t, cnt - 1));
        vzo[t] = needv ? VZ0[k] : 0.f;
        bzz[t] = needv ? m.bdt[0][k] : 0.f;
        kd[t] = ok ? m.kdt[k] : 0.f;
    }
    // halo rows of the p staging: lanes 0 .. 2H-1 load rows z0-H+lane (lane < H) and
    // z0+64+lane-H (lane >= H)
    const int hr = lane < H ? z0 - H + lane : z0 + 64 + lane - H;
    const bool hp = lane < 2 * H && hr >= b[0] - H && hr < b[1] + H;
    float hpv[CM];
#pragma unroll
    for (int t = 0; t < CM; ++t)
        hpv[t] = hp ? P0[g.org + hr + (long long)ld1 * (lo + min(t, cnt - 1))] : 0.f;
    // v_z rows just outside the wavefront that lanes 0 .. 2N-2 form: z0-N+lane (lane < N) and
    // z0+64+lane-N (lane >= N)
    const int vr = lane < N ? z0 - N + lane : z0 + 64 + lane - N;
    const bool hv = lane < 2 * N - 1 && vr >= b[0] - N && vr < b[1] + N;
    float hvz[CM], hbz[CM];
#pragma unroll
    for (int t = 0; t < CM; ++t) {
        const long long k = g.org + vr + (long long)ld1 * (lo + min(t, cnt - 1));
        hvz[t] = hv ? VZ0[k] : 0.f;
        hbz[t] = hv ? m.bdt[0][k] : 0.f;
    }

    // ---- p^n of the owned columns to LDS
#pragma unroll
    for (int t = 0; t < CM; ++t) {
        sp[wv][t][H + lane] = pw[H + t];
        if (lane < 2 * H) sp[wv][t][lane < H ? lane : 64 + lane] = hpv[t];
    }
    __builtin_amdgcn_wave_barrier();

    // ---- v_z^{n+1/2} at this lane's row (and one outside row for lanes 0 .. 2N-2)
    auto vz_new = [&](int r, int t, float vold, float bdz) -> float {
        if (r < b[0] || r >= b[1]) return vold;         // outside the box: unchanged
        const int i = r - z0 + H;                        // LDS row index
        float e = 0.f;
#pragma unroll
        for (int l = 1; l <= N; ++l) e += g.c[0][l - 1] * (sp[wv][t][i + l] - sp[wv][t][i - l + 1]);
        const int zc = slab_index(r, g.M[0], g.nb);
        if (zc >= 0) {
            const int x = lo + t;
            const float *ps = src.psp[0] + (long long)s * g.psz[0] + zc + (long long)g.W * x;
            const float psi = cp.b_h[0][r] * *ps + cp.a_h[0][r] * e;
            if (r == z && x < hi)
                dst.psp[0][(long long)s * g.psz[0] + zc + (long long)g.W * x] = psi;
            e += psi;
        }
        return vold - bdz * e;
    };
    float vzn[CM];
#pragma unroll
    for (int t = 0; t < CM; ++t) {
        vzn[t] = needv && t < cnt ? vz_new(z, t, vzo[t], bzz[t]) : 0.f;
        sv[wv][t][N + lane] = vzn[t];
        if (lane < 2 * N - 1) {
            const float o = hv && t < cnt ? vz_new(vr, t, hvz[t], hbz[t]) : 0.f;
            sv[wv][t][lane < N ? lane : 64 + lane] = o;
        }
    }
    __builtin_amdgcn_wave_barrier();
    if (!ok) return;

    // ---- v_x^{n+1/2} at columns lo-N+j on this row
    float vxn[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        const int x = lo - N + j;
        if (x < b[2] || x >= b[3] || j >= cnt + 2 * N - 1) { vxn[j] = vxo[j]; continue; }
        float e = 0.f;
#pragma unroll
        for (int l = 1; l <= N; ++l) e += g.c[1][l - 1] * (pw[j + N + l - 1] - pw[j + N - l]);
        const int xc = slab_index(x, g.M[1], g.nb);
        if (xc >= 0) {
            const long long q = (long long)s * g.psz[1] + z + (long long)ld1 * xc;
            const float psi = cp.b_h[1][x] * src.psp[1][q] + cp.a_h[1][x] * e;
            if (j >= N && j < N + cnt) dst.psp[1][q] = psi;
            e += psi;
        }
        vxn[j] = vxo[j] - bx[j] * e;
    }

    // ---- p^{n+1} on the owned cells; store the owned v
    const long long sc = src_cell[s];
    const int zc = slab_index(z, g.M[0], g.nb);
#pragma unroll
    for (int t = 0; t < CM; ++t) {
        if (t >= cnt) break;
        const int x = lo + t;
        const long long k = kz + (long long)ld1 * x;
        const int i = lane + N;
        float ez = 0.f;
#pragma unroll
        for (int l = 1; l <= N; ++l) ez += g.c[0][l - 1] * (sv[wv][t][i + l - 1] - sv[wv][t][i - l]);
        if (zc >= 0) {
            const long long q = (long long)s * g.psz[0] + zc + (long long)g.W * x;
            const float psi = cp.b_i[0][z] * src.psv[0][q] + cp.a_i[0][z] * ez;
            dst.psv[0][q] = psi;
            ez += psi;
        }
        float ex = 0.f;
#pragma unroll
        for (int l = 1; l <= N; ++l) ex += g.c[1][l - 1] * (vxn[t + N + l - 1] - vxn[t + N - l]);
        const int xc = slab_index(x, g.M[1], g.nb);
        if (xc >= 0) {
            const long long q = (long long)s * g.psz[1] + z + (long long)ld1 * xc;
            const float psi = cp.b_i[1][x] * src.psv[1][q] + cp.a_i[1][x] * ex;
            dst.psv[1][q] = psi;
            ex += psi;
        }
        float pn = pw[H + t] - kd[t] * (ez + ex);
        if (it < nt && k == sc) pn += src_amp(g.src_scale, stf[(long long)s * nt + it]);
        dst.p[so + k] = pn;
        dst.v[0][so + k] = vzn[t];
        dst.v[1][so + k] = vxn[N + t];
    }
}

// Tiled variant: a workgroup owns a tile of 64 rows x TX = 4 CW columns; its four wavefronts
// stage p^n over the tile plus a halo of H = 2N - 1 nodes along each axis (a plus-shaped
// region: the corners are never read) in LDS, form v_z^{n+1/2} over the tile's columns on
// rows z0-N .. z0+63+N-1 and v_x^{n+1/2} over the tile's rows on columns lo-N .. lo+TX+N-2
// (both staged in LDS), then p^{n+1} on the tile.  Every global load of phase 1 is issued
// before any arithmetic, and each halo value is loaded once per tile (neighbouring tiles
// share it through L2); the 8 XCDs take contiguous ranges of column tiles.
template <int N, int CW>
__global__ __launch_bounds__(256) void k_fused2d_tile(Geom g, Fields src, Fields dst, Model m,
                                                      Cpml cp, const int *__restrict__ box,
                                                      int nxc,
                                                      const long long *__restrict__ src_cell,
                                                      const float *__restrict__ stf, int nt,
                                                      int it) {
    constexpr int H = 2 * N - 1;
    constexpr int TX = 4 * CW;
    constexpr int RP = 64 + 2 * H;      // staged p rows: z0-H .. z0+63+H
    constexpr int CP = TX + 2 * H;      // staged p columns: lo-H .. lo+TX-1+H
    constexpr int RV = 64 + 2 * N - 1;  // v_z rows: z0-N .. z0+63+N-1
    constexpr int CV = TX + 2 * N - 1;  // v_x columns: lo-N .. lo+TX+N-2
    constexpr int QP = (2 * H + 3) / 4; // p halo columns per wavefront
    constexpr int QV = (2 * N - 1 + 3) / 4;  // v_x halo columns per wavefront
    __shared__ float sp[CP][RP];
    __shared__ float svz[TX][RV];
    __shared__ float svx[CV][64];

    const int lane = threadIdx.x, wv = threadIdx.y;
    const int xcd = (int)blockIdx.x & 7;
    const int bz = (int)blockIdx.x >> 3;
    const int s = (int)blockIdx.z;
    const int *b = box + 6 * s;
    const int b0 = b[0], b1 = b[1], b2 = b[2], b3 = b[3];
    const int z0 = zalign(b0) + bz * 64;
    const int lo = b2 + (xcd * nxc + (int)blockIdx.y) * TX;
    if (lo >= b3 || z0 >= b1) return;                 // uniform over the workgroup
    const int z = z0 + lane;
    const int ld1 = g.ld1;
    const long long so = (long long)s * g.P;
    const float *__restrict__ P0 = src.p + so;
    const float *__restrict__ VZ0 = src.v[0] + so;
    const float *__restrict__ VX0 = src.v[1] + so;
    const float *__restrict__ BZ = m.bdt[0];
    const float *__restrict__ BX = m.bdt[1];

    // Tiles whose halo lies inside the box and outside the absorbing slabs, without the
    // source: no masks, no CPML variables, 32-bit offsets.
    {
        const int M0 = g.M[0], M1 = g.M[1], nb = g.nb;
        const long long scell = src_cell[s];
        const int sx = scell >= 0 ? (int)((scell - g.org) / ld1) : -(1 << 30);
        const int sz = scell >= 0 ? (int)(scell - g.org - (long long)sx * ld1) : -(1 << 30);
        const bool fast = z0 - H >= max(b0, nb) && z0 + 64 + H <= min(b1, M0 - nb - 1) &&
                          lo - H >= max(b2, nb) && lo + TX + H <= min(b3, M1 - nb - 1) &&
                          !(sz >= z0 && sz < z0 + 64 && sx >= lo && sx < lo + TX);
        if (fast) {
            const int oz = (int)g.org + z;
            const int hr = lane < H ? z0 - H + lane : (lane < 2 * H ? z0 + 64 + lane - H : z);
            const int oh = (int)g.org + hr;
            const int vr = lane < N ? z0 - N + lane : (lane < 2 * N - 1 ? z0 + 64 + lane - N : z);
            const int ov = (int)g.org + vr;
            float pc[CW], ph[CW], vzc[CW], bzc[CW], vzh[CW], bzh[CW], vxc[CW], bxc[CW], kd[CW];
#pragma unroll
            for (int t = 0; t < CW; ++t) {
                const int cx = ld1 * (lo + wv * CW + t);
                pc[t] = P0[oz + cx];
                ph[t] = P0[oh + cx];
                vzc[t] = VZ0[oz + cx];
                bzc[t] = BZ[oz + cx];
                vxc[t] = VX0[oz + cx];
                bxc[t] = BX[oz + cx];
                kd[t] = m.kdt[oz + cx];
                vzh[t] = VZ0[ov + cx];
                bzh[t] = BZ[ov + cx];
            }
            float pq[QP];
#pragma unroll
            for (int q = 0; q < QP; ++q) {
                const int j = min(wv + 4 * q, 2 * H - 1);
                const int x = j < H ? lo - H + j : lo + TX + j - H;
                pq[q] = P0[oz + ld1 * x];
            }
            float vxq[QV], bxq[QV];
#pragma unroll
            for (int q = 0; q < QV; ++q) {
                const int j = min(wv + 4 * q, 2 * N - 2);
                const int x = j < N ? lo - N + j : lo + TX + j - N;
                vxq[q] = VX0[oz + ld1 * x];
                bxq[q] = BX[oz + ld1 * x];
            }
#pragma unroll
            for (int t = 0; t < CW; ++t) {
                sp[H + wv * CW + t][H + lane] = pc[t];
                if (lane < 2 * H) sp[H + wv * CW + t][lane < H ? lane : 64 + lane] = ph[t];
            }
#pragma unroll
            for (int q = 0; q < QP; ++q) {
                const int j = wv + 4 * q;
                if (j < 2 * H) sp[j < H ? j : TX + j][H + lane] = pq[q];
            }
            __syncthreads();
            float vzn[CW], vxn[CW];
#pragma unroll
            for (int t = 0; t < CW; ++t) {
                const int c = wv * CW + t;
                float e = 0.f, ex = 0.f;
#pragma unroll
                for (int l = 1; l <= N; ++l) {
                    e += g.c[0][l - 1] * (sp[H + c][H + lane + l] - sp[H + c][H + lane - l + 1]);
                    ex += g.c[1][l - 1] * (sp[H + c + l][H + lane] - sp[H + c - l + 1][H + lane]);
                }
                vzn[t] = vzc[t] - bzc[t] * e;
                vxn[t] = vxc[t] - bxc[t] * ex;
                svz[c][N + lane] = vzn[t];
                svx[N + c][lane] = vxn[t];
                if (lane < 2 * N - 1) {
                    const int i = vr - z0 + H;
                    float eh = 0.f;
#pragma unroll
                    for (int l = 1; l <= N; ++l) eh += g.c[0][l - 1] * (sp[H + c][i + l] - sp[H + c][i - l + 1]);
                    svz[c][lane < N ? lane : 64 + lane] = vzh[t] - bzh[t] * eh;
                }
            }
#pragma unroll
            for (int q = 0; q < QV; ++q) {
                const int j = wv + 4 * q;
                if (j < 2 * N - 1) {
                    const int ci = (j < N ? j - N : TX + j - N) + H;
                    float e = 0.f;
#pragma unroll
                    for (int l = 1; l <= N; ++l) e += g.c[1][l - 1] * (sp[ci + l][H + lane] - sp[ci - l + 1][H + lane]);
                    svx[j < N ? j : TX + j][lane] = vxq[q] - bxq[q] * e;
                }
            }
            __syncthreads();
            float *__restrict__ P1 = dst.p + so;
            float *__restrict__ VZ1 = dst.v[0] + so;
            float *__restrict__ VX1 = dst.v[1] + so;
#pragma unroll
            for (int t = 0; t < CW; ++t) {
                const int c = wv * CW + t;
                float ez = 0.f, ex = 0.f;
#pragma unroll
                for (int l = 1; l <= N; ++l) {
                    ez += g.c[0][l - 1] * (svz[c][lane + N + l - 1] - svz[c][lane + N - l]);
                    ex += g.c[1][l - 1] * (svx[N + c + l - 1][lane] - svx[N + c - l][lane]);
                }
                const int k = oz + ld1 * (lo + c);
                P1[k] = pc[t] - kd[t] * (ez + ex);
                VZ1[k] = vzn[t];
                VX1[k] = vxn[t];
            }
            return;
        }
    }
    auto cell = [&](int zz, int xx) -> long long { return g.org + zz + (long long)ld1 * xx; };
    auto inp = [&](int zz, int xx) { return zz >= b0 - H && zz < b1 + H && xx >= b2 - H && xx < b3 + H; };
    auto inb = [&](int zz, int xx) { return zz >= b0 && zz < b1 && xx >= b2 && xx < b3; };

    // ---- phase 1: loads
    const int hr = lane < H ? z0 - H + lane : z0 + 64 + lane - H;   // p halo row (lane < 2H)
    const int vr = lane < N ? z0 - N + lane : z0 + 64 + lane - N;   // v_z extra row (lane < 2N-1)
    float pc[CW], ph[CW], vzc[CW], bzc[CW], vzh[CW], bzh[CW], vxc[CW], bxc[CW], kd[CW];
#pragma unroll
    for (int t = 0; t < CW; ++t) {
        const int x = lo + wv * CW + t;
        const long long k = cell(z, x);
        pc[t] = inp(z, x) ? P0[k] : 0.f;
        const bool own = inb(z, x);
        vzc[t] = own ? VZ0[k] : 0.f;
        bzc[t] = own ? BZ[k] : 0.f;
        vxc[t] = own ? VX0[k] : 0.f;
        bxc[t] = own ? BX[k] : 0.f;
        kd[t] = own ? m.kdt[k] : 0.f;
        ph[t] = lane < 2 * H && inp(hr, x) ? P0[cell(hr, x)] : 0.f;
        const bool hv = lane < 2 * N - 1 && inb(vr, x);
        vzh[t] = hv ? VZ0[cell(vr, x)] : 0.f;
        bzh[t] = hv ? BZ[cell(vr, x)] : 0.f;
    }
    float pq[QP];
#pragma unroll
    for (int q = 0; q < QP; ++q) {
        const int j = wv + 4 * q;
        const int x = j < H ? lo - H + j : lo + TX + j - H;
        pq[q] = j < 2 * H && inp(z, x) ? P0[cell(z, x)] : 0.f;
    }
    float vxq[QV], bxq[QV];
#pragma unroll
    for (int q = 0; q < QV; ++q) {
        const int j = wv + 4 * q;
        const int x = j < N ? lo - N + j : lo + TX + j - N;
        const bool ok = j < 2 * N - 1 && inb(z, x);
        vxq[q] = ok ? VX0[cell(z, x)] : 0.f;
        bxq[q] = ok ? BX[cell(z, x)] : 0.f;
    }
#pragma unroll
    for (int t = 0; t < CW; ++t) {
        sp[H + wv * CW + t][H + lane] = pc[t];
        if (lane < 2 * H) sp[H + wv * CW + t][lane < H ? lane : 64 + lane] = ph[t];
    }
#pragma unroll
    for (int q = 0; q < QP; ++q) {
        const int j = wv + 4 * q;
        if (j < 2 * H) sp[j < H ? j : TX + j][H + lane] = pq[q];
    }
    __syncthreads();

    // ---- phase 2: v^{n+1/2}
    // v_z at row r of tile column c (LDS column H + c of sp); own: store the CPML variable
    auto vz_new = [&](int r, int c, float vold, float bdz, bool own) -> float {
        const int x = lo + c;
        if (!inb(r, x)) return vold;
        const int i = r - z0 + H;
        float e = 0.f;
#pragma unroll
        for (int l = 1; l <= N; ++l) e += g.c[0][l - 1] * (sp[H + c][i + l] - sp[H + c][i - l + 1]);
        const int zc = slab_index(r, g.M[0], g.nb);
        if (zc >= 0) {
            const long long q = (long long)s * g.psz[0] + zc + (long long)g.W * x;
            const float psi = cp.b_h[0][r] * src.psp[0][q] + cp.a_h[0][r] * e;
            if (own) dst.psp[0][q] = psi;
            e += psi;
        }
        return vold - bdz * e;
    };
    // v_x at column x (LDS column x - lo + H of sp) on this lane's row
    auto vx_new = [&](int x, float vold, float bdx, bool own) -> float {
        if (!inb(z, x)) return vold;
        const int ci = x - lo + H;
        float e = 0.f;
#pragma unroll
        for (int l = 1; l <= N; ++l) e += g.c[1][l - 1] * (sp[ci + l][H + lane] - sp[ci - l + 1][H + lane]);
        const int xc = slab_index(x, g.M[1], g.nb);
        if (xc >= 0) {
            const long long q = (long long)s * g.psz[1] + z + (long long)ld1 * xc;
            const float psi = cp.b_h[1][x] * src.psp[1][q] + cp.a_h[1][x] * e;
            if (own) dst.psp[1][q] = psi;
            e += psi;
        }
        return vold - bdx * e;
    };
    float vzn[CW], vxn[CW];
#pragma unroll
    for (int t = 0; t < CW; ++t) {
        const int c = wv * CW + t;
        vzn[t] = vz_new(z, c, vzc[t], bzc[t], true);
        svz[c][N + lane] = vzn[t];
        if (lane < 2 * N - 1)
            svz[c][lane < N ? lane : 64 + lane] = vz_new(vr, c, vzh[t], bzh[t], false);
        vxn[t] = vx_new(lo + c, vxc[t], bxc[t], true);
        svx[N + c][lane] = vxn[t];
    }
#pragma unroll
    for (int q = 0; q < QV; ++q) {
        const int j = wv + 4 * q;
        if (j < 2 * N - 1) {
            const int x = j < N ? lo - N + j : lo + TX + j - N;
            svx[j < N ? j : TX + j][lane] = vx_new(x, vxq[q], bxq[q], false);
        }
    }
    __syncthreads();

    // ---- phase 3: p^{n+1} on the owned cells; store the owned v
    const long long sc = src_cell[s];
    const int zc = slab_index(z, g.M[0], g.nb);
#pragma unroll
    for (int t = 0; t < CW; ++t) {
        const int c = wv * CW + t;
        const int x = lo + c;
        if (!inb(z, x)) continue;
        const long long k = cell(z, x);
        float ez = 0.f;
#pragma unroll
        for (int l = 1; l <= N; ++l) ez += g.c[0][l - 1] * (svz[c][lane + N + l - 1] - svz[c][lane + N - l]);
        if (zc >= 0) {
            const long long q = (long long)s * g.psz[0] + zc + (long long)g.W * x;
            const float psi = cp.b_i[0][z] * src.psv[0][q] + cp.a_i[0][z] * ez;
            dst.psv[0][q] = psi;
            ez += psi;
        }
        float ex = 0.f;
#pragma unroll
        for (int l = 1; l <= N; ++l) ex += g.c[1][l - 1] * (svx[N + c + l - 1][lane] - svx[N + c - l][lane]);
        const int xc = slab_index(x, g.M[1], g.nb);
        if (xc >= 0) {
            const long long q = (long long)s * g.psz[1] + z + (long long)ld1 * xc;
            const float psi = cp.b_i[1][x] * src.psv[1][q] + cp.a_i[1][x] * ex;
            dst.psv[1][q] = psi;
            ex += psi;
        }
        float pn = pc[t] - kd[t] * (ez + ex);
        if (it < nt && k == sc) pn += src_amp(g.src_scale, stf[(long long)s * nt + it]);
        dst.p[so + k] = pn;
        dst.v[0][so + k] = vzn[t];
        dst.v[1][so + k] = vxn[t];
    }
}

}  // namespace

// (not with a free surface: its mirror images would be needed between the v and p updates)
bool fused_fwd_available(const Plan &pl) { return pl.nd == 2 && pl.dbuf && !pl.g.freesurf; }

hipError_t fwd_step_fused(const StepCtx &c, const Fields &src, const Fields &dst, int it) {
    const Plan &pl = *c.pl;
    const Views &w = *c.w;
    const int cm = c.march == 8 ? 8 : 4;
    if (c.zl) {   // tiled variant: 64 rows x 4 cm columns per workgroup
        int ez = 0, ex = 0;
        for (int s = 0; s < pl.nshot; ++s) {
            const int *b = &pl.fbox[((size_t)it * pl.nshot + s) * 6];
            ez = std::max(ez, b[1] - zalign(b[0]));
            ex = std::max(ex, b[3] - b[2]);
        }
        if (ez <= 0 || ex <= 0) return hipSuccess;
        const int gz = (ez + 63) / 64, gx = (ex + 4 * cm - 1) / (4 * cm);
        const int nxc = (gx + 7) / 8;
        dim3 grid((unsigned)(8 * gz), (unsigned)nxc, (unsigned)pl.nshot), block(64, 4, 1);
        const int *box = w.fbox + (size_t)it * pl.nshot * 6;
#define SMI_TILE(N_, CW_)                                                                      \
    do {                                                                                       \
        if (c.ev)                                                                              \
            hipExtLaunchKernelGGL((k_fused2d_tile<N_, CW_>), grid, block, 0, c.st, c.ev[0],     \
                                  c.ev[1], 0, pl.geom, src, dst, w.model, w.cpml, box, nxc,    \
                                  (const long long *)w.src_cell, c.stf, pl.g.nt, it);          \
        else                                                                                   \
            hipLaunchKernelGGL((k_fused2d_tile<N_, CW_>), grid, block, 0, c.st, pl.geom, src,   \
                               dst, w.model, w.cpml, box, nxc, (const long long *)w.src_cell,  \
                               c.stf, pl.g.nt, it);                                            \
    } while (0)
        if (pl.N == 2) { if (cm == 8) SMI_TILE(2, 8); else SMI_TILE(2, 4); }
        else { if (cm == 8) SMI_TILE(4, 8); else SMI_TILE(4, 4); }
#undef SMI_TILE
        return hipGetLastError();
    }
    int ez = 0, ex = 0;
    for (int s = 0; s < pl.nshot; ++s) {
        const int *b = &pl.fbox[((size_t)it * pl.nshot + s) * 6];
        ez = std::max(ez, b[1] - zalign(b[0]));
        ex = std::max(ex, b[3] - b[2]);
    }
    if (ez <= 0 || ex <= 0) return hipSuccess;
    const int gz = (ez + 255) / 256, gx = (ex + cm - 1) / cm;
    const int nxc = (gx + 7) / 8;
    dim3 grid((unsigned)(8 * gz), (unsigned)nxc, (unsigned)pl.nshot), block(64, 4, 1);
    const int *box = w.fbox + (size_t)it * pl.nshot * 6;
#define SMI_FUSED(N_, CM_)                                                                     \
    do {                                                                                       \
        if (c.ev)                                                                              \
            hipExtLaunchKernelGGL((k_fused2d<N_, CM_>), grid, block, 0, c.st, c.ev[0], c.ev[1], 0, \
                                  pl.geom, src, dst, w.model, w.cpml, box, nxc,                \
                                  (const long long *)w.src_cell, c.stf, pl.g.nt, it);          \
        else                                                                                   \
            hipLaunchKernelGGL((k_fused2d<N_, CM_>), grid, block, 0, c.st, pl.geom, src, dst,   \
                               w.model, w.cpml, box, nxc, (const long long *)w.src_cell, c.stf, \
                               pl.g.nt, it);                                                   \
    } while (0)
    if (pl.N == 2) { if (cm == 8) SMI_FUSED(2, 8); else SMI_FUSED(2, 4); }
    else { if (cm == 8) SMI_FUSED(4, 8); else SMI_FUSED(4, 4); }
#undef SMI_FUSED
    return hipGetLastError();
}

}  // namespace smi
