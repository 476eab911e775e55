// fused2d.hip -- one kernel per 2D time step: v update, p update, CPML, source injection and
// receiver sampling (eq. 3-4, Sec. 2.1, Alg. 2 forward loop), for every shot of the batch.
//
// Work decomposition.  A workgroup owns a z-strip of one shot's computing box (lanes along
// z, one coalesced row per wavefront, 2N-1 halo lanes at each end) and a range of L columns
// along x, which it marches through in chunks of T columns.  Per lane, registers hold a
// window of p^n over the columns [xc - (2N-1), xc + T + 2N - 1) and of v_x^{n+1/2} over
// [xc - N, xc + T + N - 1); both windows slide by T per chunk, so every p and v_x value is
// loaded once per march and the x-derivatives never leave registers.  Per chunk: all global
// loads of the chunk are issued together, v_x of the T new columns is formed in registers,
// p of the chunk goes to LDS (barrier), v_z is formed from its z-neighbours and goes to LDS
// (barrier), and p^{n+1} is formed from v_z (LDS) and v_x (registers).
// Level n is read from one buffer and level n+1 written to the other, so values a workgroup
// reads in its halo are never overwritten by a neighbour during the step.  The zero ghost
// nodes around the padded grid make every stencil read valid without per-lane checks; the
// CPML memory variables are touched only on (uniform) branches for slab columns and on the
// lanes of slab rows.  Workgroups are ordered chunk-major with the shot fastest and remapped
// so that each XCD takes a contiguous range: the shots of one region share the model in L2.
#include "smi_internal.hpp"
#include "device.hpp"

namespace smi {

namespace {

struct Recv2 {
    const int *off;          // [nshot][M2 + 1]
    const int *z;
    const long long *out;
    const int *stride;
};

struct March2 {
    const float *src;        // field section at level n (p of shot 0)
    float *dst;              // field section at level n + 1
    int o_vz, o_vx;          // offsets of the v_z, v_x arrays in a section (floats)
    int o_pzp, o_pzv, o_pxp, o_pxv;   // offsets of the CPML memory variables
    int P, psz0, psz1;       // per-shot strides
    const float *model;      // dt kappa; dt beta_z at +P, dt beta_x at +2P
    const float *cpz, *cpx;  // CPML profiles per axis: a_i | b_i | a_h | b_h
    int M1, M2, nb, ld1, org, W;
    float cz[kMaxN], cx[kMaxN];
    float src_scale;
};

// One wavefront = one z-strip of 64 lanes (TZ = 64 - 2(2N-1) owned rows plus the halo rows
// each side) marching through L columns in chunks of T; the four wavefronts of a workgroup
// are independent (no workgroup barrier), each with its own LDS slice for the z-neighbour
// exchange.  The march is software-pipelined: the loads of chunk c+1 are issued before the
// arithmetic and the stores of chunk c, so the wait for a chunk's data never includes the
// completion of the previous chunk's stores (vector-memory counters retire in order).
template <int N, int T>
struct Chunk {
    float p[T], vo[T], bx[T], vz[T], bz[T], kd[T];
};

template <int N, int T>
__global__ __launch_bounds__(256) void k_fwd2d(March2 a, const int *__restrict__ box, int nshot,
                                               int ngrp, int L, int order,
                                               const long long *__restrict__ src_cell,
                                               const float *__restrict__ stf, int nt, int it,
                                               Recv2 rv, float *__restrict__ dcal) {
    constexpr int H = 2 * N - 1, TZ = 64 - 2 * H;
    constexpr int PW = T + 2 * H, VW = T + 2 * N - 1;
    __shared__ float lds[4][2][T][64];

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // order 0: shot fastest, XCD-contiguous; 1: shot slowest, XCD-contiguous; 2: shot slowest
    const int logical = order == 2 ? (int)blockIdx.x : xcd_remap(blockIdx.x, gridDim.x);
    int s, grp, cxk;
    if (order == 0) {
        s = logical % nshot;
        const int rest = logical / nshot;
        grp = rest % ngrp;
        cxk = rest / ngrp;
    } else {
        const int per = (int)gridDim.x / nshot;
        s = logical / per;
        const int rest = logical % per;
        grp = rest % ngrp;
        cxk = rest / ngrp;
    }
    const int *b = box + 6 * s;
    const int bz0 = b[0], bz1 = b[1], bx0 = b[2], bx1 = b[3];
    const int zs = bz0 + (grp * 4 + wave) * TZ, ze = min(zs + TZ, bz1);
    const int xs = bx0 + cxk * L, xe = min(xs + L, bx1);
    if (zs >= ze || xs >= xe) return;            // per wavefront: no workgroup barrier follows
    float(*sp)[64] = lds[wave][0];
    float(*svz)[64] = lds[wave][1];

    const int M2 = a.M2, nb = a.nb, ld1 = a.ld1;
    const int XM = M2 + GH - 1;                 // last column inside the ghost frame
    const int z = zs - H + lane;
    const int zl = min(z, ze + H - 1);          // lanes past the halo read a valid node
    const bool zbox = z >= bz0 && z < bz1;
    const bool own = z >= zs && z < ze;
    const bool vzc = zbox && lane >= N - 1 && lane + N < 64;
    const int zsl = zbox ? slab_index(z, a.M1, nb) : -1;
    const int k0 = a.org + zl;                  // offset of (zl, x = 0)

    const float *__restrict__ Ps = a.src + s * a.P;
    const float *__restrict__ VZs = a.src + a.o_vz + s * a.P;
    const float *__restrict__ VXs = a.src + a.o_vx + s * a.P;
    float *__restrict__ Pd = a.dst + s * a.P;
    float *__restrict__ VZd = a.dst + a.o_vz + s * a.P;
    float *__restrict__ VXd = a.dst + a.o_vx + s * a.P;
    const float *__restrict__ KD = a.model;
    const float *__restrict__ BZ = a.model + a.P;
    const float *__restrict__ BX = a.model + 2 * a.P;
    float cz[N], cx[N];
#pragma unroll
    for (int l = 0; l < N; ++l) { cz[l] = a.cz[l]; cx[l] = a.cx[l]; }
    const int srck = (int)src_cell[s];

    // v_x at column j from the p window (p(j - N + 1 + q) = pw[o + q]); only owned rows need it
    auto vx_at = [&](int j, const float *pw, int o, float vold, float bb) -> float {
        if (!(own && j >= bx0 && j < bx1)) return vold;
        float e = 0.f;
#pragma unroll
        for (int l = 1; l <= N; ++l) e += cx[l - 1] * (pw[o + N - 1 + l] - pw[o + N - l]);
        const int xsl = slab_index(j, M2, nb);
        const bool wr = j >= xs && j < xe;
        if (xsl >= 0) {
            const int q = s * a.psz1 + z + ld1 * xsl;
            const float psi = a.cpx[3 * M2 + j] * a.src[a.o_pxp + q] + a.cpx[2 * M2 + j] * e;
            if (wr) a.dst[a.o_pxp + q] = psi;
            e += psi;
        }
        const float v = vold - bb * e;
        if (wr) VXd[k0 + ld1 * j] = v;
        return v;
    };
    auto load = [&](int xc, Chunk<N, T> &d) {
#pragma unroll
        for (int c = 0; c < T; ++c) {
            const int kp = k0 + ld1 * min(xc + H + c, XM);
            const int kv = k0 + ld1 * min(xc + N - 1 + c, XM);
            const int kc = k0 + ld1 * min(xc + c, XM);
            d.p[c] = Ps[kp];
            d.vo[c] = VXs[kv];
            d.bx[c] = BX[kv];
            d.vz[c] = VZs[kc];
            d.bz[c] = BZ[kc];
            d.kd[c] = KD[kc];
        }
    };

    float pw[PW], vw[VW];
#pragma unroll
    for (int q = 0; q < 2 * H; ++q) pw[q] = Ps[k0 + ld1 * (xs - H + q)];
    {
        float vo[2 * N - 1], bb[2 * N - 1];
#pragma unroll
        for (int q = 0; q < 2 * N - 1; ++q) {
            const int kk = k0 + ld1 * (xs - N + q);
            vo[q] = VXs[kk];
            bb[q] = BX[kk];
        }
#pragma unroll
        for (int q = 0; q < 2 * N - 1; ++q) vw[q] = vx_at(xs - N + q, pw, q, vo[q], bb[q]);
    }

    auto compute = [&](int xc, const Chunk<N, T> &d) {
#pragma unroll
        for (int c = 0; c < T; ++c) pw[2 * H + c] = d.p[c];
#pragma unroll
        for (int c = 0; c < T; ++c) vw[2 * N - 1 + c] = vx_at(xc + N - 1 + c, pw, c + H, d.vo[c], d.bx[c]);
        // v_z from p of the chunk: z-neighbours through this wavefront's LDS slice
#pragma unroll
        for (int c = 0; c < T; ++c) sp[c][lane] = pw[H + c];
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int c = 0; c < T; ++c) {
            const int x = xc + c;
            float v = d.vz[c];
            if (vzc && x < xe) {
                float e = 0.f;
#pragma unroll
                for (int l = 1; l <= N; ++l) e += cz[l - 1] * (sp[c][lane + l] - sp[c][lane + 1 - l]);
                if (zsl >= 0) {
                    const int q = s * a.psz0 + zsl + a.W * x;
                    const float psi = a.cpz[3 * a.M1 + z] * a.src[a.o_pzp + q] + a.cpz[2 * a.M1 + z] * e;
                    if (own) a.dst[a.o_pzp + q] = psi;
                    e += psi;
                }
                v = v - d.bz[c] * e;
                if (own) VZd[k0 + ld1 * x] = v;
            }
            svz[c][lane] = v;
        }
        __builtin_amdgcn_wave_barrier();
        if (own) {
#pragma unroll
            for (int c = 0; c < T; ++c) {
                const int x = xc + c;
                if (x >= xe) break;
                float ez = 0.f, ex = 0.f;
#pragma unroll
                for (int l = 1; l <= N; ++l) ez += cz[l - 1] * (svz[c][lane + l - 1] - svz[c][lane - l]);
                if (zsl >= 0) {
                    const int q = s * a.psz0 + zsl + a.W * x;
                    const float psi = a.cpz[a.M1 + z] * a.src[a.o_pzv + q] + a.cpz[z] * ez;
                    a.dst[a.o_pzv + q] = psi;
                    ez += psi;
                }
#pragma unroll
                for (int l = 1; l <= N; ++l) ex += cx[l - 1] * (vw[c + N + l - 1] - vw[c + N - l]);
                const int xsl = slab_index(x, M2, nb);
                if (xsl >= 0) {
                    const int q = s * a.psz1 + z + ld1 * xsl;
                    const float psi = a.cpx[M2 + x] * a.src[a.o_pxv + q] + a.cpx[x] * ex;
                    a.dst[a.o_pxv + q] = psi;
                    ex += psi;
                }
                const int k = k0 + ld1 * x;
                float pn = pw[H + c] - d.kd[c] * (ez + ex);
                if (k == srck) pn += a.src_scale * stf[(long long)s * nt + it];
                Pd[k] = pn;
                const int r0 = rv.off[s * (M2 + 1) + x];
                const int r1 = rv.off[s * (M2 + 1) + x + 1];
                for (int r = r0; r < r1; ++r)
                    if (rv.z[r] == z) dcal[rv.out[r] + (long long)it * rv.stride[r]] = pn;
            }
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int q = 0; q < 2 * H; ++q) pw[q] = pw[q + T];
#pragma unroll
        for (int q = 0; q < 2 * N - 1; ++q) vw[q] = vw[q + T];
    };

    Chunk<N, T> A, Bc;
    load(xs, A);
    for (int xc = xs; xc < xe; xc += 2 * T) {
        load(xc + T, Bc);              // prefetch (clamped; unused past the end)
        compute(xc, A);
        if (xc + T >= xe) break;
        load(xc + 2 * T, A);
        compute(xc + T, Bc);
    }
}

}  // namespace

bool fused_fwd_available(const Plan &pl) {
    // 32-bit offsets inside one field section
    double sec = (double)pl.nshot * ((double)pl.P * 3 + 2.0 * (pl.geom.psz[0] + pl.geom.psz[1]));
    return pl.nd == 2 && sec < 2.0e9;
}

hipError_t fwd_step_fused(const StepCtx &c, const Fields &src, const Fields &dst, int it,
                          float *dcal) {
    const Plan &pl = *c.pl;
    const Views &w = *c.w;
    const int H = 2 * pl.N - 1;
    int ez = 0, ex = 0;
    for (int s = 0; s < pl.nshot; ++s) {
        const int *b = &pl.fbox[((size_t)it * pl.nshot + s) * 6];
        ez = std::max(ez, b[1] - b[0]);
        ex = std::max(ex, b[3] - b[2]);
    }
    if (ez <= 0 || ex <= 0) return hipSuccess;
    const int TZ = 64 - 2 * H;
    int nstripw = (ez + TZ - 1) / TZ;         // wavefront strips
    int ngrp = (nstripw + 3) / 4;             // 4 strips per workgroup
    // chunk option (tuning): v = 1000 * (2 order + t2) + L
    const int opt = pl.chunk > 0 ? pl.chunk : 16;
    const int order = (opt / 1000) / 2;
    const bool t2 = (opt / 1000) % 2 == 1;
    int L = opt % 1000;
    int nchunk = (ex + L - 1) / L;
    unsigned G = (unsigned)(pl.nshot * ngrp * nchunk);

    March2 a{};
    a.src = src.p;
    a.dst = dst.p;
    a.o_vz = (int)(src.v[0] - src.p);
    a.o_vx = (int)(src.v[1] - src.p);
    a.o_pzp = (int)(src.psp[0] - src.p);
    a.o_pzv = (int)(src.psv[0] - src.p);
    a.o_pxp = (int)(src.psp[1] - src.p);
    a.o_pxv = (int)(src.psv[1] - src.p);
    a.P = (int)pl.P;
    a.psz0 = (int)pl.geom.psz[0];
    a.psz1 = (int)pl.geom.psz[1];
    a.model = w.model.kdt;
    a.cpz = w.cpml.a_i[0];
    a.cpx = w.cpml.a_i[1];
    a.M1 = pl.M[0];
    a.M2 = pl.M[1];
    a.nb = pl.g.nb;
    a.ld1 = pl.ld1;
    a.org = (int)pl.org;
    a.W = pl.geom.W;
    for (int l = 0; l < kMaxN; ++l) { a.cz[l] = pl.geom.c[0][l]; a.cx[l] = pl.geom.c[1][l]; }
    a.src_scale = pl.geom.src_scale;
    const int *box = w.fbox + (size_t)it * pl.nshot * 6;
    Recv2 rv{w.rcol_off, w.rcol_z, w.rcol_out, w.rcol_stride};
#define SMI_MARCH(N_, T_)                                                                        \
    hipLaunchKernelGGL((k_fwd2d<N_, T_>), dim3(G), dim3(256), 0, c.st, a, box, pl.nshot, ngrp, L, order, \
                       (const long long *)w.src_cell, c.stf, pl.g.nt, it, rv, dcal)
    if (pl.N == 2) { if (t2) SMI_MARCH(2, 2); else SMI_MARCH(2, 4); }
    else { if (t2) SMI_MARCH(4, 2); else SMI_MARCH(4, 4); }
#undef SMI_MARCH
    return hipGetLastError();
}

}  // namespace smi
