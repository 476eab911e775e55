// step2d.hip -- the fused 2D time step: v update, p update, CPML, one-tap source injection
// (eq. 3-4, Sec. 2.1, Alg. 2 forward loop) for every shot of a batch in one launch, reading
// level n from one buffer set and writing level n + 1 to the other.
//
// A wavefront owns 64 consecutive z rows of one shot (a 256-byte storage line pair, aligned to
// 128 bytes) over a run of C columns and marches along x, one column per iteration:
//   * along x the stencils run in registers: a window of 2N values of p^n gives the new v_x at
//     column c, and a window of the last 2N new v_x gives the x part of the divergence at
//     column j = c - N + 1, where p is updated;
//   * along z the stencils read the wavefront's own LDS slice: p^n of column j (64 own rows and
//     2N - 1 rows each side, loaded by the first lanes) and the new v_z of column j (own rows
//     and the N rows above, N - 1 below, formed by lanes 0 .. 2N-2 a second time);
//   * every column is loaded once per wavefront and every cell stored once, by its owner; the
//     loads of column c + 1 are issued before the arithmetic of column c;
//   * no workgroup barrier: a wavefront reads only its own LDS slice.
// Cells outside the shot's computing box are not written, and a halo value outside the box
// keeps its old level, as in the half-step kernels, so the two give bitwise the same fields.
// The CPML memory variables exist only in the absorbing slabs; a wavefront whose rows or
// columns (with their halos) touch a slab runs the variant with the memory-variable updates,
// every other one runs a variant with none, chosen once per wavefront.
// The workgroups are ordered so that consecutive ones on an XCD take one tile of every shot:
// the model under a tile is read from HBM once per step for the whole batch.
// Side work rides on extra workgroups after the step's own: the receivers of the previous step
// (sampled from level n, which this launch only reads) and the bands of a saved level n.
#include <algorithm>

#include <hip/hip_ext.h>

#include "smi_internal.hpp"
#include "device.hpp"
#include "side.hpp"

namespace smi {

namespace {

struct S2 {
    int nshot;
    int nstrip;     // 64-row strips of the union of the shots' boxes
    int nrun;       // C-column runs of that union
    int z0;         // first row of strip 0
    int run0;       // absolute index of run 0 (run r covers columns [C r, C r + C))
    int nmain;      // workgroups of the step; blocks from nmain on carry side work
    int nrecb;      // side-work blocks sampling receivers (after the step's blocks)
    unsigned rbytes;    // bytes from the model to the end of the second field set
};

// Loads of one column of the march, kept in registers until the column is processed.
struct VCol {           // v_x column c: p(c + N), v_x(c), dt beta_x(c), memory variable of d_x p
    float p, vx, bx, ps;
};
struct PCol {           // p column j: v_z, dt beta_z, dt kappa, the halo rows (one register:
                        // p on lanes 0 .. 4N-3, v_z and dt beta_z on the next 2N-1 lanes each),
                        // memory variables
    float vz, bz, kd, h, pz, hpz, pvz, pvx;
};

// Raw buffer access through one resource over the region the step touches (the model, then
// both field sets): a loop-invariant 32-bit lane offset plus a wave-uniform byte offset per
// array and column.  Accesses past the resource's end read 0 and write nothing.
__device__ __forceinline__ float bld(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
}
__device__ __forceinline__ void bst(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, vo, so, 0);
}

// One wavefront's march over columns [x0, x1) of rows [zs, zs + 64) of shot s (all arguments
// wave-uniform).
//   ZP: the rows (with the N halo rows of v_z) touch a z slab; XP: the columns (with the N
//   halo columns of v_x) touch an x slab.  D: columns loaded ahead of the one processed.
// The main loop runs blocks of 8 columns, unrolled, so that the register windows and the ring
// of loads issued D columns ahead are renamed rather than copied; the columns of the last
// block past the run are computed and not stored.  Every byte offset is non-negative: the
// model sits in front of the fields and the ghost frame (GH columns, GH rows) in front of
// every array, so a column as low as x0 - 2N + 1 stays inside it; reads past the region's
// end return 0 and are never used.
template <int N, int C, int D, bool ZP, bool XP>
__device__ __forceinline__ void march2d(const Geom &g, const Fields &A, const Fields &B,
                                        const Model &m, const Cpml &cp, unsigned rbytes,
                                        const int b0, const int b1, const int xlo, const int xhi,
                                        int s, int zs, int x0, int x1, int scol, int sr,
                                        float amp, float *LP, float *LV) {
    constexpr int HP = 2 * N - 1;             // p halo rows per side
    constexpr int UB = 8;                     // columns per unrolled block
    static_assert(UB % (2 * N) == 0 && UB % D == 0, "block of 8 columns");
    const int lane = threadIdx.x & 63;
    const char *rb = (const char *)m.kdt;     // the region starts with the model
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void *)rb, (short)0, (int)rbytes, 0x00020000);
    auto off = [&](const float *p) { return (unsigned)((const char *)p - rb); };
    const long long so = (long long)s * g.P;
    const int ld1 = g.ld1;
    const unsigned colb = 4u * (unsigned)ld1;  // bytes per column
    const int r = zs + lane;                   // own row
    const bool own = r >= b0 && r < b1;
    const bool rowok = r >= 0 && r < g.M[0];
    // halo rows: p (lanes 0 .. 2 HP - 1), v_z (lanes 0 .. 2N - 2 compute them)
    const int rp = lane < HP ? zs - HP + lane : zs + 64 + (lane - HP);
    const bool hp = lane < 2 * HP;
    const int rv = lane < N ? zs - N + lane : zs + 64 + (lane - N);
    const bool hv = lane < 2 * N - 1;
    const bool hvbox = hv && rv >= b0 && rv < b1;
    const bool hrow = hv && rv >= 0 && rv < g.M[0];
    // CPML along z: slab rows of the own row and of the v_z halo row (-1: none), and their
    // profile values, zero outside the slabs (the memory variable then stays out of the sums)
    const int zci = ZP && rowok ? slab_index(r, g.M[0], g.nb) : -1;
    const int zch = ZP && hrow ? slab_index(rv, g.M[0], g.nb) : -1;
    float zah = 0.f, zbh = 0.f, zai = 0.f, zbi = 0.f, hah = 0.f, hbh = 0.f;
    if (ZP) {
        if (zci >= 0) {
            zah = cp.a_h[0][r];
            zbh = cp.b_h[0][r];
            zai = cp.a_i[0][r];
            zbi = cp.b_i[0][r];
        }
        if (zch >= 0) {
            hah = cp.a_h[0][rv];
            hbh = cp.b_h[0][rv];
        }
    }
    // uniform byte offsets of the arrays (this shot's fields), relative to the region
    const unsigned a_kdt = 0u, a_bdz = off(m.bdt[0]), a_bdx = off(m.bdt[1]);
    const unsigned a_pA = off(A.p + so), a_vzA = off(A.v[0] + so), a_vxA = off(A.v[1] + so);
    const unsigned a_pB = off(B.p + so), a_vzB = off(B.v[0] + so), a_vxB = off(B.v[1] + so);
    const unsigned a_pAN = a_pA + (unsigned)N * colb;                // p(c + N) at column c
    const unsigned a_pzA = off(A.psp[0] + (long long)s * g.psz[0]);
    const unsigned a_vpzA = off(A.psv[0] + (long long)s * g.psz[0]);
    const unsigned a_pzB = off(B.psp[0] + (long long)s * g.psz[0]);
    const unsigned a_vpzB = off(B.psv[0] + (long long)s * g.psz[0]);
    const unsigned a_pxA = off(A.psp[1] + (long long)s * g.psz[1]);
    const unsigned a_vpxA = off(A.psv[1] + (long long)s * g.psz[1]);
    const unsigned a_pxB = off(B.psp[1] + (long long)s * g.psz[1]);
    const unsigned a_vpxB = off(B.psv[1] + (long long)s * g.psz[1]);
    // loop-invariant lane offsets: own row; the merged halo load (relative to dt beta_z)
    const unsigned vr = 4u * (unsigned)(g.org + r);
    unsigned vh = vr;
    if (lane < 2 * HP) vh = a_pA - a_bdz + 4u * (unsigned)(g.org + rp);
    else if (lane < 2 * HP + 2 * N - 1) {
        const int h = lane - 2 * HP;
        vh = a_vzA - a_bdz + 4u * (unsigned)(g.org + (h < N ? zs - N + h : zs + 64 + (h - N)));
    } else if (lane < 2 * HP + 2 * (2 * N - 1)) {
        const int h = lane - 2 * HP - (2 * N - 1);
        vh = 4u * (unsigned)(g.org + (h < N ? zs - N + h : zs + 64 + (h - N)));
    }
    // memory variables: z slabs (zc + W x), x slabs (z + ld1 xc); rows outside the grid read
    // row 0 and their values are never used
    const unsigned vzi = 4u * (unsigned)(zci >= 0 ? zci : 0);
    const unsigned vzh = 4u * (unsigned)(zch >= 0 ? zch : 0);
    const unsigned vxr = 4u * (unsigned)(rowok ? r : 0);
    const unsigned wz = 4u * (unsigned)g.W;   // bytes per column of a z slab
    auto xslab = [&](int c) { return c >= 0 && c < g.M[1] ? slab_index(c, g.M[1], g.nb) : -1; };
    auto zcol = [&](int j) { return wz * (unsigned)min(max(j, 0), g.M[1] - 1); };
    const float samp = r == sr ? amp : 0.f;

    auto ldv = [&](int c) {
        VCol L;
        const unsigned cc = (unsigned)c * colb;
        L.p = bld(rs, vr, a_pAN + cc);
        L.vx = bld(rs, vr, a_vxA + cc);
        L.bx = bld(rs, vr, a_bdx + cc);
        L.ps = 0.f;
        if (XP) {
            const int xc = xslab(c);
            if (xc >= 0) L.ps = bld(rs, vxr, a_pxA + (unsigned)xc * colb);
        }
        return L;
    };
    auto ldp = [&](int j) {
        PCol L;
        const unsigned cj = (unsigned)j * colb;
        L.vz = bld(rs, vr, a_vzA + cj);
        L.bz = bld(rs, vr, a_bdz + cj);
        L.kd = bld(rs, vr, a_kdt + cj);
        L.h = bld(rs, vh, a_bdz + cj);
        L.pz = L.hpz = L.pvz = L.pvx = 0.f;
        if (ZP) {
            // every lane loads (from its slab row, or row 0 of the slab); the profile zeros
            // drop what lies outside
            const unsigned zc = zcol(j);
            L.pz = bld(rs, vzi, a_pzA + zc);
            L.pvz = bld(rs, vzi, a_vpzA + zc);
            L.hpz = bld(rs, vzh, a_pzA + zc);
        }
        if (XP) {
            const int xc = xslab(j);
            if (xc >= 0) L.pvx = bld(rs, vxr, a_vpxA + (unsigned)xc * colb);
        }
        return L;
    };

    // x window of p^n: pw[d + N - 1] = p(c + d), d = -(N-1) .. N
    float pw[2 * N];
    // window of new v_x: vw[d + 2N - 1] = v_x^{n+1/2}(c + d), d = -(2N-1) .. 0
    float vw[2 * N];
    const int cstart = x0 - N;                 // first v_x column
    const int cmain = x0 + N - 1;              // first column whose p update (at x0) runs
    const int cend = x1 + N - 1;               // one past the last v_x column

    // v_x^{n+1/2} at column c (eq. 3 first row, x part, CPML)
    auto vstep = [&](int c, const VCol &L) {
#pragma unroll
        for (int d = 0; d < 2 * N - 1; ++d) pw[d] = pw[d + 1];
        pw[2 * N - 1] = L.p;
        float e = 0.f;
#pragma unroll
        for (int l = 1; l <= N; ++l) e += g.c[1][l - 1] * (pw[l + N - 1] - pw[N - l]);
        const bool mine = c >= x0 && c < x1;
        if (XP) {
            const int xc = xslab(c);
            if (xc >= 0) {
                const float psi = cp.b_h[1][c] * L.ps + cp.a_h[1][c] * e;
                if (own && mine) bst(rs, vxr, a_pxB + (unsigned)xc * colb, psi);
                e += psi;
            }
        }
        const float vxn = c >= xlo && c < xhi ? L.vx - L.bx * e : L.vx;
        if (own && mine) bst(rs, vr, a_vxB + (unsigned)c * colb, vxn);
#pragma unroll
        for (int d = 0; d < 2 * N - 1; ++d) vw[d] = vw[d + 1];
        vw[2 * N - 1] = vxn;
    };
    // p^{n+1} at column j (eq. 3 second row, CPML, source); v_z^{n+1/2} of column j on the way
    auto pstep = [&](int j, const PCol &L) {
        const bool mine = j < x1;
        const float pj = pw[0];
        LP[lane + HP] = pj;
        if (hp) LP[lane < HP ? lane : lane + 64] = L.h;
        // the halo v_z rows' old value and dt beta_z, from the lanes that loaded them
        const float hvo = __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(
            4 * (lane + 2 * HP), __builtin_bit_cast(int, L.h)));
        const float hbz = __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(
            4 * (lane + 2 * HP + 2 * N - 1), __builtin_bit_cast(int, L.h)));
        __builtin_amdgcn_wave_barrier();
        float ez = 0.f;
#pragma unroll
        for (int l = 1; l <= N; ++l) ez += g.c[0][l - 1] * (LP[lane + HP + l] - LP[lane + HP - l + 1]);
        if (ZP) {
            const float psi = zbh * L.pz + zah * ez;
            if (own && mine && zci >= 0) bst(rs, vzi, a_pzB + zcol(j), psi);
            ez = zci >= 0 ? ez + psi : ez;
        }
        const float vzn = own ? L.vz - L.bz * ez : L.vz;
        float hz = 0.f;
        {
            const int i = hv ? rv - zs + HP : HP;   // LDS index of the halo v_z row's p
#pragma unroll
            for (int l = 1; l <= N; ++l) hz += g.c[0][l - 1] * (LP[i + l] - LP[i - l + 1]);
        }
        if (ZP) {
            const float psi = hbh * L.hpz + hah * hz;
            hz = zch >= 0 ? hz + psi : hz;
        }
        const float hvn = hvbox ? hvo - hbz * hz : hvo;
        __builtin_amdgcn_wave_barrier();
        LV[lane + N] = vzn;
        if (hv) LV[lane < N ? lane : lane + 64] = hvn;
        __builtin_amdgcn_wave_barrier();
        // z part first, then x (the order of the half-step kernels)
        float dz = 0.f;
#pragma unroll
        for (int l = 1; l <= N; ++l) dz += g.c[0][l - 1] * (LV[lane + N + l - 1] - LV[lane + N - l]);
        if (ZP) {
            const float psi = zbi * L.pvz + zai * dz;
            if (own && mine && zci >= 0) bst(rs, vzi, a_vpzB + zcol(j), psi);
            dz = zci >= 0 ? dz + psi : dz;
        }
        float dx = 0.f;
#pragma unroll
        for (int l = 1; l <= N; ++l) dx += g.c[1][l - 1] * (vw[l + N - 1] - vw[N - l]);
        if (XP) {
            const int xc = xslab(j);
            if (xc >= 0) {
                const float psi = cp.b_i[1][j] * L.pvx + cp.a_i[1][j] * dx;
                if (own && mine) bst(rs, vxr, a_vpxB + (unsigned)xc * colb, psi);
                dx += psi;
            }
        }
        float sdiv = 0.f;
        sdiv += dz;
        sdiv += dx;
        float pn = pj - L.kd * sdiv;
        if (j == scol) pn += samp;
        if (own && mine) {
            const unsigned cj = (unsigned)j * colb;
            bst(rs, vr, a_pB + cj, pn);
            bst(rs, vr, a_vzB + cj, vzn);
        }
        __builtin_amdgcn_wave_barrier();
    };

#pragma unroll
    for (int d = 0; d < 2 * N - 1; ++d) pw[d + 1] = bld(rs, vr, a_pA + (unsigned)(cstart - N + 1 + d) * colb);
#pragma unroll
    for (int d = 0; d < 2 * N; ++d) vw[d] = 0.f;
    // rings of the loads issued ahead: v_x column c in slot (c - cstart) % D, p column j in
    // slot (j - x0) % D
    VCol vq[D];
    PCol pq[D];
#pragma unroll
    for (int q = 0; q < D; ++q) vq[q] = ldv(cstart + q);
#pragma unroll
    for (int q = 0; q < D; ++q) pq[q] = ldp(x0 + q);
    // prologue: the N halo columns of v_x before the run and its first N - 1 own columns
#pragma unroll
    for (int u = 0; u < 2 * N - 1; ++u) {
        const VCol cv = vq[u % D];
        vq[u % D] = ldv(cstart + u + D);
        vstep(cstart + u, cv);
    }
    for (int cb = cmain; cb < cend; cb += UB) {
#pragma unroll
        for (int u = 0; u < UB; ++u) {
            const int c = cb + u, j = c - N + 1;
            const int sv = (u + 2 * N - 1) % D, sq = u % D;
            const VCol cv = vq[sv];
            const PCol cq = pq[sq];
            // the loads D columns ahead go out before this column's arithmetic
            vq[sv] = ldv(c + D);
            pq[sq] = ldp(j + D);
            vstep(c, cv);
            pstep(j, cq);
        }
    }
}

template <int N, int C, int D>
__global__ __launch_bounds__(256) void k_step2d(Geom g, Fields A, Fields B, Model m, Cpml cp,
                                                const int *__restrict__ box, S2 sg,
                                                const long long *__restrict__ src_cell,
                                                const float *__restrict__ stf, int nt, int it,
                                                Ext ex, BandArg sv) {
    __shared__ float lp[4][64 + 4 * N - 2];
    __shared__ float lv[4][64 + 2 * N - 1];
    const int bid = (int)blockIdx.x;
    if (bid >= sg.nmain) {
        // side work: the receivers of the previous step from level n (this launch writes only
        // the other buffer), then the band cells of a saved level n
        const int q = bid - sg.nmain;
        if (q < sg.nrecb) {
            const int nthr = sg.nrecb * 256;
            for (int rr = q * 256 + (int)threadIdx.x; rr < ex.rv.R; rr += nthr)
                sample_receiver(g, A.p, ex.rv, ex.dcal, ex.it, ex.status, rr);
        } else if (sv.buf) {
            band_lin(g, A, sv, q - sg.nrecb, (int)threadIdx.x, 0, 2);
        }
        return;
    }
    // the wavefront's tile: every quantity below is uniform over the wavefront
    const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int L = xcd_remap(bid, sg.nmain);
    const int W = L * 4 + wv;                  // logical wavefront: shot fastest, then strip, run
    const int s = W % sg.nshot;
    const int t = W / sg.nshot;
    const int k = t % sg.nstrip;
    const int rr = t / sg.nstrip;
    if (rr >= sg.nrun) return;
    const int *b = box + 6 * s;
    const int b0 = b[0], b1 = b[1], b2 = b[2], b3 = b[3];
    const int zs = sg.z0 + 64 * k;
    if (zs >= b1 || zs + 64 <= b0) return;
    const int run = sg.run0 + rr;
    const int x0 = max(C * run, b2), x1 = min(C * run + C, b3);
    if (x0 >= x1) return;
    const long long sc = src_cell[s];
    const float amp = sc >= 0 && it < nt ? src_amp(g.src_scale, stf[(long long)s * nt + it]) : 0.f;
    // source (one-tap): its row and column in this shot's field, or none
    const int sr = sc >= 0 ? (int)((sc - g.org) % g.ld1) : -1;
    const int scol = sc >= 0 ? (int)((sc - g.org) / g.ld1) : -1 - (1 << 20);
    const bool zp = zs - N < g.nb || zs + 64 + N - 1 > g.M[0] - g.nb - 1;
    const bool xp = x0 - N < g.nb || x1 + N - 1 > g.M[1] - g.nb - 1;
    float *LP = lp[wv];
    float *LV = lv[wv];
    // the slab variants carry more loads per column: a shallower ring keeps their registers
    // within the interior variant's
    constexpr int DS = D > 2 ? 2 : D;
    const unsigned rn = sg.rbytes;
    if (zp) {
        if (xp) march2d<N, C, DS, true, true>(g, A, B, m, cp, rn, b0, b1, b2, b3, s, zs, x0, x1, scol, sr, amp, LP, LV);
        else march2d<N, C, DS, true, false>(g, A, B, m, cp, rn, b0, b1, b2, b3, s, zs, x0, x1, scol, sr, amp, LP, LV);
    } else {
        if (xp) march2d<N, C, DS, false, true>(g, A, B, m, cp, rn, b0, b1, b2, b3, s, zs, x0, x1, scol, sr, amp, LP, LV);
        else march2d<N, C, D, false, false>(g, A, B, m, cp, rn, b0, b1, b2, b3, s, zs, x0, x1, scol, sr, amp, LP, LV);
    }
}

// ---------------------------------------------------------------------------- tiled step
// One workgroup per (shot, 64-row strip, TX-column run), NW = TX / 8 wavefronts.  Every load of
// the tile is issued at once, before any arithmetic (the workgroup's whole input is in flight,
// so a few resident workgroups per CU keep HBM busy), then:
//   1. p^n of the tile and of its halos (2N - 1 rows above and below the tile's columns,
//      2N - 1 columns either side of its rows) goes to LDS; barrier;
//   2. the new v_x on the tile's rows over the columns [xb - N, xb + TX + N - 1) (N halo
//      columns left, N - 1 right, computed again by the neighbouring tile) and the new v_z on
//      the tile's columns over the rows [zs - N, zs + 64 + N - 1), both from p^n in LDS,
//      go to LDS (and the tile's own cells to HBM); barrier;
//   3. the new p on the tile from both, plus the one-tap source.
// A lane is one row of the strip (z is the contiguous axis); wavefront w owns the p and v_z
// columns [xb + 8 w, xb + 8 w + 8) and a share of the v_x columns.  The arithmetic, the box
// rules (a cell outside the shot's computing box keeps its old level; only the tile's own
// cells inside the box are stored) and the CPML memory variables are those of the half-step
// kernels, term by term, so both give bitwise the same fields.  Loads past the padded grid
// read what lies there (or 0 past the region's resource): the values reach only cells that
// are not stored.
template <int N, int TX>
struct T2 {
    static constexpr int HP = 2 * N - 1;          // p halo (rows or columns) per side
    static constexpr int NW = TX / 8;             // wavefronts
    static constexpr int NT = 64 * NW;            // threads
    static constexpr int LDP = 64 + 2 * HP;       // LDS rows per p column
    static constexpr int PC = TX + 2 * HP;        // p columns in LDS, from xb - HP
    static constexpr int VXC = TX + 2 * N - 1;    // v_x columns, from xb - N
    static constexpr int LDZ = 64 + 2 * N - 1;    // LDS rows per v_z column, from zs - N
    static constexpr int PMC = (PC + NW - 1) / NW;     // p columns each wavefront loads
    static constexpr int VCW = (VXC + NW - 1) / NW;    // v_x columns per wavefront
    static constexpr int NH = 2 * HP * TX;             // p halo-row cells of the tile's columns
    static constexpr int HPT = (NH + NT - 1) / NT;     // of them per thread
    static constexpr int NVH = (2 * N - 1) * TX;       // v_z halo-row cells
    static constexpr int LDS = PC * LDP + VXC * 64 + TX * LDZ;    // floats
    static_assert(NVH <= NT, "one v_z halo cell per thread at most");
};

template <int N, int TX, bool ZP, bool XP>
__device__ __forceinline__ void tile2d(const Geom &g, const Fields &A, const Fields &B,
                                       const Model &m, const Cpml &cp, unsigned rbytes,
                                       const int b0, const int b1, const int b2, const int b3,
                                       int s, int zs, int xb, int x0, int x1, int scol, int sr,
                                       float amp, float *Pn, float *VX, float *VZ) {
    using K = T2<N, TX>;
    constexpr int HP = K::HP, NW = K::NW, NT = K::NT, LDP = K::LDP, PC = K::PC;
    constexpr int VXC = K::VXC, LDZ = K::LDZ, PMC = K::PMC, VCW = K::VCW;
    constexpr int NH = K::NH, HPT = K::HPT, NVH = K::NVH;
    const int t = (int)threadIdx.x;
    const int lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const char *rb = (const char *)m.kdt;     // the region starts with the model
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void *)rb, (short)0, (int)rbytes, 0x00020000);
    auto off = [&](const float *p) { return (unsigned)((const char *)p - rb); };
    const long long so = (long long)s * g.P;
    const unsigned colb = 4u * (unsigned)g.ld1;
    // column offsets are not clamped: every access goes through the region's resource, and
    // one past its end reads 0 and writes nothing; a store a lane must not make goes to such
    // an offset instead of sitting under a branch (no exec-mask juggling per store)
    constexpr unsigned OOB = 0x80000000u;
    auto col = [&](int c) { return (unsigned)c * colb; };
    const int r = zs + lane;
    const bool own = r >= b0 && r < b1;
    const bool rowok = r >= 0 && r < g.M[0];
    const unsigned vr = 4u * (unsigned)(g.org + r);
    const unsigned a_kdt = 0u, a_bdz = off(m.bdt[0]), a_bdx = off(m.bdt[1]);
    const unsigned a_pA = off(A.p + so), a_vzA = off(A.v[0] + so), a_vxA = off(A.v[1] + so);
    const unsigned a_pB = off(B.p + so), a_vzB = off(B.v[0] + so), a_vxB = off(B.v[1] + so);
    const unsigned a_pzA = off(A.psp[0] + (long long)s * g.psz[0]);
    const unsigned a_vpzA = off(A.psv[0] + (long long)s * g.psz[0]);
    const unsigned a_pzB = off(B.psp[0] + (long long)s * g.psz[0]);
    const unsigned a_vpzB = off(B.psv[0] + (long long)s * g.psz[0]);
    const unsigned a_pxA = off(A.psp[1] + (long long)s * g.psz[1]);
    const unsigned a_vpxA = off(A.psv[1] + (long long)s * g.psz[1]);
    const unsigned a_pxB = off(B.psp[1] + (long long)s * g.psz[1]);
    const unsigned a_vpxB = off(B.psv[1] + (long long)s * g.psz[1]);
    const unsigned wz = 4u * (unsigned)g.W;   // bytes per column of a z slab
    auto xslab = [&](int c) { return c >= 0 && c < g.M[1] ? slab_index(c, g.M[1], g.nb) : -1; };
    auto zcol = [&](int j) { return wz * (unsigned)min(max(j, 0), g.M[1] - 1); };
    const int zci = ZP && rowok ? slab_index(r, g.M[0], g.nb) : -1;
    const unsigned vzi = 4u * (unsigned)(zci >= 0 ? zci : 0);
    const unsigned vxr = 4u * (unsigned)(rowok ? r : 0);
    float zah = 0.f, zbh = 0.f, zai = 0.f, zbi = 0.f;
    if (ZP && zci >= 0) {
        zah = cp.a_h[0][r];
        zbh = cp.b_h[0][r];
        zai = cp.a_i[0][r];
        zbi = cp.b_i[0][r];
    }
    // the v_z halo cell of this thread: column xb + hc, row rv
    const bool hv = t < NVH;
    const int hc = hv ? t / (2 * N - 1) : 0, hh = hv ? t % (2 * N - 1) : 0;
    const int rv = hh < N ? zs - N + hh : zs + 64 + (hh - N);
    const bool hrow = hv && rv >= 0 && rv < g.M[0];
    const int zch = ZP && hrow ? slab_index(rv, g.M[0], g.nb) : -1;
    float hah = 0.f, hbh = 0.f;
    if (ZP && zch >= 0) {
        hah = cp.a_h[0][rv];
        hbh = cp.b_h[0][rv];
    }

    // ---- 1. every load of the tile
    float pm[PMC];
#pragma unroll
    for (int k = 0; k < PMC; ++k) {
        const int q = wv + NW * k;
        pm[k] = q < PC ? bld(rs, vr, a_pA + col(xb - HP + q)) : 0.f;
    }
    float ph[HPT];
#pragma unroll
    for (int k = 0; k < HPT; ++k) {
        const int i = t + NT * k;
        const int ci = i / (2 * HP), h = i % (2 * HP);
        const int row = h < HP ? zs - HP + h : zs + 64 + (h - HP);
        ph[k] = i < NH ? bld(rs, 4u * (unsigned)(g.org + row) + col(xb + ci), a_pA) : 0.f;
    }
    const int vc0 = wv * VCW;                 // first v_x column of this wavefront (from xb - N)
    float vxo[VCW], bx[VCW], psx[VCW];
#pragma unroll
    for (int k = 0; k < VCW; ++k) {
        const int c = xb - N + vc0 + k;
        const bool in = vc0 + k < VXC;
        vxo[k] = in ? bld(rs, vr, a_vxA + col(c)) : 0.f;
        bx[k] = in ? bld(rs, vr, a_bdx + col(c)) : 0.f;
        psx[k] = 0.f;
        if (XP && in) {
            const int xc = xslab(c);
            if (xc >= 0) psx[k] = bld(rs, vxr, a_pxA + (unsigned)xc * colb);
        }
    }
    const int j0 = xb + 8 * wv;               // first p / v_z column of this wavefront
    float vzo[8], bz[8], kd[8], psz[8], pvz[8], pvx[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int j = j0 + k;
        vzo[k] = bld(rs, vr, a_vzA + col(j));
        bz[k] = bld(rs, vr, a_bdz + col(j));
        kd[k] = bld(rs, vr, a_kdt + col(j));
        psz[k] = pvz[k] = pvx[k] = 0.f;
        if (ZP) {
            psz[k] = bld(rs, vzi, a_pzA + zcol(j));
            pvz[k] = bld(rs, vzi, a_vpzA + zcol(j));
        }
        if (XP) {
            const int xc = xslab(j);
            if (xc >= 0) pvx[k] = bld(rs, vxr, a_vpxA + (unsigned)xc * colb);
        }
    }
    float hvo = 0.f, hbz = 0.f, hpz = 0.f;
    if (hv) {
        const unsigned hr = 4u * (unsigned)(g.org + rv) + col(xb + hc);
        hvo = bld(rs, hr, a_vzA);
        hbz = bld(rs, hr, a_bdz);
        if (ZP) hpz = bld(rs, 4u * (unsigned)(zch >= 0 ? zch : 0), a_pzA + zcol(xb + hc));
    }
#pragma unroll
    for (int k = 0; k < PMC; ++k) {
        const int q = wv + NW * k;
        if (q < PC) Pn[q * LDP + HP + lane] = pm[k];
    }
#pragma unroll
    for (int k = 0; k < HPT; ++k) {
        const int i = t + NT * k;
        const int ci = i / (2 * HP), h = i % (2 * HP);
        if (i < NH) Pn[(ci + HP) * LDP + (h < HP ? h : 64 + h)] = ph[k];
    }
    __syncthreads();

    // ---- 2. new v_x (x part of eq. 3 first row) and new v_z (z part), CPML
    {
        float w[VCW + 2 * N - 1];             // p^n of this row at LDS columns vc0 ..
#pragma unroll
        for (int d = 0; d < VCW + 2 * N - 1; ++d)
            w[d] = vc0 + d < PC ? Pn[(vc0 + d) * LDP + HP + lane] : 0.f;
#pragma unroll
        for (int k = 0; k < VCW; ++k) {
            if (vc0 + k >= VXC) break;
            const int c = xb - N + vc0 + k;
            float e = 0.f;
#pragma unroll
            for (int l = 1; l <= N; ++l) e += g.c[1][l - 1] * (w[k + N - 1 + l] - w[k + N - l]);
            const bool mine = c >= x0 && c < x1;
            if (XP) {
                const int xc = xslab(c);
                if (xc >= 0) {
                    const float psi = cp.b_h[1][c] * psx[k] + cp.a_h[1][c] * e;
                    bst(rs, own && mine ? vxr : OOB, a_pxB + (unsigned)xc * colb, psi);
                    e += psi;
                }
            }
            const float vxn = c >= b2 && c < b3 ? vxo[k] - bx[k] * e : vxo[k];
            bst(rs, own && mine ? vr : OOB, a_vxB + col(c), vxn);
            VX[(vc0 + k) * 64 + lane] = vxn;
        }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int j = j0 + k;
        const float *P = Pn + (8 * wv + k + HP) * LDP + HP + lane;
        float ez = 0.f;
#pragma unroll
        for (int l = 1; l <= N; ++l) ez += g.c[0][l - 1] * (P[l] - P[1 - l]);
        const bool mine = j >= x0 && j < x1;
        if (ZP) {
            const float psi = zbh * psz[k] + zah * ez;
            bst(rs, own && mine && zci >= 0 ? vzi : OOB, a_pzB + zcol(j), psi);
            ez = zci >= 0 ? ez + psi : ez;
        }
        const float vzn = own ? vzo[k] - bz[k] * ez : vzo[k];
        bst(rs, own && mine ? vr : OOB, a_vzB + col(j), vzn);
        VZ[(8 * wv + k) * LDZ + N + lane] = vzn;
    }
    if (hv) {
        const float *P = Pn + (hc + HP) * LDP + (hh < N ? HP - N + hh : 64 + HP + hh - N);
        float hz = 0.f;
#pragma unroll
        for (int l = 1; l <= N; ++l) hz += g.c[0][l - 1] * (P[l] - P[1 - l]);
        if (ZP) {
            const float psi = hbh * hpz + hah * hz;
            hz = zch >= 0 ? hz + psi : hz;
        }
        VZ[hc * LDZ + (hh < N ? hh : 64 + hh)] = rv >= b0 && rv < b1 ? hvo - hbz * hz : hvo;
    }
    __syncthreads();

    // ---- 3. new p (eq. 3 second row): z part, then x part, CPML, source
    const float samp = r == sr ? amp : 0.f;
    float u[8 + 2 * N - 1];                   // new v_x of this row at columns j0 - N ..
#pragma unroll
    for (int d = 0; d < 8 + 2 * N - 1; ++d) u[d] = VX[(8 * wv + d) * 64 + lane];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int j = j0 + k;
        const float *V = VZ + (8 * wv + k) * LDZ + N + lane;
        float dz = 0.f;
#pragma unroll
        for (int l = 1; l <= N; ++l) dz += g.c[0][l - 1] * (V[l - 1] - V[-l]);
        const bool mine = j >= x0 && j < x1;
        if (ZP) {
            const float psi = zbi * pvz[k] + zai * dz;
            bst(rs, own && mine && zci >= 0 ? vzi : OOB, a_vpzB + zcol(j), psi);
            dz = zci >= 0 ? dz + psi : dz;
        }
        float dx = 0.f;
#pragma unroll
        for (int l = 1; l <= N; ++l) dx += g.c[1][l - 1] * (u[k + N + l - 1] - u[k + N - l]);
        if (XP) {
            const int xc = xslab(j);
            if (xc >= 0) {
                const float psi = cp.b_i[1][j] * pvx[k] + cp.a_i[1][j] * dx;
                bst(rs, own && mine ? vxr : OOB, a_vpxB + (unsigned)xc * colb, psi);
                dx += psi;
            }
        }
        float sdiv = 0.f;
        sdiv += dz;
        sdiv += dx;
        float pn = Pn[(8 * wv + k + HP) * LDP + HP + lane] - kd[k] * sdiv;
        if (j == scol) pn += samp;
        bst(rs, own && mine ? vr : OOB, a_pB + col(j), pn);
    }
}

template <int N, int TX>
__global__ __launch_bounds__(8 * TX) void k_tile2d(Geom g, Fields A, Fields B, Model m,
                                                          Cpml cp, const int *__restrict__ box,
                                                          S2 sg, const long long *__restrict__ src_cell,
                                                          const float *__restrict__ stf, int nt,
                                                          int it, Ext ex, BandArg sv) {
    using K = T2<N, TX>;
    static_assert(K::NT == 8 * TX, "the launch bound is the block size");
    __shared__ float lds[K::LDS];
    const int bid = (int)blockIdx.x;
    if (bid >= sg.nmain) {
        // side work, as in k_step2d, on the first 256 threads of the block
        if (threadIdx.x >= 256) return;
        const int q = bid - sg.nmain;
        if (q < sg.nrecb) {
            const int nthr = sg.nrecb * 256;
            for (int rr = q * 256 + (int)threadIdx.x; rr < ex.rv.R; rr += nthr)
                sample_receiver(g, A.p, ex.rv, ex.dcal, ex.it, ex.status, rr);
        } else if (sv.buf) {
            band_lin(g, A, sv, q - sg.nrecb, (int)threadIdx.x, 0, 2);
        }
        return;
    }
    // the workgroup's tile (uniform): shot fastest, then strip, then run
    const int L = xcd_remap(bid, sg.nmain);
    const int s = L % sg.nshot;
    const int tt = L / sg.nshot;
    const int k = tt % sg.nstrip;
    const int rr = tt / sg.nstrip;
    const int *b = box + 6 * s;
    const int b0 = b[0], b1 = b[1], b2 = b[2], b3 = b[3];
    const int zs = sg.z0 + 64 * k;
    if (zs >= b1 || zs + 64 <= b0) return;
    const int xb = TX * (sg.run0 + rr);
    const int x0 = max(xb, b2), x1 = min(xb + TX, b3);
    if (x0 >= x1) return;
    const long long sc = src_cell[s];
    const float amp = sc >= 0 && it < nt ? src_amp(g.src_scale, stf[(long long)s * nt + it]) : 0.f;
    const int sr = sc >= 0 ? (int)((sc - g.org) % g.ld1) : -1;
    const int scol = sc >= 0 ? (int)((sc - g.org) / g.ld1) : -1 - (1 << 20);
    // the slab variants when the tile with its halos touches an absorbing slab
    const bool zp = zs - N < g.nb || zs + 64 + N - 1 > g.M[0] - g.nb - 1;
    const bool xp = xb - N < g.nb || xb + TX + N - 1 > g.M[1] - g.nb - 1;
    float *Pn = lds;
    float *VX = lds + K::PC * K::LDP;
    float *VZ = VX + K::VXC * 64;
    const unsigned rn = sg.rbytes;
    if (zp) {
        if (xp) tile2d<N, TX, true, true>(g, A, B, m, cp, rn, b0, b1, b2, b3, s, zs, xb, x0, x1, scol, sr, amp, Pn, VX, VZ);
        else tile2d<N, TX, true, false>(g, A, B, m, cp, rn, b0, b1, b2, b3, s, zs, xb, x0, x1, scol, sr, amp, Pn, VX, VZ);
    } else {
        if (xp) tile2d<N, TX, false, true>(g, A, B, m, cp, rn, b0, b1, b2, b3, s, zs, xb, x0, x1, scol, sr, amp, Pn, VX, VZ);
        else tile2d<N, TX, false, false>(g, A, B, m, cp, rn, b0, b1, b2, b3, s, zs, xb, x0, x1, scol, sr, amp, Pn, VX, VZ);
    }
}

unsigned nblocks(long long n, int b = 256) { return (unsigned)((n + b - 1) / b); }

// bytes from the model to the end of the second field set: the span of the step's buffer
// resource
size_t region_bytes(const Plan &pl) {
    const size_t fset = sizeof(float) * (size_t)pl.nshot *
                        ((size_t)pl.P * (1 + pl.nd) +
                         2 * (size_t)(pl.geom.psz[0] + pl.geom.psz[1] + pl.geom.psz[2]));
    return std::max(pl.off_fields, pl.off_fields2) + fset - pl.off_model;
}

template <int N, int C, int D>
hipError_t step2d_t(const StepCtx &c, const Fields &src, const Fields &dst, int it) {
    const Plan &pl = *c.pl;
    const Views &w = *c.w;
    const int *tab = &pl.fbox[(size_t)it * pl.nshot * 6];
    int u[4] = {1 << 30, -1, 1 << 30, -1};
    for (int s = 0; s < pl.nshot; ++s) {
        const int *b = tab + 6 * s;
        if (b[1] <= b[0] || b[3] <= b[2]) continue;
        u[0] = std::min(u[0], b[0]);
        u[1] = std::max(u[1], b[1]);
        u[2] = std::min(u[2], b[2]);
        u[3] = std::max(u[3], b[3]);
    }
    S2 sg{};
    sg.nshot = pl.nshot;
    sg.rbytes = (unsigned)region_bytes(pl);
    const bool any = u[1] > u[0] && u[3] > u[2];
    if (any) {
        sg.z0 = zalign(u[0]);
        sg.nstrip = (u[1] - sg.z0 + 63) / 64;
        sg.run0 = u[2] / C;
        sg.nrun = (u[3] - 1) / C - sg.run0 + 1;
        const long long waves = (long long)pl.nshot * sg.nstrip * sg.nrun;
        sg.nmain = (int)((waves + 3) / 4);
    }
    const bool ext = c.ext_it >= 0 && w.recv.R > 0;
    sg.nrecb = ext ? (int)std::min<long long>(nblocks(w.recv.R), 1024) : 0;
    BandArg sv{};
    int nband = 0;
    if (c.save_p_slot >= 0) {   // the whole saved level (p and v) of level it, from src
        const int nqb = (int)((pl.band.B + 255) / 256);
        sv = BandArg{w.bdesc, w.bands + (size_t)c.save_p_slot * pl.band.B,
                     (long long)pl.nsave * pl.band.B, nqb, pl.nshot};
        nband = pl.nshot * nqb;
    }
    const Ext ex{w.recv, c.ext_dcal, ext ? c.ext_it : -1, w.status};
    const unsigned grid = (unsigned)(sg.nmain + sg.nrecb + nband);
    if (grid == 0) return hipSuccess;
    if (c.ev)
        hipExtLaunchKernelGGL((k_step2d<N, C, D>), dim3(grid), dim3(256), 0, c.st, c.ev[0], c.ev[1], 0,
                              pl.geom, src, dst, w.model, w.cpml, (const int *)(w.fbox + (size_t)it * pl.nshot * 6),
                              sg, (const long long *)w.src_cell, c.stf, pl.g.nt, it, ex, sv);
    else
        hipLaunchKernelGGL((k_step2d<N, C, D>), dim3(grid), dim3(256), 0, c.st, pl.geom, src, dst,
                           w.model, w.cpml, (const int *)(w.fbox + (size_t)it * pl.nshot * 6), sg,
                           (const long long *)w.src_cell, c.stf, pl.g.nt, it, ex, sv);
    return hipGetLastError();
}

template <int N, int TX>
hipError_t tile2d_t(const StepCtx &c, const Fields &src, const Fields &dst, int it) {
    using K = T2<N, TX>;
    const Plan &pl = *c.pl;
    const Views &w = *c.w;
    const int *tab = &pl.fbox[(size_t)it * pl.nshot * 6];
    int u[4] = {1 << 30, -1, 1 << 30, -1};
    for (int s = 0; s < pl.nshot; ++s) {
        const int *b = tab + 6 * s;
        if (b[1] <= b[0] || b[3] <= b[2]) continue;
        u[0] = std::min(u[0], b[0]);
        u[1] = std::max(u[1], b[1]);
        u[2] = std::min(u[2], b[2]);
        u[3] = std::max(u[3], b[3]);
    }
    S2 sg{};
    sg.nshot = pl.nshot;
    sg.rbytes = (unsigned)region_bytes(pl);
    if (u[1] > u[0] && u[3] > u[2]) {
        sg.z0 = zalign(u[0]);
        sg.nstrip = (u[1] - sg.z0 + 63) / 64;
        sg.run0 = u[2] / TX;
        sg.nrun = (u[3] - 1) / TX - sg.run0 + 1;
        sg.nmain = (int)((long long)pl.nshot * sg.nstrip * sg.nrun);
    }
    const bool ext = c.ext_it >= 0 && w.recv.R > 0;
    sg.nrecb = ext ? (int)std::min<long long>(nblocks(w.recv.R), 1024) : 0;
    BandArg sv{};
    int nband = 0;
    if (c.save_p_slot >= 0) {
        const int nqb = (int)((pl.band.B + 255) / 256);
        sv = BandArg{w.bdesc, w.bands + (size_t)c.save_p_slot * pl.band.B,
                     (long long)pl.nsave * pl.band.B, nqb, pl.nshot};
        nband = pl.nshot * nqb;
    }
    const Ext ex{w.recv, c.ext_dcal, ext ? c.ext_it : -1, w.status};
    const unsigned grid = (unsigned)(sg.nmain + sg.nrecb + nband);
    if (grid == 0) return hipSuccess;
    const int *box = (const int *)(w.fbox + (size_t)it * pl.nshot * 6);
    if (c.ev)
        hipExtLaunchKernelGGL((k_tile2d<N, TX>), dim3(grid), dim3(K::NT), 0, c.st, c.ev[0], c.ev[1], 0,
                              pl.geom, src, dst, w.model, w.cpml, box, sg,
                              (const long long *)w.src_cell, c.stf, pl.g.nt, it, ex, sv);
    else
        hipLaunchKernelGGL((k_tile2d<N, TX>), dim3(grid), dim3(K::NT), 0, c.st, pl.geom, src, dst,
                           w.model, w.cpml, box, sg, (const long long *)w.src_cell, c.stf,
                           pl.g.nt, it, ex, sv);
    return hipGetLastError();
}

}  // namespace

// 2D, two field sets, no free surface, and a region a buffer resource can span
bool step2d_available(const Plan &pl) {
    return pl.nd == 2 && pl.dbuf && !pl.g.freesurf && pl.off_fields2 > pl.off_model &&
           region_bytes(pl) < (size_t)0x7fffffff;
}

hipError_t fwd_step_2d(const StepCtx &c, const Fields &src, const Fields &dst, int it) {
    const Plan &pl = *c.pl;
    const int C = c.run == 64 ? 64 : 32;
    const int D = c.depth;
    if (D == 0) {               // the tiled step
        if (pl.N == 4) return C == 64 ? tile2d_t<4, 64>(c, src, dst, it) : tile2d_t<4, 32>(c, src, dst, it);
        if (pl.N == 2) return C == 64 ? tile2d_t<2, 64>(c, src, dst, it) : tile2d_t<2, 32>(c, src, dst, it);
        return hipErrorInvalidValue;
    }
    if (pl.N == 4) {
        if (C == 64) return D == 4 ? step2d_t<4, 64, 4>(c, src, dst, it)
                          : D == 1 ? step2d_t<4, 64, 1>(c, src, dst, it) : step2d_t<4, 64, 2>(c, src, dst, it);
        return D == 4 ? step2d_t<4, 32, 4>(c, src, dst, it)
               : D == 1 ? step2d_t<4, 32, 1>(c, src, dst, it) : step2d_t<4, 32, 2>(c, src, dst, it);
    }
    if (pl.N == 2) return step2d_t<2, 32, 2>(c, src, dst, it);
    return hipErrorInvalidValue;
}

}  // namespace smi
