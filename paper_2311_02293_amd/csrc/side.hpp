// side.hpp -- small device-side pieces of work that ride on the large step launches of libsmi:
// receiver sampling (Alg. 2 extract_wavefield) and the saved boundary bands of Sec. 4.2.
#pragma once

#include <hip/hip_runtime.h>

#include "smi_internal.hpp"

namespace smi {

// Receiver sampling of a previous step carried by a later launch that does not write the p it
// samples (it < 0: none): the seismogram row of step it (p^{it+1}) is taken by extra
// workgroups of the next step's v launch (the v update leaves p alone), or of the next fused
// step (which reads level it + 1 from one buffer and writes the other).
struct Ext {
    Recv rv;
    float *dcal;
    int it;
    unsigned *status;
};

// Band cell q of shot s.  dir 0: field -> buf; dir 1: buf -> field; dir 2: field <- (1-wt)
// buf + wt buf2.  which: 0 p blocks, 1 v blocks, 2 all.
__device__ __forceinline__ void band_cell(const Geom &g, const Fields &f, const BandDesc &bd,
                                          float *buf, const float *buf2, long long shot_stride,
                                          int s, long long q, int dir, int which, float wt) {
    if (q >= bd.B) return;
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
    // constant indices only: a dynamic index into the Fields of a reference would place a
    // copy of it in LDS
    float *base = bl.field == 0 ? f.p : (bl.axis == 0 ? f.v[0] : (bl.axis == 1 ? f.v[1] : f.v[2]));
    float *fld = base + s * g.P + k;
    long long bo = s * shot_stride + q;
    if (dir == 0) buf[bo] = *fld;
    else if (dir == 1) *fld = buf[bo];
    else *fld = (1.f - wt) * buf[bo] + wt * buf2[bo];
}

// Band cells carried by a launch of other work: saved levels (dir 0) during the forward half
// steps, restored levels (dir 1) in the two-launch reverse step.
struct BandArg {
    const BandDesc *bd; // band layout (device copy)
    float *buf;         // saved level of shot 0 (nullptr: nothing to do)
    long long stride;   // floats between shots
    int nqb;            // 256-cell blocks per shot
    int nshot;          // shots of the launch
    int s0 = 0;         // the first of them
};

// dcal[it][r] = sum over the taps of receiver r of w p (Alg. 2 recording; one tap on a node)
__device__ __forceinline__ void sample_receiver(const Geom &g, const float *__restrict__ p,
                                                const Recv &rv, float *dcal, int it,
                                                unsigned *status, int r) {
    const long long so = rv.shot[r] * g.P;
    float v = 0.f;
    for (int t = rv.toff[r]; t < rv.toff[r + 1]; ++t) v += rv.tw[t] * p[so + rv.tcell[t]];
    dcal[rv.obase[r] + (long long)it * rv.stride[r]] = v;
    if (!isfinite(v)) atomicOr(status, 2u);
}

// the band cells of every shot in 256-cell block `lin` of a launch's side work (thread t of
// 256 takes one cell)
__device__ __forceinline__ void band_lin(const Geom &g, const Fields &f, const BandArg &ba,
                                         long long lin, int t, int dir, int which) {
    const int j = (int)(lin / ba.nqb);
    if (j < ba.nshot)
        band_cell(g, f, *ba.bd, ba.buf, nullptr, ba.stride, ba.s0 + j, (lin % ba.nqb) * 256 + t, dir,
                  which, 0.f);
}

}  // namespace smi
