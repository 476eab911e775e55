// smi_internal.hpp -- plan, workspace layout and kernel launch interface of libsmi.
//
// Layout of one wavefield in HBM (per shot): z (n1) is the contiguous axis, then x, then y.
// The padded grid (M_a = n_a + 2 nb nodes per axis) is surrounded by GH ghost nodes per side
// and axis that are zero and never written, so stencil reads need no bounds checks.  Node
// (z, x, y) of the padded grid lives at org + z + ld1 x + ld2 y, with ld1 a multiple of 32
// floats (128 B); shots are stacked with a stride of P floats.  The model arrays use the same
// layout, so one offset addresses a field and its coefficients.  CPML memory variables exist
// only in the absorbing slabs: along axis a the compact index keeps planes [0, nb) and
// [M_a - nb - 1, M_a).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/smi.h"

namespace smi {

constexpr int kMaxN = 4;       // half order (orders 4 and 8)
constexpr int kMaxBlocks = 12; // band blocks per save level: 3 axes x {p, v} x {left, right}
constexpr int GH = 2 * kMaxN;  // ghost nodes per side and axis (>= the 2N-1 halo of a fused step)
constexpr int kTaps = 4;       // half-width (saved levels) of the decimated-band interpolator
constexpr int kTailCols = 32;  // columns of workspace slack after the last region (see plan.cpp)
constexpr size_t kInjMapCap = size_t(1) << 22;   // entries of the largest adjoint-source node map
constexpr double kKaiserBeta = 6.31;

// ---------------------------------------------------------------- device-side views

struct Geom {
    int nd, N;
    int n[3];           // interior extents (1 for inactive axes)
    int M[3];           // padded extents (1 for inactive axes)
    int nb;
    int ld1;            // stride of x (floats)
    long long ld2;      // stride of y (floats)
    long long org;      // offset of node (0, 0, 0)
    long long P;        // floats per field per shot
    int W;              // slab width 2 nb + 1
    long long psz[3];   // floats per slab array per shot, per axis
    long long I;        // interior cells per shot
    float c[3][kMaxN];  // a_l / d_a
    float dt;
    float src_scale;    // dt / (d1 d2 [d3])
    int fs;             // free surface on row nb (p = 0 there)
};

struct Model {
    float *kdt;         // dt * kappa, padded
    float *bdt[3];      // dt * beta_a at v_a points, padded
};

struct Cpml {           // per axis, indexed by the padded node index along that axis
    float *a_i[3], *b_i[3];   // integer nodes (p points)
    float *a_h[3], *b_h[3];   // half nodes (v points)
};

struct Fields {
    float *p, *v[3];
    float *psp[3];      // memory variables of d_a p (at v_a points), slab layout
    float *psv[3];      // memory variables of d_a v_a (at p points), slab layout
};

struct BandBlock {      // one block of a saved level: planes [start, start+w) along `axis`
    int field;          // 0: p, 1: v_axis
    int axis;
    int start, w;
    long long off;      // offset of the block inside one level
    long long cnt;      // cells in the block
    int ext[3];         // box extents (z, x, y) of the block
    int org[3];         // box origin (z, x, y) of the block
};

struct BandDesc {
    int nblk;
    long long B;        // floats per level per shot
    BandBlock blk[kMaxBlocks];
};

// Adjoint-source injection as a gather (eq. 8, the transpose of the receiver sampling): the
// distinct nodes that receiver operators touch, per shot in ascending cell order.  Node u (shot
// shot[u], cell offset cell[u] inside that shot's field) receives kappa sum_t w[t] G[rec[t]] over
// t in off[u] .. off[u+1), contributions in ascending receiver order: a fixed summation order,
// no atomics, so gradients and images are bit-stable from run to run.
struct Inj {
    int U;
    int *shot;          // [U]
    long long *cell;    // [U]
    int *off;           // [U + 1]
    int *rec;           // [T] receiver index (into Recv)
    float *w;           // [T] operator weight
};

struct Recv {           // flattened receivers of all shots
    int R;
    int *shot;          // [R]
    long long *obase;   // [R] offset of sample 0 in dcal
    int *stride;        // [R] nrec of its shot
    int *toff;          // [R + 1] point operator of receiver r: taps toff[r] .. toff[r+1]
    long long *tcell;   // [taps] cell offset inside one shot's field
    float *tw;          // [taps] weight
};

// ---------------------------------------------------------------- host plan

struct Plan {
    smi_grid g{};
    int nd = 2, N = 2;
    int n[3] = {1, 1, 1}, M[3] = {1, 1, 1};
    int ld1 = 0;
    long long ld2 = 0, org = 0;
    long long P = 0, I = 0;
    long long cell(int z, int x, int y) const { return org + z + (long long)ld1 * x + ld2 * y; }
    double vmin = 0, vmax = 0;
    int margin = 0;
    int nshot = 0;
    std::vector<int> src;          // [nshot][3] padded nodes
    std::vector<long long> src_cell;
    std::vector<int> rec_off;      // [nshot + 1]
    std::vector<int> rec;          // [R][3]
    std::vector<int> fbox;         // [nt][nshot][6] forward box (lo, hi exclusive per axis)
    std::vector<int> abox;         // [nt][nshot][6] adjoint box
    std::vector<int> rbox;         // [nt][nshot][6] reconstruction region (interior clip)
    // point operators of sources and receivers (Sec. 2.1): the Kaiser-windowed sinc of a
    // point off the grid, or its node with weight 1; CSR over shots / receivers, cells are
    // offsets inside one shot's field.  src_cell[s] is the node of a one-tap source, else -1.
    std::vector<int> src_toff, rec_toff;
    std::vector<long long> src_tcell, rec_tcell;
    std::vector<float> src_tw, rec_tw;
    bool src_multi = false;        // some source spreads over several nodes
    // the gather form of the adjoint-source injection (see Inj)
    std::vector<int> inj_shot, inj_off, inj_rec;
    std::vector<long long> inj_cell;
    std::vector<float> inj_w;
    // 2D reverse passes: the adjoint p update of reverse step it + 1 adds the injection of step
    // it itself, on the lanes that own the nodes, when every node lies inside its shot's adjoint
    // box at every step (inj_fused); with a free surface those lanes also write the images.  inj_map[(s inj_nrow + z -
    // inj_zlo) M[1] + x] is the node of shot s at padded (z, x), or -1, over the rows
    // [inj_zlo, inj_zlo + inj_nrow) that hold nodes.
    std::vector<int> inj_map;
    int inj_zlo = 0, inj_nrow = 0;
    bool inj_fused = false;
    BandDesc band{};
    int nsave = 0;      // saved band levels k dr, k = 0 .. nsave-1
    int nrun = 0;       // forward steps: nt, or past nt until the last saved level (dr > 1)
    Geom geom{};
    // workspace layout (byte offsets)
    size_t off_status = 0, off_misfit = 0, off_partial = 0, off_bdesc = 0;
    size_t off_model = 0, off_cpml = 0, off_tables = 0, off_recv = 0;
    size_t off_fields = 0, off_fields2 = 0, off_adj = 0, off_bands = 0, off_acc = 0, off_G = 0, off_dcal = 0;
    size_t off_rho = 0;
    size_t off_taps = 0, off_fin = 0, off_inj = 0, off_injmap = 0;
    size_t bytes = 0;
    int npartial = 0;
    bool save = false, adjoint = false, need_G = false, need_dcal = false;
    bool rho_acc = false;   // room for the density-gradient face sums (gradient-capable jobs)
    bool born = false;      // a perturbation field beside the background (tangent-linear job)
    bool dbuf = false;  // second source-field buffer for the fused steps
    int chunk = 0;      // columns per workgroup of the fused 2D step (0: default)
    double cnt_fwd = 0, cnt_adj = 0, cnt_rec = 0;
    double bytes_fwd = 0, bytes_rev = 0;   // algorithmic HBM bytes (see plan.cpp)
    // [nrun][3] algorithmic bytes of forward step it: the step as the method defines it
    // (fields read and written once), then the v and the p kernel as launched separately
    // (each reads the other field)
    std::vector<double> step_bytes;
    // [nt][4] algorithmic bytes of reverse step it: the part every reverse step moves (adjoint
    // and reconstructed fields, CPML variables, model, restored bands, adjoint sources), then
    // the gradient, image and illumination accumulators
    std::vector<double> rev_bytes;
};

// Build and validate a plan.  Returns SMI_OK or an error with `err` filled.
smi_status make_plan(const smi_grid *g, const smi_acq *acq, smi_job job, double vmin,
                     double vmax, Plan &pl, std::string &err);
smi_status check_grid(const smi_grid *g, double vmin, double vmax, std::string &err);
void algorithmic_bytes(Plan &pl);
// algorithmic bytes of forward step it over the shots [s0, s1), as a row of Plan::step_bytes
void step_bytes_of(const Plan &pl, int it, int s0, int s1, double row[3]);
// shot groups of a 2D forward pass of the register-blocked kernels: one group while every
// step's fields (with their memory variables) fit `budget` bytes, else the group count of least
// modelled cost over the schedule of boxes; max_per > 0 caps a group instead
std::vector<int> fwd_groups(const Plan &pl, double budget, int max_per);
// algorithmic bytes of reverse iteration it over the shots [s0, s1): out[0] the adjoint and
// reconstruction steps with band restores, adjoint sources and the model read once, out[1] the
// gradient sum, out[2] the image sum, out[3] the illumination sum
void rev_iter_bytes(const Plan &pl, int it, int s0, int s1, double out[4]);
// shot groups of a 2D reverse pass: boundaries 0 = g[0] < g[1] < ... = nshot, so that the
// reverse state one group touches on average over the reverse steps (source field and
// accumulators over the reconstruction region, adjoint field over the adjoint box, memory
// variables) stays within `budget` bytes (one group when it all fits, or outside 2D; rho: the
// pass keeps the density face sums); max_per > 0 caps a group at that many shots instead
std::vector<int> rev_groups(const Plan &pl, double budget, int max_per, bool rho);
void cpml_profiles(const Plan &pl, int axis, std::vector<float> &a_i, std::vector<float> &b_i,
                   std::vector<float> &a_h, std::vector<float> &b_h);

// ---------------------------------------------------------------- device views of a workspace

struct Views {
    unsigned *status;
    const BandDesc *bdesc;  // copy of the plan's band layout in device memory
    double *misfit_tmp;
    double *partial;
    Model model;
    Cpml cpml;
    int *fbox, *abox, *rbox;
    Recv recv;
    Inj inj;
    int *injmap;          // Plan::inj_map in device memory (null when the injection is not fused)
    long long *src_cell;  // [nshot] source cell offset inside one shot's field
    int *src_toff;        // [nshot + 1] source operators (see Plan)
    long long *src_tcell;
    float *src_tw;
    Fields f, q;        // source field, adjoint field
    Fields f2;          // second buffer of the source field (fused, double-buffered steps)
    float *bands;       // [nshot][nsave][B]
    float *acc_g, *acc_i, *acc_l;   // [nshot][I] gradient / image / illumination
    float *acc_r[3];    // [nshot][P] per axis: sum over steps of v~_a D+_a p on the faces
    float *G;           // [nt * R] adjoint source (when computed internally)
    float *dcal;        // internal dcal when the caller gave none
    float *fin;         // level-nt copy of p and v while the forward runs past nt (dr > 1)
};

Views views(const Plan &pl, void *ws);

// ---------------------------------------------------------------- launchers (kernels.hip)

hipError_t launch_model_prep(const Plan &pl, const Views &w, const float *vp, const float *rho,
                             hipStream_t st);
hipError_t launch_minmax(const float *vp, long long n, unsigned *out2, hipStream_t st);

struct StepCtx {
    const Plan *pl;
    const Views *w;
    const float *stf;       // device [nshot][nt]
    hipStream_t st;
    bool plain;
    // when set (batched sweep only): start / stop events of the v launch (ev[0], ev[1]) and of
    // the p launch (ev[2], ev[3]) of this step, taken by the device around each kernel
    const hipEvent_t *ev = nullptr;
    bool xcd = false;       // XCD-contiguous tile order of the sweep kernels
    bool ymap = false;      // 3D register-blocked kernels: XCD-contiguous z-fastest tile order
    int march = 0;          // > 0: register-blocked kernels with this many cells per lane (2, 4, 8)
    bool zl = false;        // register-blocked kernels take z-neighbours from LDS
    int y3 = 0;             // 3D: half steps marching along y, tile code 100 BX + CY (0: off)
    int yp = 0;             // 3D: plane-tiled half steps marching along y, CY planes (0: off)
    int rev = 0;            // 2D reverse step: 0 by batch size, 1 two launches, 2 five launches
    bool step2d = false;    // 2D forward: the fused marching step (step2d.hip), levels in two buffers
    int run = 32;           // its run of columns per wavefront or tile (32 or 64)
    int depth = 2;          // and the columns it loads ahead (1, 2 or 4); 0: the tiled step
    // receiver sampling of forward step ext_it into ext_dcal, carried by the next forward
    // step's v launch (register-blocked kernels only, see march_forward); -1: none pending
    int ext_it = -1;
    float *ext_dcal = nullptr;
    // band cells of saved levels carried by the register-blocked forward half steps: the p
    // cells of level it on the v launch of step it, the v cells of level it + 1 on the p launch
    // of step it (-1: none)
    int save_p_slot = -1;
    int save_v_slot = -1;
    // the shots [s0, s1) the launches of a time loop cover (s1 < 0: every shot): 2D forward and
    // reverse passes may run their shots in groups, one time loop per group (fwd_groups,
    // rev_groups)
    int s0 = 0;
    int s1 = -1;
};

inline int shot_end(const StepCtx &c) { return c.s1 < 0 ? c.pl->nshot : c.s1; }

hipError_t fwd_step(const StepCtx &c, int it);
// true when fwd_step runs the register-blocked half-step kernels (which can carry the
// previous step's receiver sampling)
bool march_forward(const StepCtx &c);
// 3D half steps marching along y (ymarch3d.hip)
bool y3_available(const Plan &pl);
hipError_t fwd_step_y3(const StepCtx &c, int it);
hipError_t adj_step_y3(const StepCtx &c, int it, bool image);
bool yp_available(const Plan &pl);
hipError_t fwd_step_yp(const StepCtx &c, int it);
hipError_t adj_step_yp(const StepCtx &c, int it, bool image);
// fused 2D forward step (v, p, CPML, source in one kernel, level n from src, level n + 1 to
// dst); false if not provided for this plan
bool fused_fwd_available(const Plan &pl);
hipError_t fwd_step_fused(const StepCtx &c, const Fields &src, const Fields &dst, int it);
// fused marching 2D forward step (step2d.hip): level it from src, level it + 1 to dst, every
// shot in one launch; carries the receivers of step c.ext_it (sampled from src) and, with
// c.save_p_slot >= 0, the bands of level it (from src) on extra workgroups
bool step2d_available(const Plan &pl);
hipError_t fwd_step_2d(const StepCtx &c, const Fields &src, const Fields &dst, int it);
hipError_t extract(const StepCtx &c, int it, float *dcal, const float *p = nullptr);
// p += sign dt stf[it] / dV through the operators of the sources that spread over several
// nodes (one-tap sources are injected inside the p kernels); nothing when there are none
hipError_t src_taps(const StepCtx &c, int it, float *p, float sign);
hipError_t band_save(const StepCtx &c, const Fields &f, int slot);
// the p (which 0) or v (which 1) cells of a saved level
hipError_t band_save_part(const StepCtx &c, const Fields &f, int slot, int which);
hipError_t band_restore(const StepCtx &c, int it, int which);
hipError_t snap(const StepCtx &c, const Fields &f, float *snaps, int k, int nsnap);
hipError_t scale_copy(const StepCtx &c, const float *in, float *out, float a);
hipError_t adj_inject(const StepCtx &c, int it, const float *G);
// reverse step it; with Gn (the adjoint sources) and it > 0, a step that can also adds the
// injection of step it - 1 (Plan::inj_fused) and sets *fused, so the caller skips that launch
hipError_t rev_step(const StepCtx &c, int it, bool grad, bool image, const float *Gn = nullptr,
                    bool *fused = nullptr);
// residual, G = dt r and misfit of the shots [s0, s1) (their slice of dcal / dobs / G)
hipError_t residual(const StepCtx &c, const float *dcal, const float *dobs, float *G,
                    double *misfit, int s0, int s1);
// shot reduction (fixed order) of the shots [s0, s1) into the outputs
hipError_t finalize(const StepCtx &c, const float *vp, float *grad, float *image, float *illum,
                    float *image_norm, int s0, int s1);
// density part of eq. (7): accumulate v~ D+p on the faces of reverse step it
hipError_t rho_faces(const StepCtx &c, int it);
// tangent-linear step: the perturbation field (q) over the forward box, with the secondary
// source -dt dkappa div v of the background (f, after its own step)
hipError_t born_step(const StepCtx &c, int it, const float *dkappa);
// gradients of a parametrisation family (1: Vp, rho; 2: Vp, Ip) from the kappa and face sums
hipError_t finalize_family(const StepCtx &c, const float *vp, const float *rho, int family,
                           float *g1, float *g2, int s0, int s1);
hipError_t launch_laplacian(const smi_grid *g, const float *in, float *out, hipStream_t st);

}  // namespace smi
