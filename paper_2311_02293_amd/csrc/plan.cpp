// plan.cpp -- host planning: validation (Sec. 3.8, eq. 5), acquisition to grid nodes,
// CPML profiles (Sec. 2.1), computing-box schedules (Sec. 4.1), boundary-band layout
// (Sec. 4.2) and the workspace layout.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "smi_internal.hpp"

namespace smi {

namespace {

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Staggered first-derivative weights of eq. (4): the a_l that make the 2N-point
// staggered difference exact on polynomials up to degree 2N-1, from Lagrange
// differentiation at the nodes +-(2m-1)/2.
void fd_weights(int N, double *a) {
    // The weight of node +x_l (x_m = (2m-1)/2) is the derivative at 0 of its Lagrange basis
    // polynomial over the nodes {+-x_m}:
    //   L_l(x) = (x + x_l)/(2 x_l) * prod_{m!=l} (x^2 - x_m^2)/(x_l^2 - x_m^2)
    //   a_l = L_l'(0) = 1/(2 x_l) * prod_{m!=l} (-x_m^2)/(x_l^2 - x_m^2)
    for (int l = 1; l <= N; ++l) {
        double xl = (2.0 * l - 1.0) / 2.0;
        double r = 1.0 / (2.0 * xl);
        for (int m = 1; m <= N; ++m) {
            if (m == l) continue;
            double xm = (2.0 * m - 1.0) / 2.0;
            r *= -xm * xm / (xl * xl - xm * xm);
        }
        a[l - 1] = r;
    }
}

int slab_width(int nb) { return 2 * nb + 1; }

}  // namespace

smi_status check_grid(const smi_grid *g, double vmin, double vmax, std::string &err) {
    if (!g) { err = "grid is NULL"; return SMI_E_ARG; }
    if (g->ndim != 2 && g->ndim != 3) { err = "ndim must be 2 or 3"; return SMI_E_ARG; }
    if (g->order != 4 && g->order != 8) {
        err = "order must be 4 or 8";
        return SMI_E_UNSUPPORTED;
    }
    if (g->freesurf != 0 && g->freesurf != 1) { err = "freesurf must be 0 or 1"; return SMI_E_ARG; }
    if (g->n1 < 1 || g->n2 < 1 || (g->ndim == 3 ? g->n3 < 1 : g->n3 != 1)) {
        err = "bad n1/n2/n3";
        return SMI_E_ARG;
    }
    if (!(g->d1 > 0) || !(g->d2 > 0) || (g->ndim == 3 && !(g->d3 > 0))) {
        err = "spacing must be positive";
        return SMI_E_ARG;
    }
    if (g->nb < g->order / 2 || g->nb > 1000) { err = "nb must be >= order/2"; return SMI_E_ARG; }
    if (g->nt < 1 || !(g->dt > 0) || !(g->fm > 0)) { err = "bad nt/dt/fm"; return SMI_E_ARG; }
    if (g->dr < 1) { err = "dr must be >= 1"; return SMI_E_ARG; }
    if (g->box != 0 && g->box != 1) { err = "box must be 0 or 1"; return SMI_E_ARG; }
    if (!(vmin > 0) || !(vmax >= vmin) || !std::isfinite(vmax)) {
        err = "model speeds must be finite and positive";
        return SMI_E_ARG;
    }
    int N = g->order / 2;
    double a[kMaxN];
    fd_weights(N, a);
    double sa = 0;
    for (int l = 0; l < N; ++l) sa += std::fabs(a[l]);
    double inv = 1.0 / (g->d1 * g->d1) + 1.0 / (g->d2 * g->d2) +
                 (g->ndim == 3 ? 1.0 / (g->d3 * g->d3) : 0.0);
    double cfl = g->dt * vmax * std::sqrt(inv) * sa;
    if (cfl > 1.0) {
        char b[160];
        snprintf(b, sizeof b, "CFL violated: dt*Vmax*sqrt(sum 1/d^2)*sum|a| = %.4f > 1", cfl);
        err = b;
        return SMI_E_CFL;
    }
    double dmax = std::max(g->d1, std::max(g->d2, g->ndim == 3 ? g->d3 : 0.0));
    double ppw = vmin / (2.5 * g->fm * dmax);
    double need = g->order == 4 ? 5.0 : 3.0;
    if (ppw < need) {
        char b[160];
        snprintf(b, sizeof b, "dispersion: %.2f points per wavelength < %.0f", ppw, need);
        err = b;
        return SMI_E_DISPERSION;
    }
    return SMI_OK;
}

void cpml_profiles(const Plan &pl, int axis, std::vector<float> &a_i, std::vector<float> &b_i,
                   std::vector<float> &a_h, std::vector<float> &b_h) {
    // Komatitsch & Martin CPML with kappa_pml = 1: b = exp(-(d + alpha) dt),
    // a = d (b - 1)/(d + alpha); d = d0 l^2 (l: normalised depth into the layer at the
    // node), d0 = -3 Vmax ln(R) / (2 nb h), Collino-Tsogka R, alpha = pi fm (1 - l).
    const smi_grid &g = pl.g;
    int nb = g.nb, n = pl.n[axis], M = pl.M[axis];
    double h = axis == 0 ? g.d1 : axis == 1 ? g.d2 : g.d3;
    double R = std::pow(10.0, -((std::log10((double)nb) - 1.0) / std::log10(2.0) + 3.0));
    double d0 = -3.0 * pl.vmax * std::log(R) / (2.0 * nb * h);
    a_i.assign(M, 0.f); b_i.assign(M, 1.f); a_h.assign(M, 0.f); b_h.assign(M, 1.f);
    for (int half = 0; half < 2; ++half)
        for (int i = 0; i < M; ++i) {
            double x = i + 0.5 * half;
            // no layer above a free surface (the rows there hold its mirror images)
            double top = g.freesurf && axis == 0 ? 0.0 : nb - x;
            double dist = x < nb ? top : (x > nb + n - 1 ? x - (nb + n - 1) : 0.0);
            double l = dist / nb;
            double dd = d0 * l * l, al = M_PI * g.fm * (1.0 - l);
            double b = std::exp(-(dd + al) * g.dt);
            double a = dist > 0 ? dd * (b - 1.0) / (dd + al) : 0.0;
            (half ? a_h : a_i)[i] = (float)a;
            (half ? b_h : b_i)[i] = (float)b;
        }
}

// Kaiser window parameter of the windowed-sinc point operators of half-width r (Hicks' table
// for a maximum wavenumber of half the Nyquist one); the half-width is order / 2.
static double kaiser_b(int r) { return r == 1 ? 1.24 : r == 2 ? 2.94 : r == 3 ? 4.53 : 6.31; }

static double bessel_i0(double x) {
    double s = 1.0, t = 1.0;
    for (int k = 1; k < 200; ++k) {
        t *= (x / (2.0 * k)) * (x / (2.0 * k));
        s += t;
        if (t < 1e-17 * s) break;
    }
    return s;
}

// Nodes and weights along one axis of the operator of a point at `pos` metres (interior
// coordinates): the node itself (weight 1) when the point is within 1e-3 of a spacing of it,
// else sinc(j - u) I0(b sqrt(1 - ((j-u)/r)^2)) / I0(b) on the 2r nodes around u, dropping
// nodes outside the padded grid.  False when the point lies outside [0, (n-1) h].
static bool axis_taps(double pos, double h, int n, int nb, int M, int r, int &near,
                      std::vector<int> &nodes, std::vector<double> &w) {
    const double q = pos / h;
    if (!(q >= -1e-3 && q <= n - 1 + 1e-3)) return false;
    const double u = nb + q;
    const double j0 = std::nearbyint(u);
    near = std::min(std::max((int)j0, nb), nb + n - 1);
    nodes.clear();
    w.clear();
    if (std::fabs(u - j0) <= 1e-3) {
        nodes.push_back(near);
        w.push_back(1.0);
        return true;
    }
    const double b = kaiser_b(r), i0b = bessel_i0(b);
    const int base = (int)std::floor(u);
    for (int j = base - r + 1; j <= base + r; ++j) {
        const double x = j - u;
        const double win = bessel_i0(b * std::sqrt(std::max(0.0, 1.0 - (x / r) * (x / r)))) / i0b;
        if (j < 0 || j >= M) continue;
        nodes.push_back(j);
        w.push_back(std::sin(M_PI * x) / (M_PI * x) * win);
    }
    return true;
}

// Tensor-product operator of one point: appends its taps; `node` receives the nearest node.
static bool point_taps(const Plan &pl, const double *pos, const double *hs, int *node,
                       std::vector<long long> &cell, std::vector<float> &wt) {
    std::vector<int> nd[3];
    std::vector<double> ww[3];
    for (int a = 0; a < 3; ++a) {
        if (a >= pl.nd) { nd[a] = {0}; ww[a] = {1.0}; node[a] = 0; continue; }
        if (!axis_taps(pos[a], hs[a], pl.n[a], pl.g.nb, pl.M[a], pl.N, node[a], nd[a], ww[a]))
            return false;
    }
    for (size_t k = 0; k < nd[2].size(); ++k)
        for (size_t j = 0; j < nd[1].size(); ++j)
            for (size_t i = 0; i < nd[0].size(); ++i) {
                cell.push_back(pl.cell(nd[0][i], nd[1][j], nd[2][k]));
                wt.push_back((float)(ww[0][i] * ww[1][j] * ww[2][k]));
            }
    return true;
}

// Algorithmic HBM bytes of the forward and reverse loops (what the method must move at
// FP32, independent of how the kernels move it):
//   per cell-step of a box: fields p and v_a read + written, 8 (nd + 1) B; CPML memory
//   variables read + written, 16 B per axis whose slab contains the cell;
//   per step: the model (dt kappa, dt beta_a) once per distinct cell of the union of the
//   shots' boxes, 4 (nd + 1) B (approximated by the largest box); receivers 8 B each
//   (read p, write dcal); saved bands 8 B per band cell (read field, write buffer).
//   Reverse: the adjoint step as above over the adjoint box; the reconstruction reads and
//   writes p and v_a on its region (8 (nd + 1) B) plus the accumulators touched (gradient:
//   read p~ + read/write acc = 12 B; image: read p + read/write acc = 12 B; illumination
//   8 B), the model again, the restored bands 8 B per band cell, adjoint sources 8 B each.
static double box_slab_cells(const Plan &pl, const int *b) {
    double tot = 0;
    for (int a = 0; a < pl.nd; ++a) {
        int nb = pl.g.nb, M = pl.M[a];
        int lo = b[2 * a], hi = b[2 * a + 1];
        // slab planes along a: [0, nb) and [M - nb - 1, M)
        int in = std::max(0, std::min(hi, nb) - lo) + std::max(0, hi - std::max(lo, M - nb - 1));
        double other = 1;
        for (int q = 0; q < 3; ++q)
            if (q != a) other *= b[2 * q + 1] - b[2 * q];
        tot += in * other;
    }
    return tot;
}

void rev_iter_bytes(const Plan &pl, int it, int s0, int s1, double out[4]) {
    const int ns = pl.nshot, nd = pl.nd;
    double rb0 = 0, rg = 0, ri = 0, rl = 0, maxa = 0;
    for (int s = s0; s < s1; ++s) {
        const int *ab = &pl.abox[((size_t)it * ns + s) * 6];
        const int *rb = &pl.rbox[((size_t)it * ns + s) * 6];
        double va = (double)std::max(0, ab[1] - ab[0]) * std::max(0, ab[3] - ab[2]) *
                    std::max(0, ab[5] - ab[4]);
        double vr = (double)(rb[1] - rb[0]) * (rb[3] - rb[2]) * (rb[5] - rb[4]);
        rb0 += 8.0 * (nd + 1) * va + 16.0 * box_slab_cells(pl, ab) + 8.0 * (nd + 1) * vr;
        rg += 12.0 * vr;                                    // p~ read, gradient
        rl += 8.0 * vr;                                     // illumination
        ri += 12.0 * va;                                    // image
        maxa = std::max(maxa, std::max(va, vr));
    }
    const double restore = pl.g.dr == 1 || it % pl.g.dr == 0 ? 8.0 : 4.0 * (2 * kTaps + 1);
    rb0 += 4.0 * (nd + 1) * maxa + 8.0 * (pl.rec_off[s1] - pl.rec_off[s0]) +
           restore * (double)(s1 - s0) * pl.band.B;
    out[0] = rb0; out[1] = rg; out[2] = ri; out[3] = rl;
}

void step_bytes_of(const Plan &pl, int it, int s0, int s1, double row[3]) {
    const int ns = pl.nshot, nd = pl.nd;
    double maxf = 0, sb = 0, sv = 0, sp = 0;
    for (int s = s0; s < s1; ++s) {
        const int *fb = &pl.fbox[((size_t)it * ns + s) * 6];
        double vf = (double)(fb[1] - fb[0]) * (fb[3] - fb[2]) * (fb[5] - fb[4]);
        const double slab = box_slab_cells(pl, fb);
        sb += 8.0 * (nd + 1) * vf + 16.0 * slab;
        sv += (4.0 + 8.0 * nd) * vf + 8.0 * slab;
        sp += (4.0 * nd + 8.0) * vf + 8.0 * slab;
        maxf = std::max(maxf, vf);
    }
    row[0] = sb + 4.0 * (nd + 1) * maxf;
    row[1] = sv + 4.0 * nd * maxf;
    row[2] = sp + 4.0 * maxf;
}

void algorithmic_bytes(Plan &pl) {
    const int nt = pl.g.nt, ns = pl.nshot;
    double R = pl.rec_off[ns];
    double bf = 0, br = 0;
    pl.step_bytes.assign((size_t)pl.nrun * 3, 0.0);
    pl.rev_bytes.assign(pl.adjoint ? (size_t)nt * 4 : 0, 0.0);
    for (int it = 0; it < pl.nrun; ++it) {
        double *row = &pl.step_bytes[3 * (size_t)it];
        step_bytes_of(pl, it, 0, ns, row);
        bf += row[0] + (it < nt ? 8.0 * R : 0.0);
        if (pl.save && it % pl.g.dr == 0) bf += 8.0 * (double)ns * pl.band.B;
        if (pl.adjoint && it < nt) {
            double *q = &pl.rev_bytes[4 * (size_t)it];
            rev_iter_bytes(pl, it, 0, ns, q);
            br += q[0] + q[1] + q[2] + q[3];
        }
    }
    pl.bytes_fwd = bf;
    pl.bytes_rev = pl.adjoint ? br : 0;
}

// equal groups of at most per shots (sizes differing by one at most)
static std::vector<int> equal_groups(int ns, int per) {
    const int ng = (ns + per - 1) / per;
    std::vector<int> off(ng + 1);
    for (int k = 0; k <= ng; ++k) off[k] = (int)((long long)ns * k / ng);
    return off;
}

// cells of a box (z0, z1, x0, x1, y0, y1)
static double box_volume(const int *b) {
    return (double)std::max(0, b[1] - b[0]) * std::max(0, b[3] - b[2]) * std::max(0, b[5] - b[4]);
}

// mean over the steps [0, nsteps) of one shot's box volume, averaged over the shots
static double mean_box_cells(const Plan &pl, const std::vector<int> &tab, int nsteps) {
    const int ns = pl.nshot;
    double v = 0;
    for (int it = 0; it < nsteps; ++it)
        for (int s = 0; s < ns; ++s) v += box_volume(&tab[((size_t)it * ns + s) * 6]);
    return nsteps > 0 ? v / ((double)nsteps * ns) : 0.0;
}

// memory variables of one shot that a box of `cells` cells touches, scaled from the slabs'
// share of the padded grid
static double psi_cells(const Plan &pl, double cells) {
    double all = 0;
    for (int a = 0; a < pl.nd; ++a) all += (double)pl.geom.psz[a];
    return all * cells / (double)((long long)pl.M[0] * pl.M[1] * pl.M[2]);
}

std::vector<int> fwd_groups(const Plan &pl, double budget, int max_per) {
    const int ns = pl.nshot, nrun = pl.nrun;
    if (pl.nd != 2 || ns <= 1) return {0, ns};
    if (max_per > 0) return equal_groups(ns, std::min(ns, max_per));
    // bytes of the fields and memory variables over `cells` box cells (the model is shared)
    auto bytes = [&](double cells) {
        return 4.0 * ((pl.nd + 1) * cells + 2.0 * psi_cells(pl, cells));
    };
    // cum[k (ns + 1) + s]: box cells of the shots [0, s) at step k * stride (the last sample
    // at the last step, where the boxes are largest); the steps are strided so that the table
    // stays within about 4 M entries (the boxes grow smoothly)
    const int stride = (int)std::max<long long>(1, (long long)nrun * (ns + 1) / (4LL << 20));
    const int nk = (nrun + stride - 1) / stride;
    std::vector<double> cum((size_t)nk * (ns + 1), 0.0);
    bool spill = false;
    for (int kk = 0; kk < nk; ++kk) {
        const int it = kk == nk - 1 ? nrun - 1 : kk * stride;
        double *c = &cum[(size_t)kk * (ns + 1)];
        for (int s = 0; s < ns; ++s) c[s + 1] = c[s] + box_volume(&pl.fbox[((size_t)it * ns + s) * 6]);
        spill = spill || bytes(c[ns]) > budget;
    }
    // one loop over every shot while all their boxes' fields stay in the cache: groups would
    // only add launches
    if (!spill) return {0, ns};
    // otherwise the group count whose loops cost least over the schedule of boxes.  A step's
    // two launches pay a fixed ramp and drain (about 6 us each), and a cell update costs 5.0 us
    // per million with its group's fields in the last-level cache, 8.4 us when they spill
    // (measured on the 2D order-8 step over 8, 16 and 32 shots of a 560 x 1560 grid)
    constexpr double kLaunches = 2 * 6.0, kHit = 5.0e-6, kMiss = 8.4e-6;
    std::vector<int> best;
    double best_cost = 0;
    for (int ng = 1; ng <= std::min(ns, 16); ++ng) {
        std::vector<int> off(ng + 1);
        for (int k = 0; k <= ng; ++k) off[k] = (int)((long long)ns * k / ng);
        double cost = 0;
        for (int kk = 0; kk < nk; ++kk) {
            const double *c = &cum[(size_t)kk * (ns + 1)];
            for (int k = 0; k < ng; ++k) {
                const double cells = c[off[k + 1]] - c[off[k]];
                if (cells > 0) cost += kLaunches + cells * (bytes(cells) > budget ? kMiss : kHit);
            }
        }
        if (best.empty() || cost < best_cost) {
            best = off;
            best_cost = cost;
        }
    }
    return best;
}

std::vector<int> rev_groups(const Plan &pl, double budget, int max_per, bool rho) {
    const int ns = pl.nshot;
    if (pl.nd != 2 || ns <= 1) return {0, ns};
    if (max_per > 0) return equal_groups(ns, std::min(ns, max_per));
    // on average over the reverse steps: the source field and the accumulators over the
    // reconstruction region, the adjoint field over the adjoint box, their memory variables,
    // and (when the pass keeps them) the density face sums
    const int nt = pl.g.nt;
    const double vr = mean_box_cells(pl, pl.rbox, nt), va = mean_box_cells(pl, pl.abox, nt);
    double fl = (pl.nd + 1) * (vr + va) + 3.0 * vr + 2.0 * (psi_cells(pl, vr) + psi_cells(pl, va));
    if (rho) fl += (double)pl.nd * vr;
    return equal_groups(ns, std::max(1, std::min(ns, (int)(budget / (4.0 * fl)))));
}

smi_status make_plan(const smi_grid *g, const smi_acq *acq, smi_job job, double vmin,
                     double vmax, Plan &pl, std::string &err) {
    smi_status st = check_grid(g, vmin, vmax, err);
    if (st != SMI_OK) return st;
    if (!acq || acq->nshot < 1 || !acq->src || !acq->rec_off) {
        err = "acquisition must have at least one shot";
        return SMI_E_ARG;
    }
    pl = Plan();
    pl.g = *g;
    pl.nd = g->ndim;
    pl.N = g->order / 2;
    pl.vmin = vmin;
    pl.vmax = vmax;
    pl.margin = g->box_margin >= 0 ? g->box_margin : 2 * pl.N;
    pl.n[0] = g->n1; pl.n[1] = g->n2; pl.n[2] = g->ndim == 3 ? g->n3 : 1;
    for (int a = 0; a < 3; ++a) pl.M[a] = a < pl.nd ? pl.n[a] + 2 * g->nb : 1;
    if ((pl.M[1] + 3) / 4 > 65535 || (long long)pl.M[2] * acq->nshot > 65535) {
        err = "grid too large for the sweep-kernel launch geometry";
        return SMI_E_UNSUPPORTED;
    }
    pl.ld1 = (int)align_up((size_t)pl.M[0] + 2 * GH, 32);
    pl.ld2 = (long long)pl.ld1 * (pl.M[1] + 2 * GH);
    pl.org = GH + (long long)pl.ld1 * GH + (pl.nd == 3 ? pl.ld2 * GH : 0);
    pl.P = pl.ld2 * (pl.nd == 3 ? pl.M[2] + 2 * GH : 1);
    pl.I = (long long)pl.n[0] * pl.n[1] * pl.n[2];
    pl.nshot = acq->nshot;
    if (acq->rec_off[0] != 0) { err = "rec_off[0] must be 0"; return SMI_E_ARG; }
    for (int s = 0; s < pl.nshot; ++s)
        if (acq->rec_off[s + 1] < acq->rec_off[s]) { err = "rec_off must not decrease"; return SMI_E_ARG; }
    int R = acq->rec_off[pl.nshot];
    if (R > 0 && !acq->rec) { err = "rec is NULL"; return SMI_E_ARG; }
    pl.rec_off.assign(acq->rec_off, acq->rec_off + pl.nshot + 1);
    double hs[3] = {g->d1, g->d2, g->ndim == 3 ? g->d3 : 1.0};
    pl.src.assign(3 * pl.nshot, 0);
    pl.src_cell.resize(pl.nshot);
    pl.src_toff.assign(1, 0);
    pl.src_tcell.clear();
    pl.src_tw.clear();
    pl.src_multi = false;
    for (int s = 0; s < pl.nshot; ++s) {
        if (!point_taps(pl, &acq->src[3 * s], hs, &pl.src[3 * s], pl.src_tcell, pl.src_tw)) {
            err = "source " + std::to_string(s) + " lies outside the model";
            return SMI_E_ARG;
        }
        pl.src_toff.push_back((int)pl.src_tcell.size());
        const bool one = pl.src_toff[s + 1] - pl.src_toff[s] == 1;
        pl.src_cell[s] = one ? pl.src_tcell[pl.src_toff[s]] : -1;
        pl.src_multi = pl.src_multi || !one;
    }
    pl.rec.assign(3 * (size_t)R, 0);
    pl.rec_toff.assign(1, 0);
    pl.rec_tcell.clear();
    pl.rec_tw.clear();
    for (int r = 0; r < R; ++r) {
        if (!point_taps(pl, &acq->rec[3 * (size_t)r], hs, &pl.rec[3 * (size_t)r], pl.rec_tcell,
                        pl.rec_tw)) {
            err = "receiver " + std::to_string(r) + " lies outside the model";
            return SMI_E_ARG;
        }
        pl.rec_toff.push_back((int)pl.rec_tcell.size());
    }
    // gather form of the adjoint-source injection: per shot, the distinct nodes of its
    // receivers' operators in ascending cell order, each with its (receiver, weight) pairs in
    // ascending receiver order
    pl.inj_shot.clear();
    pl.inj_cell.clear();
    pl.inj_rec.clear();
    pl.inj_w.clear();
    pl.inj_off.assign(1, 0);
    for (int s = 0; s < pl.nshot; ++s) {
        std::vector<std::pair<long long, int>> ct;   // (cell, tap index), taps in receiver order
        for (int r = pl.rec_off[s]; r < pl.rec_off[s + 1]; ++r)
            for (int t = pl.rec_toff[r]; t < pl.rec_toff[r + 1]; ++t) ct.emplace_back(pl.rec_tcell[t], t);
        std::stable_sort(ct.begin(), ct.end(),
                         [](const std::pair<long long, int> &a, const std::pair<long long, int> &b) {
                             return a.first < b.first;
                         });
        for (size_t i = 0; i < ct.size(); ++i) {
            if (i == 0 || ct[i].first != ct[i - 1].first) {
                if (i) pl.inj_off.push_back((int)pl.inj_rec.size());
                pl.inj_shot.push_back(s);
                pl.inj_cell.push_back(ct[i].first);
            }
            const int t = ct[i].second;
            // receiver of tap t: taps of receiver r are rec_toff[r] .. rec_toff[r+1)
            const int r = (int)(std::upper_bound(pl.rec_toff.begin(), pl.rec_toff.end(), t) -
                                pl.rec_toff.begin()) - 1;
            pl.inj_rec.push_back(r);
            pl.inj_w.push_back(pl.rec_tw[t]);
        }
        if (!ct.empty()) pl.inj_off.push_back((int)pl.inj_rec.size());
    }

    pl.save = job != SMI_JOB_FORWARD;
    pl.adjoint = pl.save;
    pl.need_G = job == SMI_JOB_GRAD || job == SMI_JOB_RTM;
    pl.need_dcal = pl.need_G;
    pl.rho_acc = job == SMI_JOB_GRAD || job == SMI_JOB_FORWARD_SAVE;
    pl.born = job == SMI_JOB_BORN;

    // computing boxes (Sec. 4.1)
    const int nt = g->nt, ns = pl.nshot;
    // decimated bands (dr > 1): the interpolator needs saved levels up to (nt-1)/dr + kTaps,
    // so the forward pass continues past nt (source off, nothing recorded) to that level
    pl.nsave = !pl.save ? 0 : (g->dr == 1 ? nt : (nt - 1) / g->dr + kTaps + 1);
    pl.nrun = pl.save && g->dr > 1 ? (pl.nsave - 1) * g->dr : nt;
    const int nrun = pl.nrun;
    pl.fbox.assign((size_t)nrun * ns * 6, 0);
    pl.abox.assign(pl.adjoint ? (size_t)nt * ns * 6 : 0, 0);
    pl.rbox.assign(pl.adjoint ? (size_t)nt * ns * 6 : 0, 0);
    pl.cnt_fwd = pl.cnt_adj = pl.cnt_rec = 0;
    for (int it = 0; it < nrun; ++it)
        for (int s = 0; s < ns; ++s) {
            const bool adj_it = pl.adjoint && it < nt;
            int *fb = &pl.fbox[((size_t)it * ns + s) * 6];
            double vf = 1, va = 1, vr = 1;
            for (int a = 0; a < 3; ++a) {
                int lo = 0, hi = pl.M[a];
                if (a < pl.nd && g->box) {
                    int r = (int)std::ceil(vmax * (it + 1) * g->dt / hs[a]) + pl.margin;
                    lo = std::max(0, pl.src[3 * s + a] - r);
                    hi = std::min(pl.M[a] - 1, pl.src[3 * s + a] + r) + 1;
                }
                fb[2 * a] = lo; fb[2 * a + 1] = hi;
                vf *= hi - lo;
                if (adj_it) {
                    int *ab = &pl.abox[((size_t)it * ns + s) * 6];
                    int *rb = &pl.rbox[((size_t)it * ns + s) * 6];
                    int alo = 0, ahi = pl.M[a];
                    int nr = pl.rec_off[s + 1] - pl.rec_off[s];
                    if (a < pl.nd && nr == 0) { alo = 0; ahi = 0; }
                    else if (a < pl.nd && g->box) {
                        int rmin = 1 << 30, rmax = -1;
                        for (int r = pl.rec_off[s]; r < pl.rec_off[s + 1]; ++r) {
                            rmin = std::min(rmin, pl.rec[3 * (size_t)r + a]);
                            rmax = std::max(rmax, pl.rec[3 * (size_t)r + a]);
                        }
                        int w = (int)std::ceil(vmax * (nt - it) * g->dt / hs[a]) + pl.margin;
                        alo = std::max(0, rmin - w);
                        ahi = std::min(pl.M[a] - 1, rmax + w) + 1;
                    }
                    ab[2 * a] = alo; ab[2 * a + 1] = ahi;
                    va *= std::max(0, ahi - alo);
                    int rlo = lo, rhi = hi;
                    if (a < pl.nd) {
                        rlo = std::max(lo, g->nb);
                        rhi = std::min(hi, g->nb + pl.n[a]);
                    }
                    if (rhi < rlo) rhi = rlo;
                    rb[2 * a] = rlo; rb[2 * a + 1] = rhi;
                    vr *= rhi - rlo;
                }
            }
            pl.cnt_fwd += vf;
            if (adj_it) { pl.cnt_adj += va; pl.cnt_rec += vr; }
        }
    algorithmic_bytes(pl);

    // boundary bands (Sec. 4.2): N planes of p and N of the face-normal v per face
    BandDesc &bd = pl.band;
    bd = BandDesc();
    long long off = 0;
    for (int a = 0; a < pl.nd; ++a) {
        int N = pl.N, nb = g->nb, na = pl.n[a];
        int starts[4] = {nb - N, nb + na, nb - N, nb + na - 1};
        for (int k = 0; k < 4; ++k) {
            BandBlock &b = bd.blk[bd.nblk++];
            b.field = k < 2 ? 0 : 1;
            b.axis = a;
            b.start = starts[k];
            b.w = N;
            long long cnt = 1;
            for (int q = 0; q < 3; ++q) {
                if (q >= pl.nd) { b.ext[q] = 1; b.org[q] = 0; }
                else if (q == a) { b.ext[q] = N; b.org[q] = b.start; }
                else { b.ext[q] = pl.n[q]; b.org[q] = nb; }
                cnt *= b.ext[q];
            }
            b.off = off;
            b.cnt = cnt;
            off += cnt;
        }
    }
    bd.B = off;
    if (bd.B >= (1LL << 31)) {
        // the band kernels index the cells of one shot's band with 32-bit integers
        err = "the saved boundary band of one shot exceeds 2^31 cells";
        return SMI_E_UNSUPPORTED;
    }


    // device geometry
    Geom &G = pl.geom;
    G.nd = pl.nd; G.N = pl.N; G.nb = g->nb; G.ld1 = pl.ld1; G.ld2 = pl.ld2; G.org = pl.org;
    G.P = pl.P; G.I = pl.I;
    for (int a = 0; a < 3; ++a) { G.n[a] = pl.n[a]; G.M[a] = pl.M[a]; }
    G.W = slab_width(g->nb);
    G.psz[0] = (long long)G.W * pl.M[1] * pl.M[2];
    G.psz[1] = pl.nd >= 2 ? (long long)pl.ld1 * G.W * pl.M[2] : 0;
    G.psz[2] = pl.nd == 3 ? (long long)pl.ld1 * pl.M[1] * G.W : 0;
    double aw[kMaxN];
    fd_weights(pl.N, aw);
    for (int a = 0; a < 3; ++a)
        for (int l = 0; l < kMaxN; ++l) G.c[a][l] = l < pl.N ? (float)(aw[l] / hs[a]) : 0.f;
    G.dt = (float)g->dt;
    G.fs = g->freesurf;
    G.src_scale = (float)(g->dt / (hs[0] * hs[1] * (pl.nd == 3 ? hs[2] : 1.0)));

    // node map of the adjoint-source gather (see Plan::inj_map): the adjoint p update of
    // reverse step it + 1 adds the injection of step it on the lanes that own the nodes when
    // every node of a shot lies inside that shot's adjoint box at every such step
    pl.inj_map.clear();
    pl.inj_zlo = pl.inj_nrow = 0;
    pl.inj_fused = false;
    if (pl.adjoint && pl.nd == 2 && !pl.inj_cell.empty()) {
        const int U = (int)pl.inj_cell.size();
        std::vector<int> nz(U), nx(U);
        std::vector<int> bb((size_t)ns * 4);   // per shot: node rows and columns, min and max
        for (int s = 0; s < ns; ++s) {
            bb[4 * s] = bb[4 * s + 2] = 1 << 30;
            bb[4 * s + 1] = bb[4 * s + 3] = -1;
        }
        int zlo = 1 << 30, zhi = -1;
        for (int u = 0; u < U; ++u) {
            const long long rel = pl.inj_cell[u] - pl.org;   // z + ld1 x, nodes inside the model
            nx[u] = (int)(rel / pl.ld1);
            nz[u] = (int)(rel - (long long)nx[u] * pl.ld1);
            zlo = std::min(zlo, nz[u]);
            zhi = std::max(zhi, nz[u]);
            int *q = &bb[4 * (size_t)pl.inj_shot[u]];
            q[0] = std::min(q[0], nz[u]);
            q[1] = std::max(q[1], nz[u]);
            q[2] = std::min(q[2], nx[u]);
            q[3] = std::max(q[3], nx[u]);
        }
        const int nrow = zhi - zlo + 1;
        bool ok = (size_t)ns * nrow * pl.M[1] <= kInjMapCap;
        for (int it = 1; ok && it < nt; ++it)
            for (int s = 0; ok && s < ns; ++s) {
                const int *q = &bb[4 * (size_t)s];
                if (q[1] < 0) continue;
                const int *ab = &pl.abox[((size_t)it * ns + s) * 6];
                ok = q[0] >= ab[0] && q[1] < ab[1] && q[2] >= ab[2] && q[3] < ab[3];
            }
        if (ok) {
            pl.inj_map.assign((size_t)ns * nrow * pl.M[1], -1);
            for (int u = 0; u < U; ++u)
                pl.inj_map[((size_t)pl.inj_shot[u] * nrow + (nz[u] - zlo)) * pl.M[1] + nx[u]] = u;
            pl.inj_zlo = zlo;
            pl.inj_nrow = nrow;
            pl.inj_fused = true;
        }
    }

    // workspace layout
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes, 256); return r; };
    pl.off_status = take(64);
    pl.off_misfit = take(16);
    pl.off_bdesc = take(sizeof(BandDesc));
    pl.npartial = std::max(1024, acq->nshot);   // also holds the per-shot peak illumination
    pl.off_partial = take(sizeof(double) * pl.npartial);
    pl.off_model = take(sizeof(float) * (size_t)pl.P * (1 + pl.nd));
    size_t cp = 0;
    for (int a = 0; a < pl.nd; ++a) cp += 4 * (size_t)pl.M[a];
    pl.off_cpml = take(sizeof(float) * cp);
    pl.off_tables = take(sizeof(int) * (pl.fbox.size() + pl.abox.size() + pl.rbox.size()));
    pl.off_recv = take((size_t)R * (sizeof(int) * 2 + sizeof(long long)) +
                       sizeof(long long) * (size_t)ns + 64);
    pl.off_taps = take(sizeof(int) * (pl.src_toff.size() + pl.rec_toff.size()) +
                       (sizeof(long long) + sizeof(float)) * (pl.src_tcell.size() + pl.rec_tcell.size()) + 64);
    pl.off_inj = take((sizeof(int) * 2 + sizeof(long long)) * pl.inj_cell.size() +
                      (sizeof(int) + sizeof(float)) * pl.inj_rec.size() + 64);
    pl.off_injmap = take(sizeof(int) * pl.inj_map.size() + 64);
    size_t fld = sizeof(float) * (size_t)ns * ((size_t)pl.P * (1 + pl.nd) +
                 2 * (size_t)(G.psz[0] + G.psz[1] + G.psz[2]));
    pl.off_fields = take(fld);
    pl.dbuf = pl.nd == 2;
    pl.off_fields2 = pl.dbuf ? take(fld) : 0;
    pl.off_adj = pl.adjoint || pl.born ? take(fld) : 0;
    pl.off_bands = pl.save ? take(sizeof(float) * (size_t)ns * pl.nsave * (size_t)bd.B) : 0;
    pl.off_fin = pl.save && g->dr > 1 ? take(sizeof(float) * (size_t)ns * (size_t)pl.P * (1 + pl.nd)) : 0;
    pl.off_acc = pl.adjoint ? take(sizeof(float) * 3 * (size_t)ns * (size_t)pl.I) : 0;
    pl.off_rho = pl.rho_acc ? take(sizeof(float) * pl.nd * (size_t)ns * (size_t)pl.P) : 0;
    pl.off_G = pl.need_G ? take(sizeof(float) * (size_t)nt * R) : 0;
    pl.off_dcal = pl.need_dcal ? take(sizeof(float) * (size_t)nt * R) : 0;
    // tail slack: the fused 2D step reads (and never uses) up to kTailCols columns of a
    // field or model array past the ghost frame of the last shot
    take(sizeof(float) * (size_t)kTailCols * pl.ld1);
    pl.bytes = o;
    return SMI_OK;
}

Views views(const Plan &pl, void *ws) {
    char *b = (char *)ws;
    Views w{};
    w.status = (unsigned *)(b + pl.off_status);
    w.bdesc = (const BandDesc *)(b + pl.off_bdesc);
    w.misfit_tmp = (double *)(b + pl.off_misfit);
    w.partial = (double *)(b + pl.off_partial);
    float *m = (float *)(b + pl.off_model);
    w.model.kdt = m;
    for (int a = 0; a < 3; ++a) w.model.bdt[a] = a < pl.nd ? m + (size_t)pl.P * (1 + a) : nullptr;
    float *c = (float *)(b + pl.off_cpml);
    for (int a = 0; a < 3; ++a) {
        if (a >= pl.nd) { w.cpml.a_i[a] = w.cpml.b_i[a] = w.cpml.a_h[a] = w.cpml.b_h[a] = nullptr; continue; }
        int M = pl.M[a];
        w.cpml.a_i[a] = c; w.cpml.b_i[a] = c + M; w.cpml.a_h[a] = c + 2 * M; w.cpml.b_h[a] = c + 3 * M;
        c += 4 * M;
    }
    int *t = (int *)(b + pl.off_tables);
    w.fbox = t;
    w.abox = pl.adjoint ? t + pl.fbox.size() : nullptr;
    w.rbox = pl.adjoint ? t + pl.fbox.size() + pl.abox.size() : nullptr;
    int R = pl.rec_off[pl.nshot];
    char *r = b + pl.off_recv;
    w.recv.R = R;
    w.recv.obase = (long long *)r;
    w.recv.shot = (int *)(r + sizeof(long long) * R);
    w.recv.stride = (int *)(r + sizeof(long long) * R + sizeof(int) * R);
    w.src_cell = (long long *)(r + align_up((sizeof(long long) + 2 * sizeof(int)) * (size_t)R, 8));
    {
        // taps: cells (8-byte) first, then weights and offsets
        char *q = b + pl.off_taps;
        w.src_tcell = (long long *)q;
        q += sizeof(long long) * pl.src_tcell.size();
        w.recv.tcell = (long long *)q;
        q += sizeof(long long) * pl.rec_tcell.size();
        w.src_tw = (float *)q;
        q += sizeof(float) * pl.src_tw.size();
        w.recv.tw = (float *)q;
        q += sizeof(float) * pl.rec_tw.size();
        w.src_toff = (int *)q;
        q += sizeof(int) * pl.src_toff.size();
        w.recv.toff = (int *)q;
    }
    {
        // injection gather: cells (8-byte) first, then shots, offsets, receivers, weights
        const size_t U = pl.inj_cell.size(), T = pl.inj_rec.size();
        char *q = b + pl.off_inj;
        w.inj.U = (int)U;
        w.inj.cell = (long long *)q;
        q += sizeof(long long) * U;
        w.inj.shot = (int *)q;
        q += sizeof(int) * U;
        w.inj.off = (int *)q;
        q += sizeof(int) * (U + 1);
        w.inj.rec = (int *)q;
        q += sizeof(int) * T;
        w.inj.w = (float *)q;
        w.injmap = pl.inj_map.empty() ? nullptr : (int *)(b + pl.off_injmap);
    }
    auto fields = [&](size_t off) {
        Fields f{};
        float *p = (float *)(b + off);
        size_t ns = pl.nshot;
        f.p = p; p += ns * pl.P;
        for (int a = 0; a < 3; ++a) {
            if (a < pl.nd) { f.v[a] = p; p += ns * pl.P; } else f.v[a] = nullptr;
        }
        for (int a = 0; a < 3; ++a) {
            if (a < pl.nd) {
                f.psp[a] = p; p += ns * pl.geom.psz[a];
                f.psv[a] = p; p += ns * pl.geom.psz[a];
            } else f.psp[a] = f.psv[a] = nullptr;
        }
        return f;
    };
    w.f = fields(pl.off_fields);
    w.f2 = pl.dbuf ? fields(pl.off_fields2) : Fields{};
    w.q = pl.adjoint || pl.born ? fields(pl.off_adj) : Fields{};
    w.bands = pl.save ? (float *)(b + pl.off_bands) : nullptr;
    if (pl.adjoint) {
        float *a = (float *)(b + pl.off_acc);
        w.acc_g = a;
        for (int q = 0; q < 3; ++q)
            w.acc_r[q] = pl.rho_acc && q < pl.nd
                             ? (float *)(b + pl.off_rho) + (size_t)q * pl.nshot * pl.P
                             : nullptr;
        w.acc_i = a + (size_t)pl.nshot * pl.I;
        w.acc_l = a + 2 * (size_t)pl.nshot * pl.I;
    }
    w.G = pl.need_G ? (float *)(b + pl.off_G) : nullptr;
    w.dcal = pl.need_dcal ? (float *)(b + pl.off_dcal) : nullptr;
    w.fin = pl.off_fin ? (float *)(b + pl.off_fin) : nullptr;
    return w;
}

}  // namespace smi
