// Host-side construction of the coarse operator and the interface lists.
//
// * Q1 elements on the uniform M x M mesh, 2 x 2 Gauss quadrature, consistent
//   capacity matrix; Galerkin form of eq. (Galerkin) plus, with supg, the
//   streamline-upwind terms of eq. (SUPG) with tau_e of eq. (SUPG_tau)
//   (h_e = mesh size, p = 1, evaluated per quadrature point; the residual has
//   no diffusion term since the Laplacian of a bilinear function vanishes).
// * Trapezoidal rule of eq. (FEM_discrete) with theta = 1/2 for the nodal
//   values: A = C + dt/2 T, B = C - dt/2 T with capacity C = M + Ms and
//   transport T = K + Ks (K includes the reaction k M).
// * Strong Dirichlet rows (diagonal only) on the outer edge and on Gamma_{f->c}.
// * A sparse approximate inverse P of A on a (2R+1)^2 stencil: row i of P
//   minimises || e_i^T - P_i A ||_2 over that pattern (normal equations,
//   Cholesky).  A P is formed once as a (2R+3)^2 stencil.
#include <cmath>
#include <cstring>

#include <array>
#include <algorithm>

#include "hyb_impl.h"

namespace hyb {
namespace {

// upwind function chi(a) = coth(a) - 1/a of eq. (SUPG_tau); for a < 0.1 the
// difference cancels badly, so the Laurent series through a^9 is summed.
double upwind_chi(double a) {
    if (a < 0.1) {
        const double a2 = a * a;
        double s = 2.0 / 93555.0;
        s = -1.0 / 4725.0 + a2 * s;
        s = 2.0 / 945.0 + a2 * s;
        s = -1.0 / 45.0 + a2 * s;
        s = 1.0 / 3.0 + a2 * s;
        return a * s;
    }
    return 1.0 / std::tanh(a) - 1.0 / a;   // tanh saturates to 1; cosh/sinh would overflow
}

struct Stencil {
    int M, W, R;
    std::vector<double> c;
    Stencil(int M_, int W_) : M(M_), W(W_), R(W_ / 2), c((size_t)(M_ + 1) * (M_ + 1) * W_ * W_, 0.0) {}
    double &at(int node, int dk, int dl) { return c[(size_t)node * W * W + (dl + R) * W + (dk + R)]; }
    double get(int node, int dk, int dl) const {
        if (dk < -R || dk > R || dl < -R || dl > R) return 0.0;
        return c[(size_t)node * W * W + (dl + R) * W + (dk + R)];
    }
};

// small dense SPD solve (Cholesky), n <= 25; returns false if not SPD.
bool chol_solve(std::vector<double> &G, std::vector<double> &b, int n) {
    for (int j = 0; j < n; ++j) {
        double d = G[j * n + j];
        for (int k = 0; k < j; ++k) d -= G[j * n + k] * G[j * n + k];
        if (!(d > 0.0)) return false;
        d = std::sqrt(d);
        G[j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            double s = G[i * n + j];
            for (int k = 0; k < j; ++k) s -= G[i * n + k] * G[j * n + k];
            G[i * n + j] = s / d;
        }
    }
    for (int i = 0; i < n; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= G[i * n + k] * b[k];
        b[i] = s / G[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = b[i];
        for (int k = i + 1; k < n; ++k) s -= G[k * n + i] * b[k];
        b[i] = s / G[i * n + i];
    }
    return true;
}

}  // namespace

// Interface lists of one patch against the mesh: coarse-to-fine weights of
// its perimeter slots and the fine-to-coarse corners of out.fc_nodes (its
// Gamma_{f->c} nodes, set by the caller), each with its transpose.
std::string patch_lists(int M, double L, const PatchGeom &g, CoarseHost &out) {
    const int m1 = M + 1;
    const int n = m1 * m1;
    const double h = L / M;
    const int N = g.N, pitch = g.pitch;
    const double x0 = g.x0, y0 = g.y0;
    const uint8_t *solid = g.solid;
    // --- coarse -> fine: containing element of each perimeter slot --------
    const int S = M + 1 + 2 * kCoarseHalo;
    auto padded = [&](int kk, int l) { return (l + kCoarseHalo) * S + (kk + kCoarseHalo); };
    const int nslots = 4 * (N - 1);
    out.c2f_idx.assign((size_t)4 * nslots, 0);
    out.c2f_w.assign((size_t)4 * nslots, 0.0);
    for (int p = 0; p < nslots; ++p) {
        int i, j;
        slot_to_node(N, p, i, j);
        const double sx = (x0 + i) / h, sy = (y0 + j) / h;
        int ex = (int)std::floor(sx), ey = (int)std::floor(sy);
        ex = ex < 0 ? 0 : (ex > M - 1 ? M - 1 : ex);
        ey = ey < 0 ? 0 : (ey > M - 1 ? M - 1 : ey);
        const double xi = sx - ex, et = sy - ey;
        const int cidx[4] = {padded(ex, ey), padded(ex + 1, ey), padded(ex + 1, ey + 1), padded(ex, ey + 1)};
        const double cw[4] = {(1 - xi) * (1 - et), xi * (1 - et), xi * et, (1 - xi) * et};
        for (int c = 0; c < 4; ++c) {
            out.c2f_idx[4 * p + c] = cidx[c];
            out.c2f_w[4 * p + c] = cw[c];
        }
    }

    // coarse -> fine transposed: per mesh node, the slots that read it
    {
        out.c2fT_ptr.assign(n + 1, 0);
        auto node_of = [&](int pidx) { return (pidx / S - kCoarseHalo) * m1 + (pidx % S - kCoarseHalo); };
        for (int e = 0; e < 4 * nslots; ++e) out.c2fT_ptr[node_of(out.c2f_idx[e]) + 1] += 1;
        for (int id = 0; id < n; ++id) out.c2fT_ptr[id + 1] += out.c2fT_ptr[id];
        out.c2fT_slot.assign((size_t)4 * nslots, 0);
        out.c2fT_w.assign((size_t)4 * nslots, 0.0);
        std::vector<int> fill(out.c2fT_ptr.begin(), out.c2fT_ptr.end() - 1);
        for (int e = 0; e < 4 * nslots; ++e) {
            const int at = fill[node_of(out.c2f_idx[e])]++;
            out.c2fT_slot[at] = e / 4;
            out.c2fT_w[at] = out.c2f_w[e];
        }
    }

    // --- fine -> coarse: four surrounding lattice nodes --------------------
    const int nfc = (int)out.fc_nodes.size();
    out.fc_idx.assign((size_t)4 * nfc, 0);
    out.fc_w.assign((size_t)4 * nfc, 0.0);
    out.fcr_idx.assign((size_t)4 * nfc, 0);
    out.fcr_w.assign((size_t)4 * nfc, 0.0);
    out.fcr_fb.assign((size_t)nfc, -1);
    auto is_solid = [&](int i, int j) { return solid && solid[(size_t)j * N + i]; };
    for (int c = 0; c < nfc; ++c) {
        const int id = out.fc_nodes[c];
        const double px = (id % m1) * h - x0, py = (id / m1) * h - y0;
        int i0 = (int)std::floor(px), j0 = (int)std::floor(py);
        i0 = i0 < 0 ? 0 : (i0 > N - 2 ? N - 2 : i0);
        j0 = j0 < 0 ? 0 : (j0 > N - 2 ? N - 2 : j0);
        const double gx = px - i0, gy = py - j0;
        const int ci[4] = {i0, i0 + 1, i0 + 1, i0}, cj[4] = {j0, j0, j0 + 1, j0 + 1};
        const double cw[4] = {(1 - gx) * (1 - gy), gx * (1 - gy), gx * gy, (1 - gx) * gy};
        double wsum = 0.0;
        for (int m = 0; m < 4; ++m) {
            if (!is_solid(ci[m], cj[m])) wsum += cw[m];
            out.fcr_idx[4 * c + m] = cj[m] * pitch + ci[m];
            out.fcr_w[4 * c + m] = cw[m];
        }
        if (wsum > 0.0) {
            for (int m = 0; m < 4; ++m) {
                out.fc_idx[4 * c + m] = cj[m] * pitch + ci[m];
                out.fc_w[4 * c + m] = is_solid(ci[m], cj[m]) ? 0.0 : cw[m] / wsum;
            }
            continue;
        }
        // all four corners solid: nearest fluid node, lowest j*N+i on ties,
        // searched in growing squares around the point
        int best = -1;
        double bd = 0.0;
        const int ic = (int)std::floor(px + 0.5), jc = (int)std::floor(py + 0.5);
        for (int r = 1; r <= 2 * N && best < 0; ++r) {
            int cand = -1;
            double cd = 0.0;
            for (int j = std::max(0, jc - r); j <= std::min(N - 1, jc + r); ++j)
                for (int i = std::max(0, ic - r); i <= std::min(N - 1, ic + r); ++i) {
                    if (is_solid(i, j)) continue;
                    const double d2 = (i - px) * (i - px) + (j - py) * (j - py);
                    if (cand < 0 || d2 < cd) { cand = j * N + i; cd = d2; }
                }
            if (cand >= 0 && std::sqrt(cd) <= r - 0.5) { best = cand; bd = cd; }
        }
        (void)bd;
        if (best < 0) return "fine-to-coarse transfer: no fluid lattice node";
        out.fc_idx[4 * c] = (best / N) * pitch + (best % N);
        out.fc_w[4 * c] = 1.0;
        out.fcr_fb[c] = out.fc_idx[4 * c];
        for (int m = 1; m < 4; ++m) {
            out.fc_idx[4 * c + m] = out.fc_idx[4 * c];
            out.fc_w[4 * c + m] = 0.0;
        }
    }

    // fine -> coarse transposed: per lattice node read with a nonzero
    // weight, the Gamma_{f->c} indices and weights (node, then index order)
    {
        std::vector<std::array<double, 3>> e;      // (pitched node, c, w)
        for (int c = 0; c < nfc; ++c)
            for (int m = 0; m < 4; ++m)
                if (out.fc_w[4 * c + m] != 0.0) e.push_back({(double)out.fc_idx[4 * c + m], (double)c, out.fc_w[4 * c + m]});
        std::sort(e.begin(), e.end(), [](const std::array<double, 3> &a, const std::array<double, 3> &b) {
            return a[0] != b[0] ? a[0] < b[0] : a[1] < b[1];
        });
        out.f2cT_node.clear();
        out.f2cT_ptr.assign(1, 0);
        out.f2cT_c.clear();
        out.f2cT_w.clear();
        for (size_t t = 0; t < e.size(); ++t) {
            if (t == 0 || e[t][0] != e[t - 1][0]) {
                if (t) out.f2cT_ptr.push_back((int)t);
                out.f2cT_node.push_back((int)e[t][0]);
            }
            out.f2cT_c.push_back((int)e[t][1]);
            out.f2cT_w.push_back(e[t][2]);
        }
        out.f2cT_ptr.push_back((int)e.size());
        if (e.empty()) out.f2cT_ptr.assign(1, 0);
    }

    // the same for a geometry that changes (dissolving solids): every raw
    // corner (slot 0..3) and fallback node (slot 4) of every Gamma_{f->c}
    // node, grouped per lattice node; the weights follow from the flag words
    // of the step being reversed
    {
        std::vector<std::array<int, 3>> e;         // (pitched node, c, slot)
        for (int c = 0; c < nfc; ++c) {
            for (int m = 0; m < 4; ++m) e.push_back({out.fcr_idx[4 * c + m], c, m});
            if (out.fcr_fb[c] >= 0) e.push_back({out.fcr_fb[c], c, 4});
        }
        std::sort(e.begin(), e.end());
        out.f2cD_node.clear();
        out.f2cD_ptr.assign(1, 0);
        out.f2cD_c.clear();
        out.f2cD_m.clear();
        for (size_t t = 0; t < e.size(); ++t) {
            if (t == 0 || e[t][0] != e[t - 1][0]) {
                if (t) out.f2cD_ptr.push_back((int)t);
                out.f2cD_node.push_back(e[t][0]);
            }
            out.f2cD_c.push_back(e[t][1]);
            out.f2cD_m.push_back(e[t][2]);
        }
        out.f2cD_ptr.push_back((int)e.size());
        if (e.empty()) out.f2cD_ptr.assign(1, 0);
    }
    return std::string();
}

std::string build_coarse(int M, double L, double D, double k, double dt, int supg, const double *vnodes,
                         int overlap_elems, const std::vector<PatchGeom> &patches, CoarseHost &out,
                         std::vector<CoarseHost> *more, int outer_natural) {
    if (patches.empty()) return "no lattice patch";
    const int m1 = M + 1;
    const int n = m1 * m1;
    const double h = L / M;
    out.M = M;
    out.L = L;
    out.h = h;

    // --- quadrature tables on the reference square [-1,1]^2 -------------
    // local nodes 0:(0,0) 1:(1,0) 2:(1,1) 3:(0,1) of element (ex, ey)
    const int lk[4] = {0, 1, 1, 0}, ll[4] = {0, 0, 1, 1};
    const double gq = 1.0 / std::sqrt(3.0);
    double Nv[4][4], Gx[4][4], Gy[4][4];   // [gauss point][local node]
    for (int g = 0; g < 4; ++g) {
        const double xi = (g & 1) ? gq : -gq, et = (g & 2) ? gq : -gq;
        for (int a = 0; a < 4; ++a) {
            const double sa = lk[a] ? 1.0 : -1.0, ta = ll[a] ? 1.0 : -1.0;
            Nv[g][a] = 0.25 * (1.0 + sa * xi) * (1.0 + ta * et);
            Gx[g][a] = 0.5 * sa * (1.0 + ta * et) / h;
            Gy[g][a] = 0.5 * ta * (1.0 + sa * xi) / h;
        }
    }
    const double wq = 0.25 * h * h;   // Gauss weight 1 times det J

    Stencil A(M, 3), B(M, 3);
    for (int ey = 0; ey < M; ++ey) {
        for (int ex = 0; ex < M; ++ex) {
            int node[4];
            for (int a = 0; a < 4; ++a) node[a] = (ey + ll[a]) * m1 + (ex + lk[a]);
            double cap[4][4] = {}, tr[4][4] = {};
            for (int g = 0; g < 4; ++g) {
                double vx = 0.0, vy = 0.0;
                for (int a = 0; a < 4; ++a) {
                    vx += Nv[g][a] * vnodes[2 * node[a]];
                    vy += Nv[g][a] * vnodes[2 * node[a] + 1];
                }
                const double speed = std::sqrt(vx * vx + vy * vy);
                double tau = 0.0;
                if (supg && speed > 0.0) tau = h / (2.0 * speed) * upwind_chi(speed * h / (2.0 * D));
                double adv[4];
                for (int a = 0; a < 4; ++a) adv[a] = vx * Gx[g][a] + vy * Gy[g][a];
                for (int a = 0; a < 4; ++a) {
                    for (int b = 0; b < 4; ++b) {
                        const double mass = Nv[g][a] * Nv[g][b];
                        const double galerkin = Nv[g][a] * adv[b] + D * (Gx[g][a] * Gx[g][b] + Gy[g][a] * Gy[g][b]) +
                                                k * mass;
                        const double stab_cap = tau * adv[a] * Nv[g][b];
                        const double stab_tr = tau * adv[a] * (adv[b] + k * Nv[g][b]);
                        cap[a][b] += wq * (mass + stab_cap);
                        tr[a][b] += wq * (galerkin + stab_tr);
                    }
                }
            }
            for (int a = 0; a < 4; ++a) {
                for (int b = 0; b < 4; ++b) {
                    const int dk = lk[b] - lk[a], dl = ll[b] - ll[a];
                    A.at(node[a], dk, dl) += cap[a][b] + 0.5 * dt * tr[a][b];
                    B.at(node[a], dk, dl) += cap[a][b] - 0.5 * dt * tr[a][b];
                }
            }
        }
    }

    // --- Dirichlet sets ---------------------------------------------------
    // Gamma_{f->c} of patch p: the coarse nodes inside it at least
    // overlap_elems elements from its boundary; indices run patch by patch
    // (each patch's transferred values are one contiguous run)
    // outer edges 0: x = 0, 1: x = L, 2: y = 0, 3: y = L; an edge whose bit
    // is set in outer_natural keeps its rows (the natural condition of the
    // weak form, zero diffusive flux); a node on a Dirichlet edge is a
    // Dirichlet row
    out.dkind.assign(n, -1);
    for (int l = 0; l < m1; ++l)
        for (int kk = 0; kk < m1; ++kk) {
            const bool dir = (kk == 0 && !(outer_natural & 1)) || (kk == M && !(outer_natural & 2)) ||
                             (l == 0 && !(outer_natural & 4)) || (l == M && !(outer_natural & 8));
            if (dir) out.dkind[l * m1 + kk] = -2;
        }
    const double ov = overlap_elems * h, tol = 1e-9 * h;
    std::vector<std::vector<int>> fcn(patches.size());
    int nfc_all = 0;
    for (size_t p = 0; p < patches.size(); ++p) {
        const PatchGeom &g = patches[p];
        const double x1 = g.x0 + (g.N - 1), y1 = g.y0 + (g.N - 1);
        for (int l = 1; l < M; ++l) {
            for (int kk = 1; kk < M; ++kk) {
                const int id = l * m1 + kk;
                const double X = kk * h, Y = l * h;
                if (X - g.x0 >= ov - tol && x1 - X >= ov - tol && Y - g.y0 >= ov - tol && y1 - Y >= ov - tol) {
                    if (out.dkind[id] != -1) return "a coarse node lies on the interface of two patches";
                    out.dkind[id] = nfc_all++;
                    fcn[p].push_back(id);
                }
            }
        }
    }
    out.fc_nodes = fcn[0];
    if (more) {
        more->assign(patches.size() - 1, CoarseHost());
        for (size_t p = 1; p < patches.size(); ++p) {
            CoarseHost &o = (*more)[p - 1];
            o.M = M;
            o.L = L;
            o.h = h;
            o.fc_nodes = fcn[p];
            std::string msg = patch_lists(M, L, patches[p], o);
            if (!msg.empty()) return msg;
        }
    }
    // A Dirichlet row becomes a_ii e_i with the assembled diagonal a_ii (the
    // right-hand side is scaled by a_ii too), so every row of A carries the
    // same scale (~h^2) and the preconditioner's local systems stay well
    // conditioned even when h is hundreds of lattice units.
    for (int id = 0; id < n; ++id) {
        if (out.dkind[id] == -1) continue;
        const double diag = A.at(id, 0, 0);
        for (int dl = -1; dl <= 1; ++dl)
            for (int dk = -1; dk <= 1; ++dk) A.at(id, dk, dl) = 0.0;
        A.at(id, 0, 0) = diag > 0.0 ? diag : 1.0;
    }

    // --- sparse approximate inverse of A ---------------------------------
    constexpr int R = kSpaiRadius, W = kSpaiW;
    Stencil P(M, W);
    std::vector<int> pk, pl;
    std::vector<double> G, rhs;
    for (int l = 0; l < m1; ++l) {
        for (int kk = 0; kk < m1; ++kk) {
            const int id = l * m1 + kk;
            pk.clear();
            pl.clear();
            for (int dl = -R; dl <= R; ++dl)
                for (int dk = -R; dk <= R; ++dk)
                    if (kk + dk >= 0 && kk + dk <= M && l + dl >= 0 && l + dl <= M) {
                        pk.push_back(dk);
                        pl.push_back(dl);
                    }
            const int np = (int)pk.size();
            G.assign((size_t)np * np, 0.0);
            rhs.assign(np, 0.0);
            for (int a = 0; a < np; ++a) {
                const int na = (l + pl[a]) * m1 + (kk + pk[a]);
                // rhs_a = A(na, id): column id lies at offset (-pk, -pl) from row na
                rhs[a] = A.get(na, -pk[a], -pl[a]);
                for (int b = a; b < np; ++b) {
                    const int nb = (l + pl[b]) * m1 + (kk + pk[b]);
                    // sum over columns c of A(na, c) A(nb, c)
                    double s = 0.0;
                    for (int dl = -1; dl <= 1; ++dl)
                        for (int dk = -1; dk <= 1; ++dk) {
                            const double va = A.get(na, dk, dl);
                            if (va == 0.0) continue;
                            s += va * A.get(nb, dk + pk[a] - pk[b], dl + pl[a] - pl[b]);
                        }
                    G[a * np + b] = s;
                    G[b * np + a] = s;
                }
            }
            if (chol_solve(G, rhs, np)) {
                for (int a = 0; a < np; ++a) P.at(id, pk[a], pl[a]) = rhs[a];
            } else {
                P.at(id, 0, 0) = 1.0 / A.get(id, 0, 0);   // Jacobi row as a fallback
            }
        }
    }
    Stencil AP(M, kApW);
    for (int l = 0; l < m1; ++l) {
        for (int kk = 0; kk < m1; ++kk) {
            const int id = l * m1 + kk;
            for (int dl = -1; dl <= 1; ++dl)
                for (int dk = -1; dk <= 1; ++dk) {
                    const double a = A.get(id, dk, dl);
                    if (a == 0.0) continue;
                    const int nk = kk + dk, nl = l + dl;
                    const int nid = nl * m1 + nk;
                    for (int el = -R; el <= R; ++el)
                        for (int ek = -R; ek <= R; ++ek) {
                            const double pv = P.get(nid, ek, el);
                            if (pv != 0.0) AP.at(id, dk + ek, dl + el) += a * pv;
                        }
                }
        }
    }
    for (double x : A.c)
        if (!std::isfinite(x)) return "coarse operator has non-finite entries";
    for (double x : P.c)
        if (!std::isfinite(x)) return "coarse preconditioner has non-finite entries";
    // transposes for the reverse mode: entry (id, offset o) of S^T is entry
    // (id + o, -o) of S (zero when id + o leaves the mesh)
    auto transpose = [&](const Stencil &S) {
        Stencil T(M, S.W);
        for (int l = 0; l < m1; ++l)
            for (int kk = 0; kk < m1; ++kk)
                for (int dl = -S.R; dl <= S.R; ++dl)
                    for (int dk = -S.R; dk <= S.R; ++dk) {
                        const int nk = kk + dk, nl = l + dl;
                        if (nk < 0 || nk > M || nl < 0 || nl > M) continue;
                        T.at(l * m1 + kk, dk, dl) = S.get(nl * m1 + nk, -dk, -dl);
                    }
        return T;
    };
    out.APT = transpose(AP).c;
    out.PT = transpose(P).c;
    out.A9 = std::move(A.c);
    out.B9 = std::move(B.c);
    out.P = std::move(P.c);
    out.AP = std::move(AP.c);

    return patch_lists(M, L, patches[0], out);
}

std::string build_coarse(int M, double L, double D, double k, double dt, int supg, const double *vnodes,
                         int overlap_elems, int N, double x0, double y0, const uint8_t *solid, int pitch,
                         CoarseHost &out, int outer_natural) {
    const std::vector<PatchGeom> one{PatchGeom{N, x0, y0, solid, pitch}};
    return build_coarse(M, L, D, k, dt, supg, vnodes, overlap_elems, one, out, nullptr, outer_natural);
}

}  // namespace hyb
