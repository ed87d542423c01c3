// Host construction of the FETI topology (see plan.hpp).
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

namespace feti {

int64_t Plan::sum_nb2() const {
    int64_t t = 0;
    for (int s = 0; s < n_sub; ++s) t += (int64_t)n_b[s] * n_b[s];
    return t;
}

int64_t Plan::sum_nb_nc() const {
    int64_t t = 0;
    for (int s = 0; s < n_sub; ++s) t += (int64_t)n_b[s] * n_c[s];
    return t;
}

namespace {

std::string fmt(const char* f, long long a = 0, long long b = 0) {
    char buf[256];
    snprintf(buf, sizeof buf, f, a, b);
    return buf;
}

}  // namespace

std::string build_plan(const feti_mesh* mesh, const feti_partition* part, const feti_opts* opts,
                       Plan& P) {
    if (!mesh || !part || !opts) return "null mesh, partition or options";
    if (mesh->dim != 2 && mesh->dim != 3) return "dim must be 2 or 3";
    const int dim = mesh->dim;
    P = Plan();
    P.dim = dim;
    P.dpn = dim;
    P.method = opts->method;
    if (P.method != FETI_TFETI && P.method != FETI_DP) return "unknown method";
    if (!(mesh->nu > -1.0 && mesh->nu < 0.5)) return "nu must lie in (-1, 0.5)";
    P.nu = mesh->nu;
    int64_t n_el = 1, n_nodes = 1;
    for (int a = 0; a < 3; ++a) {
        P.nel[a] = a < dim ? mesh->nel[a] : 0;
        P.nsub[a] = a < dim ? part->nsub[a] : 1;
        if (a < dim) {
            if (P.nel[a] < 1 || P.nel[a] > (1 << 20)) return fmt("nel[%lld] out of range", a);
            if (P.nsub[a] < 1 || P.nsub[a] > P.nel[a]) return fmt("nsub[%lld] out of range", a);
            n_el *= P.nel[a];
            n_nodes *= P.nel[a] + 1;
        }
    }
    if ((int64_t)dim * n_nodes >= (1ll << 31)) return "problem too large for 32-bit DOF numbers";
    P.n_el = (int)n_el;
    P.n_nodes = (int)n_nodes;
    P.n_dof = (int)(dim * n_nodes);
    P.n_sub = P.nsub[0] * P.nsub[1] * P.nsub[2];

    // cuts and per-axis lookup tables
    for (int a = 0; a < dim; ++a) {
        auto& c = P.cuts[a];
        c.resize(P.nsub[a] + 1);
        if (part->cuts[a]) {
            for (int k = 0; k <= P.nsub[a]; ++k) c[k] = part->cuts[a][k];
            if (c[0] != 0 || c[P.nsub[a]] != P.nel[a]) return fmt("cuts[%lld] must run from 0 to nel", a);
            for (int k = 0; k < P.nsub[a]; ++k)
                if (c[k + 1] <= c[k]) return fmt("cuts[%lld] must be strictly increasing", a);
        } else {
            if (P.nel[a] % P.nsub[a]) return fmt("nel[%lld] not divisible by nsub (give cuts)", a);
            for (int k = 0; k <= P.nsub[a]; ++k) c[k] = k * (P.nel[a] / P.nsub[a]);
        }
        P.ax_first[a].assign(P.nel[a] + 1, 0);
        P.ax_cnt[a].assign(P.nel[a] + 1, 1);
        for (int k = 0; k < P.nsub[a]; ++k)
            for (int i = c[k]; i <= c[k + 1]; ++i) {
                if (i == c[k] && k > 0) continue;  // already owned by k-1, count 2 below
                P.ax_first[a][i] = k;
            }
        for (int k = 1; k < P.nsub[a]; ++k) {
            P.ax_first[a][c[k]] = k - 1;
            P.ax_cnt[a][c[k]] = 2;
        }
    }
    for (int a = dim; a < 3; ++a) {
        P.cuts[a] = {0, 0};
        P.ax_first[a] = {0};
        P.ax_cnt[a] = {1};
    }
    int nng[3];
    for (int a = 0; a < 3; ++a) nng[a] = a < dim ? P.nel[a] + 1 : 1;

    // clamped DOFs
    std::vector<uint8_t> fixed(P.n_dof, 0);
    if (mesh->n_fixed < 0 || (mesh->n_fixed > 0 && !mesh->fixed_dofs)) return "bad fixed DOF list";
    for (int k = 0; k < mesh->n_fixed; ++k) {
        int g = mesh->fixed_dofs[k];
        if (g < 0 || g >= P.n_dof) return fmt("fixed DOF %lld out of range", g);
        fixed[g] = 1;
    }
    std::vector<std::vector<uint8_t>> is_cut(3);
    for (int a = 0; a < 3; ++a) {
        is_cut[a].assign(nng[a], a < dim ? 0 : 1);
        if (a < dim)
            for (int v : P.cuts[a]) is_cut[a][v] = 1;
    }

    auto node_coords = [&](int node, int* x) {
        x[0] = node % nng[0];
        x[1] = (node / nng[0]) % nng[1];
        x[2] = node / (nng[0] * nng[1]);
    };
    // subdomains containing a node, ascending
    auto node_subs = [&](const int* x, int* out) {
        int cnt = 0;
        for (int kz = 0; kz < P.ax_cnt[2][x[2]]; ++kz)
            for (int ky = 0; ky < P.ax_cnt[1][x[1]]; ++ky)
                for (int kx = 0; kx < P.ax_cnt[0][x[0]]; ++kx) {
                    int sx = P.ax_first[0][x[0]] + kx, sy = P.ax_first[1][x[1]] + ky,
                        sz = P.ax_first[2][x[2]] + kz;
                    out[cnt++] = sx + P.nsub[0] * (sy + P.nsub[1] * sz);
                }
        std::sort(out, out + cnt);
        return cnt;
    };
    auto is_corner_node = [&](int node) {
        if (P.method != FETI_DP) return false;
        int x[3];
        node_coords(node, x);
        int m = P.ax_cnt[0][x[0]] * P.ax_cnt[1][x[1]] * P.ax_cnt[2][x[2]];
        if (m < 2) return false;
        for (int a = 0; a < 3; ++a)
            if (!is_cut[a][x[a]]) return false;
        for (int c = 0; c < dim; ++c)
            if (!fixed[dim * node + c]) return true;
        return false;
    };

    // direction groups
    int gblk[3] = {1, 1, 1};
    bool one_per_sub = true;
    for (int a = 0; a < dim; ++a)
        if (part->group[a] > 1) one_per_sub = false;
    int nbk[3] = {P.nsub[0], P.nsub[1], P.nsub[2]};
    if (!one_per_sub) {
        for (int a = 0; a < dim; ++a) {
            gblk[a] = part->group[a] > 0 ? part->group[a] : 1;
            if (P.nsub[a] % gblk[a]) return fmt("group[%lld] must divide nsub", a);
            nbk[a] = P.nsub[a] / gblk[a];
        }
    }
    for (int a = 0; a < 3; ++a) P.group[a] = gblk[a];
    P.n_groups = nbk[0] * nbk[1] * nbk[2];

    // ---- subdomains ----
    const int n_sub = P.n_sub;
    P.lo.assign(3 * n_sub, 0);
    P.nn.assign(3 * n_sub, 1);
    P.n_loc.assign(n_sub, 0);
    P.n_i.assign(n_sub, 0);
    P.n_b.assign(n_sub, 0);
    P.n_c.assign(n_sub, 0);
    P.band.assign(n_sub, 0);
    P.grp.assign(n_sub, 0);
    P.off_loc.assign(n_sub + 1, 0);
    P.off_i.assign(n_sub + 1, 0);
    P.off_b.assign(n_sub + 1, 0);
    P.off_c.assign(n_sub + 1, 0);
    std::vector<uint8_t> corner_node(P.n_nodes, 0);
    for (int nd = 0; nd < P.n_nodes; ++nd) corner_node[nd] = is_corner_node(nd) ? 1 : 0;
    // further primal nodes (Sec. 6, item i: compatibility enforced in primal variables at nodes
    // other than the corners): each must be shared by two or more subdomains and carry a free DOF
    if (part->n_primal < 0 || (part->n_primal > 0 && !part->primal_nodes)) return "bad primal node list";
    if (part->n_primal > 0 && P.method != FETI_DP) return "primal nodes need FETI-DP";
    for (int k = 0; k < part->n_primal; ++k) {
        const int nd = part->primal_nodes[k];
        if (nd < 0 || nd >= P.n_nodes) return fmt("primal node %lld out of range", nd);
        int x[3];
        node_coords(nd, x);
        if (P.ax_cnt[0][x[0]] * P.ax_cnt[1][x[1]] * P.ax_cnt[2][x[2]] < 2)
            return fmt("primal node %lld is not shared by two subdomains", nd);
        bool free_dof = false;
        for (int c = 0; c < dim; ++c) free_dof = free_dof || !fixed[dim * nd + c];
        if (!free_dof) return fmt("primal node %lld has no free DOF", nd);
        corner_node[nd] = 1;
    }

    for (int s = 0; s < n_sub; ++s) {
        int k[3] = {s % P.nsub[0], (s / P.nsub[0]) % P.nsub[1], s / (P.nsub[0] * P.nsub[1])};
        int n = dim;
        for (int a = 0; a < 3; ++a) {
            P.lo[3 * s + a] = a < dim ? P.cuts[a][k[a]] : 0;
            P.nn[3 * s + a] = a < dim ? P.cuts[a][k[a] + 1] - P.cuts[a][k[a]] + 1 : 1;
            n *= P.nn[3 * s + a];
        }
        P.n_loc[s] = n;
        P.grp[s] = (k[0] / gblk[0]) + nbk[0] * ((k[1] / gblk[1]) + nbk[1] * (k[2] / gblk[2]));
        P.off_loc[s + 1] = P.off_loc[s] + n;
    }
    const int64_t n_loc_tot = P.off_loc[n_sub];
    P.lcls.assign(n_loc_tot, CLS_I);
    P.lidx.assign(n_loc_tot, 0);
    P.lglob.assign(n_loc_tot, 0);
    P.lown.assign(n_loc_tot, 0);
    for (int s = 0; s < n_sub; ++s) {
        const int* lo = &P.lo[3 * s];
        const int* nn = &P.nn[3 * s];
        int cnt[4] = {0, 0, 0, 0};
        int64_t base = P.off_loc[s];
        int l = 0;
        for (int z = 0; z < nn[2]; ++z)
            for (int y = 0; y < nn[1]; ++y)
                for (int x = 0; x < nn[0]; ++x) {
                    int gx[3] = {lo[0] + x, lo[1] + y, lo[2] + z};
                    int node = gx[0] + nng[0] * (gx[1] + nng[1] * gx[2]);
                    int m = P.ax_cnt[0][gx[0]] * P.ax_cnt[1][gx[1]] * P.ax_cnt[2][gx[2]];
                    int subs[8];
                    node_subs(gx, subs);
                    for (int c = 0; c < dim; ++c, ++l) {
                        int g = dim * node + c;
                        int8_t cls;
                        if (fixed[g])
                            cls = P.method == FETI_TFETI ? CLS_B : CLS_X;
                        else if (m >= 2)
                            cls = corner_node[node] ? CLS_C : CLS_B;
                        else
                            cls = CLS_I;
                        P.lcls[base + l] = cls;
                        P.lidx[base + l] = cnt[cls]++;
                        P.lglob[base + l] = g;
                        P.lown[base + l] = subs[0] == s ? 1 : 0;
                    }
                }
        P.n_i[s] = cnt[CLS_I];
        P.n_b[s] = cnt[CLS_B];
        P.n_c[s] = cnt[CLS_C];
        P.off_i[s + 1] = P.off_i[s] + cnt[CLS_I];
        P.off_b[s + 1] = P.off_b[s] + cnt[CLS_B];
        P.off_c[s + 1] = P.off_c[s] + cnt[CLS_C];
        // half-bandwidth of K_ii in the compressed interior numbering
        int w = 0;
        for (int z = 0; z < nn[2]; ++z)
            for (int y = 0; y < nn[1]; ++y)
                for (int x = 0; x < nn[0]; ++x) {
                    int la = x + nn[0] * (y + nn[1] * z);
                    for (int dz = -1; dz <= 1; ++dz)
                        for (int dy = -1; dy <= 1; ++dy)
                            for (int dx = -1; dx <= 1; ++dx) {
                                int xb = x + dx, yb = y + dy, zb = z + dz;
                                if (xb < 0 || yb < 0 || zb < 0 || xb >= nn[0] || yb >= nn[1] || zb >= nn[2])
                                    continue;
                                int lb = xb + nn[0] * (yb + nn[1] * zb);
                                for (int ca = 0; ca < dim; ++ca)
                                    for (int cb = 0; cb < dim; ++cb) {
                                        int64_t pa = base + dim * la + ca, pb = base + dim * lb + cb;
                                        if (P.lcls[pa] == CLS_I && P.lcls[pb] == CLS_I)
                                            w = std::max(w, std::abs(P.lidx[pa] - P.lidx[pb]));
                                    }
                            }
                }
        P.band[s] = w;
    }
    P.i_loc.resize(P.off_i[n_sub]);
    P.b_loc.resize(P.off_b[n_sub]);
    P.c_loc.resize(P.off_c[n_sub]);
    for (int s = 0; s < n_sub; ++s)
        for (int l = 0; l < P.n_loc[s]; ++l) {
            int64_t q = P.off_loc[s] + l;
            switch (P.lcls[q]) {
                case CLS_I: P.i_loc[P.off_i[s] + P.lidx[q]] = l; break;
                case CLS_B: P.b_loc[P.off_b[s] + P.lidx[q]] = l; break;
                case CLS_C: P.c_loc[P.off_c[s] + P.lidx[q]] = l; break;
                default: break;
            }
        }

    // local DOF of a global DOF inside subdomain s (node must belong to s)
    auto local_dof = [&](int s, const int* gx, int c) {
        const int* lo = &P.lo[3 * s];
        const int* nn = &P.nn[3 * s];
        int ln = (gx[0] - lo[0]) + nn[0] * ((gx[1] - lo[1]) + nn[1] * (gx[2] - lo[2]));
        return dim * ln + c;
    };

    // ---- corners ----
    std::vector<int> cg_of_dof;
    if (P.method == FETI_DP) {
        cg_of_dof.assign(P.n_dof, -1);
        for (int nd = 0; nd < P.n_nodes; ++nd)
            if (corner_node[nd])
                for (int c = 0; c < dim; ++c)
                    if (!fixed[dim * nd + c]) {
                        cg_of_dof[dim * nd + c] = (int)P.corner_dofs.size();
                        P.corner_dofs.push_back(dim * nd + c);
                    }
        P.n_cg = (int)P.corner_dofs.size();
        P.c_glob.resize(P.off_c[n_sub]);
        std::vector<int> cnt(P.n_cg + 1, 0);
        for (int s = 0; s < n_sub; ++s)
            for (int j = 0; j < P.n_c[s]; ++j) {
                int l = P.c_loc[P.off_c[s] + j];
                int cg = cg_of_dof[P.lglob[P.off_loc[s] + l]];
                P.c_glob[P.off_c[s] + j] = cg;
                cnt[cg + 1]++;
            }
        P.cc_ptr.assign(P.n_cg + 1, 0);
        for (int k = 0; k < P.n_cg; ++k) P.cc_ptr[k + 1] = P.cc_ptr[k] + cnt[k + 1];
        P.cc_s.resize(P.cc_ptr[P.n_cg]);
        P.cc_j.resize(P.cc_ptr[P.n_cg]);
        std::vector<int> fill(P.cc_ptr.begin(), P.cc_ptr.end() - 1);
        for (int s = 0; s < n_sub; ++s)
            for (int j = 0; j < P.n_c[s]; ++j) {
                int cg = P.c_glob[P.off_c[s] + j];
                P.cc_s[fill[cg]] = s;
                P.cc_j[fill[cg]] = j;
                fill[cg]++;
            }
    }

    // ---- lambda rows ----
    P.sh_ptr.push_back(0);
    for (int nd = 0; nd < P.n_nodes; ++nd) {
        int x[3];
        node_coords(nd, x);
        int m = P.ax_cnt[0][x[0]] * P.ax_cnt[1][x[1]] * P.ax_cnt[2][x[2]];
        bool any_fixed = false;
        for (int c = 0; c < dim; ++c) any_fixed |= fixed[dim * nd + c] != 0;
        if (m < 2 && !(any_fixed && P.method == FETI_TFETI)) continue;
        if (corner_node[nd]) continue;
        int subs[8];
        int ns = node_subs(x, subs);
        for (int c = 0; c < dim; ++c) {
            int g = dim * nd + c;
            if (fixed[g]) {
                if (P.method != FETI_TFETI) continue;
                for (int t = 0; t < ns; ++t) {
                    int s = subs[t];
                    int l = local_dof(s, x, c);
                    P.row_s.push_back(s);
                    P.row_j.push_back(P.lidx[P.off_loc[s] + l]);
                    P.row_sg.push_back(1);
                    P.row_s.push_back(-1);
                    P.row_j.push_back(-1);
                    P.row_sg.push_back(0);
                    P.row_sh.push_back(-1);
                }
                continue;
            }
            if (ns < 2) continue;
            int sh = (int)P.sh_ptr.size() - 1;
            int lv[8];
            for (int t = 0; t < ns; ++t) {
                lv[t] = local_dof(subs[t], x, c);
                P.sh_s.push_back(subs[t]);
                P.sh_l.push_back(lv[t]);
            }
            P.sh_ptr.push_back((int)P.sh_s.size());
            for (int a = 0; a < ns; ++a)
                for (int b = a + 1; b < ns; ++b) {
                    P.row_s.push_back(subs[a]);
                    P.row_j.push_back(P.lidx[P.off_loc[subs[a]] + lv[a]]);
                    P.row_sg.push_back(1);
                    P.row_s.push_back(subs[b]);
                    P.row_j.push_back(P.lidx[P.off_loc[subs[b]] + lv[b]]);
                    P.row_sg.push_back(-1);
                    P.row_sh.push_back(sh);
                }
        }
    }
    P.n_lambda = (int)P.row_sh.size();

    // gather lists: b DOF -> rows
    const int64_t nb_tot = P.off_b[n_sub];
    std::vector<int> cnt(nb_tot + 1, 0);
    for (int r = 0; r < P.n_lambda; ++r)
        for (int t = 0; t < 2; ++t)
            if (P.row_s[2 * r + t] >= 0) cnt[P.off_b[P.row_s[2 * r + t]] + P.row_j[2 * r + t] + 1]++;
    P.bg_ptr.assign(nb_tot + 1, 0);
    for (int64_t q = 0; q < nb_tot; ++q) {
        if (cnt[q + 1] == 0) return "internal: interface DOF without a constraint row";
        P.bg_ptr[q + 1] = P.bg_ptr[q] + cnt[q + 1];
    }
    P.bg_row.resize(P.bg_ptr[nb_tot]);
    P.bg_sg.resize(P.bg_ptr[nb_tot]);
    {
        std::vector<int> fill(P.bg_ptr.begin(), P.bg_ptr.end() - 1);
        for (int r = 0; r < P.n_lambda; ++r)
            for (int t = 0; t < 2; ++t) {
                int s = P.row_s[2 * r + t];
                if (s < 0) continue;
                int64_t q = P.off_b[s] + P.row_j[2 * r + t];
                P.bg_row[fill[q]] = r;
                P.bg_sg[fill[q]] = P.row_sg[2 * r + t];
                fill[q]++;
            }
    }
    if (P.method == FETI_TFETI) {
        P.n_rbm = dim == 2 ? 3 : 6;
        P.n_alpha = P.n_rbm * n_sub;
        for (int s = 0; s < n_sub; ++s)
            if (P.n_b[s] == 0) return "TFETI needs every subdomain to touch a constraint";
    }
    return "";
}

std::string adaptive_primal(const feti_mesh* mesh, const feti_partition* part, const double* rho, double p,
                            double E0, double Emin, double theta, int cap, std::vector<int>& out) {
    out.clear();
    if (!mesh || !part || !rho) return "null mesh, partition or densities";
    if (mesh->dim == 3) return "";
    if (mesh->dim != 2) return "dim must be 2 or 3";
    const int nx = mesh->nel[0], ny = mesh->nel[1];
    if (nx < 1 || ny < 1) return "bad grid";
    std::vector<int> cuts[2];
    for (int a = 0; a < 2; ++a) {
        const int ns = part->nsub[a], ne = mesh->nel[a];
        if (ns < 1 || ns > ne) return fmt("nsub[%lld] out of range", a);
        cuts[a].resize(ns + 1);
        for (int k = 0; k <= ns; ++k) cuts[a][k] = part->cuts[a] ? part->cuts[a][k] : k * (ne / ns);
        if (cuts[a][0] != 0 || cuts[a][ns] != ne) return fmt("cuts[%lld] must run from 0 to nel", a);
    }
    const int nnx = nx + 1;
    const long long n_dof = 2LL * nnx * (ny + 1);
    std::vector<uint8_t> fixed(n_dof, 0);
    for (int k = 0; k < mesh->n_fixed; ++k)
        if (mesh->fixed_dofs[k] >= 0 && mesh->fixed_dofs[k] < n_dof) fixed[mesh->fixed_dofs[k]] = 1;
    auto modulus = [&](int e) { return Emin + std::pow(rho[e], p) * (E0 - Emin); };
    auto stiffness = [&](int x, int y) {   // elements containing the node, lexicographic order
        double k = 0.0;
        for (int ey = y - 1; ey <= y; ++ey)
            for (int ex = x - 1; ex <= x; ++ex)
                if (ex >= 0 && ex < nx && ey >= 0 && ey < ny) k += modulus(ex + nx * ey);
        return k;
    };
    std::vector<std::vector<std::pair<int, int>>> edges;
    for (size_t i = 1; i + 1 < cuts[0].size(); ++i)
        for (size_t j = 0; j + 1 < cuts[1].size(); ++j) {
            std::vector<std::pair<int, int>> e;
            for (int y = cuts[1][j] + 1; y < cuts[1][j + 1]; ++y) e.push_back({cuts[0][i], y});
            edges.push_back(e);
        }
    for (size_t j = 1; j + 1 < cuts[1].size(); ++j)
        for (size_t i = 0; i + 1 < cuts[0].size(); ++i) {
            std::vector<std::pair<int, int>> e;
            for (int x = cuts[0][i] + 1; x < cuts[0][i + 1]; ++x) e.push_back({x, cuts[1][j]});
            edges.push_back(e);
        }
    std::vector<int> nodes;
    for (const auto& e : edges) {
        if (e.empty()) continue;
        std::vector<double> k(e.size());
        double kmax = 0.0;
        for (size_t t = 0; t < e.size(); ++t) {
            k[t] = stiffness(e[t].first, e[t].second);
            kmax = std::max(kmax, k[t]);
        }
        if (!(kmax > 0.0)) continue;
        struct Run {
            int a, b;
            double w;
        };
        std::vector<Run> runs;
        int a = -1;
        for (size_t t = 0; t <= e.size(); ++t) {
            const bool stiff = t < e.size() && k[t] >= theta * kmax;
            if (stiff && a < 0) {
                a = (int)t;
            } else if (!stiff && a >= 0) {
                double w = 0.0;
                for (int q = a; q < (int)t; ++q) w += k[q];
                runs.push_back({a, (int)t - 1, w});
                a = -1;
            }
        }
        std::stable_sort(runs.begin(), runs.end(), [](const Run& u, const Run& v) {
            return u.w > v.w || (u.w == v.w && u.a < v.a);
        });
        for (int r = 0; r < (int)runs.size() && r < cap; ++r) {
            const auto& xy = e[(runs[r].a + runs[r].b) / 2];
            const int nd = xy.first + nnx * xy.second;
            if (!(fixed[2LL * nd] && fixed[2LL * nd + 1])) nodes.push_back(nd);
        }
    }
    std::sort(nodes.begin(), nodes.end());
    nodes.erase(std::unique(nodes.begin(), nodes.end()), nodes.end());
    out = nodes;
    return "";
}

std::string build_plan_batched(int nd, const feti_mesh* meshes, const feti_partition* parts, const feti_opts* opts,
                               Plan& U, std::vector<DesignMeta>& D, bool segmented) {
    if (nd < 1 || !meshes || !parts) return "need at least one design";
    U = Plan();
    D.assign(nd, DesignMeta{});
    U.off_loc.assign(1, 0);
    U.off_i.assign(1, 0);
    U.off_b.assign(1, 0);
    U.off_c.assign(1, 0);
    U.sh_ptr.assign(1, 0);
    U.bg_ptr.assign(1, 0);
    U.cc_ptr.assign(1, 0);
    int n_sh = 0;
    for (int d = 0; d < nd; ++d) {
        Plan P;
        std::string err = build_plan(&meshes[d], &parts[d], opts, P);
        if (!err.empty()) return "design " + std::to_string(d) + ": " + err;
        if (d == 0) {
            U.dim = P.dim;
            U.dpn = P.dpn;
            U.method = P.method;
            U.nu = P.nu;
            U.n_rbm = P.n_rbm;
        } else if (P.dim != U.dim) {
            return "all designs must have the same dimension";
        } else if (P.nu != U.nu) {
            return "all designs must have the same Poisson ratio";
        }
        DesignMeta& M = D[d];
        M.sub0 = U.n_sub;
        M.n_sub = P.n_sub;
        M.el0 = U.n_el;
        M.n_el = P.n_el;
        M.node0 = U.n_nodes;
        M.n_nodes = P.n_nodes;
        M.dof0 = U.n_dof;
        M.n_dof = P.n_dof;
        M.lam0 = U.n_lambda;
        M.n_lambda = P.n_lambda;
        M.cg0 = U.n_cg;
        M.n_cg = P.n_cg;
        M.grp0 = segmented ? 0 : U.n_groups;
        M.n_groups = P.n_groups;
        for (int a = 0; a < 3; ++a) {
            M.nel[a] = P.nel[a];
            M.nsub[a] = P.nsub[a];
            M.ax_first[a] = P.ax_first[a];
            M.ax_cnt[a] = P.ax_cnt[a];
        }
        const int64_t loc0 = U.off_loc.back(), i0 = U.off_i.back(), b0 = U.off_b.back(), c0 = U.off_c.back();
        for (int s = 0; s < P.n_sub; ++s) {
            for (int a = 0; a < 3; ++a) {
                U.lo.push_back(P.lo[3 * s + a]);
                U.nn.push_back(P.nn[3 * s + a]);
            }
            U.n_loc.push_back(P.n_loc[s]);
            U.n_i.push_back(P.n_i[s]);
            U.n_b.push_back(P.n_b[s]);
            U.n_c.push_back(P.n_c[s]);
            U.band.push_back(P.band[s]);
            U.grp.push_back(P.grp[s] + M.grp0);
            U.off_loc.push_back(loc0 + P.off_loc[s + 1]);
            U.off_i.push_back(i0 + P.off_i[s + 1]);
            U.off_b.push_back(b0 + P.off_b[s + 1]);
            U.off_c.push_back(c0 + P.off_c[s + 1]);
        }
        U.lcls.insert(U.lcls.end(), P.lcls.begin(), P.lcls.end());
        U.lidx.insert(U.lidx.end(), P.lidx.begin(), P.lidx.end());
        U.lown.insert(U.lown.end(), P.lown.begin(), P.lown.end());
        for (int g : P.lglob) U.lglob.push_back(g + (int)M.dof0);
        U.i_loc.insert(U.i_loc.end(), P.i_loc.begin(), P.i_loc.end());
        U.b_loc.insert(U.b_loc.end(), P.b_loc.begin(), P.b_loc.end());
        U.c_loc.insert(U.c_loc.end(), P.c_loc.begin(), P.c_loc.end());
        for (int g : P.c_glob) U.c_glob.push_back(g + M.cg0);
        for (int r = 0; r < P.n_lambda; ++r) {
            for (int t = 0; t < 2; ++t) {
                const int s = P.row_s[2 * r + t];
                U.row_s.push_back(s >= 0 ? s + M.sub0 : -1);
                U.row_j.push_back(P.row_j[2 * r + t]);
                U.row_sg.push_back(P.row_sg[2 * r + t]);
            }
            U.row_sh.push_back(P.row_sh[r] >= 0 ? P.row_sh[r] + n_sh : -1);
        }
        const int sh_base = U.sh_ptr.back();
        for (size_t q = 1; q < P.sh_ptr.size(); ++q) U.sh_ptr.push_back(sh_base + P.sh_ptr[q]);
        for (int s : P.sh_s) U.sh_s.push_back(s + M.sub0);
        U.sh_l.insert(U.sh_l.end(), P.sh_l.begin(), P.sh_l.end());
        n_sh += (int)P.sh_ptr.size() - 1;
        const int bg_base = U.bg_ptr.back();
        for (size_t q = 1; q < P.bg_ptr.size(); ++q) U.bg_ptr.push_back(bg_base + P.bg_ptr[q]);
        for (int r : P.bg_row) U.bg_row.push_back(r + M.lam0);
        U.bg_sg.insert(U.bg_sg.end(), P.bg_sg.begin(), P.bg_sg.end());
        for (int g : P.corner_dofs) U.corner_dofs.push_back(g + (int)M.dof0);
        const int cc_base = U.cc_ptr.back();
        for (size_t q = 1; q < P.cc_ptr.size(); ++q) U.cc_ptr.push_back(cc_base + P.cc_ptr[q]);
        for (int s : P.cc_s) U.cc_s.push_back(s + M.sub0);
        U.cc_j.insert(U.cc_j.end(), P.cc_j.begin(), P.cc_j.end());
        U.n_sub += P.n_sub;
        U.n_el += P.n_el;
        U.n_nodes += P.n_nodes;
        U.n_dof += P.n_dof;
        U.n_lambda += P.n_lambda;
        M.n_rows = P.n_lambda;
        if (segmented) {   // empty rows up to a multiple of 256
            const int pad = (256 - P.n_lambda % 256) % 256;
            for (int q = 0; q < pad; ++q) {
                for (int t = 0; t < 2; ++t) {
                    U.row_s.push_back(-1);
                    U.row_j.push_back(0);
                    U.row_sg.push_back(0);
                }
                U.row_sh.push_back(-1);
            }
            U.n_lambda += pad;
            M.n_rows += pad;
        }
        U.n_cg += P.n_cg;
        U.n_groups = segmented ? std::max(U.n_groups, P.n_groups) : U.n_groups + P.n_groups;
        U.n_alpha += P.n_alpha;
    }
    if (nd == 1) {
        for (int a = 0; a < 3; ++a) {
            U.nel[a] = D[0].nel[a];
            U.nsub[a] = D[0].nsub[a];
            U.ax_first[a] = D[0].ax_first[a];
            U.ax_cnt[a] = D[0].ax_cnt[a];
        }
    } else {
        for (int a = 0; a < 3; ++a) U.nel[a] = U.nsub[a] = 0;
    }
    return "";
}

}  // namespace feti
