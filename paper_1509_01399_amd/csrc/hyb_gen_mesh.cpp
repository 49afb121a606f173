// Host analysis of a general tetrahedral mesh of the FEM box: conformity with
// the grid on the overlap (Sec. 3), P1 element matrices and lumped masses
// from the vertex coordinates (Sec. 7.2), the device node numbering and the
// sliced ELL tables of hyb_gen.h.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <unordered_map>

#include "hyb_gen.h"

namespace hyb {

namespace {

// Gradients of the barycentric coordinates of a tetrahedron and its volume.
double grads_p1(const double X[4][3], double Gr[4][3])
{
    double E[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) E[r][c] = X[c + 1][r] - X[0][r];
    const double det = E[0][0] * (E[1][1] * E[2][2] - E[1][2] * E[2][1]) -
                       E[0][1] * (E[1][0] * E[2][2] - E[1][2] * E[2][0]) +
                       E[0][2] * (E[1][0] * E[2][1] - E[1][1] * E[2][0]);
    if (det == 0.0) return 0.0;
    // rows of the inverse of E: the gradients of the barycentric coordinates 1..3
    double I[3][3];
    I[0][0] = (E[1][1] * E[2][2] - E[1][2] * E[2][1]) / det;
    I[0][1] = (E[0][2] * E[2][1] - E[0][1] * E[2][2]) / det;
    I[0][2] = (E[0][1] * E[1][2] - E[0][2] * E[1][1]) / det;
    I[1][0] = (E[1][2] * E[2][0] - E[1][0] * E[2][2]) / det;
    I[1][1] = (E[0][0] * E[2][2] - E[0][2] * E[2][0]) / det;
    I[1][2] = (E[0][2] * E[1][0] - E[0][0] * E[1][2]) / det;
    I[2][0] = (E[1][0] * E[2][1] - E[1][1] * E[2][0]) / det;
    I[2][1] = (E[0][1] * E[2][0] - E[0][0] * E[2][1]) / det;
    I[2][2] = (E[0][0] * E[1][1] - E[0][1] * E[1][0]) / det;
    for (int c = 0; c < 3; ++c) {
        Gr[0][c] = -(I[0][c] + I[1][c] + I[2][c]);
        for (int r = 0; r < 3; ++r) Gr[r + 1][c] = I[r][c];
    }
    return std::fabs(det) / 6.0;
}

constexpr int SL = 64;  // slice height: one wavefront

}  // namespace

hyb_status analyse_general(const hyb_fd_grid *gr, const hyb_fem_mesh *m, const int o[3], const int C[3],
                           GenHost &out, std::string &err)
{
    const double h = gr->h, tol = 1e-7;  // tolerance in cells
    const long long nn = m->n_nodes, nt = m->n_tets;
    const long long nx = gr->n_cells[0] + 1, ny = gr->n_cells[1] + 1;
    if (nn > INT32_MAX / 2 || nt > INT32_MAX / 8) {
        err = "fem mesh: too many nodes or tetrahedra";
        return HYB_E_UNSUPPORTED;
    }
    for (int d = 0; d < 3; ++d) { out.o[d] = o[d]; out.C[d] = C[d]; }
    // ---- node classes
    std::vector<int8_t> cls(nn);
    std::vector<uint8_t> plane(nn, 0);  // box-surface planes through the node (bit 2d: o, 2d+1: o+C)
    std::vector<int32_t> q3(3 * nn), cell3(3 * nn);
    std::vector<int64_t> lin(nn, -1);
    std::unordered_map<int64_t, int64_t> at;
    at.reserve((size_t)nn);
    long long n_surf = 0;
    bool all_grid = true;
    for (long long i = 0; i < nn; ++i) {
        bool grid = true, surf = false, inner = true, on_inner_surf = false;
        long long qi[3];
        for (int d = 0; d < 3; ++d) {
            const double q = (m->xyz[3 * i + d] - gr->origin[d]) / h;
            qi[d] = std::llround(q);
            if (std::fabs(q - (double)qi[d]) > tol) grid = false;
            if (std::fabs(q - o[d]) <= tol) plane[i] |= (uint8_t)(1u << (2 * d));
            if (std::fabs(q - (o[d] + C[d])) <= tol) plane[i] |= (uint8_t)(1u << (2 * d + 1));
            if (plane[i]) surf = true;
            if (q < o[d] + 2 - tol || q > o[d] + C[d] - 2 + tol) inner = false;
            if (std::fabs(q - (o[d] + 2)) <= tol || std::fabs(q - (o[d] + C[d] - 2)) <= tol) on_inner_surf = true;
            cell3[3 * i + d] = (int32_t)std::floor(q + tol);
        }
        if (surf && !grid) {
            err = "fem mesh: node on the box surface off the grid";
            return HYB_E_MESH;
        }
        all_grid = all_grid && grid;
        if (grid) {
            for (int d = 0; d < 3; ++d) q3[3 * i + d] = (int32_t)qi[d];
            lin[i] = qi[0] + nx * (qi[1] + ny * qi[2]);
            if (!at.emplace(lin[i], i).second) {
                err = "fem mesh: two nodes at one grid point";
                return HYB_E_MESH;
            }
        }
        cls[i] = surf ? 3 : (inner ? ((grid && on_inner_surf) ? 0 : 1) : 2);
        n_surf += surf;
    }
    const long long Lo = C[0] + 1, Li = C[0] - 1;
    if (n_surf != Lo * Lo * Lo - Li * Li * Li) {
        err = "fem mesh: the box surface must carry exactly its grid nodes";
        return HYB_E_MESH;
    }
    // every grid node of the inner box surface must be a mesh node
    const int L = C[0] - 4;
    for (int c = 0; c <= L; ++c)
        for (int b = 0; b <= L; ++b)
            for (int a = 0; a <= L; ++a) {
                if (!(a == 0 || a == L || b == 0 || b == L || c == 0 || c == L)) continue;
                const int64_t g = (o[0] + 2 + a) + nx * ((o[1] + 2 + b) + ny * (long long)(o[2] + 2 + c));
                if (!at.count(g)) {
                    err = "fem mesh: a grid node of the inner box surface is not a mesh node";
                    return HYB_E_MESH;
                }
            }
    // ---- device numbering: class, then the cell's z, y, x, then the node id
    std::vector<int32_t> ord(nn);
    std::iota(ord.begin(), ord.end(), 0);
    std::sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
        if (cls[a] != cls[b]) return cls[a] < cls[b];
        for (int d = 2; d >= 0; --d)
            if (cell3[3 * a + d] != cell3[3 * b + d]) return cell3[3 * a + d] < cell3[3 * b + d];
        return a < b;
    });
    std::vector<int32_t> dev(nn);
    for (long long n = 0; n < nn; ++n) dev[ord[n]] = (int32_t)n;
    long long cnt[4] = {0, 0, 0, 0};
    for (long long i = 0; i < nn; ++i) cnt[cls[i]]++;
    out.fn = nn;
    out.nA = cnt[0];
    out.nH = cnt[0] + cnt[1];
    out.nR = out.nH + cnt[2];
    out.ntet = nt;
    out.all_grid = all_grid;
    out.orig_of_dev.assign(ord.begin(), ord.end());
    out.grid_lin.resize(nn);
    out.gq.resize(3 * nn);
    for (long long n = 0; n < nn; ++n) {
        const int32_t i = ord[n];
        out.grid_lin[n] = lin[i];
        for (int d = 0; d < 3; ++d) out.gq[3 * n + d] = lin[i] >= 0 ? q3[3 * i + d] : -1;
    }
    // ---- elements: matrices, masses, free tetrahedra; vertex pairs (a < b)
    std::vector<double> mass(nn, 0.0);
    std::vector<double> ke(16 * (size_t)nt);
    out.pvol.assign(nt, 0.0);
    const double vmin = 1e-12 * h * h * h;
    std::vector<int64_t> pcount(nn + 1, 0);  // pairs per smaller vertex
    for (long long t = 0; t < nt; ++t) {
        double X[4][3], Gr[4][3];
        int32_t v[4];
        bool freet = true;
        for (int q = 0; q < 4; ++q) {
            const int32_t id = m->tet4[4 * t + q];
            if (id < 0 || id >= nn) {
                err = "fem mesh: node id out of range";
                return HYB_E_ARG;
            }
            v[q] = dev[id];
            for (int d = 0; d < 3; ++d) X[q][d] = m->xyz[3 * id + d];
            freet = freet && v[q] < out.nH;
        }
        for (int q = 0; q < 4; ++q)
            for (int r = q + 1; r < 4; ++r)
                if (v[q] == v[r]) {
                    err = "fem mesh: tetrahedron with a repeated vertex";
                    return HYB_E_MESH;
                }
        const double vol = grads_p1(X, Gr);
        if (!(vol > vmin)) {
            err = "fem mesh: degenerate tetrahedron";
            return HYB_E_MESH;
        }
        for (int q = 0; q < 4; ++q) {
            mass[v[q]] += vol / 4.0;
            for (int r = 0; r < 4; ++r)
                ke[16 * t + 4 * q + r] = vol * (Gr[q][0] * Gr[r][0] + Gr[q][1] * Gr[r][1] + Gr[q][2] * Gr[r][2]);
        }
        if (freet) out.pvol[t] = vol;
        for (int q = 0; q < 4; ++q)
            for (int r = q + 1; r < 4; ++r) pcount[std::min(v[q], v[r]) + 1]++;
    }
    for (long long n = 0; n < nn; ++n)
        if (!(mass[n] > 0)) {
            err = "fem mesh: node in no tetrahedron";
            return HYB_E_MESH;
        }
    // conformity: every face is shared by at most two tetrahedra, a face of
    // only one lies on the box surface, and the tetrahedra fill the box
    {
        double vsum = 0.0;
        for (long long t = 0; t < nt; ++t) {
            double X[4][3], Gr[4][3];
            for (int q = 0; q < 4; ++q)
                for (int d = 0; d < 3; ++d) X[q][d] = m->xyz[3 * m->tet4[4 * t + q] + d];
            vsum += grads_p1(X, Gr);
        }
        const double vbox = (double)C[0] * C[1] * C[2] * h * h * h;
        if (std::fabs(vsum - vbox) > 1e-9 * vbox) {
            err = "fem mesh: the tetrahedra do not fill the box";
            return HYB_E_MESH;
        }
        std::vector<int64_t> fptr(nn + 1, 0);
        for (long long t = 0; t < nt; ++t) {
            int32_t v[4];
            for (int q = 0; q < 4; ++q) v[q] = m->tet4[4 * t + q];
            std::sort(v, v + 4);
            fptr[v[0] + 1] += 3;  // faces {0,1,2} {0,1,3} {0,2,3} start at v0
            fptr[v[1] + 1] += 1;  // face {1,2,3}
        }
        for (long long n = 0; n < nn; ++n) fptr[n + 1] += fptr[n];
        std::vector<std::pair<int32_t, int32_t>> fbc(fptr[nn]);
        std::vector<int64_t> fill(fptr.begin(), fptr.end() - 1);
        for (long long t = 0; t < nt; ++t) {
            int32_t v[4];
            for (int q = 0; q < 4; ++q) v[q] = m->tet4[4 * t + q];
            std::sort(v, v + 4);
            fbc[fill[v[0]]++] = {v[1], v[2]};
            fbc[fill[v[0]]++] = {v[1], v[3]};
            fbc[fill[v[0]]++] = {v[2], v[3]};
            fbc[fill[v[1]]++] = {v[2], v[3]};
        }
        for (long long a = 0; a < nn; ++a) {
            std::sort(fbc.begin() + fptr[a], fbc.begin() + fptr[a + 1]);
            for (int64_t p = fptr[a]; p < fptr[a + 1];) {
                int64_t r = p + 1;
                while (r < fptr[a + 1] && fbc[r] == fbc[p]) ++r;
                const int64_t k = r - p;
                const bool on_box = (plane[a] & plane[fbc[p].first] & plane[fbc[p].second]) != 0;
                if (k > 2 || (k == 1 && !on_box) || (k == 2 && on_box)) {
                    err = "fem mesh: not conforming (a face shared by more than two tetrahedra, an inner "
                          "face of only one, or a surface face of two)";
                    return HYB_E_MESH;
                }
                p = r;
            }
        }
    }
    // pairs bucketed by the smaller vertex, then sorted by the larger one:
    // the edges (a, b), a < b, in increasing (a, b) order, with the list of
    // (tetrahedron, K^t_ab) that share each edge
    for (long long n = 0; n < nn; ++n) pcount[n + 1] += pcount[n];
    const long long npair = pcount[nn];
    std::vector<int32_t> pb(npair), pt(npair);
    std::vector<int8_t> pl(npair);  // local pair index 0..5 in its tetrahedron
    {
        std::vector<int64_t> fill(pcount.begin(), pcount.end() - 1);
        for (long long t = 0; t < nt; ++t) {
            int32_t v[4];
            for (int q = 0; q < 4; ++q) v[q] = dev[m->tet4[4 * t + q]];
            int lp = 0;
            for (int q = 0; q < 4; ++q)
                for (int r = q + 1; r < 4; ++r, ++lp) {
                    const int32_t a = std::min(v[q], v[r]), b = std::max(v[q], v[r]);
                    const int64_t p = fill[a]++;
                    pb[p] = b;
                    pt[p] = (int32_t)t;
                    pl[p] = (int8_t)lp;
                }
        }
    }
    static const int PQ[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
    std::vector<int32_t> up_ptr(nn + 1, 0), up_col;   // upper neighbours (b > a) of each a
    std::vector<int32_t> pair_edge(npair);
    out.cptr.assign(1, 0);
    out.ctet.clear();
    out.cw.clear();
    out.ctet.reserve(npair);
    out.cw.reserve(npair);
    {
        std::vector<int64_t> idx;
        for (long long a = 0; a < nn; ++a) {
            const int64_t p0 = pcount[a], p1 = pcount[a + 1];
            idx.resize(p1 - p0);
            std::iota(idx.begin(), idx.end(), p0);
            std::sort(idx.begin(), idx.end(), [&](int64_t x, int64_t y) {
                return pb[x] != pb[y] ? pb[x] < pb[y] : pt[x] < pt[y];
            });
            for (size_t u = 0; u < idx.size(); ++u) {
                const int64_t p = idx[u];
                if (u == 0 || pb[p] != pb[idx[u - 1]]) {
                    if (u > 0) out.cptr.push_back((int32_t)out.ctet.size());
                    up_col.push_back(pb[p]);
                }
                pair_edge[p] = (int32_t)up_col.size() - 1;
                const long long t = pt[p];
                const int q = PQ[pl[p]][0], r = PQ[pl[p]][1];
                out.ctet.push_back((int32_t)t);
                out.cw.push_back(ke[16 * t + 4 * q + r]);
            }
            if (!idx.empty()) out.cptr.push_back((int32_t)out.ctet.size());
            up_ptr[a + 1] = (int32_t)up_col.size();
        }
    }
    out.nedge = (long long)up_col.size();
    // lower neighbours (a < n) of each n, with their edge ids, in increasing a
    std::vector<int32_t> lo_ptr(nn + 1, 0);
    for (long long e = 0; e < out.nedge; ++e) lo_ptr[up_col[e] + 1]++;
    for (long long n = 0; n < nn; ++n) lo_ptr[n + 1] += lo_ptr[n];
    std::vector<int32_t> lo_col(out.nedge), lo_eid(out.nedge);
    {
        std::vector<int32_t> fill(lo_ptr.begin(), lo_ptr.end() - 1);
        for (long long a = 0; a < nn; ++a)
            for (int32_t e = up_ptr[a]; e < up_ptr[a + 1]; ++e) {
                const int32_t p = fill[up_col[e]]++;
                lo_col[p] = (int32_t)a;
                lo_eid[p] = e;
            }
    }
    // ---- sliced ELL: row n lists its upper neighbours inside [0, nH) first
    // (n < nH), then the rest in increasing column order
    out.nslice = (nn + SL - 1) / SL;
    out.nslice_h = (out.nH + SL - 1) / SL;
    auto nup_of = [&](long long n) -> int {
        if (n >= out.nH) return 0;
        int c = 0;
        for (int32_t e = up_ptr[n]; e < up_ptr[n + 1] && up_col[e] < out.nH; ++e) ++c;
        return c;
    };
    out.soff.assign(out.nslice + 1, 0);
    out.eoff.assign(out.nslice_h + 1, 0);
    for (long long s = 0; s < out.nslice; ++s) {
        int w = 0, we = 0;
        for (long long n = s * SL; n < std::min((s + 1) * SL, nn); ++n) {
            w = std::max(w, (up_ptr[n + 1] - up_ptr[n]) + (lo_ptr[n + 1] - lo_ptr[n]));
            if (s < out.nslice_h) we = std::max(we, nup_of(n));
        }
        if ((long long)out.soff[s] + (long long)SL * w > INT32_MAX) {
            err = "fem mesh: adjacency too large for 32-bit offsets";
            return HYB_E_UNSUPPORTED;
        }
        out.soff[s + 1] = out.soff[s] + SL * w;
        if (s < out.nslice_h) out.eoff[s + 1] = out.eoff[s] + SL * we;
    }
    out.nnz = out.soff[out.nslice];
    out.nE = out.eoff[out.nslice_h];
    out.col.assign(out.nnz, 0);
    out.eid.assign(out.nnz, -1);
    std::vector<int32_t> edge_pos(out.nedge, -1);  // E position of upper-inner edges
    std::vector<std::pair<int32_t, int32_t>> rest;
    for (long long n = 0; n < nn; ++n) {
        const long long s = n / SL, l = n % SL;
        int j = 0;
        auto put = [&](int32_t c, int32_t e) {
            const int64_t p = out.soff[s] + (int64_t)SL * j + l;
            out.col[p] = c;
            out.eid[p] = e;
            ++j;
        };
        const int nup = nup_of(n);
        for (int u = 0; u < nup; ++u) {
            const int32_t e = up_ptr[n] + u;
            edge_pos[e] = (int32_t)(out.eoff[s] + (int64_t)SL * j + l);
            put(up_col[e], e);
        }
        rest.clear();
        for (int32_t e = up_ptr[n] + nup; e < up_ptr[n + 1]; ++e) rest.emplace_back(up_col[e], e);
        for (int32_t p = lo_ptr[n]; p < lo_ptr[n + 1]; ++p) rest.emplace_back(lo_col[p], lo_eid[p]);
        std::sort(rest.begin(), rest.end());
        for (auto &ce : rest) put(ce.first, ce.second);
        const int w = (out.soff[s + 1] - out.soff[s]) / SL;
        while (j < w) put((int32_t)n, -1);
    }
    // ---- per free tetrahedron: E position and K^t entry of each vertex pair
    out.tetE.assign(6 * (size_t)nt, -1);
    out.ke6.assign(6 * (size_t)nt, 0.0);
    for (long long a = 0; a < nn; ++a)
        for (int64_t p = pcount[a]; p < pcount[a + 1]; ++p) {
            const long long t = pt[p];
            if (out.pvol[t] == 0.0) continue;
            const int q = PQ[pl[p]][0], r = PQ[pl[p]][1];
            out.tetE[6 * t + pl[p]] = edge_pos[pair_edge[p]];
            out.ke6[6 * t + pl[p]] = ke[16 * t + 4 * q + r];
        }
    for (long long t = 0; t < nt; ++t)
        if (out.pvol[t] > 0.0)
            for (int u = 0; u < 6; ++u)
                if (out.tetE[6 * t + u] < 0) {
                    err = "internal: free tetrahedron edge without accumulator";
                    return HYB_E_MESH;
                }
    out.minv.assign(nn, 0.0);
    for (long long n = 0; n < out.nR; ++n) out.minv[n] = 1.0 / mass[n];
    return HYB_OK;
}

}  // namespace hyb
