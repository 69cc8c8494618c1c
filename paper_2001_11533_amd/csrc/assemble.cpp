// Host P1 finite-element assembly (paper, Section 2: [A]_ij = a(phi_j, phi_i)
// with a(y, v) = int kappa grad y . grad v, and [M]_ij = (phi_j, phi_i)).
//
// The element matrices come from p1_element.hpp (shared with the device
// assembler).  Each global entry adds its element contributions in ascending
// element index; the pattern is the mesh graph with sorted columns and
// explicit zeros kept.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "amghess.h"
#include "p1_element.hpp"

#pragma clang fp contract(off)

namespace {

// vertex -> elements (ascending) adjacency
void vertex_elems(int nl, int32_t nv, int32_t ne, const int32_t *elems, std::vector<int64_t> &vp,
                  std::vector<int32_t> &ve) {
    vp.assign((size_t)nv + 1, 0);
    for (int64_t e = 0; e < (int64_t)ne * nl; ++e) vp[elems[e] + 1]++;
    for (int32_t v = 0; v < nv; ++v) vp[v + 1] += vp[v];
    ve.resize(vp[nv]);
    std::vector<int64_t> fill(vp.begin(), vp.end() - 1);
    for (int32_t e = 0; e < ne; ++e)
        for (int a = 0; a < nl; ++a) ve[fill[elems[(int64_t)e * nl + a]]++] = e;
}

bool row_pattern(int nl, const int32_t *elems, const std::vector<int64_t> &vp, const std::vector<int32_t> &ve,
                 int32_t v, std::vector<int32_t> &cols) {
    cols.clear();
    for (int64_t p = vp[v]; p < vp[v + 1]; ++p) {
        const int32_t e = ve[p];
        for (int a = 0; a < nl; ++a) cols.push_back(elems[(int64_t)e * nl + a]);
    }
    std::sort(cols.begin(), cols.end());
    cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
    return true;
}

bool valid_mesh(int dim, int32_t nv, int32_t ne, const int32_t *elems) {
    if ((dim != 2 && dim != 3) || nv <= 0 || ne <= 0 || !elems) return false;
    const int nl = dim + 1;
    for (int64_t e = 0; e < (int64_t)ne * nl; ++e)
        if (elems[e] < 0 || elems[e] >= nv) return false;
    return true;
}

}  // namespace

extern "C" int amg_p1_pattern(int dim, int32_t nv, int32_t ne, const int32_t *elems, int32_t *nnz) {
    if (!nnz || !valid_mesh(dim, nv, ne, elems)) return AMG_ERR_ARG;
    const int nl = dim + 1;
    std::vector<int64_t> vp;
    std::vector<int32_t> ve, cols;
    vertex_elems(nl, nv, ne, elems, vp, ve);
    int64_t tot = 0;
    for (int32_t v = 0; v < nv; ++v) {
        row_pattern(nl, elems, vp, ve, v, cols);
        tot += (int64_t)cols.size();
    }
    if (tot > INT32_MAX) return AMG_ERR_ARG;
    *nnz = (int32_t)tot;
    return AMG_OK;
}

extern "C" int amg_p1_assemble(int dim, int32_t nv, const double *coords, int32_t ne, const int32_t *elems,
                               const double *kappa, int32_t nnz, int32_t *rowptr, int32_t *col, double *valA,
                               double *valM) {
    if (!coords || !kappa || !rowptr || !col || !valA || !valM || !valid_mesh(dim, nv, ne, elems)) return AMG_ERR_ARG;
    const int nl = dim + 1;
    std::vector<int64_t> vp;
    std::vector<int32_t> ve, cols;
    vertex_elems(nl, nv, ne, elems, vp, ve);
    int64_t pos = 0;
    rowptr[0] = 0;
    double X[12];
    amg::P1Elem el;
    for (int32_t v = 0; v < nv; ++v) {
        row_pattern(nl, elems, vp, ve, v, cols);
        if (pos + (int64_t)cols.size() > nnz) return AMG_ERR_ARG;
        const int64_t base = pos;
        for (size_t q = 0; q < cols.size(); ++q) {
            col[base + q] = cols[q];
            valA[base + q] = 0.0;
            valM[base + q] = 0.0;
        }
        for (int64_t p = vp[v]; p < vp[v + 1]; ++p) {  // elements in ascending order
            const int32_t e = ve[p];
            const int32_t *ev = elems + (int64_t)e * nl;
            for (int a = 0; a < nl; ++a)
                for (int r = 0; r < dim; ++r) X[a * dim + r] = coords[(int64_t)ev[a] * dim + r];
            amg::p1_element(dim, X, kappa[e], el);
            int a = 0;
            while (ev[a] != v) ++a;
            for (int b = 0; b < nl; ++b) {
                const int32_t k = ev[b];
                const int64_t q = base + (std::lower_bound(cols.begin(), cols.end(), k) - cols.begin());
                valA[q] = valA[q] + el.K[a][b];
                valM[q] = valM[q] + el.M[a][b];
            }
        }
        pos += (int64_t)cols.size();
        rowptr[v + 1] = (int32_t)pos;
    }
    return pos == nnz ? AMG_OK : AMG_ERR_ARG;
}
