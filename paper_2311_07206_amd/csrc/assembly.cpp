// Host P1 finite-element assembly (paper Sec. 2.2, eq. "abstract monodomain").
//
// For a simplex T with vertices x_0..x_d let J be the d x d matrix whose rows
// are x_k - x_0 (k = 1..d).  The barycentric gradients are the columns of
// J^{-1} (k >= 1) and minus their sum (k = 0); |T| = |det J| / d!.
//   element stiffness  Khat_T[a][b] = |T| g_a . D_T g_b
//   stiffness          A = sum_T sigma_T Khat_T,  sigma_T = mean of node_sigma on T
//   lumped mass        ML_i = sum_{T containing i} |T| / (d+1)
// Rows are built independently ("gather" assembly: row i visits the elements
// containing i in ascending element order), so the work splits over threads
// without atomics and the summation order is fixed.
#include "internal.hpp"

#include <algorithm>
#include <cmath>
#include <thread>

namespace sdc {

namespace {

struct Geo {
  double vol;
  double g[4][3];  // gradients of the d+1 barycentric functions
};

bool geometry(int d, const double* X /*[d+1][d]*/, Geo* o) {
  double J[3][3] = {};
  for (int k = 1; k <= d; ++k)
    for (int c = 0; c < d; ++c) J[k - 1][c] = X[k * d + c] - X[c];
  double inv[3][3] = {};
  double det;
  if (d == 1) {
    det = J[0][0];
    if (det == 0.0) return false;
    inv[0][0] = 1.0 / det;
  } else if (d == 2) {
    det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    if (det == 0.0) return false;
    inv[0][0] = J[1][1] / det;
    inv[0][1] = -J[0][1] / det;
    inv[1][0] = -J[1][0] / det;
    inv[1][1] = J[0][0] / det;
  } else {
    double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    if (det == 0.0) return false;
    // inverse = adjugate / det; adj[i][j] = cofactor[j][i]
    inv[0][0] = c00 / det;
    inv[1][0] = c01 / det;
    inv[2][0] = c02 / det;
    inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
  }
  double fact = (d == 1) ? 1.0 : (d == 2 ? 2.0 : 6.0);
  o->vol = std::fabs(det) / fact;
  for (int c = 0; c < d; ++c) {
    double s = 0.0;
    for (int k = 1; k <= d; ++k) {
      o->g[k][c] = inv[c][k - 1];  // column k-1 of J^{-1}
      s += inv[c][k - 1];
    }
    o->g[0][c] = -s;
  }
  return true;
}

template <class Fn>
void parallel_ranges(int64_t n, Fn fn) {
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n < 4096) nt = 1;
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t) {
    int64_t lo = n * t / nt, hi = n * (t + 1) / nt;
    th.emplace_back([=, &fn] { fn(static_cast<int>(t), lo, hi); });
  }
  for (auto& x : th) x.join();
}

}  // namespace

std::string assemble_p1(int dim, int64_t n, const double* coords, int64_t ne,
                        const int32_t* elems, const double* elem_tensor,
                        const double* node_sigma, HostSystem* out) {
  const int nv = dim + 1;
  if (dim < 1 || dim > 3) return "dim must be 1, 2 or 3";
  if (n <= 0 || n >= (int64_t(1) << 31)) return "node count out of range";
  for (int64_t e = 0; e < ne * nv; ++e)
    if (elems[e] < 0 || elems[e] >= n) return "element vertex id out of range";

  // node -> elements (ascending element ids)
  std::vector<int64_t> eptr(n + 1, 0);
  for (int64_t e = 0; e < ne * nv; ++e) eptr[elems[e] + 1]++;
  for (int64_t i = 0; i < n; ++i) eptr[i + 1] += eptr[i];
  std::vector<int64_t> elist(eptr[n]);
  {
    std::vector<int64_t> fill(eptr.begin(), eptr.end() - 1);
    for (int64_t e = 0; e < ne; ++e)
      for (int a = 0; a < nv; ++a) elist[fill[elems[e * nv + a]]++] = e;
  }

  // row patterns, per thread range
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n < 4096) nt = 1;
  std::vector<std::vector<int32_t>> tcols(nt);
  std::vector<int32_t> rowlen(n);
  parallel_ranges(n, [&](int t, int64_t lo, int64_t hi) {
    std::vector<int32_t> nb;
    auto& cols = tcols[t];
    for (int64_t i = lo; i < hi; ++i) {
      nb.clear();
      nb.push_back(static_cast<int32_t>(i));
      for (int64_t q = eptr[i]; q < eptr[i + 1]; ++q)
        for (int a = 0; a < nv; ++a) nb.push_back(elems[elist[q] * nv + a]);
      std::sort(nb.begin(), nb.end());
      nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
      rowlen[i] = static_cast<int32_t>(nb.size());
      cols.insert(cols.end(), nb.begin(), nb.end());
    }
  });
  out->n = n;
  out->rowptr.assign(n + 1, 0);
  int64_t nnz = 0;
  for (int64_t i = 0; i < n; ++i) {
    nnz += rowlen[i];
    if (nnz >= (int64_t(1) << 31)) return "nnz exceeds int32 range";
    out->rowptr[i + 1] = static_cast<int32_t>(nnz);
  }
  out->col.resize(nnz);
  {
    int64_t pos = 0;
    for (unsigned t = 0; t < nt; ++t) {
      std::copy(tcols[t].begin(), tcols[t].end(), out->col.begin() + pos);
      pos += static_cast<int64_t>(tcols[t].size());
      std::vector<int32_t>().swap(tcols[t]);
    }
  }
  out->val.assign(nnz, 0.0);
  out->ml.assign(n, 0.0);
  out->diag.assign(n, -1);

  std::string err;
  std::vector<std::string> terr(nt);
  parallel_ranges(n, [&](int t, int64_t lo, int64_t hi) {
    double X[4 * 3];
    Geo geo;
    for (int64_t i = lo; i < hi; ++i) {
      const int32_t* rc = out->col.data() + out->rowptr[i];
      const int32_t len = out->rowptr[i + 1] - out->rowptr[i];
      double* rv = out->val.data() + out->rowptr[i];
      double ml = 0.0;
      for (int64_t q = eptr[i]; q < eptr[i + 1]; ++q) {
        const int64_t e = elist[q];
        const int32_t* ev = elems + e * nv;
        for (int a = 0; a < nv; ++a)
          for (int c = 0; c < dim; ++c) X[a * dim + c] = coords[int64_t(ev[a]) * dim + c];
        if (!geometry(dim, X, &geo)) {
          terr[t] = "degenerate element";
          return;
        }
        int la = 0;
        while (ev[la] != i) ++la;
        double sig = 0.0;
        for (int a = 0; a < nv; ++a) sig += node_sigma[ev[a]];
        sig /= nv;
        const double* D = elem_tensor + e * dim * dim;
        double Dg[4][3] = {};  // D g_a for every vertex
        for (int a = 0; a < nv; ++a)
          for (int r = 0; r < dim; ++r)
            for (int c = 0; c < dim; ++c) Dg[a][r] += D[r * dim + c] * geo.g[a][c];
        for (int b = 0; b < nv; ++b) {
          // Khat_ab = g_q . D g_p with (p, q) = (min, max)(la, b): rows la and
          // b evaluate the same expression, so A is exactly symmetric
          const int pa = std::min(la, b), qa = std::max(la, b);
          double kab = 0.0;
          for (int c = 0; c < dim; ++c) kab += geo.g[qa][c] * Dg[pa][c];
          const int32_t* p = std::lower_bound(rc, rc + len, ev[b]);
          rv[p - rc] += sig * geo.vol * kab;
        }
        ml += geo.vol / nv;
      }
      out->ml[i] = ml;
      out->diag[i] = static_cast<int32_t>(std::lower_bound(rc, rc + len, static_cast<int32_t>(i)) - rc) +
                     out->rowptr[i];
    }
  });
  for (auto& e : terr)
    if (!e.empty()) return e;
  return err;
}

std::string add_pair_couplings(HostSystem* hs, int64_t n_pairs, const int32_t* a, const int32_t* b,
                               const double* w, const double* diag) {
  const int64_t n = hs->n;
  // extra columns per row (both directions), then a merged, sorted pattern
  std::vector<std::vector<std::pair<int32_t, double>>> extra(n);
  for (int64_t q = 0; q < n_pairs; ++q) {
    const int32_t i = a[q], j = b[q];
    if (i < 0 || i >= n || j < 0 || j >= n || i == j) return "pair node out of range or repeated";
    const double wq = w ? w[q] : 0.0;
    extra[i].emplace_back(j, -wq);
    extra[j].emplace_back(i, -wq);
    extra[i].emplace_back(i, wq);
    extra[j].emplace_back(j, wq);
  }
  std::vector<int32_t> rowptr(n + 1, 0), col;
  std::vector<double> val;
  col.reserve(hs->col.size() + 2 * n_pairs);
  val.reserve(hs->col.size() + 2 * n_pairs);
  for (int64_t r = 0; r < n; ++r) {
    std::vector<std::pair<int32_t, double>> row;
    for (int32_t e = hs->rowptr[r]; e < hs->rowptr[r + 1]; ++e) row.emplace_back(hs->col[e], hs->val[e]);
    for (const auto& x : extra[r]) row.push_back(x);
    // stable sort keeps the element value first and the additions in pair order
    std::stable_sort(row.begin(), row.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
    for (size_t k = 0; k < row.size();) {
      size_t k1 = k;
      double v = 0.0;
      for (; k1 < row.size() && row[k1].first == row[k].first; ++k1) v += row[k1].second;
      col.push_back(row[k].first);
      val.push_back(v);
      k = k1;
    }
    if (static_cast<int64_t>(col.size()) >= (int64_t(1) << 31)) return "nnz exceeds int32 range";
    rowptr[r + 1] = static_cast<int32_t>(col.size());
  }
  if (diag)
    for (int64_t r = 0; r < n; ++r)
      for (int32_t e = rowptr[r]; e < rowptr[r + 1]; ++e)
        if (col[e] == r) val[e] += diag[r];
  hs->rowptr.swap(rowptr);
  hs->col.swap(col);
  hs->val.swap(val);
  for (int64_t r = 0; r < n; ++r) {
    const int32_t* rc = hs->col.data() + hs->rowptr[r];
    const int32_t len = hs->rowptr[r + 1] - hs->rowptr[r];
    hs->diag[r] = static_cast<int32_t>(std::lower_bound(rc, rc + len, static_cast<int32_t>(r)) - rc) + hs->rowptr[r];
  }
  return "";
}

std::string element_pairs(int dim, const double* coords, int64_t ne, const int32_t* elems,
                          const double* elem_tensor, std::vector<double>* w) {
  const int nv = dim + 1, np = nv * dim / 2;
  w->assign(static_cast<size_t>(ne) * np, 0.0);
  std::string err;
  std::vector<std::string> terr(16);
  parallel_ranges(ne, [&](int t, int64_t lo, int64_t hi) {
    double X[4 * 3];
    Geo geo;
    for (int64_t e = lo; e < hi; ++e) {
      const int32_t* ev = elems + e * nv;
      for (int a = 0; a < nv; ++a)
        for (int c = 0; c < dim; ++c) X[a * dim + c] = coords[int64_t(ev[a]) * dim + c];
      if (!geometry(dim, X, &geo)) {
        terr[t] = "degenerate element";
        return;
      }
      const double* D = elem_tensor + e * dim * dim;
      int q = 0;
      for (int a = 0; a < nv; ++a)
        for (int b = a + 1; b < nv; ++b, ++q) {
          double kab = 0.0;
          for (int r = 0; r < dim; ++r)
            for (int c = 0; c < dim; ++c) kab += geo.g[a][r] * D[r * dim + c] * geo.g[b][c];
          (*w)[static_cast<size_t>(e) * np + q] = geo.vol * kab;
        }
    }
  });
  for (auto& s : terr)
    if (!s.empty()) return s;
  return err;
}

}  // namespace sdc
