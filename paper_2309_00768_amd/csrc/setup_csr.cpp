// Host sparse-matrix utilities used by the setup phase (assembly, wave operator,
// AMG Galerkin products).  Plain float64 CSR with sorted rows.
#include <algorithm>
#include <atomic>
#include <functional>
#include <thread>

#include "st_internal.h"

namespace st {

int64_t Csr::find(int r, int c) const {
  const int* b = ci.data() + rp[r];
  const int* e = ci.data() + rp[r + 1];
  const int* it = std::lower_bound(b, e, c);
  if (it == e || *it != c) return -1;
  return it - ci.data();
}

Csr PatternBuilder::finish() {
  Csr a;
  a.nr = nr_;
  a.nc = nc_;
  a.rp.assign(nr_ + 1, 0);
  for (int r = 0; r < nr_; ++r) {
    auto& row = rows_[r];
    std::sort(row.begin(), row.end());
    row.erase(std::unique(row.begin(), row.end()), row.end());
    a.rp[r + 1] = a.rp[r] + int(row.size());
  }
  a.ci.resize(a.rp[nr_]);
  for (int r = 0; r < nr_; ++r) std::copy(rows_[r].begin(), rows_[r].end(), a.ci.begin() + a.rp[r]);
  a.v.assign(a.ci.size(), 0.0);
  rows_.clear();
  return a;
}

Csr csr_transpose(const Csr& a) {
  Csr t;
  t.nr = a.nc;
  t.nc = a.nr;
  t.rp.assign(t.nr + 1, 0);
  const int64_t nnz = a.nnz();
  for (int64_t p = 0; p < nnz; ++p) t.rp[a.ci[p] + 1]++;
  for (int r = 0; r < t.nr; ++r) t.rp[r + 1] += t.rp[r];
  t.ci.resize(nnz);
  const int nsets = nnz ? int(a.v.size() / nnz) : 1;
  t.v.resize(size_t(nsets) * nnz);
  std::vector<int> next(t.rp.begin(), t.rp.end() - 1);
  for (int r = 0; r < a.nr; ++r)
    for (int p = a.rp[r]; p < a.rp[r + 1]; ++p) {
      int q = next[a.ci[p]]++;
      t.ci[q] = r;
      for (int s = 0; s < nsets; ++s) t.v[size_t(s) * nnz + q] = a.v[size_t(s) * nnz + p];
    }
  return t;
}

Csr csr_matmul(const Csr& a, const Csr& b) {
  // Gustavson row-by-row product on value set 0 of each operand.
  Csr c;
  c.nr = a.nr;
  c.nc = b.nc;
  c.rp.assign(c.nr + 1, 0);
  std::vector<int> marker(b.nc, -1);
  std::vector<double> acc(b.nc, 0.0);
  std::vector<int> cols;
  for (int r = 0; r < a.nr; ++r) {
    cols.clear();
    for (int p = a.rp[r]; p < a.rp[r + 1]; ++p) {
      const int k = a.ci[p];
      const double av = a.v[p];
      for (int q = b.rp[k]; q < b.rp[k + 1]; ++q) {
        const int j = b.ci[q];
        if (marker[j] != r) {
          marker[j] = r;
          acc[j] = 0.0;
          cols.push_back(j);
        }
        acc[j] += av * b.v[q];
      }
    }
    std::sort(cols.begin(), cols.end());
    for (int j : cols) {
      c.ci.push_back(j);
      c.v.push_back(acc[j]);
    }
    c.rp[r + 1] = int(c.ci.size());
  }
  return c;
}

Csr csr_add(const Csr& a, double sa, const Csr& b, double sb) {
  Csr c;
  c.nr = a.nr;
  c.nc = a.nc;
  c.rp.assign(c.nr + 1, 0);
  for (int r = 0; r < a.nr; ++r) {
    int p = a.rp[r], q = b.rp[r];
    const int pe = a.rp[r + 1], qe = b.rp[r + 1];
    while (p < pe || q < qe) {
      if (q >= qe || (p < pe && a.ci[p] < b.ci[q])) {
        c.ci.push_back(a.ci[p]);
        c.v.push_back(sa * a.v[p]);
        ++p;
      } else if (p >= pe || b.ci[q] < a.ci[p]) {
        c.ci.push_back(b.ci[q]);
        c.v.push_back(sb * b.v[q]);
        ++q;
      } else {
        c.ci.push_back(a.ci[p]);
        c.v.push_back(sa * a.v[p] + sb * b.v[q]);
        ++p;
        ++q;
      }
    }
    c.rp[r + 1] = int(c.ci.size());
  }
  return c;
}

Csr csr_scale_cols(const Csr& a, const std::vector<double>& s) {
  Csr c = a;
  const int64_t nnz = a.nnz();
  c.v.resize(nnz);
  for (int64_t p = 0; p < nnz; ++p) c.v[p] = a.v[p] * s[a.ci[p]];
  return c;
}

void csr_spmv(const Csr& a, const double* x, double* y) {
  for (int r = 0; r < a.nr; ++r) {
    double s = 0.0;
    for (int p = a.rp[r]; p < a.rp[r + 1]; ++p) s += a.v[p] * x[a.ci[p]];
    y[r] = s;
  }
}

int host_threads() {
  unsigned h = std::thread::hardware_concurrency();
  if (h == 0) h = 4;
  return int(std::min(h, 16u));
}

void parallel_for(int n, int threads, const std::function<void(int)>& f) {
  if (n <= 0) return;
  threads = std::max(1, std::min(threads, n));
  if (threads == 1) {
    for (int i = 0; i < n; ++i) f(i);
    return;
  }
  std::atomic<int> next(0);
  std::vector<std::thread> pool;
  for (int t = 0; t < threads; ++t)
    pool.emplace_back([&]() {
      for (;;) {
        int i = next.fetch_add(1);
        if (i >= n) break;
        f(i);
      }
    });
  for (auto& th : pool) th.join();
}

}  // namespace st
