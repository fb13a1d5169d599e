// Windowed layout of an explicit matrix (host side, at lattice creation).
//
// The sparse Chebyshev step gathers phi_n at the column indices of every
// entry.  In the slice layout of the input order a slice of 128 consecutive
// rows touches a long, mostly unused column range, and each gathered value
// is read from the caches once per entry that names it.  Here the rows are
// regrouped into slices of 128 rows that are compact in the matrix graph
// (grown breadth-first from the lowest unassigned row, so a slice is a ball
// of neighbouring orbitals), and each slice records its window: the sorted
// distinct columns its entries name.  The recursion kernel stages a slice's
// window of phi_n in LDS once per step and gathers from there with 16-bit
// window-local indices; rows keep their index in every vector (only slice
// membership changes), so nothing outside the recursion kernel sees the
// regrouping.
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

#include "csp_internal.h"

namespace csp {

bool build_ell_windows(int64_t N, int D, const int32_t* col, const double* val,
                       EllWindows* w) {
  const int64_t n_sl = (N + 127) / 128;
  // entries in quads: slice, quad q of a row's entries 4q .. 4q + 3, row,
  // entry inside the quad ([n_sl][D4][128][4]); entries past D are padding
  const int D4 = (D + 3) / 4;
  const size_t n = (size_t)n_sl * D4 * 128 * 4;
  w->D4 = D4;
  w->n_slices = n_sl;
  w->rows.assign((size_t)n_sl * 128, -1);
  w->off.assign(n_sl + 1, 0);
  w->idx.clear();
  w->loc.assign(n, 0);
  w->col.assign(n, 0);
  w->v64.assign(n, 0.0);
  w->v32.assign(n, 0.0f);
  w->max_window = 0;

  // ---- slices grown breadth-first over the matrix graph
  std::vector<uint8_t> taken((size_t)N, 0);
  std::vector<int32_t> queue;
  queue.reserve(128);
  int64_t seed = 0, filler = 0;
  for (int64_t sl = 0; sl < n_sl; ++sl) {
    int32_t* rows = w->rows.data() + (size_t)sl * 128;
    int cnt = 0;
    while (seed < N && taken[seed]) ++seed;
    if (seed < N) {
      queue.clear();
      queue.push_back(static_cast<int32_t>(seed));
      taken[seed] = 1;
      size_t head = 0;
      while (head < queue.size() && cnt < 128) {
        const int32_t r = queue[head++];
        rows[cnt++] = r;
        const int32_t* cr = col + (size_t)r * D;
        for (int k = 0; k < D && (int)(queue.size() - head) + cnt < 128; ++k) {
          const int32_t j = cr[k];
          if (j >= 0 && !taken[j]) {
            taken[j] = 1;
            queue.push_back(j);
          }
        }
      }
      for (size_t q = head; q < queue.size(); ++q) taken[queue[q]] = 0;   // not used
    }
    // a slice the search could not fill takes the next free rows in order
    while (cnt < 128) {
      while (filler < N && taken[filler]) ++filler;
      if (filler >= N) break;
      taken[filler] = 1;
      rows[cnt++] = static_cast<int32_t>(filler);
    }
    // rows ascending inside the slice: neighbouring lanes then read
    // neighbouring rows of the vectors and, for matrices with a regular
    // pattern, neighbouring positions of the window (fewer LDS bank conflicts)
    std::sort(rows, rows + cnt);
  }

  // ---- windows and the entries in slice order, slices split over threads
  // (each with its own column marks)
  std::vector<std::vector<int32_t>> wins((size_t)n_sl);
  auto work = [&](int64_t sl_lo, int64_t sl_hi) {
    std::vector<int32_t> mark((size_t)N, -1);
    for (int64_t sl = sl_lo; sl < sl_hi; ++sl) {
      const int32_t* rows = w->rows.data() + (size_t)sl * 128;
      std::vector<int32_t>& win = wins[sl];
      for (int t = 0; t < 128; ++t) {
        const int32_t r = rows[t];
        if (r < 0) continue;
        const int32_t* cr = col + (size_t)r * D;
        for (int k = 0; k < D; ++k) {
          const int32_t j = cr[k];
          if (j >= 0 && mark[j] < 0) {
            mark[j] = 0;
            win.push_back(j);
          }
        }
      }
      std::sort(win.begin(), win.end());
      for (size_t q = 0; q < win.size(); ++q) mark[win[q]] = static_cast<int32_t>(q);
      const size_t o = (size_t)sl * D4 * 512;
      for (int t = 0; t < 128; ++t) {
        const int32_t r = rows[t];
        for (int k = 0; k < 4 * D4; ++k) {
          const size_t e = o + (size_t)(k >> 2) * 512 + (size_t)t * 4 + (k & 3);
          if (r < 0 || k >= D) {
            // lanes past N and entries past D: a valid index with the value 0
            w->col[e] = r < 0 ? 0 : r;
            w->loc[e] = 0;
            continue;
          }
          const int32_t j = col[(size_t)r * D + k];
          const double v = j >= 0 ? val[(size_t)r * D + k] : 0.0;
          // padding entries: the row itself with the value 0 (the row need
          // not be in its own window, so its local index is 0, also with
          // value 0)
          w->col[e] = j >= 0 ? j : r;
          w->loc[e] = j >= 0 && mark[j] <= 0xffff ? static_cast<uint16_t>(mark[j]) : 0;
          w->v64[e] = v;
          w->v32[e] = static_cast<float>(v);
        }
      }
      for (int32_t j : win) mark[j] = -1;
    }
  };
  const int64_t entries = N * (int64_t)D;
  int nt = (int)std::min<int64_t>(16, std::max<unsigned>(1u, std::thread::hardware_concurrency()));
  if (entries < (int64_t)1 << 22) nt = 1;
  nt = (int)std::min<int64_t>(nt, n_sl);
  std::vector<std::thread> pool;
  for (int q = 1; q < nt; ++q)
    pool.emplace_back(work, n_sl * q / nt, n_sl * (q + 1) / nt);
  work(0, n_sl / nt);
  for (auto& th : pool) th.join();
  for (int64_t sl = 0; sl < n_sl; ++sl) {
    const int64_t W = (int64_t)wins[sl].size();
    w->max_window = std::max(w->max_window, W);
    w->off[sl + 1] = w->off[sl] + W;
  }
  w->idx.resize((size_t)w->off[n_sl]);
  for (int64_t sl = 0; sl < n_sl; ++sl)
    std::copy(wins[sl].begin(), wins[sl].end(), w->idx.begin() + w->off[sl]);
  return true;
}

}  // namespace csp
