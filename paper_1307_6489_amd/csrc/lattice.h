// Lattice-row order of a camera's pixels (host code, plain C++): the table
// the neighbour-peak stage uses to place its staged words.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

namespace rta {

constexpr int kLatCols = 8;  // int16 [Npad][8] rows, as the device neighbour table

// Lattice-row order of the pixels for the neighbour-peak gathers: rows of
// equal y (quantised to half the smallest neighbour distance), x increasing,
// ties by index.  lat[p] holds the positions of the neighbours of the pixel
// at position p, one column per direction (0/1: row before, x below / above;
// 2/3: same row; 4/5: row after; a neighbour whose column is taken goes to
// the first free one), then the pixel index.  Only the speed of the gathers
// depends on this order.  nb: [N][8] neighbour indices, -1 padded, at most
// six per pixel; lat: [Np][8], filled with -1 by the caller; lpos: [Np].
inline void lattice_order(int N, int Np, const float* X, const float* Y, const int16_t* nb, int16_t* lat, uint16_t* lpos) {
  double pitch = 0.0;
  for (int i = 0; i < N; ++i)
    for (int k = 0; k < kLatCols; ++k) {
      const int j = nb[(size_t)i * kLatCols + k];
      if (j < 0) continue;
      const double d = std::hypot((double)X[j] - X[i], (double)Y[j] - Y[i]);
      if (std::isfinite(d) && d > 0.0 && (pitch == 0.0 || d < pitch)) pitch = d;
    }
  const double q = pitch > 0.0 ? 0.5 * pitch : 1.0;
  auto fin = [](double v) { return std::isfinite(v) ? std::min(std::max(v, -1e15), 1e15) : 0.0; };
  std::vector<long long> row(N);
  std::vector<double> xk(N);
  for (int i = 0; i < N; ++i) {
    row[i] = std::llround(fin((double)Y[i] / q));
    xk[i] = fin((double)X[i]);
  }
  std::vector<int> order(N);
  for (int i = 0; i < N; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int a, int b) {
    if (row[a] != row[b]) return row[a] < row[b];
    if (xk[a] != xk[b]) return xk[a] < xk[b];
    return a < b;
  });
  std::vector<int> pos(N);
  for (int p = 0; p < N; ++p) pos[order[p]] = p;
  for (int j = 0; j < Np; ++j) lpos[j] = (uint16_t)(j < N ? pos[j] : j);
  for (int p = 0; p < N; ++p) {
    const int i = order[p];
    int16_t* L = lat + (size_t)p * kLatCols;
    for (int k = 0; k < kLatCols; ++k) {
      const int j = nb[(size_t)i * kLatCols + k];
      if (j < 0) continue;
      const int dc = row[j] < row[i] ? 0 : (row[j] == row[i] ? 2 : 4);
      int col = dc + (xk[j] > xk[i] ? 1 : 0);
      if (L[col] >= 0) {
        col = 0;
        while (col < 6 && L[col] >= 0) ++col;
      }
      L[col] = (int16_t)pos[j];  // at most six neighbours, so a column is free
    }
    L[6] = (int16_t)i;
  }
}

}  // namespace rta
