// GPU check of the short FP64 division and square root of the face code
// (div_nr, sqrt_pos in physics.hpp) against the IEEE operations on the same
// device: on seeded random operands (mantissas uniform in [1, 2), exponents
// -20 .. 20 for quotients and -30 .. 30 for roots, plus values next to powers
// of two and exact squares) every result must equal the correctly rounded one
// bit for bit. Prints the mismatch counts; exit 1 on any mismatch or error.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "../../paper_2203_13760_amd/csrc/physics.hpp"

__global__ void k_arith(const double* __restrict__ a, const double* __restrict__ b, const double* __restrict__ x,
                        double* __restrict__ out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[4 * i + 0] = cfd::div_nr(a[i], b[i]);
  out[4 * i + 1] = a[i] / b[i];
  out[4 * i + 2] = cfd::sqrt_pos(x[i]);
  out[4 * i + 3] = sqrt(x[i]);
}

static bool same_bits(double p, double q) {
  uint64_t i, j;
  std::memcpy(&i, &p, 8);
  std::memcpy(&j, &q, 8);
  return i == j;
}

int main() {
  const int n = 1 << 22;
  std::mt19937_64 rng(2203);
  std::uniform_real_distribution<double> mant(1.0, 2.0), e20(-20.0, 20.0), e30(-30.0, 30.0);
  std::vector<double> a(n), b(n), x(n), out(4 * (size_t)n);
  for (int i = 0; i < n; ++i) {
    b[i] = mant(rng) * std::exp2(std::floor(e20(rng)));
    a[i] = (rng() & 1 ? 1.0 : -1.0) * mant(rng) * std::exp2(std::floor(e20(rng)));
    x[i] = mant(rng) * std::exp2(std::floor(e30(rng)));
  }
  for (int i = 0; i < 64; ++i) {
    b[i] = 1.0 + i * 0x1p-52;               // just above a power of two
    b[64 + i] = 2.0 - (i + 1) * 0x1p-52;    // just below one
    x[i] = 1.0 + i * 0x1p-52;
    x[64 + i] = 4.0 - (i + 1) * 0x1p-51;
  }
  for (int i = 128; i < 1128; ++i) {
    const double r = 1.0 + (i - 128) * 0x1p-40;
    x[i] = r * r;                           // near exact squares
  }
  double *da = nullptr, *db = nullptr, *dx = nullptr, *dout = nullptr;
  const size_t bytes = sizeof(double) * (size_t)n;
  if (hipMalloc(&da, bytes) != hipSuccess || hipMalloc(&db, bytes) != hipSuccess ||
      hipMalloc(&dx, bytes) != hipSuccess || hipMalloc(&dout, 4 * bytes) != hipSuccess) {
    std::printf("hipMalloc failed\n");
    return 1;
  }
  if (hipMemcpy(da, a.data(), bytes, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(db, b.data(), bytes, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dx, x.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
    std::printf("upload failed\n");
    return 1;
  }
  hipLaunchKernelGGL(k_arith, dim3((n + 255) / 256), dim3(256), 0, 0, da, db, dx, dout, n);
  if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(out.data(), dout, 4 * bytes, hipMemcpyDeviceToHost) != hipSuccess) {
    std::printf("kernel failed\n");
    return 1;
  }
  long long div_bad = 0, sqrt_bad = 0;
  for (int i = 0; i < n; ++i) {
    div_bad += !same_bits(out[4 * (size_t)i], out[4 * (size_t)i + 1]);
    sqrt_bad += !same_bits(out[4 * (size_t)i + 2], out[4 * (size_t)i + 3]);
  }
  std::printf("samples %d div_nr_mismatch %lld sqrt_pos_mismatch %lld\n", n, div_bad, sqrt_bad);
  (void)hipFree(da);
  (void)hipFree(db);
  (void)hipFree(dx);
  (void)hipFree(dout);
  return div_bad == 0 && sqrt_bad == 0 ? 0 : 1;
}
