// Rusanov-NN flux of §7.4 on gfx950: the Rusanov flux whose dissipation alpha
// is the output of a small network of four face features.
//
//   forward:  k_nn_alpha evaluates the network for every face of the active axes
//             from the WENO3-JS face states and stores alpha at the face's
//             left cell (Geom::nna); the sweeps (scheme SCH_W3_NN) read it.
//   reverse:  k_face_adj_nn recomputes the face (states, features,
//             network), reverses the flux with alpha held, the network
//             (output adjoint -> input adjoint) and the features, then the
//             WENO3-JS stencils into Wbar with atomics, as the other face
//             reverses do. It records the network's pre-activations and their
//             adjoints per face; k_nn_wgrad forms the weight gradient from the
//             records as the sums over faces of (delta_l h_{l-1}^T), one block
//             per output row, in a fixed order (bitwise repeatable for given
//             face adjoints).
//
// The layers are FP64 matrix products on the matrix cores: a wavefront takes 16
// faces, four lanes per face, and a layer of 32 units is two 16 x 16 result
// tiles, each a chain of 16x16x4 products over the layer's inputs.
#pragma once
#include "kernels_adj.hpp"

namespace cfd {

// Network of §7.4: 4 inputs, three hidden layers of 32 units with ReLU, one
// output through exp (alpha >= 0). Weights in the order W1 (32 x 4,
// row-major), b1, W2 (32 x 32), b2, W3 (32 x 32), b3, W4 (1 x 32), b4; a layer
// maps h -> W h + b.
constexpr int kNNH = 32, kNNIn = 4;
constexpr int kNNb1 = kNNH * kNNIn, kNNW2 = kNNb1 + kNNH, kNNb2 = kNNW2 + kNNH * kNNH, kNNW3 = kNNb2 + kNNH,
              kNNb3 = kNNW3 + kNNH * kNNH, kNNW4 = kNNb3 + kNNH, kNNb4 = kNNW4 + kNNH, kNNParams = kNNb4 + 1;
static_assert(kNNParams == 2305, "network size");

// Per-face records of one right-hand-side reverse, written by k_face_adj_nn
// and read by k_nn_wgrad: pre-activations z1..z3 and their adjoints d1..d3
// ([F][32] each), the inputs ([F][4]) and the output pre-activation's adjoint
// ([F]); F counts the faces of all active axes.
struct NNTape {
  double* z[3];
  double* d[3];
  double* f;
  double* d4;
  double* part;  // kNNChunks partial weight gradients (kNNParams each)
  long long F;
};
constexpr int kNNTapePerFace = 6 * kNNH + kNNIn + 1;
constexpr int kNNChunks = 4;  // face chunks of the weight gradient
constexpr int kNNRows = 3 * kNNH + 1;  // output rows of the four layers

__device__ __forceinline__ double relu(double z) { return z > 0.0 ? z : 0.0; }

// WENO3-JS states across the face whose left cell is cl (padded index),
// normal to D, from cells cl-1 .. cl+2, as in the sweeps.
template <int D>
__device__ __forceinline__ void nn_face_states(const Geom& g, const double* __restrict__ P, long long cl, double* WL,
                                               double* WR) {
  const long long st = g.s[D];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const double* q = P + v * g.vs + cl;
    const double a = q[-st], b = q[0], c = q[st], d = q[2 * st];
    WL[v] = weno3(a, b, c);
    WR[v] = weno3(d, c, b);
  }
}

// Inputs of the network: |u_R - u_L|, (u_L + u_R)/2, (c_L + c_R)/2 and
// |s_R - s_L|, u normal to the face, c = sqrt(gamma p / rho), the entropy
// s = (ln p - gamma ln rho)/(gamma - 1).
template <int D>
__device__ __forceinline__ void nn_features(const Geom& g, const double* WL, const double* WR, double* f) {
  const double uL = WL[1 + D], uR = WR[1 + D];
  const double cL = sqrt_pos(div_nr(g.gamma * WL[4], WL[0])), cR = sqrt_pos(div_nr(g.gamma * WR[4], WR[0]));
  const double sL = (log(WL[4]) - g.gamma * log(WL[0])) * g.gm1i;
  const double sR = (log(WR[4]) - g.gamma * log(WR[0])) * g.gm1i;
  f[0] = fabs(uR - uL);
  f[1] = 0.5 * (uL + uR);
  f[2] = 0.5 * (cL + cR);
  f[3] = fabs(sR - sL);
}

typedef double nn_v4 __attribute__((ext_vector_type(4)));

// Matrix layout. The 16x16x4 product D = A B + C takes A[i][k] from lane
// i + 16k, B[k][j] from lane j + 16k, and leaves D[4r + k][j] in item r of lane
// j + 16k. A wavefront holds 16 faces: lane (f, q) = f + 16q works on face f
// (f = lane % 16) in quarter q (= lane / 16). A layer's 32 units x 16 faces
// are two tiles t of 16 units; lane (f, q) holds units 16t + 4r + q, r = 0..3,
// of face f (NNTile). The next layer's B operand in its k-step s (s = 0..7)
// is then the lane's own item r = s % 4 of tile t = s / 4, input unit
// nn_unit(s, q): a layer needs no exchange between lanes.
struct NNTile {
  nn_v4 t[2];
};

__device__ __forceinline__ int nn_unit(int s, int q) { return 16 * (s >> 2) + 4 * (s & 3) + q; }

__device__ __forceinline__ nn_v4 nn_mfma(double a, double b, nn_v4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// First layer: z = W1 f + b1; lane (f, q) supplies input feature q of its face.
__device__ __forceinline__ void nn_layer1(const double* __restrict__ th, double fq, int f, int q, NNTile& z) {
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    nn_v4 c;
#pragma unroll
    for (int r = 0; r < 4; ++r) c[r] = th[kNNb1 + 16 * t + 4 * r + q];
    z.t[t] = nn_mfma(th[(16 * t + f) * kNNIn + q], fq, c);
  }
}

// Hidden layer: z = W relu(h) + b (W row-major 32 x 32).
__device__ __forceinline__ void nn_layer(const double* __restrict__ W, const double* __restrict__ b, const NNTile& h,
                                         int f, int q, NNTile& z) {
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    nn_v4 c;
#pragma unroll
    for (int r = 0; r < 4; ++r) c[r] = b[16 * t + 4 * r + q];
#pragma unroll
    for (int s = 0; s < 8; ++s) c = nn_mfma(W[(16 * t + f) * kNNH + nn_unit(s, q)], relu(h.t[s >> 2][s & 3]), c);
    z.t[t] = c;
  }
}

// Output pre-activation of the lane's face: W4 relu(z3) + b4, the four
// quarters' partial sums added across lanes (every lane of the face gets it).
__device__ __forceinline__ double nn_output(const double* __restrict__ th, const NNTile& z3, int q) {
  double s = 0.0;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) s = fma(th[kNNW4 + 16 * t + 4 * r + q], relu(z3.t[t][r]), s);
  s += __shfl_xor(s, 16, 64);
  s += __shfl_xor(s, 32, 64);
  return s + th[kNNb4];
}

// Forward pass of the lane's face; returns the output pre-activation.
__device__ __forceinline__ double nn_forward(const double* __restrict__ th, double fq, int f, int q, NNTile& z1,
                                             NNTile& z2, NNTile& z3) {
  nn_layer1(th, fq, f, q, z1);
  nn_layer(th + kNNW2, th + kNNb2, z1, f, q, z2);
  nn_layer(th + kNNW3, th + kNNb3, z2, f, q, z3);
  return nn_output(th, z3, q);
}

// Transposed layer: di = (W^T dout) masked by the ReLU of zi (a pre-activation
// of exactly zero passes, as max(z, 0) taking z there).
__device__ __forceinline__ void nn_layer_rev(const double* __restrict__ W, const NNTile& dout, const NNTile& zi,
                                             int f, int q, NNTile& di) {
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    nn_v4 c = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 8; ++s) c = nn_mfma(W[nn_unit(s, q) * kNNH + 16 * t + f], dout.t[s >> 2][s & 3], c);
#pragma unroll
    for (int r = 0; r < 4; ++r) c[r] = zi.t[t][r] >= 0.0 ? c[r] : 0.0;
    di.t[t] = c;
  }
}

// Input adjoint of the first layer: W1^T d1, one tile whose rows 0..3 are the
// four inputs; lane (f, q) receives input q's adjoint of its face.
__device__ __forceinline__ double nn_input_rev(const double* __restrict__ th, const NNTile& d1, int f, int q) {
  nn_v4 c = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < 8; ++s) c = nn_mfma(f < kNNIn ? th[nn_unit(s, q) * kNNIn + f] : 0.0, d1.t[s >> 2][s & 3], c);
  return c[0];
}

// Primitive adjoint of one side's physical flux F(W) and conservative state
// U(W) along D: Wb += (dF/dW)^T Fb + (dU/dW)^T Ub.
template <int D>
__device__ __forceinline__ void euler_state_rev(double gm1i, const double* W, const double* Fb, const double* Ub,
                                                double* Wb) {
  const double rho = W[0], p = W[4], un = W[1 + D];
  const double q2 = W[1] * W[1] + W[2] * W[2] + W[3] * W[3];
  const double E = p * gm1i + 0.5 * rho * q2;
  const double m = rho * un;
  // F0 = m, F_{1+a} = m u_a + [a == D] p, F4 = un (E + p)
  double mb = Fb[0];
  double Eb = Fb[4] * un + Ub[4];
  double unb = Fb[4] * (E + p);
  double pb = Fb[4] * un + Fb[1 + D];
  double rb = Ub[0];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    mb += Fb[1 + a] * W[1 + a];
    Wb[1 + a] += Fb[1 + a] * m + Ub[1 + a] * rho;  // also U_{1+a} = rho u_a
    rb += Ub[1 + a] * W[1 + a];
  }
  // m = rho un
  rb += mb * un;
  unb += mb * rho;
  // E = p/(gamma-1) + rho |u|^2 / 2
  pb += Eb * gm1i;
  rb += Eb * 0.5 * q2;
#pragma unroll
  for (int a = 0; a < 3; ++a) Wb[1 + a] += Eb * rho * W[1 + a];
  Wb[1 + D] += unb;
  Wb[0] += rb;
  Wb[4] += pb;
}

// Reverse of G = (F_L + F_R)/2 - alpha (U_R - U_L)/2 with alpha held:
// WLb, WRb += the state adjoints; returns alpha's adjoint.
template <int D>
__device__ __forceinline__ double rusanov_given_rev(double gm1i, const double* WL, const double* WR, double alpha,
                                                    const double* Gb, double* WLb, double* WRb) {
  double Fb[5], ULb[5], URb[5];
  double ab = 0.0;
  const double qL = WL[1] * WL[1] + WL[2] * WL[2] + WL[3] * WL[3];
  const double qR = WR[1] * WR[1] + WR[2] * WR[2] + WR[3] * WR[3];
  const double UL[5] = {WL[0], WL[0] * WL[1], WL[0] * WL[2], WL[0] * WL[3], WL[4] * gm1i + 0.5 * WL[0] * qL};
  const double UR[5] = {WR[0], WR[0] * WR[1], WR[0] * WR[2], WR[0] * WR[3], WR[4] * gm1i + 0.5 * WR[0] * qR};
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    Fb[v] = 0.5 * Gb[v];
    ULb[v] = 0.5 * alpha * Gb[v];
    URb[v] = -0.5 * alpha * Gb[v];
    ab -= 0.5 * Gb[v] * (UR[v] - UL[v]);
  }
  euler_state_rev<D>(gm1i, WL, Fb, ULb, WLb);
  euler_state_rev<D>(gm1i, WR, Fb, URb, WRb);
  return ab;
}

// Reverse of nn_features: WLb, WRb += (df/dW)^T fb. |x| takes the slope +1 at
// x = 0, as the comparison x < 0 selects -x.
template <int D>
__device__ __forceinline__ void nn_features_rev(const Geom& g, const double* WL, const double* WR, const double* fb,
                                                double* WLb, double* WRb) {
  const double uL = WL[1 + D], uR = WR[1 + D];
  const double du = uR - uL;
  const double sg0 = du < 0.0 ? -1.0 : 1.0;
  WRb[1 + D] += fb[0] * sg0 + 0.5 * fb[1];
  WLb[1 + D] += -fb[0] * sg0 + 0.5 * fb[1];
  // c = sqrt(gamma p / rho): dc/dp = c/(2p), dc/drho = -c/(2 rho)
  const double cL = sqrt_pos(div_nr(g.gamma * WL[4], WL[0])), cR = sqrt_pos(div_nr(g.gamma * WR[4], WR[0]));
  const double cb = 0.5 * fb[2];
  WLb[4] += cb * cL / (2.0 * WL[4]);
  WLb[0] -= cb * cL / (2.0 * WL[0]);
  WRb[4] += cb * cR / (2.0 * WR[4]);
  WRb[0] -= cb * cR / (2.0 * WR[0]);
  // s = (ln p - gamma ln rho)/(gamma - 1)
  const double sL = (log(WL[4]) - g.gamma * log(WL[0])) * g.gm1i;
  const double sR = (log(WR[4]) - g.gamma * log(WR[0])) * g.gm1i;
  const double sg3 = (sR - sL) < 0.0 ? -1.0 : 1.0;
  const double sRb = fb[3] * sg3, sLb = -fb[3] * sg3;
  WLb[4] += sLb * g.gm1i / WL[4];
  WLb[0] -= sLb * g.gamma * g.gm1i / WL[0];
  WRb[4] += sRb * g.gm1i / WR[4];
  WRb[0] -= sRb * g.gamma * g.gm1i / WR[0];
}

// Face and lane of a network kernel: 16 faces per wavefront, numbered as in
// the face reverses. Lanes beyond the last face take face 0 (valid addresses)
// and keep to the matrix products, which need the whole wavefront.
template <int D>
__device__ __forceinline__ bool nn_face(const Geom& g, int bx, int& t, int& i, int& j, int& k, int& f, int& q) {
  const int lane = threadIdx.x & 63;
  f = lane & 15;
  q = lane >> 4;
  t = ((bx * kBlock + (int)threadIdx.x) >> 6) * 16 + f;
  int fc = 0, col = 0;
  const bool has = face_coords<D>(g, t, i, j, k, fc, col);
  if (!has) face_coords<D>(g, 0, i, j, k, fc, col);
  return has;
}

// One launch covers the faces of every active axis: blocks [0, blk[0]) take
// x faces, the next blk[1] y faces, the last blk[2] z faces (64 faces per
// block; 0 blocks for an inactive axis), so the axes' latencies overlap.
// off[D]: first record slot of axis D in the reverse's tape.
struct NNAxes {
  int blk[3];
  long long off[3];
};

// alpha of every face normal to D, stored at the face's left cell.
template <int D>
__device__ __forceinline__ void nn_alpha_body(const double* __restrict__ P, const Geom& g, int bx) {
  int t, i, j, k, f, q;
  const bool has = nn_face<D>(g, bx, t, i, j, k, f, q);
  const long long cl = cell_at(g, i, j, k) - g.s[D];  // cell f-1 of the face
  double WL[5], WR[5], ft[kNNIn];
  nn_face_states<D>(g, P, cl, WL, WR);
  nn_features<D>(g, WL, WR, ft);
  const double fq = q == 0 ? ft[0] : q == 1 ? ft[1] : q == 2 ? ft[2] : ft[3];
  NNTile z1, z2, z3;
  const double out = nn_forward(g.nnw, fq, f, q, z1, z2, z3);
  if (has && q == 0) g.nna[D * g.vs + cl] = exp(out);
}

// Face reverse of the Rusanov-NN flux (inviscid), faces normal to D; the
// records of face t go to slot off + t of the tape. The four lanes of a face
// share the network's products; the flux reverse is the same in each, and the
// stencil reverse is split by variable (quarter q takes the variables
// v = q mod 4).
template <int D>
__device__ __forceinline__ void face_adj_nn_body(const double* __restrict__ P, const double* __restrict__ Rbar,
                                                 double rscale, double* Wbar, const Geom& g, const NNTape& tp,
                                                 long long off, int bx) {
  int t, i, j, k, f, q;
  const bool has = nn_face<D>(g, bx, t, i, j, k, f, q);
  const long long st = g.s[D];
  const long long cf = cell_at(g, i, j, k), cl = cf - st;
  const long long e = off + t;
  double Gb[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (has) face_gbar<D>(g, Rbar, rscale, cf, D == 0 ? i : D == 1 ? j : k, Gb);  // face index along D
  double WL[5], WR[5], ft[kNNIn];
  nn_face_states<D>(g, P, cl, WL, WR);
  nn_features<D>(g, WL, WR, ft);
  const double fq = q == 0 ? ft[0] : q == 1 ? ft[1] : q == 2 ? ft[2] : ft[3];
  const double* __restrict__ th = g.nnw;
  NNTile z1, z2, z3;
  const double alpha = exp(nn_forward(th, fq, f, q, z1, z2, z3));
  double WLb[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, WRb[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const double ab = rusanov_given_rev<D>(g.gm1i, WL, WR, alpha, Gb, WLb, WRb);
  // network reverse: output through exp, then the layers
  const double d4 = ab * alpha;
  NNTile d3, d2, d1;
#pragma unroll
  for (int tt = 0; tt < 2; ++tt)
#pragma unroll
    for (int r = 0; r < 4; ++r) d3.t[tt][r] = z3.t[tt][r] >= 0.0 ? th[kNNW4 + 16 * tt + 4 * r + q] * d4 : 0.0;
  nn_layer_rev(th + kNNW3, d3, z2, f, q, d2);
  nn_layer_rev(th + kNNW2, d2, z1, f, q, d1);
  const double fbq = nn_input_rev(th, d1, f, q);
  double fb[kNNIn];
#pragma unroll
  for (int m = 0; m < kNNIn; ++m) fb[m] = __shfl(fbq, f + 16 * m, 64);
  if (has) {
    // records for the weight gradient
#pragma unroll
    for (int tt = 0; tt < 2; ++tt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long long u = e * kNNH + 16 * tt + 4 * r + q;
        tp.z[0][u] = z1.t[tt][r];
        tp.z[1][u] = z2.t[tt][r];
        tp.z[2][u] = z3.t[tt][r];
        tp.d[0][u] = d1.t[tt][r];
        tp.d[1][u] = d2.t[tt][r];
        tp.d[2][u] = d3.t[tt][r];
      }
    tp.f[e * kNNIn + q] = fq;
    if (q == 0) tp.d4[e] = d4;
  }
  nn_features_rev<D>(g, WL, WR, fb, WLb, WRb);
  if (!has) return;
  // WENO3-JS reverse into the stencil cells cl-1 .. cl+2, variables v = q mod 4
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    if ((v & 3) != q) continue;
    double* w = Wbar + v * g.vs + cl;
    const double* qv = P + v * g.vs + cl;
    const double a = qv[-st], b = qv[0], c = qv[st], d = qv[2 * st];
    double gs[4] = {0.0, 0.0, 0.0, 0.0};
    weno3_rev(a, b, c, WLb[v], gs);
    double gr[3] = {0.0, 0.0, 0.0};
    weno3_rev(d, c, b, WRb[v], gr);
    gs[3] += gr[0];
    gs[2] += gr[1];
    gs[1] += gr[2];
#pragma unroll
    for (int m = 0; m < 4; ++m) atomic_add(w + (m - 1) * st, gs[m]);
  }
}

__global__ void __launch_bounds__(kBlock) k_nn_alpha(const double* __restrict__ P, Geom g, NNAxes ax) {
  int b = blockIdx.x;
  if (b < ax.blk[0]) return nn_alpha_body<0>(P, g, b);
  b -= ax.blk[0];
  if (b < ax.blk[1]) return nn_alpha_body<1>(P, g, b);
  b -= ax.blk[1];
  nn_alpha_body<2>(P, g, b);
}

__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2)))
k_face_adj_nn(const double* __restrict__ P, const double* __restrict__ Rbar,
                                                        double rscale, double* Wbar, Geom g, NNTape tp, NNAxes ax) {
  int b = blockIdx.x;
  if (b < ax.blk[0]) return face_adj_nn_body<0>(P, Rbar, rscale, Wbar, g, tp, ax.off[0], b);
  b -= ax.blk[0];
  if (b < ax.blk[1]) return face_adj_nn_body<1>(P, Rbar, rscale, Wbar, g, tp, ax.off[1], b);
  b -= ax.blk[1];
  face_adj_nn_body<2>(P, Rbar, rscale, Wbar, g, tp, ax.off[2], b);
}

// Weight gradient from the records, in two launches with every sum in a fixed
// order. k_nn_wgrad: block (r, chunk) = r + kNNRows * chunk owns output row r
// (rows 0..31 of (W1 | b1), 32..63 of (W2 | b2), 64..95 of (W3 | b3), 96 the
// output layer (W4 | b4)) over the faces of its chunk (faces e with
// e / kBlock = chunk mod kNNChunks); each lane sums its faces for the row's
// weights and bias, the wavefronts reduce by shuffles, the four partial sums
// are added in a fixed order and stored in the chunk's partial gradient.
// k_nn_wgrad_sum then adds the kNNChunks partials to thb.
__global__ void __launch_bounds__(kBlock) k_nn_wgrad(NNTape tp) {
  const int r = blockIdx.x % kNNRows, chunk = blockIdx.x / kNNRows;
  const int layer = r / kNNH, o = r - layer * kNNH;
  const double* hs = layer == 0 ? tp.f : tp.z[layer - 1];
  double acc[kNNH + 1];
#pragma unroll
  for (int m = 0; m <= kNNH; ++m) acc[m] = 0.0;
  for (long long e = (long long)chunk * kBlock + threadIdx.x; e < tp.F; e += (long long)kBlock * kNNChunks) {
    const double dd = layer < 3 ? tp.d[layer][e * kNNH + o] : tp.d4[e];
    acc[kNNH] += dd;
    if (layer == 0) {
#pragma unroll
      for (int m = 0; m < kNNIn; ++m) acc[m] = fma(dd, hs[e * kNNIn + m], acc[m]);
    } else {
#pragma unroll
      for (int m = 0; m < kNNH; ++m) acc[m] = fma(dd, relu(hs[e * kNNH + m]), acc[m]);
    }
  }
  __shared__ double part[kBlock / 64][kNNH + 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int m = 0; m <= kNNH; ++m) {
    double v = acc[m];
#pragma unroll
    for (int sft = 32; sft >= 1; sft >>= 1) v += __shfl_xor(v, sft, 64);
    if (lane == 0) part[wave][m] = v;
  }
  __syncthreads();
  const int m = threadIdx.x;
  const int nin = layer == 0 ? kNNIn : kNNH;
  if (m > kNNH || (m < kNNH && m >= nin)) return;
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) s += part[w][m];
  long long idx;
  if (layer == 0) idx = m < kNNH ? o * kNNIn + m : kNNb1 + o;
  else if (layer == 1) idx = m < kNNH ? kNNW2 + o * kNNH + m : kNNb2 + o;
  else if (layer == 2) idx = m < kNNH ? kNNW3 + o * kNNH + m : kNNb3 + o;
  else idx = m < kNNH ? kNNW4 + m : kNNb4;
  tp.part[(long long)chunk * kNNParams + idx] = s;
}

__global__ void __launch_bounds__(kBlock) k_nn_wgrad_sum(const double* __restrict__ part, double* __restrict__ thb) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= kNNParams) return;
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < kNNChunks; ++c) s += part[c * kNNParams + p];
  thb[p] += s;
}

}  // namespace cfd
