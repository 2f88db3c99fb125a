// Device kernels of the reverse (adjoint) SDC step.
//
// The forward sweep on the active set S (eq. final-sdc, implicit-explicit
// reading), written with I = I(v, w), R = R(v, w) and primes for values at
// the end of the sweep:
//   b_m  = ML (v0 - v_m) + dt sum_j Q[m][j] (-A v_j - ML I(v_j, w_j))
//          - dt ML sum_{j<m} QE[m][j] (I(v'_j, w'_j) - I(v_j, w_j)) - dt A sum_{j<m} QI[m][j] dv_j
//   dv_m = H_m[S,S]^{-1} b_m,     H_m = ML + dt QI[m][m] A
//   dw_m = w0 - w_m + dt sum_j Q[m][j] R(v_j, w_j) + dt sum_{j<m} QE[m][j] (R(v'_j, w'_j) - R(v_j, w_j))
//   v'_m = v_m + dv_m,  w'_m = w_m + dw_m   (on S; unchanged elsewhere)
// The reverse pass visits the nodes m = M-1..0 holding the adjoints Lv_j, Lw_j
// of the sweep's start values (initialised with the adjoints of its end
// values, since v' = v + dv), Ldv_j, Ldw_j of the corrections, Lv0, Lw0 of the
// step's initial state, and per-row / per-element sensitivity accumulators.
#include "kernels.hpp"
#include "device.hpp"

#include <type_traits>

namespace sdc {

namespace {

// Aliev-Panfilov partial derivatives (paper Sec. 5.1) with respect to v, w, a.
__device__ inline void ap_partials(double v, double w, const double* p, double& Iv, double& Iw,
                                   double& Ia, double& Rv, double& Rw, double& Ra) {
  const double k = p[0], a = p[1], eps0 = p[2], mu1 = p[3], mu2 = p[4], s = p[5];
  Iv = k * ((v - a) * (v - 1.0) + v * (v - 1.0) + v * (v - a)) + w;
  Iw = v;
  Ia = -k * v * (v - 1.0);
  const double den = v + mu2;
  const double e = eps0 + mu1 * w / den;
  const double g = -w - k * v * (v - a - 1.0);
  const double e_v = -mu1 * w / (den * den), e_w = mu1 / den;
  const double g_v = -k * (2.0 * v - a - 1.0);
  Rv = s * (e_v * g + e * g_v);
  Rw = s * (e_w * g - e);
  Ra = s * e * k * v;
}

template <class F>
void dispatch_m(int M, F&& f) {
  switch (M) {
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 5: f(std::integral_constant<int, 5>{}); break;
    case 6: f(std::integral_constant<int, 6>{}); break;
    default: break;
  }
}

inline dim3 grid(int n) { return dim3(static_cast<unsigned>(n > 0 ? n : 1)); }

// Sweep start: the corrections inherit the adjoints of the end values (v' = v + dv).
template <int M>
__global__ __launch_bounds__(kBlock) void k_adj_sweep_init(Map map, int64_t N, const double* __restrict__ Lv,
                                                           const double* __restrict__ Lw,
                                                           double* __restrict__ Ldv,
                                                           double* __restrict__ Ldw) {
  const Row rw = map_row(map);
  if (!rw.valid) return;
  const int i = rw.row;
#pragma unroll
  for (int j = 0; j < M; ++j) {
    Ldv[j * N + i] = Lv[j * N + i];
    Ldw[j * N + i] = Lw[j * N + i];
  }
}

// Reverse of dw_m (rows of S).  V, W: start-of-sweep values; Ve, We: end values.
template <int M>
__global__ __launch_bounds__(kBlock) void k_adj_dw(Map map, int m, int64_t N, const double* __restrict__ ionic,
                                                   const double* __restrict__ V, const double* __restrict__ W,
                                                   const double* __restrict__ Ve, const double* __restrict__ We,
                                                   double* Lv, double* Lw, double* Ldv, double* Ldw,
                                                   double* Lw0, double* ga_row, CollArgs c) {
  const Row rw = map_row(map);
  if (!rw.valid) return;
  const int i = rw.row;
  const double* p = ionic + 6 * rw.inst;
  const double mu = Ldw[m * N + i];
  Lw0[i] += mu;
  Lw[m * N + i] -= mu;
  double ga = 0.0;
#pragma unroll
  for (int j = 0; j < M; ++j) {
    const double cs = c.dt * c.Q[m][j] - (j < m ? c.dt * c.QE[m][j] : 0.0);
    double Iv, Iw, Ia, Rv, Rw, Ra;
    ap_partials(V[j * N + i], W[j * N + i], p, Iv, Iw, Ia, Rv, Rw, Ra);
    Lv[j * N + i] += cs * Rv * mu;
    Lw[j * N + i] += cs * Rw * mu;
    ga += cs * Ra * mu;
    if (j < m) {
      const double ce = c.dt * c.QE[m][j];
      ap_partials(Ve[j * N + i], We[j * N + i], p, Iv, Iw, Ia, Rv, Rw, Ra);
      const double cv = ce * Rv * mu, cw = ce * Rw * mu;
      Lv[j * N + i] += cv;
      Ldv[j * N + i] += cv;
      Lw[j * N + i] += cw;
      Ldw[j * N + i] += cw;
      ga += ce * Ra * mu;
    }
  }
  ga_row[i] += ga;
}

// Reverse of b_m given psi = H_m[S,S]^{-1} Ldv_m (zero off S), over all rows
// of the instances: the A-terms reach the neighbours of S.  Also writes
// u_m = -dt sum_j Q[m][j] v_j - dt sum_{j<=m} QI[m][j] dv_j for the
// conductivity sensitivity psi^T (dA/dsigma) u_m.
template <int M, bool DIA>
__global__ __launch_bounds__(kBlock) void k_adj_apsi(Map all, int m, int64_t N, Mat A,
                                                     const double* __restrict__ ml,
                                                     const double* __restrict__ ionic,
                                                     const uint8_t* __restrict__ in_set,
                                                     const double* __restrict__ psi,
                                                     const double* __restrict__ V, const double* __restrict__ W,
                                                     const double* __restrict__ Ve, const double* __restrict__ We,
                                                     const double* __restrict__ DV, double* Lv, double* Lw,
                                                     double* Ldv, double* Ldw, double* Lv0, double* ga_row,
                                                     double* __restrict__ u, CollArgs c) {
  const Row rw = map_row(all);
  if (!rw.valid) return;
  const int i = rw.row;
  double aps = 0.0;
  if constexpr (DIA) {
    const int h = A.nd / 2;   // symmetric diagonal storage, see kernels.hpp
    for (int d = 0; d < A.nd; ++d) {
      const int k = i + rw.off(d);
      const bool in = k >= rw.lo && k < rw.hi;
      const double a = d < h ? (in ? A.dval[(A.nd - 1 - d - h) * N + k] : 0.0) : A.dval[(d - h) * N + i];
      aps += a * psi[in ? k : i];
    }
  } else {
    for (int e = A.rowptr[i]; e < A.rowptr[i + 1]; ++e) aps += A.val[e] * psi[A.col[e]];
  }
  double ui = 0.0;
#pragma unroll
  for (int j = 0; j < M; ++j) {
    ui -= c.dt * c.Q[m][j] * V[j * N + i];
    if (j <= m) ui -= c.dt * c.QI[m][j] * DV[j * N + i];
    Lv[j * N + i] -= c.dt * c.Q[m][j] * aps;
  }
  u[i] = ui;
  if (!in_set[i]) return;
  const double ps = psi[i];
  const double mli = ml[i];
  const double* p = ionic + 6 * rw.inst;
  Lv0[i] += mli * ps;
  Lv[m * N + i] -= mli * ps;
  double ga = 0.0;
#pragma unroll
  for (int j = 0; j < M; ++j) {
    if (j < m) Ldv[j * N + i] -= c.dt * c.QI[m][j] * aps;
    const double cs = -c.dt * c.Q[m][j] * mli + (j < m ? c.dt * c.QE[m][j] * mli : 0.0);
    double Iv, Iw, Ia, Rv, Rw, Ra;
    ap_partials(V[j * N + i], W[j * N + i], p, Iv, Iw, Ia, Rv, Rw, Ra);
    Lv[j * N + i] += ps * cs * Iv;
    Lw[j * N + i] += ps * cs * Iw;
    ga += ps * cs * Ia;
    if (j < m) {
      const double ce = -c.dt * c.QE[m][j] * mli;
      ap_partials(Ve[j * N + i], We[j * N + i], p, Iv, Iw, Ia, Rv, Rw, Ra);
      const double cv = ps * ce * Iv, cw = ps * ce * Iw;
      Lv[j * N + i] += cv;
      Ldv[j * N + i] += cv;
      Lw[j * N + i] += cw;
      Ldw[j * N + i] += cw;
      ga += ps * ce * Ia;
    }
  }
  ga_row[i] += ga;
}

// Per element: q_T += psi_T^T Khat_T u_T = -sum_{a<b} Khat_ab (psi_a - psi_b)(u_a - u_b).
template <int NV>
__global__ __launch_bounds__(kBlock) void k_adj_elem(int64_t ne, const int32_t* __restrict__ elems,
                                                     const double* __restrict__ pairw,
                                                     const double* __restrict__ psi,
                                                     const double* __restrict__ u, double* __restrict__ qe) {
  const int64_t e = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x;
  if (e >= ne) return;
  constexpr int NP = NV * (NV - 1) / 2;
  int vtx[NV];
  double ps[NV];
  bool any = false;
#pragma unroll
  for (int a = 0; a < NV; ++a) {
    vtx[a] = elems[e * NV + a];
    ps[a] = psi[vtx[a]];
    any |= ps[a] != 0.0;
  }
  if (!any) return;
  double us[NV];
#pragma unroll
  for (int a = 0; a < NV; ++a) us[a] = u[vtx[a]];
  double q = 0.0;
  int t = 0;
#pragma unroll
  for (int a = 0; a < NV; ++a)
#pragma unroll
    for (int b = a + 1; b < NV; ++b, ++t) q -= pairw[e * NP + t] * (ps[a] - ps[b]) * (us[a] - us[b]);
  qe[e] += q;
}

// End of the reverse step (all rows): the spread v_j = v0, w_j = w0 of the
// step start passes the node adjoints to the initial state.
template <int M>
__global__ __launch_bounds__(kBlock) void k_adj_spread(int64_t N, const double* __restrict__ Lv,
                                                       const double* __restrict__ Lw, double* Lv0,
                                                       double* Lw0) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x;
  if (i >= N) return;
  double a = Lv0[i], b = Lw0[i];
#pragma unroll
  for (int j = 0; j < M; ++j) {
    a += Lv[j * N + i];
    b += Lw[j * N + i];
  }
  Lv0[i] = a;
  Lw0[i] = b;
}

// g_sigma[n] += sum_{T containing n} q_T / (d + 1)  (node-to-element lists, fixed order).
__global__ __launch_bounds__(kBlock) void k_adj_gather_sigma(int64_t N, int nv, const int32_t* __restrict__ nptr,
                                                             const int32_t* __restrict__ nel,
                                                             const double* __restrict__ qe,
                                                             double* __restrict__ g) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x;
  if (i >= N) return;
  double s = 0.0;
  for (int q = nptr[i]; q < nptr[i + 1]; ++q) s += qe[nel[q]];
  g[i] += s / nv;
}

// g_a[i] += sum of ga_row over instance i's rows (one block per instance).
__global__ __launch_bounds__(kBlock) void k_adj_reduce_a(const int64_t* __restrict__ node_off,
                                                         const double* __restrict__ ga_row,
                                                         double* __restrict__ g_a) {
  __shared__ double sh[kBlock / 64];
  const int inst = blockIdx.x;
  double s = 0.0;
  for (int64_t i = node_off[inst] + threadIdx.x; i < node_off[inst + 1]; i += kBlock) s += ga_row[i];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) g_a[inst] += (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ __launch_bounds__(kBlock) void k_set_flags(Map map, uint8_t* flags, uint8_t value) {
  const Row rw = map_row(map);
  if (rw.valid) flags[rw.row] = value;
}

__global__ void k_zero_values(const int32_t* __restrict__ nodes, int64_t n, double* v) {
  const int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (t < n) v[nodes[t]] = 0.0;
}

}  // namespace

void launch_adj_sweep_init(hipStream_t s, int M, const Map& map, int64_t N, const double* Lv,
                           const double* Lw, double* Ldv, double* Ldw) {
  if (map.nblk <= 0) return;
  dispatch_m(M, [&](auto mm) {
    k_adj_sweep_init<decltype(mm)::value><<<grid(map.nblk), kBlock, 0, s>>>(map, N, Lv, Lw, Ldv, Ldw);
  });
}

void launch_adj_dw(hipStream_t s, int M, int m, const Map& map, int64_t N, const double* ionic,
                   const double* V, const double* W, const double* Ve, const double* We, double* Lv,
                   double* Lw, double* Ldv, double* Ldw, double* Lw0, double* ga_row, const CollArgs& c) {
  if (map.nblk <= 0) return;
  dispatch_m(M, [&](auto mm) {
    k_adj_dw<decltype(mm)::value><<<grid(map.nblk), kBlock, 0, s>>>(map, m, N, ionic, V, W, Ve, We, Lv, Lw,
                                                                   Ldv, Ldw, Lw0, ga_row, c);
  });
}

void launch_adj_apsi(hipStream_t s, int M, int m, const Map& all, int64_t N, const Mat& A,
                     const double* ml, const double* ionic, const uint8_t* in_set, const double* psi,
                     const double* V, const double* W, const double* Ve, const double* We,
                     const double* DV, double* Lv, double* Lw, double* Ldv, double* Ldw, double* Lv0,
                     double* ga_row, double* u, const CollArgs& c) {
  if (all.nblk <= 0) return;
  dispatch_m(M, [&](auto mm) {
    if (A.nd > 0)
      k_adj_apsi<decltype(mm)::value, true><<<grid(all.nblk), kBlock, 0, s>>>(
          all, m, N, A, ml, ionic, in_set, psi, V, W, Ve, We, DV, Lv, Lw, Ldv, Ldw, Lv0, ga_row, u, c);
    else
      k_adj_apsi<decltype(mm)::value, false><<<grid(all.nblk), kBlock, 0, s>>>(
          all, m, N, A, ml, ionic, in_set, psi, V, W, Ve, We, DV, Lv, Lw, Ldv, Ldw, Lv0, ga_row, u, c);
  });
}

void launch_adj_elem(hipStream_t s, int nv, int64_t ne, const int32_t* elems, const double* pairw,
                     const double* psi, const double* u, double* qe) {
  if (ne <= 0) return;
  const dim3 g(static_cast<unsigned>((ne + kBlock - 1) / kBlock));
  switch (nv) {
    case 2: k_adj_elem<2><<<g, kBlock, 0, s>>>(ne, elems, pairw, psi, u, qe); break;
    case 3: k_adj_elem<3><<<g, kBlock, 0, s>>>(ne, elems, pairw, psi, u, qe); break;
    case 4: k_adj_elem<4><<<g, kBlock, 0, s>>>(ne, elems, pairw, psi, u, qe); break;
    default: break;
  }
}

void launch_adj_spread(hipStream_t s, int M, int64_t N, const double* Lv, const double* Lw, double* Lv0,
                       double* Lw0) {
  const dim3 g(static_cast<unsigned>((N + kBlock - 1) / kBlock));
  dispatch_m(M, [&](auto mm) { k_adj_spread<decltype(mm)::value><<<g, kBlock, 0, s>>>(N, Lv, Lw, Lv0, Lw0); });
}

void launch_adj_gather_sigma(hipStream_t s, int64_t N, int nv, const int32_t* nptr, const int32_t* nel,
                             const double* qe, double* g) {
  k_adj_gather_sigma<<<dim3(static_cast<unsigned>((N + kBlock - 1) / kBlock)), kBlock, 0, s>>>(N, nv, nptr, nel,
                                                                                              qe, g);
}

void launch_adj_reduce_a(hipStream_t s, int n_inst, const int64_t* node_off, const double* ga_row, double* g_a) {
  k_adj_reduce_a<<<dim3(static_cast<unsigned>(n_inst)), kBlock, 0, s>>>(node_off, ga_row, g_a);
}

void launch_set_flags(hipStream_t s, const Map& map, uint8_t* flags, uint8_t value) {
  if (map.nblk <= 0) return;
  k_set_flags<<<grid(map.nblk), kBlock, 0, s>>>(map, flags, value);
}

void launch_zero_values(hipStream_t s, const int32_t* nodes, int64_t n, double* v) {
  if (n <= 0) return;
  k_zero_values<<<dim3(static_cast<unsigned>((n + 255) / 256)), 256, 0, s>>>(nodes, n, v);
}

}  // namespace sdc
