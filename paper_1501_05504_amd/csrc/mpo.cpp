// MPO builders of the model Hamiltonians (host C++).
//
// Layout: W[w][v][s][t], (w_{i-1}, w_i, d, d), s = output (bra) index.
// Finite-state construction: bond index 0 = "nothing placed yet", the last
// index = "term complete", and for every operator kind k and distance r a
// channel "kind k placed r sites to the left" (index 1 + k*range + r - 1).
// A pair term c_ij A_i B_j (i < j <= i + range) starts with A at site i,
// passes the string operator through the sites in between and is completed
// by c_ij B at site j.  Fermions carry Jordan-Wigner strings F = (-1)^n; the
// starting operators are c+ F (for c+_i c_j) and F c (for c+_j c_i).
#include <cstring>
#include <vector>

#include "../../include/dmrg3s.h"

namespace {

struct Op {
  int d;
  std::vector<double> a;   // d x d, row = out
  explicit Op(int dd) : d(dd), a((size_t)dd * dd, 0.0) {}
  double& at(int s, int t) { return a[(size_t)s * d + t]; }
  double at(int s, int t) const { return a[(size_t)s * d + t]; }
};

Op identity(int d) {
  Op o(d);
  for (int i = 0; i < d; ++i) o.at(i, i) = 1.0;
  return o;
}

Op mul(const Op& x, const Op& y) {
  Op o(x.d);
  for (int i = 0; i < x.d; ++i)
    for (int j = 0; j < x.d; ++j) {
      double s = 0;
      for (int k = 0; k < x.d; ++k) s += x.at(i, k) * y.at(k, j);
      o.at(i, j) = s;
    }
  return o;
}

Op transpose(const Op& x) {
  Op o(x.d);
  for (int i = 0; i < x.d; ++i)
    for (int j = 0; j < x.d; ++j) o.at(i, j) = x.at(j, i);
  return o;
}

Op scaled(const Op& x, double f) {
  Op o = x;
  for (double& v : o.a) v *= f;
  return o;
}

// Generic builder.  coupling(i, r) = amplitude of the pair (i, i + r).
template <typename Coupling, typename Onsite>
d3s_status build(int l, int d, int range, const std::vector<Op>& start, const std::vector<Op>& string,
                 const std::vector<Op>& finish, Coupling coupling, Onsite onsite, double* out, long* offsets,
                 int* dims, long* total) {
  if (l < 1 || range < 1 || !total) return D3S_EINVAL;
  const int nk = (int)start.size();
  const int w = 2 + nk * range;
  const int last = w - 1;
  std::vector<int> wd(l + 1, w);
  wd[0] = 1;
  wd[l] = 1;
  long off = 0;
  std::vector<long> offs(l);
  for (int i = 0; i < l; ++i) {
    offs[i] = off;
    off += (long)wd[i] * wd[i + 1] * d * d;
  }
  *total = off;
  if (dims)
    for (int i = 0; i <= l; ++i) dims[i] = wd[i];
  if (offsets)
    for (int i = 0; i < l; ++i) offsets[i] = offs[i];
  if (!out) return D3S_OK;
  std::memset(out, 0, sizeof(double) * (size_t)off);
  const Op I = identity(d);
  for (int j = 0; j < l; ++j) {
    // full bulk block, then keep the boundary row / column
    std::vector<double> blk((size_t)w * w * d * d, 0.0);
    auto put = [&](int a, int b, const Op& o) {
      for (int s = 0; s < d; ++s)
        for (int t = 0; t < d; ++t) blk[(((size_t)a * w + b) * d + s) * d + t] += o.at(s, t);
    };
    put(0, 0, I);
    put(last, last, I);
    put(0, last, onsite(j));
    for (int k = 0; k < nk; ++k) {
      const int base = 1 + k * range;
      put(0, base, start[k]);
      for (int r = 1; r < range; ++r) put(base + r - 1, base + r, string[k]);
      for (int r = 1; r <= range; ++r) {
        const int i = j - r;
        if (i < 0) continue;
        const double cij = coupling(i, r);
        if (cij != 0.0) put(base + r - 1, last, scaled(finish[k], cij));
      }
    }
    // the first site keeps row 0 only, the last site column `last` only
    const int nr = wd[j], nc = wd[j + 1];
    const int c0 = (j == l - 1) ? last : 0;
    double* dst = out + offs[j];
    for (int a = 0; a < nr; ++a)
      for (int b = 0; b < nc; ++b)
        std::memcpy(dst + (((size_t)a * nc + b) * d) * d, blk.data() + (((size_t)a * w + c0 + b) * d) * d,
                    sizeof(double) * d * d);
  }
  return D3S_OK;
}

}  // namespace

extern "C" {

d3s_status d3s_mpo_spin_exchange(int l, int range, const double* J, double* out, long* offsets, int* dims,
                                 long* total) {
  if (!J) return D3S_EINVAL;
  Op sz(2), sp(2);
  sz.at(0, 0) = 0.5;
  sz.at(1, 1) = -0.5;
  sp.at(0, 1) = 1.0;   // |up><down|
  const Op sm = transpose(sp);
  std::vector<Op> start{sp, sm, sz};
  std::vector<Op> str{identity(2), identity(2), identity(2)};
  std::vector<Op> fin{scaled(sm, 0.5), scaled(sp, 0.5), sz};
  return build(l, 2, range, start, str, fin, [&](int i, int r) { return J[(size_t)i * range + r - 1]; },
               [&](int) { return Op(2); }, out, offsets, dims, total);
}

d3s_status d3s_mpo_fermion_hopping(int l, int range, const double* t, double U, const double* mu, double* out,
                                   long* offsets, int* dims, long* total) {
  if (!t) return D3S_EINVAL;
  // basis 0 = |0>, 1 = |up>, 2 = |dn>, 3 = |updn> = c+_up c+_dn |0>
  Op cu(4), cd(4), F(4);
  cu.at(0, 1) = 1.0;
  cu.at(2, 3) = 1.0;
  cd.at(0, 2) = 1.0;
  cd.at(1, 3) = -1.0;
  F.at(0, 0) = 1.0;
  F.at(1, 1) = -1.0;
  F.at(2, 2) = -1.0;
  F.at(3, 3) = 1.0;
  const Op cuT = transpose(cu), cdT = transpose(cd);
  const Op nu = mul(cuT, cu), nd = mul(cdT, cd);
  const Op nn = mul(nu, nd);
  std::vector<Op> start{mul(cuT, F), mul(cdT, F), mul(F, cu), mul(F, cd)};
  std::vector<Op> str{F, F, F, F};
  std::vector<Op> fin{scaled(cu, -1.0), scaled(cd, -1.0), scaled(cuT, -1.0), scaled(cdT, -1.0)};
  auto onsite = [&](int i) {
    Op o(4);
    const double m = mu ? mu[i] : 0.0;
    for (int s = 0; s < 4; ++s)
      for (int q = 0; q < 4; ++q) o.at(s, q) = U * nn.at(s, q) - m * (nu.at(s, q) + nd.at(s, q));
    return o;
  };
  return build(l, 4, range, start, str, fin, [&](int i, int r) { return t[(size_t)i * range + r - 1]; }, onsite,
               out, offsets, dims, total);
}

/* Channel charges Delta of the MPO bond channels in the builders' channel
 * order (0 = identity before, 1 + k*range + r - 1 = kind k placed r sites
 * before, last = complete).  Spin kinds S+, S-, Sz carry 2Sz = +2, -2, 0
 * (nq = 1); fermion kinds c+_up F, c+_dn F, F c_up, F c_dn carry
 * (N, 2Sz) = (1, 1), (1, -1), (-1, -1), (-1, 1) (nq = 2). */
d3s_status d3s_mpo_spin_charges(int range, int* out) {
  if (range < 1 || !out) return D3S_EINVAL;
  const int kinds[3] = {2, -2, 0};
  const int w = 2 + 3 * range;
  for (int c = 0; c < w; ++c) out[c] = 0;
  for (int k = 0; k < 3; ++k)
    for (int r = 1; r <= range; ++r) out[1 + k * range + r - 1] = kinds[k];
  return D3S_OK;
}

d3s_status d3s_mpo_fermion_charges(int range, int* out) {
  if (range < 1 || !out) return D3S_EINVAL;
  const int kinds[4][2] = {{1, 1}, {1, -1}, {-1, -1}, {-1, 1}};
  const int w = 2 + 4 * range;
  for (int c = 0; c < 2 * w; ++c) out[c] = 0;
  for (int k = 0; k < 4; ++k)
    for (int r = 1; r <= range; ++r) {
      out[2 * (1 + k * range + r - 1)] = kinds[k][0];
      out[2 * (1 + k * range + r - 1) + 1] = kinds[k][1];
    }
  return D3S_OK;
}

}  // extern "C"
