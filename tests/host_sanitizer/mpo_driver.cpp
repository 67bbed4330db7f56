// Host driver for the sanitizer build of the MPO builders (mpo.cpp): every
// builder and charge table over a range of chain lengths and interaction
// ranges, each output in a buffer of exactly the announced size, so that
// AddressSanitizer sees any write past it and UndefinedBehaviorSanitizer
// any overflow or bad shift.  Prints "ok" and returns 0 when every call
// succeeds and every invariant below holds.
#include <cmath>
#include <cstdio>
#include <vector>

#include "../../include/dmrg3s.h"

static int fail(const char* what, int l, int range) {
  std::printf("FAIL %s l=%d range=%d\n", what, l, range);
  return 1;
}

int main() {
  for (int l : {1, 2, 3, 5, 8, 17}) {
    for (int range = 1; range <= 5; ++range) {
      std::vector<double> J((size_t)l * range), t((size_t)l * range), mu(l);
      for (size_t i = 0; i < J.size(); ++i) J[i] = t[i] = 0.1 * (double)(i % 7) - 0.2;
      for (int i = 0; i < l; ++i) mu[i] = 0.05 * i;
      for (int kind = 0; kind < 2; ++kind) {
        long total = -1;
        std::vector<long> offsets(l);
        std::vector<int> dims(l + 1);
        d3s_status st = kind == 0 ? d3s_mpo_spin_exchange(l, range, J.data(), nullptr, offsets.data(), dims.data(), &total)
                                  : d3s_mpo_fermion_hopping(l, range, t.data(), 4.0, mu.data(), nullptr, offsets.data(),
                                                            dims.data(), &total);
        if (st != D3S_OK || total <= 0) return fail("size query", l, range);
        if (dims[0] != 1 || dims[l] != 1) return fail("boundary bonds", l, range);
        std::vector<double> out((size_t)total);
        st = kind == 0 ? d3s_mpo_spin_exchange(l, range, J.data(), out.data(), offsets.data(), dims.data(), &total)
                       : d3s_mpo_fermion_hopping(l, range, t.data(), 4.0, mu.data(), out.data(), offsets.data(),
                                                 dims.data(), &total);
        if (st != D3S_OK) return fail("build", l, range);
        const int d = kind == 0 ? 2 : 4;
        long expect = 0;
        for (int i = 0; i < l; ++i) {
          if (offsets[i] != expect) return fail("offsets", l, range);
          expect += (long)dims[i] * dims[i + 1] * d * d;
        }
        if (expect != total) return fail("total", l, range);
        for (double v : out)
          if (!std::isfinite(v)) return fail("finite", l, range);
      }
      const int ws = 2 + 3 * range, wf = 2 + 4 * range;
      std::vector<int> qs(ws), qf(2 * wf);
      if (d3s_mpo_spin_charges(range, qs.data()) != D3S_OK) return fail("spin charges", l, range);
      if (d3s_mpo_fermion_charges(range, qf.data()) != D3S_OK) return fail("fermion charges", l, range);
      if (qs[0] != 0 || qs[ws - 1] != 0 || qf[0] != 0 || qf[2 * wf - 1] != 0) return fail("identity channels", l, range);
    }
  }
  // argument checks
  long total = 0;
  double J = 1.0;
  if (d3s_mpo_spin_exchange(0, 1, &J, nullptr, nullptr, nullptr, &total) != D3S_EINVAL) return fail("l = 0", 0, 1);
  if (d3s_mpo_spin_exchange(3, 0, &J, nullptr, nullptr, nullptr, &total) != D3S_EINVAL) return fail("range 0", 3, 0);
  if (d3s_mpo_spin_charges(0, nullptr) != D3S_EINVAL) return fail("charges range 0", 0, 0);
  std::printf("ok\n");
  return 0;
}
