// CPU driver for the library's multiple-double arithmetic (md.hpp, compiled
// for the host): reads cases "m count" then per case the limbs of s, a, b
// (complex: s.re, s.im, a.re, a.im, b.re, b.im, m limbs each, hex floats),
// prints per case c_fmadd(s, a, b) (re, im), c_add(s, c_mul(a, b)) (re, im)
// and md_mul(a.re, b.re), m limbs each, hex floats.
#include <cstdio>
#include <cstdlib>

#include "md.hpp"

using namespace mds;

template <int M>
static void run(int count) {
  for (int t = 0; t < count; ++t) {
    mdr<M> v[6];
    for (auto &x : v)
      for (int i = 0; i < M; ++i)
        if (scanf("%la", &x.v[i]) != 1) exit(2);
    const mdc<M> s{v[0], v[1]}, a{v[2], v[3]}, b{v[4], v[5]};
    const mdc<M> f = c_fmadd<M>(s, a, b), u = c_add<M>(s, c_mul<M>(a, b));
    const mdr<M> p = md_mul<M>(a.re, b.re);
    const mdr<M> out[5] = {f.re, f.im, u.re, u.im, p};
    for (const auto &x : out)
      for (int i = 0; i < M; ++i) printf("%a ", x.v[i]);
    printf("\n");
  }
}

int main() {
  int m, count;
  while (scanf("%d %d", &m, &count) == 2) {
    switch (m) {
      case 2: run<2>(count); break;
      case 3: run<3>(count); break;
      case 4: run<4>(count); break;
      case 5: run<5>(count); break;
      case 8: run<8>(count); break;
      case 10: run<10>(count); break;
      default: return 1;
    }
  }
  return 0;
}
