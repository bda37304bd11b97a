// Host driver for the library's Stockham FFT passes (csrc/fft_core.h):
// reads "N dir order" then N complex values (re im) from stdin, runs every pass of
// the plan sequentially on the CPU and prints the transform.  Used by
// tests/test_fft_host.py to check the butterflies against numpy.fft.
#include <cmath>
#include <cstdio>
#include <vector>

#include "fft_core.h"

using namespace cbp;

int main() {
  int N, dir, order;
  if (std::scanf("%d %d %d", &N, &dir, &order) != 3) return 2;
  fft_plan p;
  if (!make_fft_plan(N, &p, order)) { std::printf("BADPLAN\n"); return 3; }
  std::vector<cplx<double>> a(N), b(N), tw(N);
  for (int i = 0; i < N; ++i)
    if (std::scanf("%lf %lf", &a[i].re, &a[i].im) != 2) return 2;
  for (int t = 0; t < N; ++t) {
    const double ang = -2.0 * M_PI * (double)t / (double)N;
    tw[t] = {std::cos(ang), std::sin(ang)};
  }
  cplx<double>* src = a.data();
  cplx<double>* dst = b.data();
  int Ns = 1;
  for (int s = 0; s < p.npass; ++s) {
    if (dir < 0) fft_pass<-1>(src, dst, N, plan_radix(p, s), Ns, tw.data(), 1, N, 0, 1);
    else fft_pass<+1>(src, dst, N, plan_radix(p, s), Ns, tw.data(), 1, N, 0, 1);
    Ns *= plan_radix(p, s);
    cplx<double>* t = src; src = dst; dst = t;
  }
  for (int i = 0; i < N; ++i) std::printf("%.17g %.17g\n", src[i].re, src[i].im);
  return 0;
}
