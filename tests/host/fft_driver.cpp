// Host driver for the library's Stockham FFT passes (csrc/fft_core.h):
// reads "N dir order split" then N complex values (re im) from stdin, runs
// every pass of the plan sequentially on the CPU (twiddles from the full table,
// or with split = 1 from tw_split's two short tables) and prints the
// transform.  Used by tests/test_fft_host.py to check the butterflies against
// numpy.fft.
#include <cmath>
#include <cstdio>
#include <vector>

#include "fft_core.h"

using namespace cbp;

int main() {
  int N, dir, order, split;
  if (std::scanf("%d %d %d %d", &N, &dir, &order, &split) != 4) return 2;
  fft_plan p;
  if (!make_fft_plan(N, &p, order)) { std::printf("BADPLAN\n"); return 3; }
  std::vector<cplx<double>> a(N), b(N), tw(N);
  for (int i = 0; i < N; ++i)
    if (std::scanf("%lf %lf", &a[i].re, &a[i].im) != 2) return 2;
  for (int t = 0; t < N; ++t) {
    const double ang = -2.0 * M_PI * (double)t / (double)N;
    tw[t] = {std::cos(ang), std::sin(ang)};
  }
  std::vector<cplx<double>> lo(64), hi((N + 63) / 64);
  for (int i = 0; i < 64; ++i) {
    const double ang = -2.0 * M_PI * (double)i / (double)N;
    lo[i] = {std::cos(ang), std::sin(ang)};
  }
  for (int j = 0; j < (int)hi.size(); ++j) {
    const double ang = -2.0 * M_PI * (double)(64 * j) / (double)N;
    hi[j] = {std::cos(ang), std::sin(ang)};
  }
  const tw_split<double> ts{lo.data(), hi.data()};
  const cplx<double>* full = tw.data();
  cplx<double>* src = a.data();
  cplx<double>* dst = b.data();
  int Ns = 1;
  for (int s = 0; s < p.npass; ++s) {
    const int R = plan_radix(p, s);
    if (split) {
      if (dir < 0) fft_pass<-1>(src, dst, N, R, Ns, ts, 1, N, 0, 1);
      else fft_pass<+1>(src, dst, N, R, Ns, ts, 1, N, 0, 1);
    } else {
      if (dir < 0) fft_pass<-1>(src, dst, N, R, Ns, full, 1, N, 0, 1);
      else fft_pass<+1>(src, dst, N, R, Ns, full, 1, N, 0, 1);
    }
    Ns *= R;
    cplx<double>* t = src; src = dst; dst = t;
  }
  for (int i = 0; i < N; ++i) std::printf("%.17g %.17g\n", src[i].re, src[i].im);
  return 0;
}
