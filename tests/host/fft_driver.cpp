// Host driver for the library's Stockham butterflies (csrc/fft_core.h):
// reads "N dir order with9" then N complex values (re im) from stdin and runs every
// pass of the plan on the CPU the way the kernels do, in place: each pass
// reads all of its butterflies (stockham_read, with k = j mod Ns split by the
// kernels' FP32 reciprocal, twiddles from the plan's pass tables) before
// writing their outputs over the input.
// Prints the transform; tests/test_fft_host.py checks it against numpy.fft.
#include <cmath>
#include <cstdio>
#include <vector>

#include "fft_core.h"

using namespace cbp;

template <int R, int DIR>
void pass(std::vector<cplx<double>>& buf, int N, int Ns, const cplx<double>* tw) {
  const int NR = N / R;
  const float rns = 1.0f / (float)Ns;
  std::vector<cplx<double>> out(N);
  std::vector<int> base(NR);
  std::vector<cplx<double>> v((size_t)NR * R);
  for (int j = 0; j < NR; ++j) {
    const int k = j - fdiv_floor(j, rns) * Ns;
    base[j] = Ns > 1 ? stockham_read<R, DIR, true>(buf.data(), NR, tw, j, k, &v[(size_t)j * R])
                     : stockham_read<R, DIR, false>(buf.data(), NR, tw, j, k, &v[(size_t)j * R]);
  }
  for (int j = 0; j < NR; ++j)
    for (int r = 0; r < R; ++r) buf[base[j] + r * Ns] = v[(size_t)j * R + r];
}

template <int DIR>
void run_pass(int R, std::vector<cplx<double>>& buf, int N, int Ns, const cplx<double>* tw) {
  switch (R) {
    case 2: pass<2, DIR>(buf, N, Ns, tw); break;
    case 3: pass<3, DIR>(buf, N, Ns, tw); break;
    case 4: pass<4, DIR>(buf, N, Ns, tw); break;
    case 5: pass<5, DIR>(buf, N, Ns, tw); break;
    case 7: pass<7, DIR>(buf, N, Ns, tw); break;
    case 9: pass<9, DIR>(buf, N, Ns, tw); break;
    default: pass<8, DIR>(buf, N, Ns, tw); break;
  }
}

int main() {
  int N, dir, order, with9;
  if (std::scanf("%d %d %d %d", &N, &dir, &order, &with9) != 4) return 2;
  fft_plan p;
  if (!make_fft_plan(N, &p, order, with9 != 0)) { std::printf("BADPLAN\n"); return 3; }
  std::vector<cplx<double>> a(N);
  for (int i = 0; i < N; ++i)
    if (std::scanf("%lf %lf", &a[i].re, &a[i].im) != 2) return 2;
  // the pass tables (fft_core.h tw_pitch), padding entries poisoned: a read
  // of one spoils the transform
  std::vector<cplx<double>> tw((size_t)pass_table_entries(p) + 1);
  {
    int Ns = 1;
    size_t off = 0;
    for (int s = 0; s < p.npass; ++s) {
      const int R = plan_radix(p, s), P = tw_pitch(R);
      if (Ns > 1) {
        for (int k = 0; k < Ns; ++k)
          for (int r = 1; r <= P; ++r) {
            const double ang = -2.0 * M_PI * (double)(r * k) / (double)(Ns * R);
            tw[off + (size_t)k * P + r - 1] = r < R ? cplx<double>{std::cos(ang), std::sin(ang)}
                                                    : cplx<double>{NAN, NAN};
          }
        off += (size_t)Ns * P;
      }
      Ns *= R;
    }
    if (off != tw.size() - 1) return 4;
  }
  int Ns = 1;
  size_t off = 0;
  for (int s = 0; s < p.npass; ++s) {
    const int R = plan_radix(p, s);
    if (dir < 0) run_pass<-1>(R, a, N, Ns, tw.data() + off);
    else run_pass<+1>(R, a, N, Ns, tw.data() + off);
    if (Ns > 1) off += (size_t)Ns * tw_pitch(R);
    Ns *= R;
  }
  for (int i = 0; i < N; ++i) std::printf("%.17g %.17g\n", a[i].re, a[i].im);
  return 0;
}
