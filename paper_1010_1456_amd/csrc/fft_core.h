// Register-level FFT building blocks for the grid passes.
//
// A length-P transform is factored into stages of radix r (Stockham
// autosort). With L the product of the radices already applied and
// M' = P / (L r), butterfly beta = j M' + k' (j < L, k' < M') of a stage reads
//     x[j r M' + q M' + k'],               q = 0..r-1,
// multiplies element q by exp(-+2 pi i j q M' / P), applies a length-r DFT and
// writes element p to
//     x[(j + L p) M' + k'],                p = 0..r-1.
// The first stage (L = 1) reads plain strided input; the last (M' = 1) writes
// natural order. Small DFTs are unrolled at compile time: primes 2, 3, 5, 7
// directly, composite radices as two smaller DFTs (prime-factor split for
// coprime factors, else with compile-time twiddles).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#define AIM_AI __attribute__((always_inline))

namespace aim {
namespace fftc {

// ---- compile-time trigonometry (Taylor series after reduction to [-pi, pi])
constexpr double kPiD = 3.14159265358979323846264338327950288;

constexpr double ce_reduce(double x) {
  while (x > kPiD) x -= 2.0 * kPiD;
  while (x < -kPiD) x += 2.0 * kPiD;
  return x;
}
constexpr double ce_sin(double x) {
  x = ce_reduce(x);
  double term = x, sum = x;
  for (int n = 1; n < 30; ++n) {
    term *= -x * x / ((2.0 * n) * (2.0 * n + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double ce_cos(double x) {
  x = ce_reduce(x);
  double term = 1.0, sum = 1.0;
  for (int n = 1; n < 30; ++n) {
    term *= -x * x / ((2.0 * n - 1.0) * (2.0 * n));
    sum += term;
  }
  return sum;
}

template <int N, typename F, int... Is>
__host__ __device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, typename F>
__host__ __device__ __forceinline__ void static_for(F &&f) {
  static_for_impl<N>(f, std::make_integer_sequence<int, N>{});
}

template <typename V>
struct real_of;
template <>
struct real_of<float2> {
  using type = float;
};
template <>
struct real_of<double2> {
  using type = double;
};

template <typename V>
__host__ __device__ __forceinline__ V mk(typename real_of<V>::type x, typename real_of<V>::type y) {
  V v;
  v.x = x;
  v.y = y;
  return v;
}
template <typename V>
__host__ __device__ __forceinline__ V add(V a, V b) {
  return mk<V>(a.x + b.x, a.y + b.y);
}
template <typename V>
__host__ __device__ __forceinline__ V sub(V a, V b) {
  return mk<V>(a.x - b.x, a.y - b.y);
}
template <typename V>
__host__ __device__ __forceinline__ V cmul(V a, V b) {
  return mk<V>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename V>
__host__ __device__ __forceinline__ V cmulc(V a, V b) {  // a * conj(b)
  return mk<V>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
// multiply by -i (forward sense) or +i (inverse sense)
template <bool INV, typename V>
__host__ __device__ __forceinline__ V mul_mi(V a) {
  return INV ? mk<V>(-a.y, a.x) : mk<V>(a.y, -a.x);
}

// a * exp(-+ 2 pi i E / R), E and R compile-time
template <int R, int E, bool INV, typename V>
__host__ __device__ __forceinline__ V twc(V a) {
  using T = typename real_of<V>::type;
  constexpr int e = ((E % R) + R) % R;
  if constexpr (e == 0) {
    return a;
  } else if constexpr (2 * e == R) {
    return mk<V>(-a.x, -a.y);
  } else if constexpr (4 * e == R) {
    return mul_mi<INV>(a);
  } else if constexpr (4 * e == 3 * R) {
    return mul_mi<!INV>(a);
  } else {
    constexpr double ang = 2.0 * kPiD * (double)e / (double)R;
    constexpr double c = ce_cos(ang);
    constexpr double s = INV ? ce_sin(ang) : -ce_sin(ang);
    return mk<V>((T)c * a.x - (T)s * a.y, (T)c * a.y + (T)s * a.x);
  }
}

constexpr int smallest_factor(int n) {
  for (int f = 2; f * f <= n; ++f)
    if (n % f == 0) return f;
  return n;
}

template <int R, bool INV, typename V, typename Enable = void>
struct Dft;

template <bool INV, typename V>
struct Dft<1, INV, V> {
  __host__ __device__ __forceinline__ static void run(V *) {}
};

template <bool INV, typename V>
struct Dft<2, INV, V> {
  __host__ __device__ __forceinline__ static void run(V *v) {
    V a = v[0], b = v[1];
    v[0] = add(a, b);
    v[1] = sub(a, b);
  }
};

template <bool INV, typename V>
struct Dft<3, INV, V> {
  __host__ __device__ __forceinline__ static void run(V *v) {
    using T = typename real_of<V>::type;
    const T s3 = (T)0.86602540378443864676372317075294;
    V t1 = add(v[1], v[2]);
    V d = sub(v[1], v[2]);
    V t2 = mk<V>(v[0].x - (T)0.5 * t1.x, v[0].y - (T)0.5 * t1.y);
    // X1, X2 = t2 -+ i s3 d (forward) / t2 +- i s3 d (inverse); written as
    // multiply-adds so the scaled difference is never formed on its own
    const T sg = INV ? -s3 : s3;
    v[0] = add(v[0], t1);
    v[1] = mk<V>(t2.x + sg * d.y, t2.y - sg * d.x);
    v[2] = mk<V>(t2.x - sg * d.y, t2.y + sg * d.x);
  }
};

// odd prime R: symmetric pairs a_m = v_m + v_{R-m}, b_m = v_m - v_{R-m};
// X_k = v0 + sum_m a_m cos(2 pi k m / R) -+ i sum_m b_m sin(2 pi k m / R)
template <int R, bool INV, typename V>
struct DftOddPrime {
  __host__ __device__ __forceinline__ static void run(V *v) {
    using T = typename real_of<V>::type;
    constexpr int H = (R - 1) / 2;
    V a[H], b[H];
    static_for<H>([&](auto m_) AIM_AI {
      constexpr int m = decltype(m_)::value + 1;
      a[m - 1] = add(v[m], v[R - m]);
      b[m - 1] = sub(v[m], v[R - m]);
    });
    V x0 = v[0];
    V sum = x0;
    static_for<H>([&](auto m_) AIM_AI { sum = add(sum, a[decltype(m_)::value]); });
    V out[R];
    out[0] = sum;
    static_for<H>([&](auto k_) AIM_AI {
      constexpr int k = decltype(k_)::value + 1;
      V re = x0, im = mk<V>((T)0, (T)0);
      static_for<H>([&](auto m_) AIM_AI {
        constexpr int m = decltype(m_)::value + 1;
        constexpr double c = ce_cos(2.0 * kPiD * (double)(k * m % R) / (double)R);
        constexpr double s = ce_sin(2.0 * kPiD * (double)(k * m % R) / (double)R);
        re = mk<V>(re.x + (T)c * a[m - 1].x, re.y + (T)c * a[m - 1].y);
        im = mk<V>(im.x + (T)s * b[m - 1].x, im.y + (T)s * b[m - 1].y);
      });
      V rot = mul_mi<INV>(im);  // -+ i * im
      out[k] = add(re, rot);
      out[R - k] = sub(re, rot);
    });
    static_for<R>([&](auto i_) AIM_AI { v[decltype(i_)::value] = out[decltype(i_)::value]; });
  }
};

template <bool INV, typename V>
struct Dft<5, INV, V> : DftOddPrime<5, INV, V> {};
template <bool INV, typename V>
struct Dft<7, INV, V> : DftOddPrime<7, INV, V> {};

constexpr int prime_power_part(int n, int p) {
  int q = 1;
  while (n % p == 0) {
    n /= p;
    q *= p;
  }
  return q;
}
constexpr int inverse_mod(int a, int m) {  // a^-1 mod m for coprime a, m (m > 1)
  for (int x = 1; x < m; ++x)
    if ((a * x) % m == 1) return x;
  return 0;
}

// composite R. With N1 the power of R's smallest prime and N2 = R / N1:
//  * N2 > 1 (coprime factors): prime-factor (Good-Thomas) split. Input n =
//    (N2 n1 + N1 n2) mod R, N2 DFTs of length N1 over n1, then N1 DFTs of
//    length N2 over n2; output k = (N2 t1 k1 + N1 t2 k2) mod R with
//    t1 = N2^-1 mod N1, t2 = N1^-1 mod N2 (Chinese remainder indexing). The
//    cross terms of n k are multiples of R, so no twiddles are needed
//    between the layers.
//  * N2 = 1 (prime power): Cooley-Tukey split A * B, A the prime: stage 1
//    runs B DFTs of length A (L = 1, M' = B), stage 2 runs A DFTs of length
//    B (L = A, M' = 1) after compile-time twiddles.
template <int R, bool INV, typename V>
struct Dft<R, INV, V, std::enable_if_t<(R > 3 && smallest_factor(R) != R)>> {
  static constexpr int p = smallest_factor(R);
  static constexpr int N1 = prime_power_part(R, p);
  static constexpr int N2 = R / N1;

  __host__ __device__ __forceinline__ static void run(V *v) {
    if constexpr (N2 > 1) {
      constexpr int t1 = inverse_mod(N2 % N1, N1), t2 = inverse_mod(N1 % N2, N2);
      V a[N1 * N2];  // a[k1 N2 + n2]
      static_for<N2>([&](auto n2_) AIM_AI {
        constexpr int n2 = decltype(n2_)::value;
        V s[N1];
        static_for<N1>([&](auto n1_) AIM_AI {
          constexpr int n1 = decltype(n1_)::value;
          s[n1] = v[(N2 * n1 + N1 * n2) % R];
        });
        Dft<N1, INV, V>::run(s);
        static_for<N1>([&](auto k1_) AIM_AI { a[decltype(k1_)::value * N2 + n2] = s[decltype(k1_)::value]; });
      });
      static_for<N1>([&](auto k1_) AIM_AI {
        constexpr int k1 = decltype(k1_)::value;
        V s[N2];
        static_for<N2>([&](auto n2_) AIM_AI { s[decltype(n2_)::value] = a[k1 * N2 + decltype(n2_)::value]; });
        Dft<N2, INV, V>::run(s);
        static_for<N2>([&](auto k2_) AIM_AI {
          constexpr int k2 = decltype(k2_)::value;
          v[(N2 * t1 * k1 + N1 * t2 * k2) % R] = s[k2];
        });
      });
    } else {
      constexpr int A = p;
      constexpr int B = R / A;
      V u[R];
      static_for<B>([&](auto kp_) AIM_AI {
        constexpr int kp = decltype(kp_)::value;
        V s[A];
        static_for<A>([&](auto q_) AIM_AI { s[decltype(q_)::value] = v[decltype(q_)::value * B + kp]; });
        Dft<A, INV, V>::run(s);
        static_for<A>([&](auto p_) AIM_AI { u[decltype(p_)::value * B + kp] = s[decltype(p_)::value]; });
      });
      static_for<A>([&](auto j_) AIM_AI {
        constexpr int j = decltype(j_)::value;
        V s[B];
        static_for<B>([&](auto q_) AIM_AI {
          constexpr int q = decltype(q_)::value;
          s[q] = twc<R, j * q, INV>(u[j * B + q]);
        });
        Dft<B, INV, V>::run(s);
        static_for<B>([&](auto p_) AIM_AI { v[j + A * decltype(p_)::value] = s[decltype(p_)::value]; });
      });
    }
  }
};

// Length-R DFT (R even) of a vector whose upper half v[R/2..R-1] is zero and
// is not read. Outputs in natural order as Dft<R>::run.
//  * R = 2 * odd: prime-factor split with N1 = 2. Each length-2 DFT pairs
//    inputs n and n + R/2, exactly one of which lies in the lower half, so
//    the layer reduces to copies and sign changes, leaving two DFTs of
//    length R/2.
//  * R divisible by 4: the radix-2 first layer of the Cooley-Tukey split
//    degenerates to copies, leaving the two half-length DFTs of v and of v
//    twisted by exp(-+ 2 pi i q / R).
template <int R, bool INV, typename V>
__host__ __device__ __forceinline__ void dft_upper_zero(V *v) {
  static_assert(R % 2 == 0, "upper-half-zero DFT needs an even length");
  constexpr int B = R / 2;
  if constexpr (R == 2) {
    v[1] = v[0];
  } else if constexpr (B % 2 == 1) {
    constexpr int t2 = inverse_mod(2 % B, B);
    V e[B], o[B];
    static_for<B>([&](auto n2_) AIM_AI {
      constexpr int n2 = decltype(n2_)::value;
      constexpr int i0 = (2 * n2) % R;  // n1 = 0; n1 = 1 is i0 + B mod R
      if constexpr (i0 < B) {           // (x_i0 + 0, x_i0 - 0)
        e[n2] = v[i0];
        o[n2] = v[i0];
      } else {                          // (0 + x_i1, 0 - x_i1)
        constexpr int i1 = (B + 2 * n2) % R;
        e[n2] = v[i1];
        o[n2] = mk<V>(-v[i1].x, -v[i1].y);
      }
    });
    Dft<B, INV, V>::run(e);
    Dft<B, INV, V>::run(o);
    // k = (B t1 k1 + 2 t2 k2) mod R with t1 = B^-1 mod 2 = 1
    static_for<B>([&](auto k2_) AIM_AI {
      constexpr int k2 = decltype(k2_)::value;
      v[(2 * t2 * k2) % R] = e[k2];
      v[(B + 2 * t2 * k2) % R] = o[k2];
    });
  } else {
    V e[B], o[B];
    static_for<B>([&](auto q_) AIM_AI {
      constexpr int q = decltype(q_)::value;
      e[q] = v[q];
      o[q] = twc<R, q, INV>(v[q]);
    });
    Dft<B, INV, V>::run(e);
    Dft<B, INV, V>::run(o);
    static_for<B>([&](auto p_) AIM_AI {
      constexpr int p = decltype(p_)::value;
      v[2 * p] = e[p];
      v[2 * p + 1] = o[p];
    });
  }
}

// Twiddle exp(-+ 2 pi i e / P) from a table of exp(-2 pi i e / P).
template <bool INV, typename V>
__host__ __device__ __forceinline__ V tw_mul(V a, const V *tw, int e) {
  V w = tw[e];
  return INV ? cmulc(a, w) : cmul(a, w);
}

// One Stockham stage for butterfly beta. ld(i) / st(i, v) access element i
// of the line. Barrier placement is the caller's.
template <int R, bool INV, typename V, class Ld>
__device__ __forceinline__ void stage_load(V *v, int beta, int Mp, Ld &ld) {
  int j = beta / Mp, kp = beta - j * Mp;
  int base = j * R * Mp + kp;
  static_for<R>([&](auto q_) AIM_AI { v[decltype(q_)::value] = ld(base + decltype(q_)::value * Mp); });
}
// first NIN inputs only (the others are known to be zero)
template <int R, int NIN, typename V, class Ld>
__device__ __forceinline__ void stage_load_p(V *v, int beta, int Mp, Ld &ld) {
  int j = beta / Mp, kp = beta - j * Mp;
  int base = j * R * Mp + kp;
  static_for<NIN>([&](auto q_) AIM_AI { v[decltype(q_)::value] = ld(base + decltype(q_)::value * Mp); });
}

// UZ: the upper half of the butterfly's inputs is zero (first stage of a
// transform whose line holds at most P/2 inputs, R even). NOUT: only outputs
// p < NOUT are stored (last stage of a transform of which at most the first
// P/2 outputs are kept: NOUT = R/2); the rest is never computed. ROWS: tw is
// a per-stage table of rows tw[j (R - 1) + q - 1] = exp(-2 pi i j M' q / P)
// (one row per butterfly group j, so a thread reads its twiddles at fixed
// offsets from one address) instead of the table of exp(-2 pi i e / P).
template <int R, bool INV, bool UZ, int NOUT, bool ROWS, typename V, class St>
__device__ __forceinline__ void stage_compute_store_p(V *v, int beta, int L, int Mp, const V *tw,
                                                      St &st) {
  int j = beta / Mp, kp = beta - j * Mp;
  if (L > 1) {
    if constexpr (ROWS) {
      const V *row = tw + j * (R - 1);
      static_for<R - 1>([&](auto q_) AIM_AI {
        constexpr int q = decltype(q_)::value + 1;
        v[q] = tw_mul<INV>(v[q], row, q - 1);
      });
    } else {
      int step = j * Mp;
      static_for<R - 1>([&](auto q_) AIM_AI {
        constexpr int q = decltype(q_)::value + 1;
        v[q] = tw_mul<INV>(v[q], tw, step * q);
      });
    }
  }
  if constexpr (UZ) dft_upper_zero<R, INV, V>(v);
  else Dft<R, INV, V>::run(v);
  static_for<NOUT>([&](auto p_) AIM_AI {
    constexpr int p = decltype(p_)::value;
    st((j + L * p) * Mp + kp, v[p]);
  });
}
template <int R, bool INV, typename V, class St>
__device__ __forceinline__ void stage_compute_store(V *v, int beta, int L, int Mp, const V *tw,
                                                    St &st) {
  stage_compute_store_p<R, INV, false, R, false>(v, beta, L, Mp, tw, st);
}

// Supported radices; the dispatch macro expands a body once per radix with
// the constant RADIX defined.
#define AIM_FOR_EACH_RADIX(X) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(12) X(14) X(16) X(18)

}  // namespace fftc
}  // namespace aim
