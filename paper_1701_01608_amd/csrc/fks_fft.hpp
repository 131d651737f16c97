// Register-resident mixed-radix DFTs for gfx950 (compile-time lengths 2^a 3^b).
//
// Every loop is a compile-time recursion, so a transform of length n is fully
// unrolled into straight-line VALU code on values held in VGPRs, and each
// twiddle factor is a literal.  Inputs known to be zero (pruned transforms) and
// outputs never read are removed by the compiler; this file is compiled with
// -fno-signed-zeros -ffinite-math-only so that products with the literal 0 and
// 1 twiddle components fold away.
//
// Convention: dft<n, sign>(x) computes X[k] = sum_j x[j] exp(sign * 2 pi i j k / n)
// in place (no scaling); sign = -1 is the forward and +1 the inverse transform.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

namespace fks {

template <typename T>
struct cpx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cpx<T> conj(cpx<T> a) { return {a.re, -a.im}; }
// multiply by sign * i
template <int sign, typename T>
__device__ __forceinline__ cpx<T> mul_si(cpx<T> a) {
  if constexpr (sign > 0) return {-a.im, a.re};
  else return {a.im, -a.re};
}

// ---- compile-time trigonometry (Taylor series on [0, pi/4], octant symmetry) ----
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double taylor_sin(double x) {
  double x2 = x * x, term = x, sum = x;
  for (int i = 1; i < 14; ++i) {
    term *= -x2 / double((2 * i) * (2 * i + 1));
    sum += term;
  }
  return sum;
}
constexpr double taylor_cos(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int i = 1; i < 14; ++i) {
    term *= -x2 / double((2 * i - 1) * (2 * i));
    sum += term;
  }
  return sum;
}

struct sc {
  double c, s;
};

// cos and sin of 2 pi k / n, exact at multiples of pi/2
constexpr sc sincos2pi(long k, long n) {
  k %= n;
  if (k < 0) k += n;
  const long q = (4 * k) / n;      // quadrant
  const long rem = 4 * k - q * n;  // angle inside the quadrant = rem/n * pi/2
  double cb = 1.0, sb = 0.0;
  if (rem != 0) {
    if (2 * rem <= n) {
      const double x = double(rem) / double(n) * (kPi / 2);
      cb = taylor_cos(x);
      sb = taylor_sin(x);
    } else {
      const double x = double(n - rem) / double(n) * (kPi / 2);
      cb = taylor_sin(x);
      sb = taylor_cos(x);
    }
  }
  switch (q) {
    case 0: return {cb, sb};
    case 1: return {-sb, cb};
    case 2: return {-cb, -sb};
    default: return {sb, -cb};
  }
}

// Scheduling fence: no instruction is moved across it.  Used inside long unrolled load
// sequences so that the scheduler does not hoist every load (and its destination
// registers) to the top of the sequence.
__device__ __forceinline__ void sched_fence() { __builtin_amdgcn_sched_barrier(0); }

// ---- static loops ----
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// x * exp(sign * 2 pi i e / n) with e a compile-time exponent
template <int n, int sign, long e, typename T>
__device__ __forceinline__ cpx<T> twiddle(cpx<T> x) {
  constexpr long em = ((e % n) + n) % n;
  if constexpr (em == 0) {
    return x;
  } else if constexpr (4 * em == n) {
    return mul_si<sign>(x);
  } else if constexpr (2 * em == n) {
    return {-x.re, -x.im};
  } else if constexpr (4 * em == 3 * n) {
    return mul_si<-sign>(x);
  } else {
    constexpr sc w = sincos2pi(em, n);
    constexpr T c = T(w.c);
    constexpr T s = T(sign > 0 ? w.s : -w.s);
    return {x.re * c - x.im * s, x.re * s + x.im * c};
  }
}

constexpr int first_radix(int n) { return (n % 4 == 0) ? 4 : ((n % 3 == 0) ? 3 : 2); }
constexpr int pow2_part(int n) { return (n % 2 == 0) ? 2 * pow2_part(n / 2) : 1; }
// inverse of a modulo m (a, m coprime, small)
constexpr int inv_mod(int a, int m) {
  for (int t = 1; t < m; ++t)
    if ((a * t) % m == 1) return t;
  return 1;
}

template <int n, int sign, typename T>
__device__ __forceinline__ void dft(cpx<T>* x);

// Good-Thomas prime-factor DFT for n = N1 N2 with N1 = 2^a, N2 = 3^b coprime: input
// index (N2 n1 + N1 n2) mod n and output index (N2 t1 k1 + N1 t2 k2) mod n (t1 = N2^-1
// mod N1, t2 = N1^-1 mod N2) turn the length-n DFT into an N1 x N2 two-dimensional DFT
// without inter-stage twiddle factors.
template <int n, int sign, typename T>
__device__ __forceinline__ void dft_pfa(cpx<T>* x) {
  constexpr int N1 = pow2_part(n), N2 = n / N1;
  constexpr int t1 = inv_mod(N2 % N1, N1), t2 = inv_mod(N1 % N2, N2);
  cpx<T> a[N2][N1];
  static_for<0, N2>([&](auto i2) {
    static_for<0, N1>([&](auto i1) {
      a[decltype(i2)::value][decltype(i1)::value] = x[(N2 * decltype(i1)::value + N1 * decltype(i2)::value) % n];
    });
    dft<N1, sign>(a[decltype(i2)::value]);
  });
  static_for<0, N1>([&](auto k1) {
    cpx<T> b[N2];
    static_for<0, N2>([&](auto i2) { b[decltype(i2)::value] = a[decltype(i2)::value][decltype(k1)::value]; });
    dft<N2, sign>(b);
    static_for<0, N2>([&](auto k2) {
      x[(N2 * t1 * decltype(k1)::value + N1 * t2 * decltype(k2)::value) % n] = b[decltype(k2)::value];
    });
  });
}

template <int n, int sign, typename T>
__device__ __forceinline__ void dft(cpx<T>* x) {
  static_assert(n >= 1, "bad length");
  if constexpr (n == 1) {
  } else if constexpr (n == 2) {
    const cpx<T> a = x[0], b = x[1];
    x[0] = a + b;
    x[1] = a - b;
  } else if constexpr (n == 3) {
    constexpr T h = T(0.86602540378443864676372317075293618);  // sin(2 pi / 3)
    const cpx<T> a = x[0], t = x[1] + x[2], d = x[1] - x[2];
    const cpx<T> u = {a.re - T(0.5) * t.re, a.im - T(0.5) * t.im};
    const cpx<T> v = mul_si<sign>(cpx<T>{h * d.re, h * d.im});
    x[0] = a + t;
    x[1] = u + v;
    x[2] = u - v;
  } else if constexpr (n == 4) {
    const cpx<T> s02 = x[0] + x[2], d02 = x[0] - x[2];
    const cpx<T> s13 = x[1] + x[3], d13 = mul_si<sign>(x[1] - x[3]);
    x[0] = s02 + s13;
    x[1] = d02 + d13;
    x[2] = s02 - s13;
    x[3] = d02 - d13;
  } else if constexpr (pow2_part(n) > 1 && pow2_part(n) < n) {
    dft_pfa<n, sign>(x);
  } else {
    constexpr int r = first_radix(n);
    constexpr int m = n / r;
    static_assert(r * m == n, "length must be 2^a 3^b");
    cpx<T> sub[r][m];
    static_for<0, r>([&](auto s) {
      static_for<0, m>([&](auto j) { sub[s][j] = x[r * decltype(j)::value + decltype(s)::value]; });
    });
    static_for<0, r>([&](auto s) { dft<m, sign>(sub[decltype(s)::value]); });
    static_for<0, m>([&](auto k) {
      constexpr int kk = decltype(k)::value;
      cpx<T> t[r];
      static_for<0, r>([&](auto s) {
        constexpr int ss = decltype(s)::value;
        t[ss] = twiddle<n, sign, long(ss) * kk>(sub[ss][kk]);
      });
      dft<r, sign>(t);
      static_for<0, r>([&](auto q) { x[kk + m * decltype(q)::value] = t[decltype(q)::value]; });
    });
  }
}

}  // namespace fks

namespace fks {

// Half of an inverse DFT of even length n with pruned input (radix-2 decimation in
// frequency).  Outputs X[2j + h], j < n/2, of X[m] = sum_k c_k exp(+2 pi i k m / n), where
// the only nonzero inputs are c_k for signed k in [-kh, kh] (stored at k mod n) and
// load(i) returns c for k = i - kh.  fold_half forms u[k'] = w^{k' h} (c[k'] + (-1)^h
// c[k' + n/2]) (w = exp(2 pi i / n)); the n/2-point inverse DFT of u then gives the half.
// Only n/2 complex values are live.
template <int n, int kh, int h, typename T, class Load>
__device__ __forceinline__ void fold_half(cpx<T>* u, Load&& load) {
  constexpr int m = n / 2;
  // bin by bin: the (at most two) inputs of u[k'] sit at positions k' and k' + m
  static_for<0, m>([&](auto kk) {
    constexpr int kp = decltype(kk)::value;
    constexpr int p0 = kp, p1 = kp + m;
    constexpr bool has0 = (p0 <= kh) || (p0 >= n - kh);
    constexpr bool has1 = (p1 <= kh) || (p1 >= n - kh);
    constexpr int i0 = (p0 <= kh ? p0 : p0 - n) + kh;
    constexpr int i1 = (p1 <= kh ? p1 : p1 - n) + kh;
    cpx<T> v = {T(0), T(0)};
    if constexpr (has0) v = load(i0);
    if constexpr (has1) {
      const cpx<T> c = load(i1);
      if constexpr (h == 1) v = v - c;
      else v = v + c;
    }
    u[kp] = (h == 1) ? twiddle<n, +1, kp>(v) : v;
    if constexpr (kp % 6 == 5) sched_fence();
  });
}

// The same split into R parts (R divides n): outputs X[R j + h], j < n/R, from the
// n/R-point inverse DFT of u[k'] = w^{k' h} sum_{q < R} c[k' + q n/R] exp(2 pi i q h / R).
// R = 2 is fold_half.  More parts hold fewer values per thread (n/R) at the price of
// every part reading all nonzero inputs.
template <int n, int R, int kh, int h, typename T, class Load, class Pin>
__device__ __forceinline__ void fold_part(cpx<T>* u, Load&& load, Pin&& pin) {
  static_assert(n % R == 0, "parts must divide the length");
  constexpr int m = n / R;
  static_for<0, m>([&](auto kk) {
    constexpr int kp = decltype(kk)::value;
    cpx<T> v = {T(0), T(0)};
    bool any = false;
    static_for<0, R>([&](auto qq) {
      constexpr int q = decltype(qq)::value;
      constexpr int pos = kp + q * m;
      if constexpr ((pos <= kh) || (pos >= n - kh)) {
        constexpr int idx = (pos <= kh ? pos : pos - n) + kh;
        const cpx<T> c = twiddle<R, +1, long(q) * h>(load(idx));
        v = any ? v + c : c;
        any = true;
      }
    });
    u[kp] = twiddle<n, +1, long(kp) * h>(v);
    pin(u[kp], kk);
    if constexpr (kp % 6 == 5) sched_fence();
  });
}
template <int n, int R, int kh, int h, typename T, class Load>
__device__ __forceinline__ void fold_part(cpx<T>* u, Load&& load) {
  fold_part<n, R, kh, h>(u, load, [](const cpx<T>&, auto) {});
}

// Forward (sign -1) counterpart with every input present: outputs Y[R j + h], j < n/R, of
// Y[k] = sum_y a[y] exp(-2 pi i y k / n) from the n/R-point forward DFT of
// u[k'] = w^{-k' h} sum_{q < R} a[k' + q n/R] exp(-2 pi i q h / R); load(i) returns a[i].
template <int n, int R, int h, typename T, class Load>
__device__ __forceinline__ void fold_part_fwd(cpx<T>* u, Load&& load) {
  static_assert(n % R == 0, "parts must divide the length");
  constexpr int m = n / R;
  static_for<0, m>([&](auto kk) {
    constexpr int kp = decltype(kk)::value;
    cpx<T> v = load(kp);
    static_for<1, R>([&](auto qq) {
      constexpr int q = decltype(qq)::value;
      v = v + twiddle<R, -1, long(q) * h>(load(kp + q * m));
    });
    u[kp] = twiddle<n, -1, long(kp) * h>(v);
    if constexpr (kp % 6 == 5) sched_fence();
  });
}

// f(std::integral_constant<int, h>) for a run-time part index h < R, as one if/else chain:
// exactly one part's code runs (independent ifs may be if-converted into selects that
// evaluate every part, with all of their loads live at once)
template <int R, int H = 0, class F>
__device__ __forceinline__ void part_dispatch(int h, F&& f) {
  if constexpr (H == R - 1) {
    f(std::integral_constant<int, H>{});
  } else {
    if (h == H) f(std::integral_constant<int, H>{});
    else part_dispatch<R, H + 1>(h, f);
  }
}

template <int n, int kh, int h, typename T, class Load>
__device__ __forceinline__ void idft_half(cpx<T>* u, Load&& load) {
  fold_half<n, kh, h>(u, load);
  dft<n / 2, +1>(u);
}

// Lowest modes k < nk of the forward DFT (sign -1) of n real samples r[0..n-1], n even,
// by one complex DFT of n/2 packed samples z_j = r_{2j} + i r_{2j+1}.
template <int n, int nk, typename T>
__device__ __forceinline__ void rdft_low(const T* r, cpx<T>* out) {
  constexpr int m = n / 2;
  static_assert(nk <= m, "rdft_low returns at most n/2 modes");
  cpx<T> z[m];
  static_for<0, m>([&](auto j) { z[j] = cpx<T>{r[2 * decltype(j)::value], r[2 * decltype(j)::value + 1]}; });
  dft<m, -1>(z);
  static_for<0, nk>([&](auto kk) {
    constexpr int k = decltype(kk)::value;
    constexpr int kc = (m - k) % m;
    const cpx<T> a = z[k], b = conj(z[kc]);
    const cpx<T> e = {T(0.5) * (a.re + b.re), T(0.5) * (a.im + b.im)};    // even-sample DFT
    const cpx<T> d = {T(0.5) * (a.re - b.re), T(0.5) * (a.im - b.im)};
    const cpx<T> o = {d.im, -d.re};                                         // (a - b) / 2i
    out[k] = e + twiddle<n, -1, k>(o);
  });
}

}  // namespace fks
