// zeus_user_elem.h -- hands a user objective (the function template
// `objective` defined by the user's source, see zeus_user.h) to the kernels
// as the whole-form objective kUser.  Included by the run-time program after
// the user's source; not part of the library build.
#pragma once

#include "zeus_user.h"

namespace zeus {

template <>
struct Elem<kUser> {
  static constexpr int K = 1, W = 1;
  static constexpr bool kWhole = true;
  __host__ __device__ __forceinline__ static int terms(int) { return 1; }
  // In number type T (double, or float for the FP32 evaluations of mixed
  // precision), returned as a double.
  // f at the point xs[0..d)
  template <class T>
  __device__ __forceinline__ static double value(const double *xs, int d) {
    using N = UserNum<T>;
    return N::val(::objective<typename N::S>(PlainView<T>{xs}, d));
  }
  // f and df/dx_j (pass j of Alg. 5; j < 0: no seed, *g = 0)
  template <class T>
  __device__ __forceinline__ static double value_grad(const double *xs, int d, int j, double *g) {
    using N = UserNum<T>;
    const typename N::D r = ::objective<typename N::D>(SeededView<T>{xs, j}, d);
    *g = N::tan(r);
    return N::val(r);
  }
  // f at the trial point xs + alpha ps
  template <class T>
  __device__ __forceinline__ static double trial(const double *xs, const double *ps, double alpha,
                                                 int d) {
    using N = UserNum<T>;
    return N::val(::objective<typename N::S>(TrialView<T>{xs, ps, alpha}, d));
  }
};

}  // namespace zeus
