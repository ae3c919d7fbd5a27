"""User-defined objectives without a GPU: every example source compiles for
gfx950 through the library's run-time compiler (the embedded kernel
templates included), a broken source is refused with the compiler's message, a source that is
not generic over the number type (FP64 overloads only) is refused because the
mixed-precision instantiations need the FP32 types too, and the entry points
other than zeus_minimize_user refuse ZEUS_USER."""
import pytest

from paper_2603_28770_amd import user_objectives as UO
from paper_2603_28770_amd import workloads as W


@pytest.fixture(scope="module")
def Z():
    from paper_2603_28770_amd import zeus
    return zeus


@pytest.mark.parametrize("name", ["ROSENBROCK", "GOLDSTEIN_PRICE", "RASTRIGIN", "CHAIN_LOG", "poisson"])
def test_example_sources_compile(Z, name):
    src = UO.poisson_fit_source() if name == "poisson" else getattr(UO, name)
    Z.zeus_objective_check(src)


def test_broken_source_is_refused_with_message(Z):
    with pytest.raises(Z.ZeusError) as e:
        Z.zeus_objective_check("template <class T, class X> ZEUS_FN T objective(const X &x, int d) "
                               "{ return x[0] * no_such_thing; }")
    assert e.value.code == Z.EINVAL and "no_such_thing" in str(e.value)


def test_fp64_only_source_is_refused(Z):
    src = """
ZEUS_FN double sq(double a) { return a * a; }
ZEUS_FN Dual sq(Dual a) { return a * a; }
template <class T, class X>
ZEUS_FN T objective(const X &x, int d) {
  T s = T(0.0);
  for (int i = 0; i < d; ++i) s = s + sq(x[i]);
  return s;
}
"""
    with pytest.raises(Z.ZeusError) as e:
        Z.zeus_objective_check(src)
    assert e.value.code == Z.EINVAL and "F32" in str(e.value)
    # the same function written over T compiles
    Z.zeus_objective_check(src.replace("ZEUS_FN double sq(double a) { return a * a; }\n"
                                       "ZEUS_FN Dual sq(Dual a) { return a * a; }",
                                       "template <class T> ZEUS_FN T sq(T a) { return a * a; }"))


def test_user_problems_need_the_user_entry_point(Z):
    p = Z.make_problem(W.problem(objective="user", dim=3, n=10, lower=-1.0, upper=1.0))
    assert Z.zeus_validate(p) == Z.EINVAL
    assert "zeus_minimize_user" in Z.zeus_last_error()
