"""The binding's argument checks, which run before the library is called
(no GPU needed): arrays on the host, of the wrong type or shape are refused
instead of reaching a kernel."""
import pytest

torch = pytest.importorskip("torch")

from paper_0908_3889_amd import api  # noqa: E402


def _host(*shape):
    return torch.zeros(*shape, dtype=torch.float64)


def test_integrate_refuses_host_arrays():
    with pytest.raises(TypeError, match="on the GPU"):
        api.pn_integrate(_host(2, 4), _host(6, 4), _host(3, 4), _host(4), 0.05, 1e-8)


def test_record_and_observables_refuse_host_arrays():
    with pytest.raises(TypeError):
        api.pn_integrate_record(_host(2, 4), _host(6, 4), _host(3, 4), _host(4), 0.05, 1e-8)
    with pytest.raises(TypeError):
        api.pn_observables(_host(10, 4))
    with pytest.raises(TypeError):
        api.pn_rhs(_host(2, 4), _host(10, 4))


def test_statistics_refuse_host_arrays():
    x = _host(3, 100)
    for call in (lambda: api.pn_histogram(x), lambda: api.pn_histogram2d(x, x), lambda: api.pn_pearson(x, x),
                 lambda: api.pn_kde(x, _host(3)), lambda: api.pn_ks_uniform(x)):
        with pytest.raises(TypeError, match="on the GPU"):
            call()


def test_generate_refuses_host_outputs():
    out = {"m": _host(2, 8), "S": _host(6, 8), "L": _host(3, 8), "omega0": _host(8)}
    with pytest.raises(TypeError):
        api.pn_generate(8, api.gen_spec(), out=out)


def test_options_are_checked():
    with pytest.raises(KeyError):
        api.make_opts(schedule="sometimes")
    with pytest.raises(KeyError):
        api.make_opts(precision="fp16")


def test_adjoint_refuses_host_and_strided_arrays():
    rec = {"status": torch.zeros(4, dtype=torch.int32), "ckpt_every": 16}
    with pytest.raises(TypeError):
        api.pn_integrate_adjoint(_host(2, 4), 0.05, rec, _host(10, 4))


def test_missing_library_fails_loudly_and_the_package_never_imports_the_oracle():
    """Without libpn.so the binding raises (there is no CPU fallback), and
    importing the package pulls in nothing from the oracle."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys\n"
            "from paper_0908_3889_amd import api, _lib, population\n"
            "assert not any(m == 'oracle' or m.startswith('oracle.') for m in sys.modules), 'oracle imported'\n"
            "try:\n"
            "    _lib.load()\n"
            "except _lib.PnError as e:\n"
            "    assert 'no fallback' in str(e), e\n"
            "    print('raised')\n")
    env = dict(os.environ, PN_LIB=os.path.join(root, "no-such-dir", "libpn.so"))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=root, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.strip() == "raised"


def test_packed_records_are_checked():
    """opts.packed takes only a contiguous float64 [n, 16] tensor; None clears it."""
    o = api.make_opts()
    assert not o.packed
    for bad in (torch.zeros(4, 12, dtype=torch.float64), torch.zeros(4, 16, dtype=torch.float32),
                torch.zeros(16, 4, dtype=torch.float64).t(), torch.zeros(64, dtype=torch.float64)):
        with pytest.raises(ValueError):
            api.set_packed(o, bad)
    good = torch.zeros(4, 16, dtype=torch.float64)
    api.set_packed(o, good)
    assert o.packed == good.data_ptr()
    api.set_packed(o, None)
    assert not o.packed
