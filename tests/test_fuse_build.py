"""The fusing compiler on the host (no GPU): program text from the front
end, the kernel partition and which values reach memory, error reporting,
and the generated source."""
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def F():
    from paper_2107_00555_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2107_00555_amd import build
        build.build(verbose=False)
    from paper_2107_00555_amd import fuse
    return fuse


def step_program(F, dtype="f64", h=1.0):
    P = F.Program(dtype)
    u, f = P.input("u", "f")
    alpha, beta, gamma, dt = P.param("alpha", "beta", "gamma", "dt")
    lap = F.lap7(u, h)
    u3 = (u * u) * u
    P.output("unew", u + dt * ((alpha * lap - beta * u3) + gamma * f))
    return P


def test_step_program_fuses_into_one_kernel(F):
    P = step_program(F)
    fused = P.compile()
    assert (fused.n_inputs, fused.n_params, fused.n_outputs) == (2, 4, 1)
    assert fused.n_kernels == 1 and fused.n_buffers == 0      # no temporary reaches memory
    assert fused.workspace_bytes((8, 8, 8)) == 0
    naive = P.compile(fuse=False)
    assert naive.n_kernels > 15 and naive.n_buffers == naive.n_kernels - 1   # every value but the output
    assert naive.workspace_bytes((8, 8, 8)) == naive.n_buffers * 8 * 8 * 8 * 8


def test_shift_of_a_temporary_starts_a_kernel(F):
    P = F.Program("f32")
    u, = P.input("u")
    t = u * u                       # kernel 0, read shifted later: stored
    s = t.shift(1, 0, 0)            # kernel 1
    v = u + 2.0                     # kernel 0, read point-wise by kernel 1: stored
    P.output("y", s + v)            # kernel 1
    P.output("z", v * 3.0)          # kernel 0 (its operand is there)
    fz = P.compile()
    assert fz.n_kernels == 2 and fz.n_buffers == 2
    src = fz.source
    assert "dcp_gen_f32_fused_k0" in src and "dcp_gen_f32_fused_k1" in src and "float" in src


def test_chain_of_shifted_temporaries(F):
    P = F.Program()
    u, = P.input("u")
    a = u.shift(1, 0, 0) * 0.5
    b = a.shift(0, 1, 0) + a
    c = b.shift(0, 0, -1) - u
    P.output("c", c)
    assert P.compile().n_kernels == 3


@pytest.mark.parametrize("text,msg", [
    ("input u\ny = add u u\noutput y\n", "missing dtype"),
    ("dtype f64\ninput u\ny = add u v\noutput y\n", "undefined"),
    ("dtype f64\ninput u\ny = add u u\ny = mul u u\noutput y\n", "defined twice"),
    ("dtype f64\ninput u\nparam p\ny = shift p 1 0 0\noutput y\n", "shift of a scalar"),
    ("dtype f64\ninput u\ny = pow u u\noutput y\n", "unknown operation"),
    ("dtype f64\ninput u\ny = add u u\n", "no output"),
    ("dtype f64\ninput u\noutput u\n", "is an input"),
    ("dtype f64\ninput u\nparam p\ns = mul p 2\noutput s\n", "scalar"),
    ("dtype f16\ninput u\n", "dtype"),
    ("dtype f64\ninput u\ny = shift u 1 x 0\noutput y\n", "bad shift"),
    ("dtype f64\ninput 9u\n", "bad name"),
    ("dtype f64\ninput u\ny = mul u 1e999\noutput y\n", "not a finite"),
])
def test_program_errors(F, text, msg):
    with pytest.raises(F.FuseError, match=msg):
        F.compile_text(text)


def test_literals_are_exact_in_the_source(F):
    P = F.Program()
    u, = P.input("u")
    P.output("y", u * 0.1)
    src = P.compile().source
    assert "0x1.999999999999ap-4" in src          # 0.1 as a hex float, exact


def test_build_status_codes(F):
    import ctypes
    L = F._load()
    h = ctypes.c_void_p()
    err = ctypes.create_string_buffer(256)
    assert L.dcp_fuse_build(None, 1, ctypes.byref(h), err, 256) == -1
    assert L.dcp_fuse_build(b"dtype f64\n", 1, ctypes.byref(h), err, 256) == -5
    assert b"no output" in err.value


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_random_programs_compile_with_torch_loaded(F, seed, dtype):
    # run-time compilation goes through whichever device compiler the process
    # has loaded; with torch imported first that is torch's own, which must
    # accept every generated construct (an inline-asm select crashed it)
    import sys
    import torch  # noqa: F401
    assert "torch" in sys.modules
    from fuse_programs import random_program
    P = random_program(seed, dtype)
    for fuse in (True, False):
        prog = P.compile(fuse)
        assert prog.n_kernels >= 1
        assert "asm" not in prog.source


def test_run_argument_checks_on_the_host(F):
    # every case below is rejected before any device call (placeholder
    # addresses are never dereferenced); an empty grid is a no-op.  Run only
    # where no GPU is visible, so a regression could never reach a launch
    import ctypes
    import torch
    if torch.cuda.is_available():
        pytest.skip("placeholder device addresses: host-only check")
    L = F._load()
    P = step_program(F)                                  # 2 inputs, 4 params, 1 output
    p = P.compile()
    vp = ctypes.c_void_p
    ins = (vp * 2)(0x10000, 0x20000)
    outs = (vp * 1)(0x30000)
    prm = (ctypes.c_double * 4)(1.0, 0.1, 0.5, 0.1)
    h = p._h

    def run(i=ins, q=prm, o=outs, n=(8, 8, 8), bc=1, ws=None, wsb=0):
        return L.dcp_fuse_run(h, i, q, o, n[0], n[1], n[2], bc, ws, wsb, None)

    assert run(n=(0, 8, 8)) == 0 and run(i=None, q=None, o=None, n=(8, 0, 8)) == 0   # empty grid
    assert run(n=(-1, 8, 8)) == -2
    assert run(n=(1 << 40, 1 << 20, 8)) == -2                                        # size overflows
    assert run(bc=2) == -4
    assert run(i=None) == -1 and run(o=None) == -1 and run(q=None) == -1
    assert run(i=(vp * 2)(0x10000, None)) == -1
    nan = (ctypes.c_double * 4)(1.0, float("nan"), 0.5, 0.1)
    assert run(q=nan) == -5
    # the output overlaps an input (8^3 float64 = 4096 bytes from each address)
    assert run(o=(vp * 1)(0x10000 + 4088)) == -7
    # a program with a stored temporary needs a workspace
    Q = F.Program("f64")
    (u,) = Q.input("u")
    Q.output("y", (u * u).shift(1, 0, 0))
    q2 = Q.compile()
    need = q2.workspace_bytes((8, 8, 8))
    assert need == 4096
    one = (vp * 1)(0x10000)
    assert L.dcp_fuse_run(q2._h, one, None, outs, 8, 8, 8, 1, None, 0, None) == -1
    assert L.dcp_fuse_run(q2._h, one, None, outs, 8, 8, 8, 1, vp(0x80000), need - 1, None) == -6
    assert L.dcp_fuse_run(q2._h, one, None, outs, 8, 8, 8, 1, vp(0x30000 + 256), need, None) == -7


def test_compile_cache(F):
    P = step_program(F)
    a = P.compile()
    assert P.compile() is a                              # same text and mode: the same program
    assert P.compile(fuse=False) is not a
    b = P.compile(cache=False)
    assert b is not a and b.n_kernels == a.n_kernels and b.source == a.source
