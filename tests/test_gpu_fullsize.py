"""Parity where the kernels run at full size, through the C ABI.

* Interior 256x256 tiles (the tile of every FP16/BF16 problem with t >= 2p, FP8
  t >= 8p): integer inputs, every operand contiguity, data-parallel and Stream-K (both fixups),
  row- and column-major C -- bit-exact against the oracle.
* The precision set (BF16 and FP8 e4m3 with per-tensor absmax scales, N(0,1)
  from seed 2, BF16 output) on 8192^3, 256x256x65536 and 4096x1024x4096 in
  the library's default configuration, against the FP64 oracle on the
  stored inputs: ||C - Cref||_F / (||A||_F ||B||_F) <= 5e-5 plus the BF16
  output's own rounding (which the bound does not cover); the measured errors
  are printed.  Every element is compared on the two smaller shapes; on
  8192^3 (minutes of CPU time for the whole oracle) 128 seeded rows of C are
  compared in full and the numerator is estimated from them.
* k = 65536, the edge of the 5e-5 bound, with FP16 inputs and FP32 output.
* The geometry sweep exactly as the benchmark launches it (2048 FP16 GEMMs,
  default configuration): sampled elements against the oracle's element
  function, each within the worst-case bound gamma_k * sum_l |a_il b_lj| of
  any FP32 summation order.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from paper_2301_03598_amd import runtime as R
from paper_2301_03598_amd import streamk as S
from tests.gpu_util import LOWP_BOUND, dev, rel_err, run_gemm, say
from tests.test_gpu_parity import check_case

pytestmark = pytest.mark.gpu

BIG = {"f16": (256, 256, 64), "bf16": (256, 256, 64), "f8e4m3": (256, 256, 128)}


@pytest.fixture(scope="module")
def ws():
    return R.Workspace("cuda")


@pytest.mark.parametrize("ab,ct", [("f16", "f32"), ("bf16", "bf16"), ("f8e4m3", "f32")])
@pytest.mark.parametrize("ao,bo", [("row", "row"), ("row", "col"), ("col", "row"), ("col", "col")])
def test_interior_256_tiles_integer_exact(ab, ct, ao, bo, ws):
    # 4 x 3 tiles of 256 x 256, all interior; 10 (5 for FP8) MAC iterations
    m, n, k = 1024, 768, 640
    for co in ("row", "col"):
        for sched, grid, fx in (("dp", 0, "auto"), ("sk", 19, "serial"), ("sk", 19, "spread")):
            cfg = S.make_config(sched=sched, blk=BIG[ab], grid=grid, fixup=fx)
            _, plan = check_case(m, n, k, ab, ct, dist="int4", a_order=ao, b_order=bo, c_order=co, cfg=cfg,
                                 ws=ws, trace=sched == "sk")
            assert (plan.blk_m, plan.blk_n) == (256, 256)


# Above this many multiply-adds the oracle runs on a seeded sample of rows:
# the plain FP64 triple loop takes minutes of CPU time on 8192^3.
FULL_ORACLE_MACS = 1 << 36
SAMPLE_ROWS = 128


def precision_case(name, ab, ws, cfg=None):
    """The precision-set GEMM in the library's default configuration (or
    cfg) against the FP64 oracle on the stored inputs.  The statistic is
    ||C - Cref||_F / (||A||_F ||B||_F); on 8192^3 its numerator comes from
    SAMPLE_ROWS uniformly drawn rows of C, each compared in full (the sum of
    squares scaled by m / rows: an unbiased estimate of the whole), the
    denominator is exact."""
    m, n, k = W.PRECISION_SHAPES[name]
    say(f"precision set ({name}) {m}x{n}x{k} {ab}->bf16")
    A, B = W.gemm_operands(m, n, k, ab, 2, "normal")
    Ct, plan, _ = run_gemm(m, n, k, dev(A), dev(B), c_type="bf16", cfg=cfg, ws=ws)
    sampled = m * n * k > FULL_ORACLE_MACS
    if sampled:
        rows = np.sort(np.random.default_rng(12).choice(m, SAMPLE_ROWS, replace=False))
        got = Ct[torch.from_numpy(rows).cuda()].cpu().double().numpy()
        At = A.tensor[torch.from_numpy(rows)].contiguous()
        As = W.Operand(At, len(rows), k, A.dtype, "row", k, A.scale)
        cref = oracle.gemm(len(rows), n, k, As, B, c_type="bf16")
        scale = m / len(rows)
    else:
        got = Ct.cpu().double().numpy()
        cref = oracle.gemm(m, n, k, A, B, c_type="bf16")
        scale = 1.0
    del Ct
    Ad, Bd = oracle.decode_operand(A), oracle.decode_operand(B)
    den = np.linalg.norm(Ad) * np.linalg.norm(Bd)
    err = math.sqrt(scale) * np.linalg.norm(got - cref) / den
    rnd = math.sqrt(scale) * np.linalg.norm(oracle.decode(oracle.round_to(cref, "bf16"), "bf16") - cref) / den
    say(f"  {name} {ab}: rel err {err:.3e} (output rounding alone {rnd:.3e}; bound {LOWP_BOUND + rnd:.3e}; "
        f"{'rows sampled: ' + str(len(cref)) if sampled else 'every element'}) "
        f"sched={S.SCHED_NAME.get(plan.sched)} grid={plan.grid} tile={plan.blk_m}x{plan.blk_n} "
        f"fixup={S.FIXUP_NAME.get(plan.fixup)}")
    assert err <= LOWP_BOUND + rnd
    return err, plan


@pytest.mark.timeout(900)
@pytest.mark.parametrize("ab", ["bf16", "f8e4m3"])
@pytest.mark.parametrize("name", ["a", "b", "c"])
def test_precision_set_full_size(name, ab, ws):
    precision_case(name, ab, ws)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("fixup", ["serial", "spread"])
def test_deep_k_streamk_both_fixups(fixup, ws):
    # 256 x 256 x 65536 as basic Stream-K on the model grid with each fixup
    precision_case("b", "bf16", ws, S.make_config(sched="sk", fixup=fixup))


@pytest.mark.timeout(300)
def test_k65536_fp16_fp32_bound(ws):
    # the edge of the 5e-5 bound: FP16 inputs U[-1,1], FP32 output, k = 65536
    for sched in ("auto", "dp"):
        check_case(256, 384, 65536, "f16", "f32", dist="uniform", seed=3, cfg=S.make_config(sched=sched),
                   ws=ws, trace=False)
    check_case(256, 384, 65536, "f16", "f32", dist="int4", seed=3, cfg=S.make_config(sched="sk", grid=64),
               ws=ws, trace=False)


@pytest.mark.timeout(900)
def test_geometry_sweep_sampled_default_config(ws):
    # all 2048 sweep problems, FP16 U[-1,1] inputs, FP32 output, each launched
    # through sk_gemm with the default configuration (as the benchmark does);
    # 8 sampled elements per problem against the oracle's element function
    shapes = W.sweep_shapes()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1)
    rng = np.random.default_rng(11)
    u = 2.0 ** -24
    worst = 0.0
    for i, (m, n, k) in enumerate(shapes):
        A = torch.empty((m, k), dtype=torch.float16, device="cuda")
        B = torch.empty((k, n), dtype=torch.float16, device="cuda")
        A.uniform_(-1.0, 1.0, generator=gen)
        B.uniform_(-1.0, 1.0, generator=gen)
        C = torch.empty((m, n), dtype=torch.float32, device="cuda")
        d = S.make_desc(m, n, k, A, B, C, ab_type="f16", c_type="f32")
        st, plan = S.sk_plan(d, None)
        S.check(st, "sk_plan")
        ws.ensure(plan.workspace_bytes)
        S.check(S.sk_gemm(d, None, ws.ptr, ws.nbytes, torch.cuda.current_stream().cuda_stream), "sk_gemm")
        rows = rng.integers(0, m, 8)
        cols = rng.integers(0, n, 8)
        # the sampled rows of A and columns of B, stored as the library saw them
        Ar = W.Operand(A[rows].contiguous().cpu(), 8, k, "f16", "row", k)
        Bc = W.Operand(B[:, cols].t().contiguous().cpu(), k, 8, "f16", "col", k)
        got = C[rows, cols].cpu().double().numpy()
        want = oracle.gemm_elems(list(range(8)), list(range(8)), k, Ar, Bc)
        absdot = np.abs(oracle.decode_operand(Ar)) @ np.abs(oracle.decode_operand(Bc))
        gamma = k * u / (1 - k * u)
        bound = gamma * np.diag(absdot)
        err = np.abs(got - want)
        assert np.all(err <= bound), f"problem {i} {m}x{n}x{k}: {err.max()} > {bound[err.argmax()]}"
        worst = max(worst, float(np.max(err / np.maximum(bound, 1e-300))))
        if i % 256 == 0:
            say(f"sweep {i}/{len(shapes)} ok (worst error / bound so far {worst:.3f})")
    ws.check()
