"""Host logic of the HIP library on the CPU: the work plans the library
computes for the mode-k contraction kernel are read back (debug dump of the
planner) and the kernel's index arithmetic is replayed in numpy, showing that
every launch touches each tensor element exactly once, stays inside X, the LDS
tile and the split-partial buffer, and writes every U_k entry exactly once per
split.  No GPU is needed."""
import os
import re
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2511_16358_amd", "libifctn.so")

SHAPES = [
    ((30, 30, 30), 2), ((256, 256, 31), 6), ((214, 61, 144), 4), ((144, 176, 3, 50), 5),
    ((7, 13, 5), 3), ((9, 11), 4), ((5, 6, 7, 3), 2), ((4, 3, 5, 2, 3), 2), ((1, 1, 1), 1),
    ((3, 1, 4), 2), ((17, 33, 9), 8), ((144, 176, 50, 3), 5), ((16, 16, 16, 16, 16), 6),
    ((45, 44, 46, 43), 4), ((20, 19, 21, 18, 22), 6), ((4, 4, 4, 4, 4), 8),
    # long fibres: split into chunks over workgroups, or another fibre mode
    ((40000, 3), 2), ((3, 40000), 2), ((20000, 4, 3), 2), ((5, 3, 30000), 2), ((3, 4, 5, 3000), 2),
]

PLAN_RE = re.compile(r"\[ifctn plan\] (.*?) \|")


def plans_for(dims, R, precision=0):
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_2511_16358_amd import ifctn, workloads as W\n"
        "print(ifctn.workspace_bytes(%r, W.uniform_ranks(%d, %d), precision=%d))\n"
    ) % (ROOT, tuple(dims), len(dims), R, precision)
    env = dict(os.environ, IFCTN_DEBUG_PLAN="1")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stderr
    assert int(r.stdout.strip().splitlines()[-1]) > 0, r.stdout + r.stderr
    plans = []
    for line in r.stderr.splitlines():
        m = PLAN_RE.search(line)
        if not m:
            continue
        kv = {}
        for tok in m.group(1).split():
            key, val = tok.split("=")
            kv[key] = val
        plans.append(kv)
    assert len(plans) == len(dims)
    return plans


def simulate(dims, R, plan):
    """Replay k_contract's indexing for one plan; returns coverage counts."""
    N = len(dims)
    k, f = int(plan["k"]), int(plan["f"])
    ordr = [int(c) for c in plan["ord"]]
    Ik, If, LDF = int(plan["Ik"]), int(plan["If"]), int(plan["LDF"])
    jn, JT, S, PPW, PB = (int(plan[x]) for x in ("jn", "JT", "S", "PPW", "PB"))
    nplanes = int(plan["nplanes"])
    Rprod = int(plan["Rprod"])
    strides = [int(np.prod(dims[m + 1:])) for m in range(N)]
    cm = [m for m in range(N) if m not in (k, f)]
    cdim = [dims[m] for m in cm]
    nX = int(np.prod(dims))
    assert nplanes * Ik * If == nX
    Rk = {m: R for m in range(N) if m != k}
    ust, acc = {}, 1
    for m in reversed([m for m in range(N) if m != k]):
        ust[m] = acc
        acc *= Rk[m]
    Rf = Rk[f]
    slot_to_col = []
    for sl in range(Rprod):
        rc, col = sl // Rf, (sl % Rf) * ust[f]
        for c in reversed(range(len(cm))):
            col += (rc % Rk[cm[c]]) * ust[cm[c]]
            rc //= Rk[cm[c]]
        slot_to_col.append(col)
    assert sorted(slot_to_col) == list(range(Rprod))
    kind = int(plan.get("kind", 0))
    FS = int(plan.get("FS", 1))
    if kind != 0:
        return simulate_fast(dims, plan, kind, FS, strides, cm, cdim, slot_to_col)
    count = np.zeros(nX, dtype=np.int64)
    ucount = np.zeros((S, Ik, Rprod), dtype=np.int64)
    for blk in range(JT * S):
        jt, sp = blk % JT, blk // JT
        j0 = jt * jn
        jcnt = min(jn, Ik - j0)
        assert jcnt >= 1
        pb, pe = sp * PPW, min(nplanes, sp * PPW + PPW)
        assert pe > pb
        # slot ownership: s = q*256 + tid < jcnt*Rprod -> (j, slot) -> canonical
        # U column (modes != k ascending, row-major) as the kernel computes it
        psplit = int(plan["psplit"])
        assert jcnt * Rprod * psplit <= int(plan["spt"]) * 256
        for s in range(0, jcnt * Rprod * psplit, psplit):     # the psub == 0 owner writes
            b = s // psplit
            ucount[sp, j0 + b // Rprod, slot_to_col[b % Rprod]] += 1
        for pb0 in range(pb, pe, PB):
            npl = min(PB, pe - pb0)
            p = np.arange(pb0, pb0 + npl)
            base = np.zeros(npl, dtype=np.int64)
            t = p.copy()
            for c in reversed(range(len(cm))):
                base += (t % cdim[c]) * strides[cm[c]]
                t //= cdim[c]
            ext = {0: jcnt, 1: npl, 2: If}
            D = [ext[o] for o in ordr]
            e = np.arange(D[0] * D[1] * D[2])
            idx = {ordr[0]: e // (D[1] * D[2]), ordr[1]: (e // D[2]) % D[1], ordr[2]: e % D[2]}
            jl, pl, ff = idx[0], idx[1], idx[2]
            assert jl.max() < jcnt and pl.max() < npl and ff.max() < If
            assert ((pl * jn + jl) * LDF + ff).max() < PB * jn * LDF    # LDS tile
            L = base[pl] + (j0 + jl) * strides[k] + ff * strides[f]
            assert L.min() >= 0 and L.max() < nX
            np.add.at(count, L, 1)
    return count, ucount


def simulate_fast(dims, plan, kind, FS, strides, cm, cdim, slot_to_col):
    """Replay k_contract_rows (kind 1) / k_contract_cols (kind 2)."""
    N = len(dims)
    k, f = int(plan["k"]), int(plan["f"])
    Ik, If = int(plan["Ik"]), int(plan["If"])
    jn, JT, S, PPW, PB = (int(plan[x]) for x in ("jn", "JT", "S", "PPW", "PB"))
    nplanes, Rprod, psplit = int(plan["nplanes"]), int(plan["Rprod"]), int(plan["psplit"])
    plfast, fch = int(plan["plfast"]), int(plan["fch"])
    nX = int(np.prod(dims))
    if kind == 1:
        assert strides[f] == 1
    else:
        assert strides[k] == 1
    count = np.zeros(nX, dtype=np.int64)
    ucount = np.zeros((S * FS, Ik, Rprod), dtype=np.int64)
    for blk in range(JT * S * FS):
        jt, spf = blk % JT, blk // JT
        sp, fs = spf // FS, spf % FS
        j0 = jt * jn
        jcnt = min(jn, Ik - j0)
        assert jcnt >= 1
        pb, pe = sp * PPW, min(nplanes, sp * PPW + PPW)
        assert pe > pb
        assert jcnt * Rprod * psplit <= int(plan["spt"]) * 256
        for s in range(0, jcnt * Rprod * psplit, psplit):
            b = s // psplit
            ucount[spf, j0 + b // Rprod, slot_to_col[b % Rprod]] += 1
        fcs = -(-If // FS)
        flo, fhi = fs * fcs, min(If, fs * fcs + fcs)
        assert fhi > flo
        for pb0 in range(pb, pe, PB):
            npl = min(PB, pe - pb0)
            p = np.arange(pb0, pb0 + npl)
            base = np.zeros(npl, dtype=np.int64)
            t = p.copy()
            for c in reversed(range(len(cm))):
                base += (t % cdim[c]) * strides[cm[c]]
                t //= cdim[c]
            if kind == 1:
                rows = np.arange(npl * jcnt)
                pl = rows % npl if plfast else rows // jcnt
                jl = rows // npl if plfast else rows % jcnt
                chunk = -(-(fhi - flo) // fch)             # fibre lanes share the chunk
                assert chunk * fch >= fhi - flo
                ff = np.arange(flo, fhi)
                assert (ff - flo).max() < fcs                # chunk-relative LDS tables
                L = (base[pl] + (j0 + jl) * strides[k])[:, None] + ff[None, :]
            else:
                NI = npl * jcnt
                fg = 1 if NI >= 256 else 256 // NI
                fchunk = -(-(fhi - flo) // fg)
                assert fg * fchunk >= fhi - flo and fg * NI <= 256 or fg == 1
                it = np.arange(NI)
                pl, jl = it // jcnt, it % jcnt
                ff = np.arange(flo, fhi)
                L = (base[pl] + j0 + jl)[:, None] + ff[None, :] * strides[f]
            assert L.min() >= 0 and L.max() < nX
            np.add.at(count, L.ravel(), 1)
    if FS > 1 or kind == 2:
        pass
    return count, ucount


@pytest.mark.skipif(not os.path.exists(LIB), reason="libifctn.so not built")
@pytest.mark.parametrize("dims,R", SHAPES, ids=[f"{'x'.join(map(str, d))}_R{r}" for d, r in SHAPES])
def test_contract_plan_covers_tensor_once(dims, R):
    for prec in (0, 2):
        for plan in plans_for(dims, R, prec):
            count, ucount = simulate(dims, R, plan)
            assert np.all(count == 1), (plan, np.unique(count))
            # every split writes each (j, column) of its partial exactly once
            assert np.all(ucount == 1), plan
            assert int(plan["smem"]) <= 64 * 1024
            assert int(plan["spt"]) * 256 >= int(plan["jn"]) * int(plan["Rprod"])
            if int(plan["kind"]) != 0:
                assert int(plan["spt"]) <= 8        # the layout-specialised kernels are built for <= 8
            if int(plan["stage"]):
                # staged accumulation: every batch and workgroup holds whole
                # groups of the last c-mode, so the group products line up
                cdl = int(plan["cdl"])
                assert int(plan["nc"]) >= 2 and int(plan["kind"]) in (1, 2)
                assert int(plan["PB"]) % cdl == 0 and int(plan["PPW"]) % cdl == 0
                assert int(plan["nplanes"]) % cdl == 0
