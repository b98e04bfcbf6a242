"""Precision pattern of the fKK-EC fit on paper-size tissue-like cubes.

The 703,026 x 1,000 cube and a 262,144 x 1,600 cube (512 x 512 pixels) are
fitted on the device with the Gram and the projection / reconstruction
contractions in FP32 and in BF16 (FP32 accumulation), with an FP64 Gram or
the int8 split Gram and FP32 projection / reconstruction; FP64 eigensolve
and basis-vector KK / PEC / SEC always.  For each fit the per-spectrum
relative error of the retrieved Raman spectrum (Im K_CARS),
max_j |y - y*| / max_j |y*|, is taken against the FP64 oracle's fit of the
same FP32 input, and its maximum and RMS over all spectra are reported.

test_precision_pattern_k50 runs at k = 50 with one oracle fit per cube and
asserts, for every mode:
  * the output is Eq. 23 of the fit's own exported basis (sampled spectra;
    1e-5 with FP32 operands, the BF16 operand model for BF16);
  * the Davis-Kahan sin-theta bound (Davis & Kahan 1970): the largest
    principal angle between the device's and the oracle's leading r
    eigenvectors obeys sin(theta) <= ||E||_2 / (lam_r - lam_{r+1} - ||E||_2),
    E the device Gram of A = l diag(f) minus the FP64 Gram, r the signal
    subspace (the largest relative eigenvalue gap among the first k); the
    same bound at r = k is reported, and is vacuous where lam_k sits in the
    noise bulk;
  * with the FP64 and the split Gram, every spectrum within 1e-5 of the
    oracle's own fit and the same sub-sampled rows.
FP32 and BF16 fits are not held to the oracle's own fit: past the signal
subspace their eigenvectors move within the noise bulk, which the bound
above allows.

test_precision_sweep takes k in {20, 100} on the same two cubes (one FP64
oracle fit per cube and k, about a minute of host time per cube), with the
same five modes: with the FP64 and the split Gram every spectrum within 1e-5
of the oracle's fit and the same sub-sampled rows; FP32 and BF16 are
reported.  Each cube's report is written as JSON to the directory
FKK_SWEEP_OUT (default gpurun_out).
"""
import json
import os
import sys
import time

import numpy as np
import pytest

import synth
from oracle import precision as pr
from oracle import workflows as wf

torch = pytest.importorskip("torch")
fk = pytest.importorskip("paper_2005_07132_amd")

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
TOL = 1e-5
FRAC = 0.9
MODES = (("fp64 gram + fp32", fk.PREC_FP64, fk.PREC_FP32),
         ("split gram + fp32", fk.PREC_SPLIT, fk.PREC_FP32),
         ("split gram + split", fk.PREC_SPLIT, fk.PREC_SPLIT),
         ("fp32", fk.PREC_FP32, fk.PREC_FP32),
         ("bf16", fk.PREC_BF16, fk.PREC_BF16))


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def errors(y, ref, chunk=65536):
    per = np.empty(ref.shape[0])
    num = den = 0.0
    for i in range(0, ref.shape[0], chunk):
        a, b = y[i:i + chunk].astype(np.float64), ref[i:i + chunk]
        d = np.abs(a - b)
        per[i:i + chunk] = d.max(axis=1) / np.maximum(np.abs(b).max(axis=1), 1e-30)
        num += float(np.sum(d * d))
        den += float(np.sum(b * b))
    return {"max": float(per.max()), "rms": float(np.sqrt(np.mean(per ** 2))),
            "p99": float(np.percentile(per, 99)), "global_rel_rms": float(np.sqrt(num / den))}


def sin_theta(v, w):
    """Sine of the largest principal angle between the column spaces of two
    matrices with orthonormal columns."""
    sv = np.linalg.svd(v.T @ w, compute_uv=False)
    return float(np.sqrt(max(0.0, 1.0 - sv.min() ** 2)))


def davis_kahan(o, norm_e, r):
    """sin-theta bound for the leading r eigenvectors of G + E against those
    of G (lam: G's spectrum, descending); None where the gap does not exceed
    ||E||_2 (no bound)."""
    den = o.lam[r - 1] - o.lam[r] - norm_e
    return norm_e / den if den > 0 else None


@pytest.mark.parametrize("case", ["tissue703_oracle", "tissue262_oracle"])
def test_precision_pattern_k50(request, case):
    o = request.getfixturevalue(case)
    cube, k = o.cube, o.p.k
    m, n = cube.shape
    ctx = fk.Context(0)
    t = torch.from_numpy(cube.i_cars).cuda()
    out = torch.empty_like(t)
    # signal subspace: the last of the first k eigenvalues that exceeds the
    # next by a factor of 2
    r = max(j for j in range(1, k + 1) if o.lam[j - 1] >= 2 * o.lam[j])
    rows = np.sort(synth.rng_for(m, 7).choice(m, min(m, 16384), replace=False))
    rows_t = torch.from_numpy(rows).cuda()
    i_rows = cube.i_cars[rows].astype(np.float64)
    for label, gprec, rprec in MODES:
        say(f"precision pattern {case} k={k} {label}")
        p = fk.params(k=k, f_mode=fk.F_NOISE, alpha=cube.alpha, sigma_g=cube.sigma_g,
                      gram_prec=gprec, recon_prec=rprec)
        b, _, rep = ctx.fit(t, cube.i_ref, p, out=out)
        e = b.export()
        got_rows = out[rows_t].cpu().numpy().astype(np.float64)
        e_all = errors(out.cpu().numpy(), o.im)
        # Eq. 23 of the fit's own basis
        ell, _ = wf.log_ratio(i_rows, e["i_ref"], e["ratio_floor"])
        if rprec in (fk.PREC_FP32, fk.PREC_SPLIT):  # FP32-accurate projection and reconstruction
            own = wf.reconstruct((ell * e["f"]) @ e["v"], e)["im"]
            e_own = spectrum_err(got_rows, own)
            assert e_own.max() < TOL, (label, e_own.max())
        else:
            # projection: the device's Z against the BF16 operand model, to
            # a bound for the entries of l whose FP32 value may round to the
            # other BF16 neighbour, plus FP32 summation; reconstruction: the
            # output against Eq. 23 of the device's own Z with BF16 operands
            # (the library rounds its FP32 copies of W = diag(f) V and of
            # B_re, B_im to BF16, so the model takes the same FP32 values)
            z_dev = ctx.project(b, t[rows_t], want_q=False).cpu().numpy().astype(np.float64)
            w16 = pr.round_bf16(np.float32(e["f"][:, None] * e["v"]))
            l16 = pr.round_bf16(ell)
            bound = z_flip_bound(ell, w16) + (n + 2) * 2.0 ** -24 * (np.abs(l16) @ np.abs(w16))
            assert np.all(np.abs(z_dev - l16 @ w16) <= bound), (label, np.abs(z_dev - l16 @ w16).max())
            e32 = dict(e, b_re=np.float32(e["b_re"]).astype(np.float64), b_im=np.float32(e["b_im"]).astype(np.float64))
            own = pr.reconstruct(z_dev, e32)["im"]
            e_own = spectrum_err(got_rows, own)
            assert e_own.max() < TOL, (label, e_own.max())
        # Davis-Kahan on the device's own Gram, for every leading subspace
        # whose gap exceeds the perturbation; the device eigensolve adds its
        # own backward error (FP64, taken as 64 N eps lam_1)
        g_l, _, _ = ctx.gram(t, cube.i_ref, prec=gprec)
        norm_e = float(np.linalg.norm(e["f"][:, None] * g_l * e["f"][None, :] - o.g_a, 2))
        norm_e += 64 * n * np.finfo(np.float64).eps * o.lam[0]
        checked = []
        for j in range(1, k + 1):
            bound_j = davis_kahan(o, norm_e, j)
            if bound_j is not None:
                sin_j = sin_theta(e["v"][:, :j], o.basis["v"][:, :j])
                assert sin_j <= bound_j, (label, j, sin_j, bound_j)
                checked.append((j, sin_j, bound_j))
        sin_k = sin_theta(e["v"], o.basis["v"])
        sig = [c for c in checked if c[0] == r]
        say(f"  {label}: vs oracle fit max {e_all['max']:.3e} rms {e_all['rms']:.3e}; own basis max "
            f"{e_own.max():.2e}; ||E||_2/lam_1 {norm_e / o.lam[0]:.2e}; bound holds at {len(checked)} of {k} "
            f"leading subspaces; r={r}: {sig}; k sin {sin_k:.2e} bound {davis_kahan(o, norm_e, k)}; "
            f"fit {rep['ms_total']:.1f} ms")
        if gprec != fk.PREC_BF16:
            assert sig, (label, "no bound at the signal subspace")
        if gprec in (fk.PREC_FP64, fk.PREC_SPLIT):
            assert e_all["max"] < TOL, (label, e_all["max"])
            np.testing.assert_array_equal(np.sort(e["q"]), np.sort(o.basis["q"]))
        assert np.isfinite(e_all["max"]) and e_all["max"] < 1.0
        b.free()
    del t, out
    torch.cuda.empty_cache()
    ctx.close()


def z_flip_bound(ell, w16):
    """Bound on |Z_dev - Z_model| from the entries of l (FP64 here, FP32 on
    the device: at most a few units in the last place of FP32 apart) that
    lie within 2^-20 max(|l|, 1) of a midpoint between BF16 neighbours and
    may round to the other one: each moves Z by at most one BF16 spacing
    times |W|."""
    m_, e_ = np.frexp(ell)
    spacing = np.ldexp(1.0 / 256.0, e_)              # BF16 spacing at |l| (8 significant bits)
    frac = np.abs(m_ * 256.0)
    near = np.abs(frac - np.floor(frac) - 0.5) * spacing < 2.0 ** -20 * np.maximum(np.abs(ell), 1.0)
    return (near * spacing) @ np.abs(w16)


def spectrum_err(y, ref):
    return np.abs(y - ref).max(axis=1) / np.maximum(np.abs(ref).max(axis=1), 1e-30)


@pytest.mark.parametrize("case", ["tissue703_oracle", "tissue262_oracle"])
def test_precision_sweep(request, case):
    o = request.getfixturevalue(case)
    cube = o.cube
    m, n = cube.shape
    ctx = fk.Context(0)
    report = {"description": "per-spectrum relative error of Im K_CARS vs the FP64 oracle fit of the same FP32 "
                             "input; max / RMS / 99th percentile over spectra, plus the global relative RMS",
              "cube": case, "M": m, "N": n, "cases": []}
    I = torch.from_numpy(cube.i_cars).cuda()
    out = torch.empty_like(I)
    i64 = cube.i_cars.astype(np.float64)
    for k in (20, 100):
        t0 = time.perf_counter()
        ref = wf.fit(i64, cube.i_ref, o.p.with_(k=k), svd="gram")
        say(f"sweep {case} k={k}: oracle fit {time.perf_counter() - t0:.1f} s")
        for label, gprec, rprec in MODES:
            p = fk.params(k=k, f_mode=fk.F_NOISE, alpha=cube.alpha, sigma_g=cube.sigma_g,
                          gram_prec=gprec, recon_prec=rprec)
            b, _, rep = ctx.fit(I, cube.i_ref, p, out=out)
            q = b.export()["q"]
            b.free()
            torch.cuda.synchronize()
            e = errors(out.cpu().numpy(), ref["im"])
            report["cases"].append({"k": k, "precision": label, "fit_ms": rep["ms_total"], **e})
            say(f"sweep {case} k={k} {label}: max {e['max']:.3e} rms {e['rms']:.3e} "
                f"p99 {e['p99']:.3e} global {e['global_rel_rms']:.3e} ({rep['ms_total']:.1f} ms)")
            if gprec in (fk.PREC_FP64, fk.PREC_SPLIT):
                assert e["max"] < TOL, (label, k, e["max"])
                np.testing.assert_array_equal(np.sort(q), np.sort(ref["basis"]["q"]))
            assert np.isfinite(e["max"]) and e["max"] < 1.0
        del ref
    del I, out, i64
    torch.cuda.empty_cache()
    ctx.close()
    path = os.environ.get("FKK_SWEEP_OUT", "gpurun_out")
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, f"precision_sweep_{case}.json"), "w") as fh:
        json.dump(report, fh, indent=1)
