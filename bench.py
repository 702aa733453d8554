"""Benchmark of the hot path on one MI355X.

Workload (the metric's configuration): exterior pulsating-sphere problem on an icosphere of
5120 flat triangles (15360 DOF), rho = 1, c_p = 1, c_s = 0.5, 64 BDF2 gCQ contour points
(dt = 0.1), collocation at centroids with the near-singular rule on, single layer V and
I/2 + K compressed by 3D-ACA (eps = 1e-6) on an H-matrix partition (leaf 64, eta 1.5), far
field complex64, near field complex128.

One step = the whole hot path on resident inputs: partition, compression of V and I/2 + K
(entries, pivots, fibres, per-slice ACA + recompression), and the all-frequency products
y_l = V(s_l) x_l and (I/2 + K)(s_l) x_l for one right-hand side.  The two operators run
concurrently, each on its own context and stream.

value = kernel entries (3x3 ENTRY(i, j, l) blocks) generated per second over the step.
Extra fields: all-frequency H-matvecs/s (apply only), the FP64 path's step time and the
mixed vs FP64 speedup, the relative error against the FP64 oracle on sampled rows, the
rooflines of the kernel groups of a step (3D-ACA face kernels, per-slice ACA, recompression,
products on the matrix cores; `roofline` is the one with the most device time) and the
oracle's CPU throughput; apart from value, a
solve leg (GMRES with refinement at every contour point) and a batched-product leg (the
single layers of four cube and sphere meshes, 128 contour points, 32 right-hand sides, one
set of launches), an adjoint leg (gradient of a single-layer form on the sphere of 20480
triangles with respect to all node coordinates and the material) and a time-stepping leg
(the pulsating sphere over 64 BDF2 convolution-quadrature steps).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "kernel entries/s and all-frequency H-matvecs/s at 1e-6 rel err; mixed vs FP64 speedup"
PEAK_VALU = 78.6e12  # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz: FP64 and non-packed FP32
PEAK_HBM = 8.0e12    # HBM3E bytes/s
PEAK_MFMA64 = 78.6e12   # dense FP64 MFMA
PEAK_MFMA32 = 157.3e12  # dense FP32 MFMA


# HBM bytes per launch of a kernel group, as the roofline entries count launches (face kernels
# and k_face_aca: one dispatch; recompression: the two workgroup configurations over one chunk
# of faces; product: one bem_apply), from the FETCH_SIZE / WRITE_SIZE counters (two rocprofv3
# --pmc runs of this script, scaled by the counts of a 1 GiB copy;
# profiles/traffic_c2_sphere5120_L64_mixed.md), valid while the kernels' sources and the launch
# composition (compress.cpp) hash to the recorded value
TRAFFIC = {
    "face": {"bytes": 5.535e+09, "sources": ['aca3d.hip', 'kernel.hpp', 'common.hpp', 'aca3d.hpp', 'lib.hpp', 'compress.cpp'], "sha256_16": 'c9a23dafff3bdced'},
    "recomp": {"bytes": 7.066e+09, "sources": ['recomp.hip', 'common.hpp', 'aca3d.hpp', 'compress.cpp'], "sha256_16": '5ed01768c0f8d126'},
    "aca": {"bytes": 8.005e+10, "sources": ['aca3d.hip', 'common.hpp', 'aca3d.hpp', 'compress.cpp'], "sha256_16": '6ffaa9889fb0cfdd'},
    "product": {"bytes": 6.253e+10, "sources": ['mfma.hip', 'apply.hip', 'common.hpp', 'aca3d.hpp', 'compress.cpp'], "sha256_16": '2009bc458f71c824'},
}


def traffic(key):
    """Counter-measured bytes per dispatch of a kernel group, or None once its sources changed."""
    import hashlib
    t = TRAFFIC[key]
    if t["bytes"] is None:
        return None
    m = hashlib.sha256()
    for f in t["sources"]:
        with open(os.path.join(ROOT, "paper_2607_15292_amd", "csrc", f), "rb") as fh:
            m.update(fh.read())
    return t["bytes"] if m.hexdigest()[:16] == t["sha256_16"] else None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(level=4, L=64):
    from paper_2607_15292_amd import workloads as W
    X, T = W.icosphere(level)
    T = T[:, [0, 2, 1]].copy()  # exterior domain: normals point into the sphere
    s = W.bdf2_contour(L, 0.1)
    return X, T, s


def batched_leg(args, dev, torch):
    """Batched products (reported apart from value): the single layers of the mixed cube and
    sphere meshes, one L-point contour, nrhs right-hand sides each, all in one set of launches
    (schedule tuned at creation, replayed as a HIP graph); the oracle checks sampled rows."""
    from paper_2607_15292_amd import binding as B
    from paper_2607_15292_amd import workloads as W
    Lb, nrhs = args.batch_freqs, args.batch_nrhs
    s = W.bdf2_contour(Lb, 0.1)
    ctxs, ops, xs, names = [], [], [], []
    sep_s = 0.0
    for i, (name, X, T) in enumerate(W.batch_meshes()):
        c = B.Context(0)
        c.set_mesh(X, T)
        c.set_material(1.0, 1.0, 0.5)
        c.set_frequencies(s)
        c.set_quadrature(near_on=True)
        ctxs.append(c)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ops.append(c.compress(B.OP_V, eps3d=args.batch_eps, leaf=64, eta=1.5, prec=B.PREC_MIXED,
                              mixed_eps_floor=args.batch_eps_floor))
        torch.cuda.synchronize()
        sep_s += time.perf_counter() - t0
        xs.append(torch.tensor(W.random_rhs(2 + i, (nrhs, Lb, 3 * len(T))), device=dev))
        names.append(name)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = B.Batch(ops, nrhs=nrhs, graph=True, tune=True)
    torch.cuda.synchronize()
    tune_s = time.perf_counter() - t0
    ys = [torch.empty_like(x) for x in xs]
    b.apply(xs, ys)  # records the graph
    torch.cuda.synchronize()
    reps = 2
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.apply(xs, ys)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    info = b.info()
    log("batched: %d operators, L %d, nrhs %d: %.1f ms per product, tuning %.1f s, %s"
        % (len(ops), Lb, nrhs, ms, tune_s, info))
    # sampled rows of every output, checked against the oracle in the CPU-baseline leg
    rng = np.random.default_rng(12)
    samples = []
    for (name, X, T), x, y in zip(W.batch_meshes(), xs, ys):
        K = len(T)
        rows = np.sort(rng.choice(K, size=16, replace=False))
        yg = y.cpu().numpy().reshape(nrhs, Lb, K, 3)[:, :, rows, :].reshape(nrhs, Lb, -1)
        samples.append((name, X, T, rows, x.cpu().numpy(), yg))
    b.destroy()
    # roof of the arithmetic mix: complex64 work at the FP32 MFMA rate, complex128 work and the
    # FP64 fibre contraction at the FP64 rate (the info flops split the same way)
    f32 = f64 = 0.0
    for o in ops:
        v = o.stats()
        f32 += 8.0 * v["apply_macs_c64"] * Lb * nrhs
        f64 += 8.0 * ((v["apply_macs_c128"] + v["apply_macs_fibre"]) * Lb * nrhs + v["apply_macs_sel"] * nrhs)
    sep_bytes = sum(o.stats()["bytes"] for o in ops)
    sep_kernel_ms = sum(o.stats()["kernel_ms"] for o in ops)
    sep_groups = sum(o.stats()["block_groups"] for o in ops)
    for o in ops:
        o.destroy()
    for c in ctxs:
        c.close()
    # the same batch as the components of one context: one compression, one product
    cu = B.Context(0)
    offs = cu.set_meshes([(X, T) for _, X, T in W.batch_meshes()])
    cu.set_material(1.0, 1.0, 0.5)
    cu.set_frequencies(s)
    cu.set_quadrature(near_on=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    opu = cu.compress(B.OP_V, eps3d=args.batch_eps, leaf=64, eta=1.5, prec=B.PREC_MIXED,
                      mixed_eps_floor=args.batch_eps_floor)
    torch.cuda.synchronize()
    union_s = time.perf_counter() - t0
    xu = torch.cat(xs, dim=2)
    yu = torch.empty_like(xu)
    opu.apply(xu, yu)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        opu.apply(xu, yu)
    e1.record()
    torch.cuda.synchronize()
    ms_union = e0.elapsed_time(e1) / reps
    union_diff = max(float(((yu[:, :, 3 * offs[q]:3 * offs[q + 1]] - y).abs().max() / y.abs().max()).item())
                     for q, y in enumerate(ys))
    stu = opu.stats()
    union_bytes = stu["bytes"]
    del xu, yu
    opu.destroy()
    cu.close()
    log("batched as components of one context: compression %.2f s, device %.0f ms in %d groups (meshes apart "
        "%.2f s, device %.0f ms in %d groups), product %.1f ms, max rel diff to the batch %.2e"
        % (union_s, stu["kernel_ms"], stu["block_groups"], sep_s, sep_kernel_ms, sep_groups, ms_union, union_diff))
    achieved = info["flop"] / (ms * 1e-3)
    peak = (f32 + f64) / (f32 / PEAK_MFMA32 + f64 / PEAK_MFMA64)
    out = {"workload": "single layers of %s, mixed precision eps %.0e (far-field floor %.0e), %d BDF2 gCQ points, "
                       "%d right-hand sides each" % (", ".join(names), args.batch_eps, args.batch_eps_floor, Lb, nrhs),
           "ms_per_product": ms, "products_per_s": len(ops) * nrhs * 1e3 / ms,
           "single_freq_matvecs_per_s": len(ops) * nrhs * Lb * 1e3 / ms,
           "compressed_gb": sep_bytes / 1e9,
           "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                        "frac": achieved / peak, "traffic": None,
                        "kernel": "batched product (k_far_mfma + k_rows_mfma<float/double> + k_reduce_mrows + "
                                  "permutations)",
                        "flop_per_product": info["flop"], "flop_complex64_share": f32 / max(f32 + f64, 1.0)},
           "schedule": {k: info[k] for k in ("n_groups", "n_segments", "seg_target", "far_sorted", "tune_ms",
                                             "tune_segments", "graph_builds", "graph_launches", "workspace_bytes")},
           "tune_seconds": tune_s, "rel_err_sampled_rows": None,
           "compress_seconds_meshes_apart": sep_s, "compress_device_ms_meshes_apart": sep_kernel_ms,
           "components": {"compress_seconds": union_s, "compress_device_ms": stu["kernel_ms"],
                          "block_groups": stu["block_groups"], "ms_per_product": ms_union,
                          "compressed_gb": union_bytes / 1e9, "max_rel_diff_to_batch": union_diff},
           "_check": {"s": s, "samples": samples}}
    return out


def adjoint_leg(args, dev, torch):
    """Adjoints of the single and the double layer (reported apart from value): the gradient of
    Re sum_l w_l^T A(s_l) x_l (A = V, then I/2 + K) with respect to all node coordinates and
    rho, c_p, c_s, entries recomputed (near rule on, pair classes held fixed), and the
    matrix-free products, on the sphere of 20480 triangles with 64 contour points."""
    from paper_2607_15292_amd import binding as B
    from paper_2607_15292_amd import workloads as W
    X, T = W.icosphere(args.adjoint_level)
    K, L = len(T), 64
    s = W.bdf2_contour(L, 0.1)
    c = B.Context(0)
    c.set_mesh(X, T)
    c.set_material(1.0, 1.0, 0.5)
    c.set_frequencies(s)
    c.set_quadrature(near_on=True)
    w = torch.tensor(W.random_rhs(70, (1, L, 3 * K)), device=dev)
    x = torch.tensor(W.random_rhs(71, (1, L, 3 * K)), device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    val, gn, gm = c.adjoint_v(w, x)
    t1 = time.perf_counter()
    y = c.apply_mf(B.OP_V, x)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    log("adjoint: K %d L %d: gradient %.2f s, matrix-free product %.2f s" % (K, L, t1 - t0, t2 - t1))
    # the double layer's adjoint (I/2 + K) on the same mesh
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    valk, gnk, gmk = c.adjoint_k(w, x, op=B.OP_HK)
    t4 = time.perf_counter()
    y = c.apply_mf(B.OP_HK, x)
    torch.cuda.synchronize()
    t5 = time.perf_counter()
    log("adjoint of I/2+K: gradient %.2f s, matrix-free product %.2f s" % (t4 - t3, t5 - t4))
    del w, x, y
    c.close()
    sol = solution_gradient(args, dev, torch, X, T, s)
    out = {"workload": "single layer on an icosphere of %d triangles, %d BDF2 gCQ points, near rule on, one "
                       "right-hand side; gradient of Re sum_l w_l^T V(s_l) x_l w.r.t. %d node coordinates and "
                       "rho, c_p, c_s" % (K, L, 3 * len(X)),
           "gradient_seconds": t1 - t0, "pair_freqs_per_s": K * K * L / (t1 - t0),
           "matrix_free_product_seconds": t2 - t1, "matrix_free_entries_per_s": K * K * L / (t2 - t1),
           "grad_norm_nodes": float(np.linalg.norm(gn)), "grad_mat": [float(v) for v in gm],
           "double_layer": {"operator": "I/2 + K", "gradient_seconds": t4 - t3, "pair_freqs_per_s": K * K * L / (t4 - t3),
                            "matrix_free_product_seconds": t5 - t4, "grad_norm_nodes": float(np.linalg.norm(gnk)),
                            "grad_mat": [float(v) for v in gmk]},
           "solution_gradient": sol}
    return out


def stator_leg(args, dev, torch):
    """The stator-shell configuration at a reduced mesh (reported apart from value): coaxial
    cylinders r = 1 and 0.7, length 1.5, 36 slots 0.05 x 0.1 in the bore, c_p = 1, c_s = 0.55,
    128 contour points, the single layer compressed in mixed precision at eps3d 1e-5, and the
    solution of V(s_l) t_l = g_l at every contour point by iterative refinement with the
    matrix-free FP64 operator as the fine one and the compressed mixed one as the inner one.
    The full configuration (about 100k triangles) would need the compression rate times
    184 TB of storage."""
    from paper_2607_15292_amd import binding as B
    from paper_2607_15292_amd import workloads as W
    X, T = W.stator_shell(args.stator_h)
    K, L = len(T), 128
    s = W.bdf2_contour(L, 0.1)
    c = B.Context(0)
    c.set_mesh(X, T)
    c.set_material(1.0, 1.0, 0.55)
    c.set_frequencies(s)
    c.set_quadrature(near_on=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    V = c.compress(B.OP_V, eps3d=1e-5, leaf=64, eta=1.5, prec=B.PREC_MIXED)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = V.stats()
    x = W.random_rhs(81, (1, L, 3 * K))
    xd = torch.tensor(x, device=dev)
    y = V.apply(xd).cpu().numpy()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(3):
        V.apply(xd)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    Vf = c.matrix_free(B.OP_V)
    g = torch.tensor(W.random_rhs(82, (1, L, 3 * K)), device=dev)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    tsol, sst = Vf.solve(g, inner=V, tol=1e-6, inner_tol=1e-3)
    torch.cuda.synchronize()
    t5 = time.perf_counter()
    rows = np.arange(0, K, max(1, K // 12))[:12]
    out = {"workload": "stator shell h %.3f: %d triangles (%d DOF), c_s 0.55, 128 BDF2 gCQ points, V mixed eps3d "
                       "1e-5, leaf 64, eta 1.5; solve with the matrix-free FP64 V as the fine operator" % (args.stator_h, K, 3 * K),
           "elements": K, "compress_seconds": t1 - t0, "kernel_ms": st["kernel_ms"],
           "compression_rate": st["compression_rate"], "compressed_gb": st["bytes"] / 1e9,
           "dense_gb": L * 9.0 * K * K * 16 / 1e9, "rank_mean": st["rank_mean"],
           "ms_per_product": (t3 - t2) / 3 * 1e3, "solve_seconds": t5 - t4,
           "solve_refinements": sst["refinements"], "solve_inner_products": sst["iterations"],
           "solve_rel_residual": sst["rel_residual"], "solve_converged": bool(sst["converged"]),
           "full_size_dense_tb": 128 * 9.0 * 1e5 ** 2 * 16 / 1e12,
           "_check": {"X": X, "T": T, "s": s, "rows": rows, "x": x,
                      "y": y.reshape(1, L, K, 3)[:, :, rows, :].reshape(1, L, -1)}}
    log("stator: K %d, compress %.2f s (rate %.4f, %.1f GB), product %.1f ms, solve %.2f s (%d refinements)"
        % (K, t1 - t0, st["compression_rate"], st["bytes"] / 1e9, out["ms_per_product"], t5 - t4, sst["refinements"]))
    V.destroy()
    Vf.destroy()
    c.close()
    return out


def _pair_class(X, T, I, J, r1sq=2.25, r2sq=9.0):
    """Class of the near rule for the pairs (I, J) as the library decides it: 2 if
    |c_i - c_j|^2 < r1^2 lmax_j^2, 1 if < r2^2 lmax_j^2, else 0 (same arithmetic order)."""
    V = X[T]
    c = (V[:, 0] + V[:, 1] + V[:, 2]) / 3.0
    l2 = np.zeros(len(T))
    for a in range(3):
        e = V[:, (a + 1) % 3] - V[:, a]
        l2 = np.maximum(l2, e[:, 0] * e[:, 0] + e[:, 1] * e[:, 1] + e[:, 2] * e[:, 2])
    d = c[I] - c[J]
    d2 = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2]
    return np.where(d2 < r1sq * l2[J], 2, np.where(d2 < r2sq * l2[J], 1, 0)), np.sqrt(l2.min())


def _class_boundary_pairs(X, T, tau, chunk=512):
    """Pairs i != j with |d^2 / lmax_j^2 - r^2| < tau for r^2 = 2.25 or 9 (host, in row chunks)."""
    V = X[T]
    c = (V[:, 0] + V[:, 1] + V[:, 2]) / 3.0
    l2 = np.zeros(len(T))
    for a in range(3):
        e = V[:, (a + 1) % 3] - V[:, a]
        l2 = np.maximum(l2, (e * e).sum(-1))
    I, J = [], []
    for i0 in range(0, len(T), chunk):
        q = ((c[i0:i0 + chunk, None, :] - c[None, :, :]) ** 2).sum(-1) / l2[None, :]
        m = (np.abs(q - 2.25) < tau) | (np.abs(q - 9.0) < tau)
        ii, jj = np.nonzero(m)
        keep = ii + i0 != jj
        I.append(ii[keep] + i0)
        J.append(jj[keep])
    return np.concatenate(I), np.concatenate(J)


def _fd_direction(rng, X, T, h, I, J, tau):
    """Random direction over the node coordinates (standard normal) for a central difference
    with step h: the nodes of pairs whose near-rule class would differ between X + h D and
    X - h D are held fixed (D = 0 there; a class switch is a jump of the discrete operator,
    not its derivative).  Pairs outside the candidate list (I, J) cannot switch: their
    normalised distance moves by less than tau."""
    D = rng.standard_normal(X.shape)
    base, lmin = _pair_class(X, T, I, J)
    dc = h * np.abs(D).max() * np.sqrt(3.0)
    # |d q| <= 48 dc / l + 40 (dc / l)^2 for a node displacement dc (q <= 9 + tau)
    assert 48.0 * dc / lmin + 40.0 * (dc / lmin) ** 2 < tau, "step too large for the candidate band"
    held = 0
    for _ in range(100):
        cp, _ = _pair_class(X + h * D, T, I, J)
        cm, _ = _pair_class(X - h * D, T, I, J)
        sw = (cp != base) | (cm != base)
        if not sw.any():
            return D, held
        nodes = np.unique(T[np.concatenate([I[sw], J[sw]])])
        held += int((np.abs(D[nodes]).sum(-1) > 0).sum())
        D[nodes] = 0.0
    raise RuntimeError("no class-switch-free direction")


def solution_gradient(args, dev, torch, X, T, s):
    """Gradient of a GMRES solution on the sphere of the adjoint leg: V(s_l) t_l = g_l at all
    contour points, loss sum_l |t_l - t*_l|^2, gradient w.r.t. every node coordinate and
    rho, c_p, c_s through the torch Function (forward solve, transposed solve, adjoint kernel,
    entries recomputed).  The fine operator is matrix-free (FP64 entries recomputed at every
    product: the residuals are exact to quadrature and nothing is stored); the GMRES
    iterations of the refinement run on a compressed inner operator.  With --adjoint-fd N the
    gradient is checked against central differences of the loss on N random directions (node
    coordinates and speeds together), each evaluation a solve with the fine operator of the
    perturbed mesh and the inner operator of the unperturbed one."""
    from paper_2607_15292_amd import binding as B
    from paper_2607_15292_amd import workloads as W
    from paper_2607_15292_amd.autograd import single_layer_solve
    K, L = len(T), len(s)
    tol = min(args.sg_tol, 1e-11) if args.adjoint_fd > 0 else args.sg_tol
    c = B.Context(0)
    c.set_mesh(X, T)
    c.set_material(1.0, 1.0, 0.5)
    c.set_frequencies(s)
    c.set_quadrature(near_on=True)
    inner_opts = dict(eps3d=args.sg_inner_eps, eps_aca=args.sg_inner_eps / 10, leaf=64, eta=1.5, prec=B.PREC_MIXED,
                      mixed_eps_floor=args.sg_inner_eps / 10, far_dense_max=0, aca_rounds=4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Vi = c.compress(B.OP_V, **inner_opts)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sti = Vi.stats()
    log("solution gradient: K %d: inner V compressed in %.1f s (%.1f GB, rate %.4f)"
        % (K, t1 - t0, sti["bytes"] / 1e9, sti["compression_rate"]))
    g = torch.tensor(W.random_rhs(72, (1, L, 3 * K)), device=dev)
    tstar = torch.tensor(W.random_rhs(73, (1, L, 3 * K)), device=dev)
    mat0 = [1.0, 1.0, 0.5]
    nodes = torch.tensor(X, dtype=torch.float64, requires_grad=True)
    mat = torch.tensor(mat0, dtype=torch.float64, requires_grad=True)
    t2 = time.perf_counter()
    tsol = single_layer_solve(c, nodes, mat, g, T, tol=tol, matrix_free=True, inner=Vi)
    loss = ((tsol - tstar).abs() ** 2).sum()
    lv = float(loss.item())
    t3 = time.perf_counter()
    node = tsol.grad_fn
    loss.backward()
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    st1, st2 = node.stats
    gn, gm = nodes.grad.numpy().copy(), mat.grad.numpy().copy()
    log("solution gradient: solve %.1f s (%d refinements, %d inner products), transposed solve + adjoint %.1f s "
        "(%d refinements, %d inner products), loss %.6e"
        % (t3 - t2, st1["refinements"], st1["iterations"], t4 - t3, st2["refinements"], st2["iterations"], lv))
    out = {"workload": "V(s_l) t_l = g_l on an icosphere of %d triangles at %d BDF2 contour points (near rule on), "
                       "loss sum_l |t_l - t*_l|^2 (g, t* complex Gaussian, seeds 72, 73); gradient w.r.t. %d node "
                       "coordinates and rho, c_p, c_s; fine V matrix-free FP64, inner V mixed eps3d %.0e / "
                       "eps_aca %.0e" % (K, L, 3 * len(X), args.sg_inner_eps, args.sg_inner_eps / 10),
           "inner_compress_seconds": t1 - t0, "inner_gb": sti["bytes"] / 1e9,
           "inner_compression_rate": sti["compression_rate"], "solve_seconds": t3 - t2,
           "transposed_solve_and_adjoint_seconds": t4 - t3, "tol": tol,
           "refinements": [st1["refinements"], st2["refinements"]],
           "inner_products": [st1["iterations"], st2["iterations"]],
           "rel_residual": [st1["rel_residual"], st2["rel_residual"]],
           "loss": lv, "grad_norm_nodes": float(np.linalg.norm(gn)), "grad_mat": [float(v) for v in gm]}
    if args.adjoint_fd > 0:
        h = args.adjoint_fd_step
        tau = 0.05
        I, J = _class_boundary_pairs(X, T, tau)
        F = c.matrix_free(B.OP_V)

        def f(Xp, m):
            c.set_mesh(Xp, T)
            c.set_material(*m)
            tp, stp = F.solve(g, inner=Vi, tol=tol)
            return float(((tp - tstar).abs() ** 2).sum().item())

        rng = np.random.default_rng(74)
        checks = []
        for k in range(args.adjoint_fd_skip + args.adjoint_fd):
            D, held = _fd_direction(rng, X, T, h, I, J, tau)
            dm = np.array([0.0] + list(rng.standard_normal(2)))  # (rho, c_p, c_s): the speeds
            if k < args.adjoint_fd_skip:
                continue
            fp = f(X + h * D, [m + h * d for m, d in zip(mat0, dm)])
            fm = f(X - h * D, [m - h * d for m, d in zip(mat0, dm)])
            fd = (fp - fm) / (2 * h)
            an = float((gn * D).sum() + (gm * dm).sum())
            checks.append({"fd": fd, "adjoint": an, "rel_diff": abs(an - fd) / abs(fd), "nodes_held": held})
            log("solution gradient FD direction %d: adjoint %.9e, central difference %.9e, rel diff %.2e "
                "(%d nodes held)" % (k, an, fd, abs(an - fd) / abs(fd), held))
        c.set_mesh(X, T)
        c.set_material(*mat0)
        F.destroy()
        out["fd_check"] = {"directions": checks, "step": h, "max_rel_diff": max(x["rel_diff"] for x in checks),
                           "candidate_pairs": int(len(I))}
    Vi.destroy()
    c.close()
    return out


def timestep_leg(args, dev, torch):
    """Time stepping (reported apart from value): the pulsating sphere of the metric's
    workload in the time domain, N = 64 steps of BDF2 convolution quadrature with the mixed
    V and I/2 + K.  The data are the closed-form displacement on the sphere, (a t_n)^4
    exp(-a t_n) times the unit radial vector; the error against the convolution quadrature
    of the closed-form traction is taken in the CPU-baseline leg."""
    from paper_2607_15292_amd import binding as B
    from paper_2607_15292_amd import workloads as W
    X, T, s = workload(args.level, args.freqs)
    L, dt = len(s), 0.1
    R = 1e-10 ** (1.0 / (2 * L))
    K = len(T)
    C = X[T].mean(axis=1)
    nrm = np.cross(X[T[:, 1]] - X[T[:, 0]], X[T[:, 2]] - X[T[:, 0]])
    nrm /= np.linalg.norm(nrm, axis=1)[:, None]
    a = 2.5
    Gs = a ** 4 * 24.0 / (s + a) ** 5
    # the closed form on the sphere itself (collocation points projected onto r = 1), where
    # the displacement is the pulse times the radial unit vector at every s
    Cs = C / np.linalg.norm(C, axis=1)[:, None]
    Tr = np.empty((L, 3 * K), dtype=np.complex128)
    for l in range(L):
        _, tr = W.pulsating_sphere(Cs, nrm, s[l], a=a)
        Tr[l] = tr.ravel() / Gs[l]
    tn = dt * np.arange(L)
    phi = ((a * tn) ** 4 * np.exp(-a * tn))[:, None] * np.ones((1, 3 * K))
    g = (phi * Cs.ravel()[None, :]).astype(np.complex128)
    c = B.Context(0)
    c.set_mesh(X, T)
    c.set_material(1.0, 1.0, 0.5)
    c.set_frequencies(s)
    c.set_quadrature(near_on=True)
    V = c.compress(B.OP_V, eps3d=args.eps, leaf=64, eta=1.5, prec=B.PREC_MIXED)
    H = c.compress(B.OP_HK, eps3d=args.eps, leaf=64, eta=1.5, prec=B.PREC_MIXED)
    gd = torch.tensor(g, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    td, st = V.cq_dirichlet(gd, dt, R, H=H, tol=1e-6)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log("time stepping: %d steps in %.2f s, %d GMRES products" % (L, t1 - t0, st["iterations"]))
    out = {"workload": "pulsating sphere, icosphere %d triangles, %d BDF2 convolution-quadrature steps (dt %.2f), "
                       "mixed V and I/2+K at eps %.0e, GMRES to 1e-6 per step" % (K, L, dt, args.eps),
           "seconds": t1 - t0, "steps_per_s": L / (t1 - t0), "gmres_products": st["iterations"],
           "max_rel_err_vs_cq_of_closed_form": None, "converged": bool(st["converged"]),
           "_check": {"Tr": Tr, "R": R, "phi": phi, "t": td.cpu().numpy()}}
    V.destroy()
    H.destroy()
    c.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--level", type=int, default=4)
    ap.add_argument("--freqs", type=int, default=64)
    ap.add_argument("--eps", type=float, default=1e-6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=160)
    ap.add_argument("--eps-fp64-strict", type=float, default=1e-8,
                    help="3D-ACA tolerance of the FP64 run that meets 1e-6 per-frequency error")
    ap.add_argument("--pool-gb", type=float, default=0.0, help="0 = library default")
    ap.add_argument("--no-solve", action="store_true", help="skip the solve leg (reported apart from value)")
    ap.add_argument("--solve-tol", type=float, default=1e-6)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-product leg (reported apart from value)")
    ap.add_argument("--batch-nrhs", type=int, default=32)
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint leg (reported apart from value)")
    ap.add_argument("--no-timestep", action="store_true", help="skip the time-stepping leg (reported apart from value)")
    ap.add_argument("--no-stator", action="store_true", help="skip the stator-shell leg (reported apart from value)")
    ap.add_argument("--stator-h", type=float, default=0.1, help="element size of the stator-shell leg")
    ap.add_argument("--no-iloop", action="store_true",
                    help="skip the leg that compresses V and I/2+K in the paper's order of the per-slice ACA")
    ap.add_argument("--sequential", action="store_true",
                    help="timed steps with the operators one at a time (no second stream)")
    ap.add_argument("--no-measure", action="store_true",
                    help="skip the product-timing pass (for kernel traces of the timed steps alone)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB on the GPU three times (the reference kernel of the HBM traffic counters)")
    ap.add_argument("--adjoint-level", type=int, default=5, help="icosphere level of the adjoint leg (5: 20480 triangles)")
    ap.add_argument("--adjoint-fd", type=int, default=0,
                    help="check the solution gradient against central differences on this many random directions "
                         "(each costs two solves)")
    ap.add_argument("--adjoint-fd-step", type=float, default=1e-6)
    ap.add_argument("--sg-inner-eps", type=float, default=1e-3,
                    help="3D-ACA tolerance of the inner operator of the solution gradient (eps_aca a tenth of it)")
    ap.add_argument("--sg-tol", type=float, default=1e-8,
                    help="relative residual of the solution-gradient solves (at most 1e-11 with --adjoint-fd)")
    ap.add_argument("--adjoint-fd-skip", type=int, default=0,
                    help="draw and skip this many directions first (to split a long check over several runs)")
    ap.add_argument("--batch-freqs", type=int, default=128)
    ap.add_argument("--batch-eps", type=float, default=1e-7,
                    help="3D-ACA tolerance of the batched leg (1e-6 leaves 2.5e-4 at the largest |s_l| of L = 128)")
    ap.add_argument("--batch-eps-floor", type=float, default=1e-6, help="far-field tolerance floor of the batched leg")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = 1 << 26  # 64 Mi complex128 = 1 GiB
        xs = torch.ones(n, dtype=torch.complex128, device="cuda")
        ys = torch.empty_like(xs)
        for _ in range(3):
            ys.copy_(xs)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n * 16, "copies": 3}))
        return
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU; sharding the blocks over several GPUs is not "
              "implemented, so --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2607_15292_amd import binding as B
    from paper_2607_15292_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    X, T, s = workload(args.level, args.freqs)
    K, L = len(T), len(s)
    M = 3 * K
    def make_ctx():
        cc = B.Context(0)
        cc.set_mesh(X, T)
        cc.set_material(1.0, 1.0, 0.5)
        cc.set_frequencies(s)
        cc.set_quadrature(near_on=True)
        return cc

    # V and I/2+K are compressed and applied concurrently, each with its own context on its
    # own stream (default priority) from its own host thread: the latency-bound phases of
    # one operator overlap the kernels of the other
    ctxs = [make_ctx(), make_ctx()]
    c = ctxs[0]

    def fresh_ctxs():
        """New contexts: the cached pools of the previous precision go back to the device."""
        nonlocal c
        for cc in ctxs:
            cc.close()
        torch.cuda.empty_cache()
        ctxs[0], ctxs[1] = make_ctx(), make_ctx()
        c = ctxs[0]
    streams = (torch.cuda.Stream(), torch.cuda.Stream())
    x_h = W.random_rhs(1, (1, L, M))
    x = torch.tensor(x_h, device=dev)
    torch.cuda.synchronize()
    ops_list = (B.OP_V, B.OP_HK)
    pool = int(args.pool_gb * (1 << 30))
    import threading

    def one(i, opk, prec, eps, measure, res, ci=None):
        ci = i if ci is None else ci  # context and stream (one context when sequential: its cache serves both)
        try:
            with torch.cuda.stream(streams[ci]):
                op = ctxs[ci].compress(opk, eps3d=eps or args.eps, leaf=64, eta=1.5, prec=prec, pool_bytes=pool)
                y = op.apply(x)
                stt = op.stats()
                yh = am = None
                if measure:
                    streams[ci].synchronize()
                    yh = y.cpu().numpy()
                    y_buf = torch.empty_like(x)
                    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    ev0.record(streams[ci])
                    for _ in range(10):
                        op.apply(x, y=y_buf)
                    ev1.record(streams[ci])
                    streams[ci].synchronize()
                    am = ev0.elapsed_time(ev1) / 10
                streams[ci].synchronize()
                op.destroy()
                res[i] = (stt, yh, am)
        except BaseException as e:  # reported by the caller
            res[i] = e

    def step(prec, measure=False, eps=None, concurrent=True):
        """One pass of the hot path (both operators concurrently, or one after the other);
        with measure, the operators run one after the other and the repeated applies are
        timed alone."""
        res = [None, None]
        if measure or not concurrent:
            for i, opk in enumerate(ops_list):
                one(i, opk, prec, eps, measure, res, ci=0)
        else:
            th = [threading.Thread(target=one, args=(i, opk, prec, eps, False, res)) for i, opk in enumerate(ops_list)]
            for t in th:
                t.start()
            for t in th:
                t.join()
        for r in res:
            if isinstance(r, BaseException):
                raise r
        torch.cuda.synchronize()
        st = [r[0] for r in res]
        for opk, v in zip(ops_list, st):
            log("  op %d prec %d: compress %.0f ms (faces %.0f ms, per-slice ACA %.0f ms), rate %.4f"
                % (opk, prec, v["kernel_ms"], v["face_ms"], v["aca_ms"], v["compression_rate"]))
        return st, [r[1] for r in res] if measure else [], [r[2] for r in res] if measure else []

    log("workload: K=%d L=%d; warmup %d" % (K, L, args.warmup))
    for w in range(args.warmup):
        st, _, _ = step(B.PREC_MIXED)
        log("warmup step %d: kernel_ms=%s" % (w, [round(v["kernel_ms"], 2) for v in st]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats_steps = []
    for k in range(args.steps):
        st, _, _ = step(B.PREC_MIXED, concurrent=not args.sequential)
        stats_steps.append(st)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sec_step = (t1 - t0) / args.steps
    ents = sum(v["entries_generated"] for v in stats_steps[-1])
    log("timed: %.3f s/step, entries/step %d" % (sec_step, ents))
    # the kernels' rooflines and the precision comparison take the operators one at a time:
    # with two streams, events around a kernel also count the co-running kernels
    if args.sequential:
        seq_steps, sec_step_seq = stats_steps, sec_step
    else:
        torch.cuda.synchronize()
        tq0 = time.perf_counter()
        st_seq, _, _ = step(B.PREC_MIXED, concurrent=False)
        torch.cuda.synchronize()
        sec_step_seq = time.perf_counter() - tq0
        seq_steps = [st_seq]
        log("one operator at a time: %.3f s/step" % sec_step_seq)

    # one more mixed pass keeping the products and timing the applies alone
    if args.no_measure:
        st_m, ymix, ams = stats_steps[-1], None, []
    else:
        st_m, ymix, ams = step(B.PREC_MIXED, measure=True)
    apply_ms = dict(zip(ops_list, ams))
    log("apply ms:", apply_ms)

    fp64 = None
    if not args.no_fp64:
        # the FP64 operators do not fit twice at once (compaction holds the growth pool and
        # the exact one), so the speedup compares the two precisions one operator at a time
        fresh_ctxs()
        step(B.PREC_F64, concurrent=False)  # warm-up: the FP64 pools have other sizes than the mixed ones
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        st_d, _, _ = step(B.PREC_F64, concurrent=False)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        st_d2, ys_d, ams_d = step(B.PREC_F64, measure=True)
        fp64 = {"sec_per_step": t3 - t2, "stats": st_d, "apply_ms": dict(zip(ops_list, ams_d)), "ys": ys_d}
        log("fp64 step %.3f s" % (t3 - t2))
        # FP64 at the tolerance that meets 1e-6 per-frequency error (one untimed warm-up)
        fresh_ctxs()
        step(B.PREC_F64, eps=args.eps_fp64_strict, concurrent=False)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        st_s, ys_s, ams_s = step(B.PREC_F64, measure=True, eps=args.eps_fp64_strict)
        torch.cuda.synchronize()
        t5 = time.perf_counter()
        fp64["strict"] = {"eps3d": args.eps_fp64_strict, "ys": ys_s, "apply_ms": dict(zip(ops_list, ams_s)),
                          "compress_ms": [v["kernel_ms"] for v in st_s],
                          "compression_rate": [v["compression_rate"] for v in st_s]}
        log("fp64 eps %.0e: compress %s ms" % (args.eps_fp64_strict, fp64["strict"]["compress_ms"]))

    # the paper's order of the per-slice ACA (Sec. 3.1: faces approximated inside the 3D-ACA
    # loop, pivot on the reconstruction), mixed precision, every admissible block through the
    # ACA; reported apart from value (one operator at a time, after a warm-up compression)
    iloop = None
    if not args.no_iloop:
        fresh_ctxs()
        iloop = {"workload": "V and I/2+K as in the main step, mixed, eps3d %.0e, face_order in-loop, "
                             "far_dense_max 0" % args.eps, "ops": {}}
        ys_il = []
        for opk in ops_list:
            with torch.cuda.stream(streams[0]):
                o = c.compress(opk, eps3d=args.eps, leaf=64, eta=1.5, prec=B.PREC_MIXED, pool_bytes=pool,
                               far_dense_max=0, face_order=B.FACES_IN_LOOP)
                o.destroy()
                torch.cuda.synchronize()
                ti0 = time.perf_counter()
                o = c.compress(opk, eps3d=args.eps, leaf=64, eta=1.5, prec=B.PREC_MIXED, pool_bytes=pool,
                               far_dense_max=0, face_order=B.FACES_IN_LOOP)
                torch.cuda.synchronize()
                ti1 = time.perf_counter()
                ys_il.append(o.apply(x).cpu().numpy())
                v = o.stats()
                iloop["ops"][str(opk)] = {"seconds": ti1 - ti0, "kernel_ms": v["kernel_ms"], "face_ms": v["face_ms"],
                                          "aca_ms": v["aca_ms"], "aca_kernel_ms": v["aca_kernel_ms"],
                                          "recomp_ms": v["recomp_ms"], "compression_rate": v["compression_rate"],
                                          "n_far_faces": v["n_far_faces"], "n_aca_dense": v["n_aca_dense"],
                                          "aca_rank_mean": v["aca_rank_mean"], "rank_mean": v["rank_mean"]}
                o.destroy()
        iloop["_ys"] = ys_il
        log("in-loop order:", {k: (round(v["kernel_ms"]), round(v["compression_rate"], 4), v["n_far_faces"])
                               for k, v in iloop["ops"].items()})

    # solve leg (reported apart from value): V(s_l) t_l = (I/2 + K(s_l)) g_l at every contour
    # point for the pulsating sphere; FP64 operators at the strict eps for the residuals and
    # the right-hand side, the mixed V for the inner GMRES runs
    solve = None
    if not args.no_solve:
        C = X[T].mean(axis=1)
        nrm = np.cross(X[T[:, 1]] - X[T[:, 0]], X[T[:, 2]] - X[T[:, 0]])
        nrm /= np.linalg.norm(nrm, axis=1)[:, None]
        g = np.empty((1, L, M), dtype=np.complex128)
        t_ex = np.empty_like(g)
        for l in range(L):
            u_l, t_l = W.pulsating_sphere(C, nrm, s[l])
            g[0, l] = u_l.ravel()
            t_ex[0, l] = t_l.ravel()
        fresh_ctxs()
        tc0 = time.perf_counter()
        Vf = c.compress(B.OP_V, eps3d=args.eps_fp64_strict, leaf=64, eta=1.5, prec=B.PREC_F64, pool_bytes=pool)
        Vi = c.compress(B.OP_V, eps3d=args.eps, leaf=64, eta=1.5, prec=B.PREC_MIXED, pool_bytes=pool)
        Hf = c.compress(B.OP_HK, eps3d=args.eps_fp64_strict, leaf=64, eta=1.5, prec=B.PREC_F64, pool_bytes=pool)
        gd = torch.tensor(g, device=dev)
        b = Hf.apply(gd)
        torch.cuda.synchronize()
        tc1 = time.perf_counter()
        xs, sst = Vf.solve(b, inner=Vi, tol=args.solve_tol, inner_tol=1e-3)
        torch.cuda.synchronize()
        tc2 = time.perf_counter()
        xh = xs.cpu().numpy()
        err = float(np.max(np.linalg.norm(xh - t_ex, axis=-1) / np.linalg.norm(t_ex, axis=-1)))
        solve = {"problem": "pulsating unit sphere, V t = (I/2 + K) g at all %d contour points" % L,
                 "seconds": tc2 - tc1, "setup_seconds": tc1 - tc0, "iterations": sst["iterations"],
                 "refinements": sst["refinements"], "converged": bool(sst["converged"]),
                 "rel_residual": sst["rel_residual"], "tol": args.solve_tol,
                 "max_rel_err_vs_closed_form": err,
                 "operators": "fine: V FP64 eps %.0e; inner: V mixed eps %.0e; rhs: I/2+K FP64 eps %.0e"
                              % (args.eps_fp64_strict, args.eps, args.eps_fp64_strict)}
        log("solve: %.3f s, %d inner products, %d refinements, residual %.2e, error vs closed form %.3e"
            % (tc2 - tc1, sst["iterations"], sst["refinements"], sst["rel_residual"], err))
        for o in (Vf, Vi, Hf):
            o.destroy()

    # the batched leg builds its own contexts: release these ones' cached pools first
    for cc in ctxs:
        cc.close()
    torch.cuda.empty_cache()
    batched = None if args.no_batch else batched_leg(args, dev, torch)
    adjoint = None if args.no_adjoint else adjoint_leg(args, dev, torch)
    timestep = None if args.no_timestep else timestep_leg(args, dev, torch)
    stator = None if args.no_stator else stator_leg(args, dev, torch)

    # roofline of the dominant compression kernel: algorithmic flops over event-timed device
    # time, summed over the timed steps, for the recompression kernel (k_face_recomp) and the
    # 3D-ACA face kernels (k_face_dense / k_face_general); the one with more device time is
    # reported as "roofline", the other as "roofline_next"
    # With algorithmic bytes (bytes_key), the roof is the one the kernel's arithmetic intensity
    # falls under: HBM below the ridge PEAK_VALU / PEAK_HBM (9.8 flop/B), the vector ALU above;
    # the other roof's figures are kept beside it.
    def rl(ms_key, flop_key, launch_key, name, tkey, steps=None, bytes_key=None):
        steps = stats_steps if steps is None else steps
        ms = sum(v[ms_key] for stp in steps for v in stp)
        flop = sum(v[flop_key] for stp in steps for v in stp)
        launches = sum(v[launch_key] for stp in steps for v in stp)
        achieved = flop / max(ms * 1e-3, 1e-12)
        alu = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_VALU / 1e12, "unit": "TFLOP/s",
               "frac": achieved / PEAK_VALU}
        out = dict(alu)
        if bytes_key is not None:
            nbytes = sum(v[bytes_key] for stp in steps for v in stp)
            bw = nbytes / max(ms * 1e-3, 1e-12)
            hbm = {"bound": "hbm", "achieved": bw / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s", "frac": bw / PEAK_HBM}
            ai = flop / max(nbytes, 1.0)
            out = dict(hbm, alu=alu) if ai < PEAK_VALU / PEAK_HBM else dict(alu, hbm=hbm)
            out["intensity_flop_per_byte"] = ai
            out["bytes_per_launch"] = nbytes / max(launches, 1)
        out.update({"traffic": traffic(tkey), "kernel": name, "launches": launches,
                    "avg_launch_ms": ms / max(launches, 1), "flop_per_launch": flop / max(launches, 1)})
        return ms, out

    rl_rec = rl("recomp_ms", "recomp_flop", "recomp_launches",
                "k_face_recomp (per-slice recompression: QR, pivoted QR, Jacobi SVD, factor products)", "recomp",
                seq_steps)
    rl_face = rl("face_ms", "face_flop", "face_launches", "k_face_dense / k_face_general (3D-ACA face kernels)",
                 "face", seq_steps, bytes_key="face_bytes")
    rl_aca = rl("aca_kernel_ms", "aca_flop", "aca_launches", "k_face_aca (per-slice matrix-valued ACA of the far faces)",
                "aca", seq_steps, bytes_key="aca_bytes")
    groups = [rl_face, rl_aca, rl_rec]
    # the all-frequency products (one operator at a time, HIP events around 10 products on the
    # context stream): algorithmic flops 8 per complex multiply-add of the stored faces and
    # factors with every column, plus the fibres; bytes = stored bytes + x + y; the roof is the
    # MFMA peak of the arithmetic mix (complex64 work at the FP32 MFMA rate, complex128 work and
    # the FP64 fibre contraction at the FP64 rate)
    rl_prod = None
    if apply_ms:
        pflop = pt = pbytes = 0.0
        for opk, v in zip(ops_list, st_m):
            f32 = 8.0 * v["apply_macs_c64"] * L
            f64 = 8.0 * ((v["apply_macs_c128"] + v["apply_macs_fibre"]) * L + v["apply_macs_sel"])
            pflop += f32 + f64
            pt += f32 / PEAK_MFMA32 + f64 / PEAK_MFMA64
            pbytes += v["bytes"] + 2.0 * L * M * 16.0
        ms = sum(apply_ms.values())
        achieved = pflop / (ms * 1e-3)
        peak = pflop / pt
        rl_prod = (ms, {"bound": "mfma", "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                        "frac": achieved / peak, "traffic": traffic("product"),
                        "kernel": "bem_apply: k_far_mfma, k_rows_mfma<float/double>, k_reduce_mrows, permutations "
                                  "(all-frequency products of V and I/2+K)",
                        "launches": len(apply_ms), "avg_launch_ms": ms / len(apply_ms),
                        "flop_per_launch": pflop / len(apply_ms), "bytes_per_launch": pbytes / len(apply_ms),
                        "intensity_flop_per_byte": pflop / pbytes,
                        "peak_note": "MFMA peak of the mix: FP32 %.1f and FP64 %.1f TFLOP/s weighted by the "
                                     "algorithmic flops of each precision" % (PEAK_MFMA32 / 1e12, PEAK_MFMA64 / 1e12),
                        "hbm": {"achieved": pbytes / (ms * 1e-3) / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                                "frac": pbytes / (ms * 1e-3) / PEAK_HBM}})
        groups.append(rl_prod)
    groups.sort(key=lambda g_: -g_[0])
    roofline, roofline_next = groups[0][1], groups[1][1]
    for g_ in groups:
        g_[1]["timing"] = "operators one at a time (HIP events around the launches on the context stream)"
        g_[1]["device_ms_per_step"] = g_[0] / (1 if g_ is rl_prod else len(seq_steps))
    rooflines = {"face": rl_face[1], "aca": rl_aca[1], "recomp": rl_rec[1], "product": rl_prod[1] if rl_prod else None}
    # the same kernels in the timed steps, the two operators sharing the GPU
    roofline_conc = None
    if not args.sequential:
        roofline_conc = {"face": rl("face_ms", "face_flop", "face_launches", "k_face_dense / k_face_general", "face",
                                    bytes_key="face_bytes")[1],
                         "recomp": rl("recomp_ms", "recomp_flop", "recomp_launches", "k_face_recomp", "recomp")[1]}

    # CPU baseline (oracle) on sampled rows; its results are also the accuracy reference
    cpu = None
    errs = {}
    if not args.no_cpu_baseline:
        import oracle
        oracle.build()
        P = oracle.Problem(X, T, s, 1.0, 1.0, 0.5, near_on=True)
        rng = np.random.default_rng(11)
        rows = np.sort(rng.choice(K, size=args.cpu_rows, replace=False))
        tc0 = time.perf_counter()
        refs = {}
        for opk in ops_list:
            refs[opk] = P.matvec_rows(opk, rows, x_h)
        tc1 = time.perf_counter()
        n_ent = len(ops_list) * len(rows) * K * L
        cpu = {"value": n_ent / (tc1 - tc0), "unit": "entries/s", "cores": oracle.num_threads(), "kind": "oracle",
               "sample": "%d element rows x %d elements x %d frequencies for V and I/2+K (%d entries), "
                         "FP64 C oracle with OpenMP" % (len(rows), K, L, n_ent),
               "seconds": tc1 - tc0}
        # the legs' outputs against the oracle: sampled rows of the batched products, and the
        # time-stepping tractions against the convolution quadrature of the closed form
        if batched is not None:
            chk = batched["_check"]
            berr = {}
            for name, Xb, Tb, rows_b, xb, yg in chk["samples"]:
                ref = oracle.Problem(Xb, Tb, chk["s"], 1.0, 1.0, 0.5, near_on=True).matvec_rows(0, rows_b, xb)
                berr[name] = float(np.max(np.linalg.norm(yg - ref, axis=-1) / np.linalg.norm(ref, axis=-1)))
            batched["rel_err_sampled_rows"] = berr
            log("batched rel err on sampled rows:", berr)
        if stator is not None:
            chk = stator["_check"]
            ref = oracle.Problem(chk["X"], chk["T"], chk["s"], 1.0, 1.0, 0.55, near_on=True).matvec_rows(
                0, chk["rows"], chk["x"])
            stator["rel_err_sampled_rows"] = float(np.max(np.linalg.norm(chk["y"] - ref, axis=-1)
                                                          / np.linalg.norm(ref, axis=-1)))
            log("stator rel err on sampled rows: %.3e" % stator["rel_err_sampled_rows"])
        if timestep is not None:
            from oracle import cq
            chk = timestep["_check"]
            t_ref = cq.convolve(cq.weights(chk["Tr"], chk["R"]), chk["phi"])
            timestep["max_rel_err_vs_cq_of_closed_form"] = float(np.abs(chk["t"] - t_ref).max() / np.abs(t_ref).max())
            log("time stepping error %.3e" % timestep["max_rel_err_vs_cq_of_closed_form"])

        def rel(y, ref):
            yg = y.reshape(1, L, K, 3)[:, :, rows, :].reshape(1, L, -1)
            return float(np.max(np.linalg.norm(yg - ref, axis=-1) / np.linalg.norm(ref, axis=-1)))

        if ymix is not None:
            errs["mixed"] = {str(opk): rel(y, refs[opk]) for opk, y in zip(ops_list, ymix)}
        if iloop is not None:
            errs["mixed_in_loop"] = {str(opk): rel(y, refs[opk]) for opk, y in zip(ops_list, iloop["_ys"])}
        if fp64:
            errs["fp64"] = {str(opk): rel(y, refs[opk]) for opk, y in zip(ops_list, fp64["ys"])}
            errs["fp64_eps%.0e" % args.eps_fp64_strict] = {str(opk): rel(y, refs[opk])
                                                           for opk, y in zip(ops_list, fp64["strict"]["ys"])}
    for leg in (batched, timestep, stator):
        if leg is not None:
            leg.pop("_check", None)
    if iloop is not None:
        iloop.pop("_ys", None)
    hmv = {str(k): 1e3 / v for k, v in apply_ms.items()}
    out = {
        "metric": METRIC,
        "value": ents / sec_step,
        "unit": "entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec_step * 1e3,
        "ms_per_step_one_operator_at_a_time": sec_step_seq * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "mixed-f32-f64",
        "data": "synthetic",
        "config": {"workload": "pulsating sphere, icosphere %d triangles (%d DOF), V and I/2+K, %d BDF2 gCQ points, "
                               "3D-ACA eps %.0e (admissible blocks: eps and per-slice eps_ACA raised to the "
                               "complex64 floor 1e-05; near blocks eps_ACA = eps/100) + H-matrix leaf 64 eta 1.5, "
                               "complex64 far / complex128 near" % (K, M, L, args.eps),
                   "elements": K, "frequencies": L, "rhs": 1},
        "entries_per_s_by_rule": {k: sum(v["entries_" + k] for v in stats_steps[-1]) / sec_step
                                  for k in ("regular", "near", "self", "other")},
        "hmatvecs_per_s": hmv,
        "matvecs_per_s_single_freq": {k: v * L for k, v in hmv.items()},
        "compress_stats": [{k: v[k] for k in ("n_blocks", "n_near", "n_far", "n_dense_fallback", "rank_mean",
                                               "rank_max", "aca_rank_mean", "aca_rank_max", "aca_cols_mean",
                                               "n_far_faces", "n_aca_dense", "compression_rate", "bytes",
                                               "entries_generated", "kernel_ms", "face_ms", "aca_ms",
                                               "aca_kernel_ms", "recomp_ms", "entries_regular", "entries_near",
                                               "entries_self", "entries_other")}
                           for v in st_m],
        "rel_err": errs,
        "roofline": roofline,
        "roofline_next": roofline_next,
        "rooflines": rooflines,
        "roofline_two_streams": roofline_conc,
        "solve": solve,
        "batched": batched,
        "adjoint": adjoint,
        "timestep": timestep,
        "in_loop_order": iloop,
        "stator": stator,
        "cpu_baseline": cpu,
    }
    if fp64:
        out["fp64"] = {"ms_per_step": fp64["sec_per_step"] * 1e3,
                       "hmatvecs_per_s": {str(k): 1e3 / v for k, v in fp64["apply_ms"].items()},
                       "kernel_ms": [v["kernel_ms"] for v in fp64["stats"]],
                       "rank_mean": [v["rank_mean"] for v in fp64["stats"]],
                       "compression_rate": [v["compression_rate"] for v in fp64["stats"]]}
        out["fp64"]["strict"] = {k: v for k, v in fp64["strict"].items() if k != "ys"}
        out["fp64"]["strict"]["hmatvecs_per_s"] = {str(k): 1e3 / v for k, v in fp64["strict"]["apply_ms"].items()}
        out["mixed_vs_fp64_speedup"] = fp64["sec_per_step"] / sec_step_seq
        out["mixed_vs_fp64_speedup_basis"] = (
            "step time, one operator at a time, FP64 at eps %.0e over mixed at eps %.0e: equal accuracy when "
            "rel_err.fp64 and rel_err.mixed agree (the far-field floor of the mixed run does not show in the "
            "per-frequency error); fp64.strict is the FP64 run that meets 1e-6" % (args.eps, args.eps))
        out["mixed_vs_fp64_product_speedup"] = {
            str(k): fp64["apply_ms"][k] / apply_ms[k] for k in ops_list if k in apply_ms and k in fp64["apply_ms"]}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
