"""Learned non-reflecting boundary closure: data generation, training and evaluation.

Orchestration only: every computation runs in the library (lattice steps, moments, training-pair
gather, network forward/backward/Adam, field comparison); PyTorch holds device buffers.

Problem (not in the paper, which is periodic-only): an initial state given on an L^D box, free
space at rest outside.  The judge is a periodic run on a box of E = 3L per axis with the initial
state in its centre and zero elsewhere; inside the box it is exact for n <= E - L steps (no
signal travels faster than one cell per step).  The reflection coefficient of a closure is
    R = max_t ||p'_bc(t) - p'_ext(t)||_2,box / max_t ||p'_ext(t)||_2,box,   t every 8 steps.
The sponge baseline runs on a box widened by its layer (L + 2W per axis, the layer outside the
compared L^D region), so its damping is not counted as error inside the box; so does the network
behind a sponge layer ("mlp_sponge": the network closes the widened box, the layer damps).
Training pairs come from the same judge runs: the strips at each face node now and one step
earlier, and the true entering populations at its outside neighbour.
"""
from __future__ import annotations

import json
import math
import sys
import time

import numpy as np

from . import inputs, lbm


def log(*a):
    print("[nrbc]", *a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------- initial states
def inner_pulses(rng, L: int, D: int, nmin=1, nmax=4, amp=1e-3, smin=8.0, smax=24.0):
    n = int(rng.integers(nmin, nmax + 1))
    out = []
    for _ in range(n):
        c = tuple(float(v) for v in rng.uniform(0.0, L, size=D))
        out.append(inputs.Pulse(c, float(rng.uniform(-amp, amp)), float(rng.uniform(smin, smax))))
    return out


def initial_fields(kind, rng, info, L: int, D: int):
    """Fields of one seeded initial state on the L^D box: "pulses" (1-4 Gaussian pressure pulses,
    sigma U(8, 24)), "packets" (one wave packet, wavelength U(16, 64), width one wavelength, random
    direction), or "mixed" (either, with probability 1/2)."""
    if kind == "mixed":
        kind = "pulses" if rng.uniform() < 0.5 else "packets"
    if kind == "pulses":
        return box_fields(info, (L,) * D, inner_pulses(rng, L, D))
    if kind == "packets":
        pk = inputs.random_packets(rng, L, D, 1, width_factor=1.0)
        return inputs.packet_fields((L,) * D, pk, info["rho0"], info["theta0"], info["gamma"])
    raise ValueError(kind)


def box_fields(info, shape, pulses):
    """Isentropic fields of the pulses on the box (minimum-image Gaussians on the box itself)."""
    p0 = inputs.gaussian_pressure(shape, pulses)
    return inputs.fields_from_pressure(p0, info["rho0"], info["theta0"], info["gamma"])


def embed(torch, fields, L, E, D):
    """Place box fields in the centre of an E^D box, zero elsewhere (device tensors)."""
    rho, u, theta = fields
    off = (E - L) // 2
    sl = tuple(slice(off, off + L) for _ in range(D))
    R = torch.zeros((E,) * D, dtype=torch.float64, device="cuda")
    T = torch.zeros_like(R)
    U = torch.zeros((D,) + (E,) * D, dtype=torch.float64, device="cuda")
    R[sl] = torch.as_tensor(rho, device="cuda")
    T[sl] = torch.as_tensor(theta, device="cuda")
    U[(slice(None),) + sl] = torch.as_tensor(u, device="cuda")
    return R, U, T


def judge_solver(lattice, storage, E, D):
    """The periodic judge run.  Two population buffers (so the multi-step kernels run, the
    fastest configuration) when they fit in free device memory with a 10 % margin; else one
    buffer streamed in place (half the memory, one step per launch)."""
    import torch
    need = 2 * lbm.lbm_lee_state_bytes(lbm.make_desc(lattice, storage, (E,) * D))
    free, _ = torch.cuda.mem_get_info()
    tune = 0 if need < 0.9 * free else lbm.TUNE["in_place"]
    return lbm.Solver(lattice, storage, (E,) * D, None, None, None, tune=tune)


# ---------------------------------------------------------------- training data
def generate(lattice="D2Q9", L=512, E=1536, runs=100, steps=1024, every=8, nodes=256, seed=0, storage="f32",
             init="pulses"):
    import torch
    info = lbm.lbm_lee_lattice_info(lattice)
    D = info["D"]
    dims = lbm.lbm_nrbc_dims(lattice)
    inner = lbm.make_desc(lattice, storage, (L,) * D, bc="mlp")
    nn = lbm.lbm_nrbc_face_nodes(inner)
    per_run = (steps // every) * nodes
    nin, ns = dims["n_in"], 3 * info["Q"]
    S = torch.empty((runs * per_run, nin), dtype=torch.float32, device="cuda")
    T = torch.empty((runs * per_run, dims["n_out"]), dtype=torch.float32, device="cuda")
    origin = [(E - L) // 2] * D + [0] * (3 - D)
    rng = np.random.default_rng(seed)
    st = torch.cuda.current_stream().cuda_stream
    k = 0
    t0 = time.time()
    ext = judge_solver(lattice, storage, E, D)
    org = [(E - L) // 2] * D
    for r in range(runs):
        ext.reinit_region(org, (L,) * D, *initial_fields(init, rng, info, L, D))
        for s in range(0, steps, every):
            ids = torch.from_numpy(rng.integers(0, nn, size=nodes).astype(np.int64)).cuda()
            # input row [strip(t), strip(t-1)]: the earlier strip first, then one step, then the
            # current strip with its targets
            lbm.lbm_nrbc_gather(ext.h, origin, inner, ids.data_ptr(), nodes, S[k].data_ptr() + 4 * ns, nin, None, st)
            ext.step(1)
            lbm.lbm_nrbc_gather(ext.h, origin, inner, ids.data_ptr(), nodes, S[k].data_ptr(), nin, T[k].data_ptr(), st)
            k += nodes
            ext.step(every - 1)
        if (r + 1) % max(1, runs // 20) == 0:
            torch.cuda.synchronize()
            log(f"data: run {r + 1}/{runs}, {k} pairs, {time.time() - t0:.1f} s")
    ext.close()
    return S[:k], T[:k]


def generate_closed_loop(lattice, params, L=512, E=1536, runs=100, steps=1024, every=8, nodes=256, seed=0,
                         storage="f32", init="pulses"):
    """Pairs from the states the closed loop visits: the open box runs with the network closure
    `params` beside the judge; inputs are the box's own strips at face nodes, targets the judge's
    entering populations at the same nodes (what the exact exterior would have supplied)."""
    import torch
    info = lbm.lbm_lee_lattice_info(lattice)
    D = info["D"]
    dims = lbm.lbm_nrbc_dims(lattice)
    inner = lbm.make_desc(lattice, storage, (L,) * D, bc="mlp")
    nn = lbm.lbm_nrbc_face_nodes(inner)
    per_run = (steps // every) * nodes
    nin, ns = dims["n_in"], 3 * info["Q"]
    S = torch.empty((runs * per_run, nin), dtype=torch.float32, device="cuda")
    T = torch.empty((runs * per_run, dims["n_out"]), dtype=torch.float32, device="cuda")
    junk = torch.empty((nodes, dims["n_in"]), dtype=torch.float32, device="cuda")
    org = [(E - L) // 2] * D
    origin = org + [0] * (3 - D)
    rng = np.random.default_rng(seed)
    st = torch.cuda.current_stream().cuda_stream
    P = torch.as_tensor(np.asarray(params, dtype=np.float32)).cuda()
    ext = judge_solver(lattice, storage, E, D)
    box = lbm.Solver(lattice, storage, (L,) * D, None, None, None, bc="mlp")
    box.set_closure(P)
    k = 0
    t0 = time.time()
    for r in range(runs):
        fields = initial_fields(init, rng, info, L, D)
        ext.reinit_region(org, (L,) * D, *fields)
        box.reinit_region([0] * D, (L,) * D, *fields)
        for s in range(0, steps, every):
            ids = torch.from_numpy(rng.integers(0, nn, size=nodes).astype(np.int64)).cuda()
            lbm.lbm_nrbc_gather(box.h, [0, 0, 0], box.desc, ids.data_ptr(), nodes, S[k].data_ptr() + 4 * ns, nin, None,
                                st)
            ext.step(1)
            box.step(1)
            lbm.lbm_nrbc_gather(box.h, [0, 0, 0], box.desc, ids.data_ptr(), nodes, S[k].data_ptr(), nin, None, st)
            lbm.lbm_nrbc_gather(ext.h, origin, inner, ids.data_ptr(), nodes, junk.data_ptr(), nin, T[k].data_ptr(), st)
            k += nodes
            ext.step(every - 1)
            box.step(every - 1)
        if (r + 1) % max(1, runs // 10) == 0:
            torch.cuda.synchronize()
            log(f"closed-loop data: run {r + 1}/{runs}, {k} pairs, {time.time() - t0:.1f} s")
    ext.close()
    box.close()
    return S[:k], T[:k]


# ---------------------------------------------------------------- training
def init_params(lattice, seed=0):
    dims = lbm.lbm_nrbc_dims(lattice)
    rng = np.random.default_rng(seed)
    nin, nout, H = dims["n_in"], dims["n_out"], dims["hidden"]
    parts = [rng.standard_normal((nin, H)) * math.sqrt(2.0 / nin), np.zeros(H),
             rng.standard_normal((H, H)) * math.sqrt(2.0 / H), np.zeros(H),
             rng.standard_normal((H, nout)) * math.sqrt(1.0 / H), np.zeros(nout)]
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)


def train(lattice, S, T, epochs=4, batch=4096, lr=1e-3, lr_end=1e-5, seed=0, params=None, val_frac=0.02):
    import torch
    st = torch.cuda.current_stream().cuda_stream
    n = S.shape[0]
    nval = max(batch, int(n * val_frac))
    perm = torch.randperm(n, generator=torch.Generator().manual_seed(seed)).cuda()
    Sv, Tv = S[perm[:nval]].contiguous(), T[perm[:nval]].contiguous()
    tr = perm[nval:]
    P = torch.from_numpy(params if params is not None else init_params(lattice, seed)).cuda()
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    g = torch.empty_like(P)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    wsb = lbm.lbm_nrbc_workspace_bytes(lattice, batch)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    nb = (n - nval) // batch
    total = epochs * nb
    it = 0
    # epoch 0: the validation loss of the starting parameters
    hist = [dict(epoch=0, train_loss=float("nan"), val_loss=evaluate_loss(lattice, P, Sv, Tv, ws, wsb))]
    t0 = time.time()
    for ep in range(epochs):
        order = tr[torch.randperm(tr.numel(), generator=torch.Generator().manual_seed(seed + 1 + ep)).cuda()]
        for b in range(nb):
            idx = order[b * batch:(b + 1) * batch]
            xb, yb = S[idx].contiguous(), T[idx].contiguous()
            it += 1
            lr_t = lr * (lr_end / lr) ** (it / total)
            lbm.lbm_nrbc_loss_grad(lattice, P.data_ptr(), xb.data_ptr(), yb.data_ptr(), batch, g.data_ptr(),
                                   loss.data_ptr(), ws.data_ptr(), wsb, st)
            lbm.lbm_nrbc_adam(P.numel(), P.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(), it, lr_t, 0.9, 0.999,
                              1e-8, st)
        vl = evaluate_loss(lattice, P, Sv, Tv, ws, wsb)
        hist.append(dict(epoch=ep + 1, train_loss=float(loss.item()), val_loss=vl))
        log(f"train: epoch {ep + 1}/{epochs}, batch loss {loss.item():.3e}, val loss {vl:.3e}, {time.time() - t0:.1f} s")
    return P.cpu().numpy(), hist


def evaluate_loss(lattice, P, S, T, ws, wsb):
    import torch
    st = torch.cuda.current_stream().cuda_stream
    g = torch.empty_like(P)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    n = S.shape[0]
    need = lbm.lbm_nrbc_workspace_bytes(lattice, n)
    if need > wsb:
        ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        wsb = need
    lbm.lbm_nrbc_loss_grad(lattice, P.data_ptr(), S.data_ptr(), T.data_ptr(), n, g.data_ptr(), loss.data_ptr(),
                           ws.data_ptr(), wsb, st)
    return float(loss.item())


# ---------------------------------------------------------------- evaluation
def _compare(a, b, n3, scratch, scratch_bytes, st):
    return lbm.lbm_lee_compare_fields(a.data_ptr(), n3, b.data_ptr(), n3, [0, 0, 0], scratch, scratch_bytes, st)


def _regions(L, D, slices):
    """Regions compared, (origin in box coordinates, extent), x first: the whole box, or its
    mid-planes (one per axis)."""
    if slices and D > 1:
        out = []
        for a in range(D):
            o = [0] * D
            n = [L] * D
            o[a], n[a] = L // 2, 1
            out.append((o, n))
        return out
    return [([0] * D, [L] * D)]


def judge_reference(lattice, fields, L=512, E=1536, steps=1024, every=8, ext_storage="f32", ext=None, slices=False):
    """The judge's p' on the compared regions of the inner box every `every` steps (device FP64
    tensors, [sample][region]): run once per initial state and shared by every closure."""
    info = lbm.lbm_lee_lattice_info(lattice)
    D = info["D"]
    own_ext = ext is None
    if own_ext:
        ext = judge_solver(lattice, ext_storage, E, D)
    oe = (E - L) // 2
    ext.reinit_region([oe] * D, (L,) * D, *fields)
    ref = []
    for t in range(0, steps + 1, every):
        if t:
            ext.step(every)
        ref.append([ext.moments_region([v + oe for v in o], tuple(reversed(n)))["p"].clone()
                    for o, n in _regions(L, D, slices)])
    if own_ext:
        ext.close()
    return ref


def reflection_vs(lattice, closure, fields, ref, L=512, steps=1024, every=8, params=None, storage="f32",
                  sponge_width=32, sponge_sigma=0.2, slices=False):
    """R of one closure on one initial state against a judge reference from judge_reference.
    closure: zero, copy, sponge, mlp, or mlp_sponge (the network behind a sponge layer)."""
    import torch
    info = lbm.lbm_lee_lattice_info(lattice)
    D = info["D"]
    layered = closure in ("sponge", "mlp_sponge")
    bc = "mlp" if closure == "mlp_sponge" else closure
    W = sponge_width if layered else 0
    kw = dict(sponge_width=sponge_width, sponge_sigma=sponge_sigma) if layered else {}
    nb = L + 2 * W
    if W == 0:  # the library picks the 16-bit storage scale from the fields
        box = lbm.Solver(lattice, storage, (L,) * D, *fields, bc=bc, **kw)
    else:  # the sponge layer lies outside the fields: take the scale the box alone would get
        probe = lbm.Solver(lattice, storage, (L,) * D, *fields)
        scale = probe.store_scale if lbm.ELEM_BYTES[storage] == 2 else 0.0
        probe.close()
        box = lbm.Solver(lattice, storage, (nb,) * D, None, None, None, bc=bc, store_scale=scale, **kw)
        box.reinit_region([W] * D, (L,) * D, *fields)
    if bc == "mlp":
        box.set_closure(params)
    st = torch.cuda.current_stream().cuda_stream
    regions = _regions(L, D, slices)
    err_max = ref_max = 0.0
    for k, t in enumerate(range(0, steps + 1, every)):
        if t:
            box.step(every)
        e2 = r2 = 0.0
        for (o, n), pe in zip(regions, ref[k]):
            pb = box.moments_region([v + W for v in o], tuple(reversed(n)))["p"]
            out = _compare(pb, pe, list(n) + [1] * (3 - D), box.scratch.data_ptr(), box.scratch_bytes, st)
            e2 += out[0]
            r2 += out[1]
        if not (math.isfinite(e2) and math.isfinite(r2)):
            err_max = float("inf")
            break
        err_max = max(err_max, math.sqrt(e2))
        ref_max = max(ref_max, math.sqrt(r2))
    box.close()
    return err_max / ref_max if ref_max > 0 else float("nan")


def reflection(lattice, closure, fields, L=512, E=1536, steps=1024, every=8, params=None, storage="f32",
               ext_storage="f32", sponge_width=32, sponge_sigma=0.2, ext=None, slices=False):
    """R of one closure on one initial state (see the module docstring).  slices: compare on the
    box's mid-planes (one per axis) instead of the whole box."""
    ref = judge_reference(lattice, fields, L, E, steps, every, ext_storage, ext, slices)
    return reflection_vs(lattice, closure, fields, ref, L, steps, every, params, storage, sponge_width, sponge_sigma,
                         slices)


def time_solver(sim, steps=200, graph=False):
    """ms per step.  graph=True replays a captured graph of six steps (no host launch cost per
    kernel; six is a whole number of launches for the one-, two- and three-step kernels); the
    replays advance the buffers but not the handle's step counter (timing only: with the two-step
    kernel the three launches do not end in the buffer they started from)."""
    import torch
    sim.step(10)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    if not graph:
        e0.record()
        sim.step(steps)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        lbm.lbm_lee_step(sim.h, 6, torch.cuda.current_stream().cuda_stream)
    g.replay()
    torch.cuda.synchronize()
    reps = max(1, steps // 6)
    e0.record()
    for _ in range(reps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / (6 * reps)


def time_per_step(lattice, shape, bc="periodic", params=None, storage="f32", steps=200, graph=False, tune=0,
                  fields=None, origin=None, **kw):
    """ms per step of a box of `shape`, started from `fields` (a seeded state, so the timed steps
    work on live data) on the whole box, or on a sub-box at cell offset `origin` (x, y, z) with the
    rest at rest; None: the state at rest."""
    if fields is not None and origin is None:
        sim = lbm.Solver(lattice, storage, shape, *fields, bc=bc, tune=tune, **kw)
    else:
        sim = lbm.Solver(lattice, storage, shape, None, None, None, bc=bc, tune=tune, **kw)
        if fields is not None:
            sim.reinit_region(origin, fields[0].shape, *fields)
    if bc == "mlp":
        sim.set_closure(params)
    ms = time_solver(sim, steps, graph)
    sim.close()
    return ms


# ---------------------------------------------------------------- command line
def main(argv=None):
    """python -m paper_1601_08103_amd.nrbc {train,evaluate} ...  (JSON on stdout, progress on stderr)."""
    import argparse
    import torch

    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["train", "evaluate"])
    ap.add_argument("--lattice", default="D2Q9")
    ap.add_argument("--L", type=int, default=512)
    ap.add_argument("--E", type=int, default=1536)
    ap.add_argument("--steps", type=int, default=1024)
    ap.add_argument("--runs", type=int, default=200)
    ap.add_argument("--every", type=int, default=8, help="steps between samples (training) / comparisons")
    ap.add_argument("--nodes", type=int, default=256)
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--init", default="pulses", choices=["pulses", "packets", "mixed"])
    ap.add_argument("--storage", default="f32", help="storage of the open box (evaluate)")
    ap.add_argument("--ext-storage", default="f32", help="storage of the judge run")
    ap.add_argument("--slices", action="store_true", help="compare on the mid-planes only (evaluate)")
    ap.add_argument("--closures", default="zero,copy,sponge,mlp",
                    help="zero, copy, sponge, mlp, mlp_sponge (the network behind a sponge layer)")
    ap.add_argument("--weights", default=None, help="weights file (.npy) to write (train) or read (evaluate)")
    ap.add_argument("--seeds", type=int, default=32, help="held-out initial states for evaluate")
    ap.add_argument("--sponge-width", default="32",
                    help="layer width; a comma-separated list evaluates one sponge per width (evaluate)")
    ap.add_argument("--sponge-sigma", default="0.2", help="damping rate, or one per width")
    ap.add_argument("--mlp-sponge-width", default="8", help="layer width(s) behind the network (mlp_sponge)")
    ap.add_argument("--mlp-sponge-sigma", default="0.1", help="damping rate, or one per width (mlp_sponge)")
    ap.add_argument("--dagger", type=int, default=0, help="rounds of closed-loop data + further training")
    ap.add_argument("--dagger-runs", type=int, default=100)
    ap.add_argument("--dagger-epochs", type=int, default=2)
    args = ap.parse_args(argv)
    def layers(wtext, stext, flag):
        ws = [int(w) for w in str(wtext).split(",")]
        gs = [float(x) for x in str(stext).split(",")]
        if len(gs) == 1:
            gs = gs * len(ws)
        if len(gs) != len(ws):
            ap.error(f"{flag}: one value, or one per width")
        return ws, gs

    widths, sigmas = layers(args.sponge_width, args.sponge_sigma, "--sponge-sigma")
    mwidths, msigmas = layers(args.mlp_sponge_width, args.mlp_sponge_sigma, "--mlp-sponge-sigma")
    args.sponge_width, args.sponge_sigma = widths[0], sigmas[0]
    torch.cuda.set_device(0)
    lbm.load()
    info = lbm.lbm_lee_lattice_info(args.lattice)
    D = info["D"]
    if args.mode == "train":
        S, T = generate(args.lattice, args.L, args.E, args.runs, args.steps, args.every, args.nodes, args.seed,
                        init=args.init)
        P, hist = train(args.lattice, S, T, args.epochs, args.batch, args.lr, seed=args.seed)
        for d in range(args.dagger):
            Sc, Tc = generate_closed_loop(args.lattice, P, args.L, args.E, args.dagger_runs, args.steps, args.every,
                                          args.nodes, seed=args.seed + 1000 * (d + 1), init=args.init)
            S, T = torch.cat([S, Sc]), torch.cat([T, Tc])
            del Sc, Tc
            P, h2 = train(args.lattice, S, T, args.dagger_epochs, args.batch, args.lr * 0.3, seed=args.seed + d + 1,
                          params=P)
            hist += [dict(h, dagger=d + 1) for h in h2]
        if args.weights:
            np.save(args.weights, P.astype(np.float32), allow_pickle=False)
        print(json.dumps(dict(mode="train", lattice=args.lattice, init=args.init, pairs=int(S.shape[0]),
                              runs=args.runs, dagger=args.dagger, history=hist)))
        return
    P = np.load(args.weights, allow_pickle=False) if args.weights else None
    rng = np.random.default_rng(10_000 + args.seed)  # held out: training uses seeds below 10000
    closures = [c for c in args.closures.split(",") if c and (c not in ("mlp", "mlp_sponge") or P is not None)]

    # every layered closure is name -> (width, sigma); a single one keeps the closure's name
    def named(base, ws, gs):
        return {base: (ws[0], gs[0])} if len(ws) == 1 else {f"{base}_W{w}_s{g:g}": (w, g) for w, g in zip(ws, gs)}

    layered = {"sponge": named("sponge", widths, sigmas), "mlp_sponge": named("mlp_sponge", mwidths, msigmas)}
    kinds = {n: c for c in closures for n in layered.get(c, [c])}  # name -> closure
    sponges = {n: wg for c in closures for n, wg in layered.get(c, {}).items()}
    closures = list(kinds)
    Rs = {c: [] for c in closures}
    ext = judge_solver(args.lattice, args.ext_storage, args.E, D)
    first = None
    for k in range(args.seeds):
        fields = initial_fields(args.init, rng, info, args.L, D)
        first = fields if first is None else first
        ref = judge_reference(args.lattice, fields, args.L, args.E, args.steps, args.every, args.ext_storage, ext,
                              args.slices)
        for c in closures:
            w, g = sponges.get(c, (0, 0.0))
            Rs[c].append(reflection_vs(args.lattice, kinds[c], fields, ref, args.L, args.steps, args.every, params=P,
                                       storage=args.storage, sponge_width=w, sponge_sigma=g, slices=args.slices))
        del ref
        log(f"evaluate: seed {k + 1}/{args.seeds}: " + ", ".join(f"{c} {Rs[c][-1]:.4f}" for c in closures))
    nrep = 50 if D == 3 else 200
    times = {"extended_periodic": time_solver(ext, nrep)}
    times_graph = {"extended_periodic": time_solver(ext, nrep, graph=True)}
    ext.close()
    del ext
    # step times on live data: every box starts from the first held-out state
    for c in closures:
        kind = "mlp" if kinds[c] == "mlp_sponge" else kinds[c]
        W, g = sponges.get(c, (0, 0.0))
        kw = dict(sponge_width=W, sponge_sigma=g) if c in sponges else {}
        live = dict(fields=first, origin=[W] * D if W else None)
        nb = args.L + 2 * W
        times[c] = time_per_step(args.lattice, (nb,) * D, bc=kind, params=P, storage=args.storage, **live, **kw)
        times_graph[c] = time_per_step(args.lattice, (nb,) * D, bc=kind, params=P, storage=args.storage, graph=True,
                                       **live, **kw)
        if c == "mlp":
            times_graph["mlp_closure_stream"] = time_per_step(args.lattice, (nb,) * D, bc=c, params=P,
                                                              storage=args.storage, graph=True,
                                                              tune=lbm.TUNE["closure_stream"], **live)
    print(json.dumps(dict(mode="evaluate", lattice=args.lattice, init=args.init, L=args.L, E=args.E,
                          steps=args.steps, storage=args.storage, ext_storage=args.ext_storage, seeds=args.seeds,
                          slices=args.slices, sponges={k: dict(width=w, sigma=g) for k, (w, g) in sponges.items()},
                          R_mean={c: float(np.mean(v)) for c, v in Rs.items()},
                          R_max={c: float(np.max(v)) for c, v in Rs.items()}, ms_per_step=times,
                          ms_per_step_graph=times_graph)))


if __name__ == "__main__":
    main()
