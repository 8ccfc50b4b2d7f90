"""Learned warm start of FEAST for a parameterised Hamiltonian family.

The project's extension of the subspace reuse of Sec. IV.C (Example III, where
each k-point starts from the previous one's subspace): members of a family of
block-tridiagonal pencils differ in the 16 Fourier amplitudes a of their
onsite potential; a network trained on FEAST's own converged subspaces maps a
to a start block Y0, and random Y0 stays the fallback (the FEAST residual
judges every result).

Every step runs in the HIP library through its C ABI (feast.py): the FEAST
solves, the targets T = X_in X_in^T B Y_ref (feast_cross_gram,
feast_tall_gemm), the per-cell Gram sums (feast_cell_gram_accumulate), the
coefficients (feast_basis_project), the network's training and inference
(feast_mlp_*) and the start block (feast_basis_expand).  Host code only
draws inputs, builds each member's diagonal blocks from the family's base
blocks (input generation), takes the per-cell bases from 500 64x64
symmetric eigenproblems (numpy), shuffles mini-batches and times.

Usage: python -m paper_0901_2665_amd.warmstart [--train 10000 --test 1000
       --epochs 60 --out results.json]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import feast as F
from . import workloads as W

RANK = 4          # basis vectors per cell (r)
MIX = 0.1         # random admixture of a start block, relative to the rms of the targets
HIDDEN = 512      # hidden widths d1 = d2
YREF_SEED = 4999  # the fixed start block of the targets
INPUT_SCALE = 1.0 / W.FAMILY_SIGMA


class Family:
    """Device-resident base blocks of the family and a reusable member pencil."""

    def __init__(self, ctx: F.Context, name: str = "fam32k"):
        import torch
        w = W.WORKLOADS[name]
        self.ctx = ctx
        self.nc, self.b, self.M0, self.Ne = w["nc"], w["b"], w["M0"], w["Ne"]
        self.n = self.nc * self.b
        self.emin, self.emax = W.load_interval(name)
        p0 = W.make_pencil(name)  # the member with a zero potential
        dev = "cuda"
        t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
        self.A0, self.Au, self.Bd, self.Bu = t(p0.Ad), t(p0.Au), t(p0.Bd), t(p0.Bu)
        self.modes = t(W.onsite_modes(self.nc))
        self.Ad = torch.empty_like(self.A0)
        self.pencil = F.Pencil.from_tensors(self.Ad, self.Au, self.Bd, self.Bu)
        self.Yref = t(W.random_subspace(self.n, self.M0, YREF_SEED))
        self.BYref = ctx.bt_multiply(self.pencil, 1, self.Yref)  # B is the same for every member

    def set_member(self, a: np.ndarray) -> F.Pencil:
        """Diagonal blocks of member a: base blocks plus V(s_i) on the diagonal."""
        import torch
        V = self.modes @ torch.as_tensor(a, dtype=torch.float64, device="cuda")
        self.Ad.copy_(self.A0)
        self.Ad.diagonal(dim1=1, dim2=2).add_(V[:, None])
        return self.pencil

    def solve(self, Y0=None, seed: int = 0, **kw) -> F.SolveResult:
        return self.ctx.solve(self.pencil, self.emin, self.emax, self.M0, self.Ne, Y0,
                              seed=seed, **kw)

    def target(self, r: F.SolveResult):
        """T = X_in X_in^T B Y_ref from the counted pairs of a converged solve."""
        G = self.ctx.cross_gram(r.X, self.BYref, m=r.M)
        return self.ctx.tall_gemm(r.X, G, m=r.M)


def log(msg: str) -> None:
    print(msg, flush=True)


def build_dataset(fam: Family, members, pca_members: int):
    """Solve every member from a random start, form its target, fit the
    per-cell bases on the first ``pca_members`` targets, and project every
    target on them.  Returns (inputs [K][16] f32, coefficients [K][d3] f32
    normalised, U, coefficient scale, rms of the targets, energy fraction the
    bases keep, per-member solve records)."""
    import torch
    ctx = fam.ctx
    nc, b, m0 = fam.nc, fam.b, fam.M0
    d3 = nc * RANK * m0
    K = len(members)
    X_in = torch.empty((K, W.FAMILY_MODES), dtype=torch.float32, device="cuda")
    C = torch.empty((K, d3), dtype=torch.float32, device="cuda")
    Gc = torch.zeros((nc, b, b), dtype=torch.float64, device="cuda")
    first = []
    recs = []
    U = None
    scale = None
    t_rms = kept = None
    t0 = time.time()
    for i, s in enumerate(members):
        a = W.family_amplitudes(s)
        X_in[i] = torch.as_tensor(a * INPUT_SCALE, dtype=torch.float32)
        fam.set_member(a)
        r = fam.solve(None, seed=s)
        recs.append(dict(s=s, status=r.status, M=r.M, loops=r.loops, max_res=r.max_res))
        if r.status not in (0, 2) or r.M < 1:
            raise RuntimeError(f"member {s}: FEAST status {r.status}, M {r.M}")
        T = fam.target(r)
        if i < pca_members:
            ctx.cell_gram_accumulate(nc, b, T, Gc)
            first.append(T)
            if i == pca_members - 1:
                # per-cell bases: the r leading eigenvectors of sum_s T_c T_c^T
                g = Gc.cpu().numpy()
                w, v = np.linalg.eigh(g)
                U_h = np.ascontiguousarray(v[:, :, ::-1][:, :, :RANK])
                U = torch.as_tensor(U_h, dtype=torch.float64, device="cuda")
                for j, Tj in enumerate(first):
                    ctx.basis_project(nc, b, U, Tj, 1.0, out=C[j])
                scale = float(torch.sqrt(torch.mean(C[:pca_members].double() ** 2)))
                C[:pca_members] /= scale
                first = []
                kept = float(np.sum(w[:, -RANK:]) / np.sum(w))
                t_rms = float(np.sqrt(np.sum(w) / (pca_members * fam.n * m0)))
                log(f"warm: bases from {pca_members} targets keep {kept:.3f} of their energy; "
                    f"coefficient scale {scale:.3e}, target rms {t_rms:.3e}")
        else:
            ctx.basis_project(nc, b, U, T, 1.0 / scale, out=C[i])
        if (i + 1) % 250 == 0 or i + 1 == K:
            log(f"warm: data {i + 1}/{K} members, {time.time() - t0:.1f} s")
    return X_in, C, U, scale, t_rms, kept, recs


def train(ctx: F.Context, X_in, C, epochs: int, batch: int = 64, lr: float = 1e-3,
          seed: int = 0, log_every: int = 5):
    """Adam on mini-batches of the training pairs; learning rate lr for the
    first 80% of the epochs and lr/10 after."""
    import torch
    K, d0 = X_in.shape
    d3 = C.shape[1]
    dims = (d0, HIDDEN, HIDDEN, d3)
    rng = np.random.default_rng(seed)
    parts = []
    for rows, cols in ((dims[1], dims[0]), (dims[2], dims[1]), (dims[3], dims[2])):
        parts.append(rng.standard_normal(rows * cols) * np.sqrt(2.0 / cols))  # He initialisation
        parts.append(np.zeros(rows))
    parts[-2] *= 0.1  # small output layer: the first predictions sit near the mean
    p0 = torch.as_tensor(np.concatenate(parts), dtype=torch.float32, device="cuda")
    net = F.Mlp(ctx, dims, p0, max_batch=batch)
    gen = torch.Generator(device="cpu").manual_seed(seed)
    steps = K // batch
    t0 = time.time()
    hist = []
    for ep in range(epochs):
        perm = torch.randperm(K, generator=gen).cuda()
        rate = lr if ep < int(0.8 * epochs) else lr / 10
        tot = 0.0
        for j in range(steps):
            idx = perm[j * batch:(j + 1) * batch]
            tot += net.train_step(X_in[idx].contiguous(), C[idx].contiguous(), rate)
        hist.append(tot / steps)
        if (ep + 1) % log_every == 0 or ep + 1 == epochs:
            log(f"warm: epoch {ep + 1}/{epochs} loss {hist[-1]:.4e} ({time.time() - t0:.1f} s)")
    torch.cuda.synchronize()
    return net, hist, time.time() - t0


def start_block(fam: Family, U, coef, scale: float, t_rms: float, seed: int):
    """Y0 = per-cell expansion of the coefficients plus MIX t_rms times the
    random start block of ``seed`` (a prediction of T spans only the M
    in-interval directions; the random part gives the other M0 - M columns
    theirs, as a random start would)."""
    R = fam.ctx.random_start(seed, fam.n, fam.M0)
    return fam.ctx.basis_expand(fam.nc, fam.b, U, coef, fam.M0, scale, R=R, rscale=MIX * t_rms)


def predict_start(fam: Family, net: F.Mlp, U, scale: float, t_rms: float, a: np.ndarray,
                  seed: int, xbuf, ybuf):
    """Start block of member a from the network (batch of one)."""
    import torch
    xbuf[0] = torch.as_tensor(a * INPUT_SCALE, dtype=torch.float32)
    net.forward(xbuf[:1], out=ybuf[:1])
    return start_block(fam, U, ybuf[0], scale, t_rms, seed)


def loops_to_residual(fam: Family, Y0, seed: int, M_final: int, bar: float = 1e-10,
                      kmax: int = 6) -> int:
    """Smallest loop count k whose k-loop run already has the final count of
    pairs, all with residual <= bar."""
    for k in range(1, kmax + 1):
        r = fam.solve(Y0, seed=seed, max_loops=k)
        if r.M == M_final and r.max_res <= bar:
            return k
    return kmax + 1


def evaluate(fam: Family, net: F.Mlp, U, scale: float, t_rms: float, members,
             k_study: int = 200):
    """Held-out members: random start against the learned start (random start
    again if the learned one does not converge).  For the first ``k_study``
    members also the loops each start needs to reach residual 1e-10, and
    those of the start built from the exact coefficients of the member's own
    target (what a perfect network would give with these bases)."""
    import torch
    xbuf = torch.zeros((16, W.FAMILY_MODES), dtype=torch.float32, device="cuda")
    ybuf = torch.empty((16, net.dims[3]), dtype=torch.float32, device="cuda")
    cbuf = torch.empty(net.dims[3], dtype=torch.float32, device="cuda")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = []
    t0 = time.time()
    for i, s in enumerate(members):
        a = W.family_amplitudes(s)
        fam.set_member(a)
        ev0.record()
        rr = fam.solve(None, seed=s)
        ev1.record()
        ev1.synchronize()
        t_rand = ev0.elapsed_time(ev1)
        ev0.record()
        Y0 = predict_start(fam, net, U, scale, t_rms, a, s, xbuf, ybuf)
        rl = fam.solve(Y0, seed=s)
        fallback = rl.status not in (0, 2)
        if fallback:
            rl = fam.solve(None, seed=s)
        ev1.record()
        ev1.synchronize()
        t_learn = ev0.elapsed_time(ev1)
        rec = dict(s=s, M_rand=rr.M, M_learn=rl.M, loops_rand=rr.loops, loops_learn=rl.loops,
                   ms_rand=t_rand, ms_learn=t_learn, res_rand=rr.max_res, res_learn=rl.max_res,
                   status_rand=rr.status, status_learn=rl.status, fallback=fallback)
        if i < k_study:
            T = fam.target(rr)
            fam.ctx.basis_project(fam.nc, fam.b, U, T, 1.0 / scale, out=cbuf)
            Ye = start_block(fam, U, cbuf, scale, t_rms, s)
            re = fam.solve(Ye, seed=s)
            rec.update(loops_exact=re.loops, M_exact=re.M,
                       k_rand=loops_to_residual(fam, None, s, rr.M),
                       k_learn=loops_to_residual(fam, Y0, s, rr.M),
                       k_exact=loops_to_residual(fam, Ye, s, rr.M))
        out.append(rec)
        if (i + 1) % 100 == 0 or i + 1 == len(members):
            log(f"warm: evaluated {i + 1}/{len(members)} ({time.time() - t0:.1f} s)")
    return out


def summarize(recs):
    g = lambda k: np.array([r[k] for r in recs], dtype=float)
    s = dict(members=len(recs),
             loops_rand=float(g("loops_rand").mean()), loops_learn=float(g("loops_learn").mean()),
             ms_rand=float(g("ms_rand").mean()), ms_learn=float(g("ms_learn").mean()),
             same_M=int(np.sum(g("M_rand") == g("M_learn"))),
             max_res_learn=float(g("res_learn").max()), max_res_rand=float(g("res_rand").max()),
             fallbacks=int(np.sum(g("fallback"))))
    ks = [r for r in recs if "k_rand" in r]
    if ks:
        s["k_study_members"] = len(ks)
        for key in ("rand", "learn", "exact"):
            s[f"loops_to_1e-10_{key}"] = float(np.mean([r[f"k_{key}"] for r in ks]))
        s["loops_exact"] = float(np.mean([r["loops_exact"] for r in ks]))
    return s


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=W.FAMILY_TRAIN)
    ap.add_argument("--test", type=int, default=W.FAMILY_TEST)
    ap.add_argument("--pca", type=int, default=1000)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--k-study", type=int, default=200)
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    ctx = F.Context(0)
    fam = Family(ctx)
    train_members = list(range(args.train))
    test_members = list(range(W.FAMILY_TRAIN, W.FAMILY_TRAIN + args.test))
    t0 = time.time()
    X_in, C, U, scale, t_rms, kept, recs = build_dataset(fam, train_members,
                                                         min(args.pca, args.train))
    t_data = time.time() - t0
    net, hist, t_train = train(ctx, X_in, C, args.epochs, lr=args.lr)
    ev = evaluate(fam, net, U, scale, t_rms, test_members, args.k_study)
    summ = summarize(ev)
    summ.update(train_members=args.train, data_s=t_data, train_s=t_train, epochs=args.epochs,
                basis_energy_kept=kept, rank=RANK, mix=MIX,
                final_loss=hist[-1], first_loss=hist[0],
                train_loops_mean=float(np.mean([r["loops"] for r in recs])))
    log("warm: " + json.dumps(summ))
    if args.out:
        with open(args.out, "w") as f:
            json.dump(dict(summary=summ, loss=hist, eval=ev), f)
    net.close()
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
