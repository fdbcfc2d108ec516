"""Residual check at sizes beyond the oracle: a small system S embedded in a large one.

Size-extensivity of CCSD for non-interacting parts: the full system is a small
part S (occupied 0..o_s-1, holding the core orbital 0, and the first v_s
virtuals) plus the rest S', with Cholesky vectors block-diagonal over orbitals
*and* on disjoint ranges of Q (S uses Q < q_s), so every integral joining S and
S' vanishes, and so does the Fock matrix between them.  With amplitudes inside
S and inside S' only, the residual
  * on S equals the oracle's residual of the small system, element by element;
  * on every element joining S and S' is zero;
  * on S' has the antisymmetry of the same-spin blocks;
and the energy splits: E(T) - E(T with T_S = 0) = E_S(T_S).  Every kernel,
tile and launch shape of the full size runs; a transposed operand or a wrong
offset anywhere mixes S' data into S or into the zero elements.
"""
import numpy as np

import blocks
from oracle import ccsd, reference
from synthetic import draw_system, rng_for


def build(shape, cfg, o_s, v_s, q_s):
    o, n = shape.o, shape.n
    eps, chol = draw_system(shape, cfg=cfg)
    in_s = np.zeros(n, dtype=bool)
    in_s[:o_s] = True
    in_s[o:o + v_s] = True
    chol[:q_s] *= in_s[:, None] & in_s[None, :]
    chol[q_s:] *= ~in_s[:, None] & ~in_s[None, :]
    sel = np.flatnonzero(in_s)
    small = reference.n_minus_one_reference(eps[sel], np.ascontiguousarray(chol[:q_s][:, sel][:, :, sel]),
                                            o_s, o_s, 0, 1)
    t1s, t2s = blocks.random_spin_orbital_amplitudes(small, 23, scale=0.05)
    r = ccsd.residual(small, t1s, t2s)
    return dict(shape=shape, cfg=cfg, eps=eps, chol=chol, in_s=in_s, small=small, t=(t1s, t2s), r=r,
                e_s=ccsd.energy(small, t1s, t2s))


def check(P, emb, prec, tol):
    """Set embedded amplitudes on propagator P (built from emb's eps/chol) and assert the properties."""
    no, nv = P.t1_shape()[1:]
    occ, vir = np.array(P.occ_list), np.array(P.vir_list)
    os_, vs_ = emb["in_s"][occ], emb["in_s"][vir]
    ks, vs = int(os_.sum()), int(vs_.sum())
    assert os_[:ks].all() and vs_[:vs].all()      # S leads both lists (orbital 0 heads V)
    rank = np.cumsum(emb["in_s"]) - 1             # orbital -> index in the small system
    small = emb["small"]
    b1s, b2s = blocks.to_blocks(small, rank[occ[:ks]], rank[vir[:vs]], *emb["t"])
    t1 = np.zeros((2, no, nv), dtype=np.complex128)
    t1[:, :ks, :vs] = b1s
    rng = rng_for(emb["cfg"], 77)
    t1[:, ks:, vs:] = (rng.standard_normal((2, no - ks, nv - vs))
                       + 1j * rng.standard_normal((2, no - ks, nv - vs))) * 1e-3
    t2 = np.zeros((3, no, no, nv, nv), dtype=np.complex128)
    t2[:, :ks, :ks, :vs, :vs] = b2s
    for k in range(3):
        x = (rng.standard_normal((no - ks, no - ks, nv - vs, nv - vs))
             + 1j * rng.standard_normal((no - ks, no - ks, nv - vs, nv - vs))) * 1e-3
        if k != 1:
            x = 0.5 * (x - x.transpose(1, 0, 2, 3))
            x = 0.5 * (x - x.transpose(0, 1, 3, 2))
        t2[k, ks:, ks:, vs:, vs:] = x
        del x
    P.set_amplitudes(t1, t2)
    r1, r2 = P.residual()
    e_full = P.energy()

    e1, e2 = blocks.to_blocks(small, rank[occ[:ks]], rank[vir[:vs]], *emb["r"])
    scale = max(np.abs(e1).max(), np.abs(e2).max())
    g1, g2 = r1[:, :ks, :vs], r2[:, :ks, :ks, :vs, :vs]
    if prec == "fp64":
        err = max(np.abs(g1 - e1).max(), np.abs(g2 - e2).max()) / scale
        print(f"S block: max |R - R_oracle| / max |R_oracle| = {err:.3e}", flush=True)
    else:
        err = np.sqrt(np.sum(np.abs(g1 - e1) ** 2) + np.sum(np.abs(g2 - e2) ** 2)) / np.sqrt(
            np.sum(np.abs(e1) ** 2) + np.sum(np.abs(e2) ** 2))
        print(f"S block ({prec}): residual relative Frobenius error {err:.3e}", flush=True)
    assert err < tol

    part_o = (slice(None, ks), slice(ks, None))     # S, S' along occupied indices
    part_v = (slice(None, vs), slice(vs, None))     # S, S' along virtual indices
    mixed = max(np.abs(r1[:, part_o[0], part_v[1]]).max(), np.abs(r1[:, part_o[1], part_v[0]]).max())
    full = scale
    for k in range(3):
        for gi, gj, ga, gb in np.ndindex(2, 2, 2, 2):
            x = r2[k, part_o[gi], part_o[gj], part_v[ga], part_v[gb]]
            if gi == gj == ga == gb:
                full = max(full, np.abs(x).max())
            else:
                mixed = max(mixed, np.abs(x).max())
    print(f"max |R| joining S and S': {mixed:.3e} (max |R| {full:.3e})", flush=True)
    assert mixed <= 1e-13 * full

    for k in (0, 2):
        x = r2[k, ks:, ks:, vs:, vs:]
        asym = max(np.abs(x + x.transpose(1, 0, 2, 3)).max(), np.abs(x + x.transpose(0, 1, 3, 2)).max())
        assert asym <= (1e-12 if prec == "fp64" else 10 * tol) * np.abs(x).max()
    del r1, r2

    # the energy is float64 in every precision (resident integrals and the reduction)
    t1[:, :ks, :vs] = 0
    t2[:, :ks, :ks, :vs, :vs] = 0
    P.set_amplitudes(t1, t2)
    e_p = P.energy()
    es = emb["e_s"]
    print(f"E_S: library {e_full - e_p:.14e}, oracle {es:.14e}", flush=True)
    assert abs((e_full - e_p) - es) <= 1e-11 * max(abs(es), abs(e_full))


def pidx(i, j, n):
    """Position of the pair i < j among the pairs of n (the library's lexicographic order)."""
    return i * (2 * n - i - 1) // 2 + j - i - 1


def check_device(P, emb, tol, run):
    """The same properties at sizes where host copies of the amplitudes would not fit: the
    amplitudes are written in place into the device set (rteom_device_sets), the residual is
    read where the library leaves it, and every comparison runs on the device.  `run` wraps
    the residual evaluation (e.g. to let its progress lines through).  Returns the errors."""
    import torch
    no, nv = P.no, P.nv
    occ, vir = np.array(P.occ_list), np.array(P.vir_list)
    os_, vs_ = emb["in_s"][occ], emb["in_s"][vir]
    ks, vs = int(os_.sum()), int(vs_.sum())
    assert os_[:ks].all() and vs_[:vs].all()      # S leads both lists (orbital 0 heads V)
    rank = np.cumsum(emb["in_s"]) - 1
    small = emb["small"]
    b1s, b2s = blocks.to_blocks(small, rank[occ[:ks]], rank[vir[:vs]], *emb["t"])
    e1, e2 = blocks.to_blocks(small, rank[occ[:ks]], rank[vir[:vs]], *emb["r"])
    npo, npv, n1 = no * (no - 1) // 2, nv * (nv - 1) // 2, no * nv
    nss, nab = npo * npv, no * no * nv * nv
    size = 2 * n1 + 2 * nss + nab
    x, r = P.device_sets()
    assert x.numel() == 2 * size
    dev = x.device

    def parts(buf, plane):
        b = buf[plane * size:(plane + 1) * size]
        return (b[:2 * n1].view(2, no, nv), b[2 * n1:2 * n1 + 2 * nss].view(2, npo, npv),
                b[2 * n1 + 2 * nss:].view(no, no, nv, nv))

    ij_s = [(i, j) for i in range(ks) for j in range(i + 1, ks)]
    ab_s = [(a, b) for a in range(vs) for b in range(a + 1, vs)]
    ps = torch.tensor([pidx(i, j, no) for i, j in ij_s], device=dev, dtype=torch.long)
    qs = torch.tensor([pidx(a, b, nv) for a, b in ab_s], device=dev, dtype=torch.long)
    p0, q0 = pidx(ks, ks + 1, no), pidx(vs, vs + 1, nv)     # first pair with both indices in S'
    pm = torch.tensor([pidx(i, j, no) for i in range(ks) for j in range(ks, no)], device=dev, dtype=torch.long)
    qm = torch.tensor([pidx(a, b, nv) for a in range(vs) for b in range(vs, nv)], device=dev, dtype=torch.long)
    gen = torch.Generator(device=dev)
    gen.manual_seed(77)

    def randn(*shape):
        return torch.randn(shape, generator=gen, device=dev, dtype=torch.float64) * 1e-3

    def write(with_s):
        x.zero_()
        for plane, part in ((0, np.real), (1, np.imag)):
            t1v, tssv, tabv = parts(x, plane)
            if with_s:
                t1v[:, :ks, :vs] = torch.from_numpy(np.ascontiguousarray(part(b1s))).to(dev)
                tabv[:ks, :ks, :vs, :vs] = torch.from_numpy(np.ascontiguousarray(part(b2s[1]))).to(dev)
                for s, blk in ((0, 0), (1, 2)):
                    vals = np.array([[part(b2s[blk][i, j, a, b]) for a, b in ab_s] for i, j in ij_s])
                    tssv[s][ps[:, None], qs[None, :]] = torch.from_numpy(vals).to(dev)
            t1v[:, ks:, vs:] = randn(2, no - ks, nv - vs)
            for i in range(ks, no):
                tabv[i, ks:, vs:, vs:] = randn(no - ks, nv - vs, nv - vs)
            for s in range(2):
                for p in range(p0, npo, 128):
                    m = min(128, npo - p)
                    tssv[s][p:p + m, q0:] = randn(m, npv - q0)
        P.amplitudes_written()

    write(True)
    e_full = P.energy()
    run(lambda: P.residual(want=False))
    if x.is_cuda:
        torch.cuda.synchronize()

    def cplx(fn):
        re, im = fn(parts(r, 0)), fn(parts(r, 1))
        return re.cpu().numpy() + 1j * im.cpu().numpy()

    g1 = cplx(lambda t: t[0][:, :ks, :vs])
    gab = cplx(lambda t: t[2][:ks, :ks, :vs, :vs])
    gss = [cplx(lambda t, s=s: t[1][s][ps][:, qs]) for s in range(2)]
    ess = [np.array([[e2[blk][i, j, a, b] for a, b in ab_s] for i, j in ij_s]) for blk in (0, 2)]
    scale = max(np.abs(e1).max(), np.abs(e2).max())
    err = max(np.abs(g1 - e1).max(), np.abs(gab - e2[1]).max(),
              max(np.abs(g - e).max() for g, e in zip(gss, ess))) / scale
    print(f"S block: max |R - R_oracle| / max |R_oracle| = {err:.3e}", flush=True)

    # every element joining S and S' vanishes (largest |Re|, |Im| on the device)
    def amax(t):
        if t.numel() == 0:
            return 0.0
        if t.numel() <= (1 << 26) or t.shape[0] == 1:
            return float(t.abs().max())
        step = max(1, t.shape[0] * (1 << 26) // t.numel())
        return max(float(t[k:k + step].abs().max()) for k in range(0, t.shape[0], step))

    mixed, full = 0.0, 0.0
    S, Sp = slice(None, ks), slice(ks, None)
    A, Ap = slice(None, vs), slice(vs, None)
    for plane in (0, 1):
        t1v, tssv, tabv = parts(r, plane)
        mixed = max(mixed, amax(t1v[:, S, Ap]), amax(t1v[:, Sp, A]))
        for gi, gj, ga, gb in np.ndindex(2, 2, 2, 2):
            blk = tabv[(S, Sp)[gi], (S, Sp)[gj], (A, Ap)[ga], (A, Ap)[gb]]
            if gi == gj == ga == gb:
                full = max(full, amax(blk))
            else:
                mixed = max(mixed, amax(blk))
        for s in range(2):
            occ_cls = [ps, pm, torch.arange(p0, npo, device=dev)]
            vir_cls = [qs, qm, torch.arange(q0, npv, device=dev)]
            for co, oi in enumerate(occ_cls):
                for cv, vi in enumerate(vir_cls):
                    if (co, cv) in ((0, 0), (2, 2)):
                        continue
                    for k in range(0, oi.numel(), 256):
                        mixed = max(mixed, amax(tssv[s][oi[k:k + 256]][:, vi]))
            full = max(full, amax(tssv[s][p0:, q0:]))
    print(f"max |R| joining S and S': {mixed:.3e} (max |R| {full:.3e})", flush=True)

    # the energy splits: E(T) - E(T with T_S = 0) = E_S(T_S)
    gen.manual_seed(77)
    write(False)
    e_s = e_full - P.energy()
    print(f"E_S: library {e_s:.14e}, oracle {emb['e_s']:.14e}", flush=True)
    return err, mixed / full, abs(e_s - emb["e_s"]) / max(abs(emb["e_s"]), abs(e_full))
