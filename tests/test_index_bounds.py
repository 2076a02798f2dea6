"""Host replica of the global-memory index arithmetic of the fused and plain kernels,
with a bounds check on every access (CPU only).

For each kernel the replica computes, for every thread of every workgroup of a
launch, the element index of every global load and store the device code issues --
the same expressions as the kernels (clamped fetch rows and columns, vector and scalar
paths, prologue and epilogue, the stages fetched past the last tile of a sweep) --
and asserts that each index lies inside its buffer, and that every 16-byte access is
16-byte aligned.  The buffers' extents follow the plan's workspace layout and the
caller's packed layout.  Shapes: every width 1..256 with row counts on and off the
tile boundaries, single-sample layers, and element offsets that are not multiples of
four (the unaligned paths)."""
import numpy as np
import pytest

WAVE = 64


def cdiv(a, b):
    return -(-a // b)


def nkc_bucket(D):
    need = cdiv(D, 16)
    return next(b for b in (1, 2, 3, 4, 5, 6, 7, 8, 12, 16) if b >= need)


class Buffers:
    """Extents (elements) of the regions a launch touches; check() records violations."""

    def __init__(self, **sizes):
        self.size = dict(sizes)
        self.bad = []

    def check(self, name, idx, width=1, mask=None, vec=False, block=None):
        """Every index (where mask) in [0, size) of its buffer, and in [lo, hi) of the
        block it belongs to when `block` = (lo, hi) is given (a read of a neighbouring
        layer's block would not fault but would be a wrong value)."""
        idx = np.asarray(idx, dtype=np.int64)
        if mask is not None:
            idx = idx[np.broadcast_to(np.asarray(mask), idx.shape)]
        if idx.size == 0:
            return
        n = self.size[name]
        lo, hi = int(idx.min()), int(idx.max())
        if lo < 0 or hi + width > n:
            self.bad.append((name, lo, hi + width, n))
        if block is not None and (lo < block[0] or hi + width > block[1]):
            self.bad.append((name, "outside its block", lo, hi + width, block))
        if vec and np.any(idx % 4 != 0):
            self.bad.append((name, "misaligned float4", int(idx[idx % 4 != 0][0])))


def layout(shapes, z_shift=0):
    """Layer table of the ragged packing (tmc.ragged_problem) and the fused engine's
    workspace offsets (tmc_api.cpp build_plan, fused.cpp fused_build).  z_shift moves
    every z, mu and u block by that many elements (unaligned rows)."""
    layers, zo, uo, mo, so = [], z_shift, z_shift, z_shift, 0
    sumK = sum_w = sq = ev = dsp = 0
    for Ks, Ds in shapes:
        L = len(Ks)
        first = len(layers)
        for l in range(L):
            top = l == L - 1
            d = dict(K=Ks[l], D=Ds[l], z_off=zo, u_off=uo, top=top, first=first, L=L, depth=l)
            zo += Ks[l] * Ds[l]
            uo += Ks[l]
            d.update(alpha_off=sumK, wmax_off=sum_w)
            sumK += Ks[l]
            sum_w += cdiv(Ks[l], 128)
            if not top:
                d.update(Kc=Ks[l + 1], mu_off=mo, s_off=so)
                mo += Ks[l + 1] * Ds[l]
                so += Ds[l]
            else:
                d.update(Kc=0, mu_off=0, s_off=0)
            layers.append(d)
        for l in range(L - 1):
            d, U = layers[first + l], layers[first + l + 1]
            d.update(alpha_up_off=U["alpha_off"], wmax_up_off=U["wmax_off"],
                     nwmax_up=cdiv(U["K"], 128), u_up_off=U["u_off"], up_top=U["top"])
    for d in layers:
        if d["top"]:
            continue
        d["ev_off"] = ev
        d["dz_aligned"] = d["D"] % 4 == 0 and d["z_off"] % 4 == 0 and ev % 4 == 0
        ev += d["K"] * d["D"]
        d["q_off"] = sq
        sq += d["Kc"]
        d["dsp_parts"] = cdiv(d["Kc"], 128) + cdiv(d["K"], 64)
        d["dsp_off"] = dsp
        dsp += d["D"] * d["dsp_parts"]
    bufs = dict(z=max(zo, 1), u=max(uo, 1), mu=max(mo, 1), s=max(so, 1), alpha=sumK, rl=sumK,
                lam=sumK, p=sumK, wmax=sum_w, q=max(sq, 1), ev=max(ev, 1), dsp=max(dsp, 1),
                dz=max(zo, 1), dmu=max(mo, 1), du=max(uo, 1))
    return layers, bufs


# ---------------------------------------------------------------------------
# fused engine (fused_kernels.h)
# ---------------------------------------------------------------------------

def pair_preload(B, L, tid):
    lane = tid & 63
    wb = (L["wmax_up_off"], L["wmax_up_off"] + L["nwmax_up"])
    sb = (L["s_off"], L["s_off"] + L["D"])
    B.check("wmax", L["wmax_up_off"] + np.minimum(lane, L["nwmax_up"] - 1), block=wb)
    for k in range(4):
        B.check("s", L["s_off"] + np.minimum(lane + 64 * k, L["D"] - 1), block=sb)
    B.check("s", L["s_off"] + np.minimum(tid, L["D"] - 1), block=sb)
    for k in range(64, L["nwmax_up"] + 64, 64):          # pair_maxa's strided loop
        kk = lane + k
        B.check("wmax", L["wmax_up_off"] + kk, mask=kk < L["nwmax_up"], block=wb)


def wave_load(B, buf, off, n, D, r0, tid, nkc):
    lane = tid & 63
    h = lane >> 5
    r = np.minimum(r0 + (lane & 31), n - 1)
    row = off + r * D
    blk = (off, off + n * D)
    if D % 4 == 0 and off % 4 == 0:
        for kc in range(nkc):
            for e in range(2):
                B.check(buf, row + np.minimum(kc * 16 + 8 * h + 4 * e, D - 4), 4, vec=True, block=blk)
    else:
        for kc in range(nkc):
            for s_ in range(8):
                B.check(buf, row + np.minimum(kc * 16 + 8 * h + s_, D - 1), block=blk)


def fetch_tile(B, L, tid, r0, nkc, wv, cols, dzw=False):
    """fetch_cols (cols=True: mu rows and alpha_{l+1}) / fetch_rows (z rows, row shifts,
    and with dzw the e rows and marginals of the rows)."""
    TPR = 2 * wv
    NF = cdiv(nkc, 2)
    NFT = NF * 8 // TPR
    sub = tid % TPR
    D = L["D"]
    n = L["Kc"] if cols else L["K"]
    off = L["mu_off"] if cols else L["z_off"]
    buf = "mu" if cols else "z"
    vec = D % 4 == 0 and off % 4 == 0
    gr = r0 + tid // TPR
    blk = (off, off + n * D)
    ab = (L["alpha_up_off"], L["alpha_up_off"] + L["Kc"])
    rb = (L["alpha_off"], L["alpha_off"] + L["K"])
    eb = (L["ev_off"], L["ev_off"] + L["K"] * D)
    if vec:
        gc = np.minimum(gr, n - 1)
        rowp = off + gc * D
        for m in range(NFT):
            B.check(buf, rowp + np.minimum(4 * (sub + TPR * m), D - 4), 4, vec=True, block=blk)
        if cols:
            B.check("alpha", L["alpha_up_off"] + gc, block=ab)
        elif dzw:
            erow = L["ev_off"] + gc * D
            for m in range(NFT):
                B.check("ev", erow + np.minimum(4 * (sub + TPR * m), D - 4), 4, vec=True, block=eb)
            B.check("p", L["alpha_off"] + gc, block=rb)
    else:
        gc = np.where(gr < n, gr, n - 1)
        rowp = off + gc * D
        for m in range(NFT):
            d = 4 * (sub + TPR * m)
            for e in range(4):
                B.check(buf, rowp + np.minimum(d + e, D - 1), block=blk)
        if cols:
            B.check("alpha", L["alpha_up_off"] + gc, block=ab)
    if not cols:
        rr = r0 + (tid & 31)
        B.check("lam", L["alpha_off"] + np.minimum(rr, L["K"] - 1), block=rb)


def sweep_starts(n_tiles, stages):
    """Tile starts (in tiles) a sweep fetches: the pipelined sweep (three stages) also
    fetches up to three tiles past the last one (clamped), the two-stage sweep one."""
    if stages == 3:
        return list(range(0, n_tiles + 3))
    return list(range(0, n_tiles + (1 if stages == 2 else 0)))


def fused_fwd_item(B, L, start, wv, prec, grad=True):
    nkc = nkc_bucket(L["D"])
    stages = (3 if prec == "bf16x3" else 2) if nkc <= 8 else 1
    tid = np.arange(64 * wv)
    w, lane = tid >> 6, tid & 63
    h = lane >> 5
    i = start + 32 * w + (lane & 31)
    pair_preload(B, L, tid)
    B.check("u", L["u_off"] + np.minimum(i, L["K"] - 1), block=(L["u_off"], L["u_off"] + L["K"]))
    wave_load(B, "z", L["z_off"], L["K"], L["D"], start + 32 * w, tid, nkc)
    nt = cdiv(L["Kc"], 32)
    for t in sweep_starts(nt, stages):
        fetch_tile(B, L, tid, 32 * t, nkc, wv, cols=True)
        j = 32 * t + tid // (2 * wv)
        if grad and start == 0:
            B.check("q", L["q_off"] + j, mask=(tid % (2 * wv) == 0) & (j < L["Kc"]),
                    block=(L["q_off"], L["q_off"] + L["Kc"]))
    iv = i < L["K"]
    rb = (L["alpha_off"], L["alpha_off"] + L["K"])
    B.check("rl", L["alpha_off"] + i, mask=iv & (h == 0), block=rb)
    B.check("alpha", L["alpha_off"] + i, mask=iv & (h == 0), block=rb)
    p128 = tid[: wv // 4]
    B.check("wmax", L["wmax_off"] + start // 128 + p128, mask=start + 128 * p128 < L["K"],
            block=(L["wmax_off"], L["wmax_off"] + cdiv(L["K"], 128)))
    if grad:
        D = L["D"]
        erow = L["ev_off"] + i * D
        vec = D % 4 == 0 and L["ev_off"] % 4 == 0
        for q in range(cdiv(nkc, 2)):
            for g in range(4):
                d = 32 * q + 8 * g + 4 * h
                eb = (L["ev_off"], L["ev_off"] + L["K"] * D)
                if vec:
                    B.check("ev", erow + d, 4, mask=iv & (d < D), vec=True, block=eb)
                else:
                    for e in range(4):
                        B.check("ev", erow + d + e, mask=iv & (d + e < D), block=eb)


def fused_bwd_item(B, L, start, wv, prec, rows):
    nkc = nkc_bucket(L["D"])
    stages = (3 if prec == "bf16x3" else 2) if nkc <= 8 else 1
    tid = np.arange(64 * wv)
    w, lane = tid >> 6, tid & 63
    h = lane >> 5
    jw = start + 32 * w
    j = jw + (lane & 31)
    jc = np.minimum(j, L["Kc"] - 1)
    pair_preload(B, L, tid)
    B.check("q", L["q_off"] + jc, block=(L["q_off"], L["q_off"] + L["Kc"]))
    B.check("alpha", L["alpha_up_off"] + jc, block=(L["alpha_up_off"], L["alpha_up_off"] + L["Kc"]))
    wave_load(B, "mu", L["mu_off"], L["Kc"], L["D"], jw, tid, nkc)
    nt = cdiv(L["K"], 32)
    dzw = wv == 8 and rows and L.get("dz_fused", False)
    wg_c, nwg = start // 256, cdiv(L["Kc"], 256)
    TPR = 2 * wv
    NFT = cdiv(nkc, 2) * 8 // TPR
    D = L["D"]
    for t in sweep_starts(nt, stages):
        own = dzw and t % nwg == wg_c and t < nt
        fetch_tile(B, L, tid, 32 * t, nkc, wv, cols=False, dzw=own)
        if own:   # the 8-wave row terms: dz rows of the staged tile
            row = 32 * t + tid // TPR
            sub = tid % TPR
            for m in range(NFT):
                c = 4 * (sub + TPR * m)
                B.check("dz", L["z_off"] + row * D + c, 4, mask=(row < L["K"]) & (c < D), vec=True,
                        block=(L["z_off"], L["z_off"] + L["K"] * D))
    jv = j < L["Kc"]
    ub = (L["alpha_up_off"], L["alpha_up_off"] + L["Kc"])
    B.check("p", L["alpha_up_off"] + j, mask=jv & (h == 0), block=ub)
    B.check("du", L["u_up_off"] + j, mask=jv & (h == 0), block=(L["u_up_off"], L["u_up_off"] + L["Kc"]))
    if not L["up_top"]:
        B.check("rl", L["alpha_up_off"] + j, mask=jv & (h == 0), block=ub)
        B.check("lam", L["alpha_up_off"] + j, mask=jv & (h == 0), block=ub)
    murow = L["mu_off"] + jc * D
    vec = D % 4 == 0 and L["mu_off"] % 4 == 0
    mb = (L["mu_off"], L["mu_off"] + L["Kc"] * D)
    for q in range(cdiv(nkc, 2)):
        for g in range(4):
            d = 32 * q + 8 * g + 4 * h
            if vec:
                B.check("mu", murow + np.minimum(d, D - 4), 4, vec=True, block=mb)
                B.check("dmu", murow + d, 4, mask=jv & (d < D), vec=True, block=mb)
            else:
                for e in range(4):
                    B.check("mu", murow + np.minimum(d + e, D - 1), block=mb)
                    B.check("dmu", murow + d + e, mask=jv & (d + e < D), block=mb)
    ncol = cdiv(L["Kc"], 128)
    nrow = cdiv(L["K"], 64)
    dd = np.arange(D)
    db = (L["dsp_off"], L["dsp_off"] + L["dsp_parts"] * D)
    if dzw:
        B.check("dsp", L["dsp_off"] + (ncol + wg_c) * D + dd, block=db)
        if wg_c == 0:
            e = np.arange((nrow - nwg) * D)
            B.check("dsp", L["dsp_off"] + (ncol + wg_c) * D + nwg * D + e, block=db)
    for hh in range(wv // 4):
        if start + 128 * hh >= L["Kc"]:
            break
        B.check("dsp", L["dsp_off"] + (start // 128 + hh) * D + dd, block=db)


def fused_dz_item(B, L, r0):
    tid = np.arange(256)
    D, K = L["D"], L["K"]
    cw = 4
    while cw < 32 and 4 * cw < D:
        cw *= 2
    c4, rg = tid & (cw - 1), tid // cw
    nrg = 256 // cw
    assert 64 % nrg == 0
    B.check("s", L["s_off"] + np.arange(D))
    B.check("p", L["alpha_off"] + r0 + tid, mask=(tid < 64) & (r0 + tid < K))
    vec = D % 4 == 0 and L["z_off"] % 4 == 0 and L["ev_off"] % 4 == 0
    for d0 in range(0, D, 4 * cw):
        d = d0 + 4 * c4
        for rr in range(64 // nrg):
            i = r0 + rg + nrg * rr
            ok = (d < D) & (i < K)
            B.check("p", L["alpha_off"] + i, mask=ok)
            o = i * D + d
            srcs = (("z", L["z_off"]), ("ev", L["ev_off"]), ("dz", L["z_off"]))
            if vec:
                full = ok & (d + 3 < D)
                for buf, base in srcs:
                    B.check(buf, base + o, 4, mask=full, vec=True, block=(base, base + K * D))
                part = ok & ~(d + 3 < D)
            else:
                part = ok
            for e in range(4):
                for buf, base in srcs:
                    B.check(buf, base + o + e, mask=part & (d + e < D), block=(base, base + K * D))
        ncol = cdiv(L["Kc"], 128)
        for e in range(4):
            B.check("dsp", L["dsp_off"] + (ncol + r0 // 64) * D + d + e,
                    mask=(rg == 0) & (d + e < D), block=(L["dsp_off"], L["dsp_off"] + L["dsp_parts"] * D))


def check_fused(shapes, prec, z_shift=0):
    layers, sizes = layout(shapes, z_shift)
    bad = []
    for wide in (False, True):
        B = Buffers(**sizes)
        covered = set()
        for li, L in enumerate(layers):
            if L["top"]:
                continue
            nkc = nkc_bucket(L["D"])
            wok = nkc in (7, 8)
            wvf = 8 if wide and wok and L["K"] >= 256 else 4
            wvb = 8 if wide and wok and L["Kc"] >= 256 else 4
            if wvb == 8 and L["dz_aligned"] and cdiv(L["Kc"], 256) <= cdiv(L["K"], 64):
                covered.add(li)
            L["dz_fused"] = li in covered
            for st in range(0, L["K"], 32 * wvf):
                fused_fwd_item(B, L, st, wvf, prec)
            for st in range(0, L["Kc"], 32 * wvb):
                fused_bwd_item(B, L, st, wvb, prec, rows=True)
            if li not in covered:
                for r in range(0, L["K"], 64):
                    fused_dz_item(B, L, r)
        bad += B.bad
    return bad


# ---------------------------------------------------------------------------
# plain engine (k_plain.hip): stored factors
# ---------------------------------------------------------------------------

PLAIN_FWD_R, PLAIN_FWD_W = 4, 16  # forward log-sum-exp: rows per wave, waves per workgroup


def check_plain(shapes, esz):
    layers, sizes = layout(shapes)
    VV = 4 if esz == 4 else 2
    wf = 0
    for L in layers:
        if not L["top"]:
            L["wf_off"] = wf
            wf += cdiv(L["K"] * L["Kc"], 4) * 4
    B = Buffers(**sizes, wf=max(wf, 1), anchor=sizes["alpha"])
    for L in layers:
        if L["top"]:
            continue
        K, Kc, D = L["K"], L["Kc"], L["D"]
        # factor tiles: 32 rows x 64 columns
        tid = np.arange(256)
        col, rsub = tid % 64, tid // 64
        for it in range(cdiv(K, 32) * cdiv(Kc, 64)):
            i0, j0 = (it // cdiv(Kc, 64)) * 32, (it % cdiv(Kc, 64)) * 64
            j = j0 + col
            for q in range(8):
                i = i0 + rsub + 4 * q
                B.check("wf", L["wf_off"] + i * Kc + j, mask=(j < Kc) & (i < K),
                        block=(L["wf_off"], L["wf_off"] + K * Kc))
            B.check("anchor", L["alpha_off"] + i0 + tid, mask=(j0 == 0) & (tid < 32) & (i0 + tid < K))
        # forward row sweeps: PLAIN_FWD_R rows per wave, PLAIN_FWD_W waves
        vec = Kc % VV == 0 and L["wf_off"] % VV == 0
        V = VV if vec else 1
        for start in range(0, K, PLAIN_FWD_R * PLAIN_FWD_W):
            for w in range(PLAIN_FWD_W):
                i0 = start + PLAIN_FWD_R * w
                if i0 >= K:
                    continue
                nrow = min(PLAIN_FWD_R, K - i0)
                lane = np.arange(64)
                for base in range(0, Kc, 64 * V):
                    jj = base + lane * V
                    ok = jj < Kc
                    for r in range(PLAIN_FWD_R):
                        rr = min(r, nrow - 1)
                        B.check("wf", L["wf_off"] + (i0 + rr) * Kc + jj, V, mask=ok,
                                vec=V == 4 and esz == 4, block=(L["wf_off"], L["wf_off"] + K * Kc))
        # backward column strips
        vecb = Kc >= 64 * VV and Kc % VV == 0 and L["wf_off"] % VV == 0
        Vb = VV if vecb else 1
        for j0 in range(0, Kc, 64 * Vb):
            tid = np.arange(64 * 16)
            w, lane = tid // 64, tid % 64
            j = j0 + lane * Vb
            active = j < Kc
            jc = np.where(active, j, 0)
            for i0 in range(0, K, 16 * 4):
                for r in range(4):
                    i = np.minimum(i0 + w + 16 * r, K - 1)
                    fb = (L["wf_off"], L["wf_off"] + K * Kc)
                    B.check("wf", L["wf_off"] + i * Kc + jc, Vb, block=fb)
                    live = (i0 + w + 16 * r < K) & active
                    B.check("wf", L["wf_off"] + (i0 + w + 16 * r) * Kc + j, Vb, mask=live, block=fb)
    return B.bad


# ---------------------------------------------------------------------------

SWEEP = [((K0, K1), (D, D2)) for D in list(range(1, 130)) + [131, 160, 192, 200, 255, 256]
         for (K0, K1, D2) in [(1, 1, 1), (33, 257, 3), (256, 31, 64)]]
TEST_SHAPES = [((3,), (2,)), ((17, 3), (5, 1)), ((63, 65, 130), (33, 3, 65)),
               ((1, 1, 1), (4, 4, 4)), ((257, 17, 64, 5, 9), (100, 7, 2, 1, 3)),
               ((130, 257), (200, 16)), ((40, 300, 33), (256, 129, 64)), ((31, 32, 33), (16, 17, 15)),
               ((300, 256, 257), (100, 112, 128)), ((257, 300), (128, 97)),
               ((256, 64, 256), (104, 100, 120)), ((129, 520), (128, 100)),
               ((300, 256), (99, 64)), ((64, 600), (128, 64)), ((256,) * 6, (100,) * 6),
               ((2048, 2048, 2048), (128, 128, 128))]


@pytest.mark.parametrize("prec", ["bf16x3", "fp32"])
@pytest.mark.parametrize("z_shift", [0, 1, 2])
def test_fused_accesses_in_bounds(prec, z_shift):
    bad = check_fused(TEST_SHAPES, prec, z_shift)
    assert not bad, bad[:5]


@pytest.mark.parametrize("prec", ["bf16x3", "fp32"])
def test_fused_accesses_in_bounds_every_width(prec):
    for k in range(0, len(SWEEP), 16):
        bad = check_fused(SWEEP[k:k + 16], prec, z_shift=k % 3)
        assert not bad, (SWEEP[k:k + 16], bad[:5])


@pytest.mark.parametrize("esz", [4, 8])
def test_plain_accesses_in_bounds(esz):
    bad = check_plain(TEST_SHAPES[:12], esz)
    assert not bad, bad[:5]


def test_replica_detects_unclamped_rows(monkeypatch):
    """The check itself: with the row clamps taken out of the replica (the indices a
    fetch or a wave load without them would touch) accesses outside their blocks and
    past the buffers are reported."""
    mod = __import__(__name__, fromlist=["x"])

    def fetch_unclamped(B, L, tid, r0, nkc, wv, cols, dzw=False):
        TPR, D = 2 * wv, L["D"]
        off = L["mu_off"] if cols else L["z_off"]
        n = L["Kc"] if cols else L["K"]
        gr = r0 + tid // TPR
        B.check("mu" if cols else "z", off + gr * D, block=(off, off + n * D))

    monkeypatch.setattr(mod, "fetch_tile", fetch_unclamped)
    assert check_fused([((33, 3), (5, 5))], "fp32")

    def wave_unclamped(B, buf, off, n, D, r0, tid, nkc):
        B.check(buf, off + (r0 + (tid & 31)) * D, block=(off, off + n * D))

    monkeypatch.undo()
    monkeypatch.setattr(mod, "wave_load", wave_unclamped)
    assert check_fused([((33, 3), (5, 5))], "fp32")


# ---------------------------------------------------------------------------
# star-model kernels
# ---------------------------------------------------------------------------

STAR_LANES, STAR_WAVES, STAR_TARGET = 64, 4, 2048


def star_layout(S, N, Kt, K, D):
    """The plan's point grouping (points per group P, groups, local-sample blocks)."""
    nkt = cdiv(Kt, STAR_LANES)
    P = max(min(N, STAR_WAVES), min(N, S * N * nkt // STAR_TARGET))
    return dict(S=S, N=N, Kt=Kt, K=K, D=D, P=P, ngrp=cdiv(N, P), nkb=cdiv(K, STAR_LANES), nkt=nkt)


def check_star(S, N, Kt, K, D):
    """Every global access of the six star kernels, per wave (vectorised over its lanes;
    rows that a whole wave reads are scalar loads at one address), against the caller's
    buffers and the workspace arrays."""
    a = star_layout(S, N, Kt, K, D)
    P, ngrp, nkb, nkt = a["P"], a["ngrp"], a["nkb"], a["nkt"]
    B = Buffers(mth=S * Kt * D, s=S * D, z=S * N * K * D, u=S * N * K, uth=S * Kt,
                msg=S * N * Kt, gsum=S * ngrp * Kt, w=S * Kt, dm=S * ngrp * Kt * D,
                dsp=S * N * nkb * D, dz=S * N * K * D, du=S * N * K, dmth=S * Kt * D,
                ds=S * D, duth=S * Kt, nsh=S * N * Kt, wT=S * Kt)
    lane = np.arange(STAR_LANES)
    stride = 1 if D == 1 else D
    assert S * ngrp < 2 ** 31 and nkt <= 65535 and nkb <= 65535
    # k_star_msg and k_star_bwd_global: grid (S ngrp, nkt) of 4 waves, lane -> kt; wave wv
    # walks points grp P + wv, + 4, ... and all K rows of each (scalar loads)
    for bx in range(S * ngrp):
        inst, grp = bx // ngrp, bx % ngrp
        assert inst < S
        for by in range(nkt):
            kt = by * STAR_LANES + lane
            ktv = kt < Kt
            for d in range(D):
                B.check("mth", (inst * Kt + kt) * D + d, mask=ktv)
                B.check("dm", ((inst * ngrp + grp) * Kt + kt) * D + d, mask=ktv)
            B.check("wT", inst * Kt + kt, mask=ktv)
            B.check("gsum", (inst * ngrp + grp) * Kt + kt, mask=ktv)
            for wv in range(STAR_WAVES):
                for pt in range(grp * P + wv, min(N, (grp + 1) * P), STAR_WAVES):
                    pi = inst * N + pt
                    B.check("msg", pi * Kt + kt, mask=ktv)
                    B.check("nsh", pi * Kt + kt, mask=ktv)
                    k = np.arange(K)
                    zb = (pi * K * D, (pi + 1) * K * D)
                    for d in range(D):
                        B.check("z", pi * K * D + k * stride + d, block=zb)
                    B.check("u", pi * K + k, block=(pi * K, (pi + 1) * K))
    # k_star_colsum: grid (S, nkt); lanes past Kt read column 0
    for inst in range(S):
        for by in range(nkt):
            kt = by * STAR_LANES + lane
            kc = np.where(kt < Kt, kt, 0)
            for g in range(ngrp):
                B.check("gsum", (inst * ngrp + g) * Kt + kc)
            B.check("uth", inst * Kt + kt, mask=kt < Kt)
    # k_star_bwd_local: one wave per (instance and point, 64 local samples), grid of 4-wave
    # workgroups over the S N nkb tasks (waves past the last task return at once)
    tasks = S * N * nkb
    for task in range(cdiv(tasks, STAR_WAVES) * STAR_WAVES):
        if task >= tasks:
            continue
        pi, kb = task // nkb, task % nkb
        inst = pi // N
        k = kb * STAR_LANES + lane
        kv = k < K
        for d in range(D):
            B.check("z", (pi * K + k) * D + d, mask=kv)
            B.check("dz", (pi * K + k) * D + d, mask=kv)
            B.check("dsp", (pi * nkb + kb) * D + d)
        B.check("u", pi * K + k, mask=kv)
        B.check("du", pi * K + k, mask=kv)
        t = np.arange(Kt)
        for d in range(D):
            B.check("mth", inst * Kt * D + t * stride + d, block=(inst * Kt * D, (inst + 1) * Kt * D))
        B.check("wT", inst * Kt + t)
        B.check("nsh", pi * Kt + t, block=(pi * Kt, (pi + 1) * Kt))
    # k_star_reduce: grid (S, ceil(Kt D / 64) + 1); lanes past Kt D read entry 0
    KD = Kt * D
    ny = cdiv(KD, STAR_LANES) + 1
    assert ny <= 65535
    for inst in range(S):
        for by in range(ny - 1):
            e = by * STAR_LANES + lane
            ec = np.where(e < KD, e, 0)
            for gi in range(ngrp):
                B.check("dm", (inst * ngrp + gi) * KD + ec)
            B.check("dmth", inst * KD + e, mask=e < KD)
            B.check("s", inst * D + e % D, mask=e < KD)
        j = np.arange(N * nkb)
        for d in range(D):
            B.check("dsp", inst * N * nkb * D + j * D + d)
            B.check("ds", inst * D + d)
        B.check("duth", inst * Kt + np.arange(Kt))
        B.check("w", inst * Kt + np.arange(Kt))
        B.check("wT", inst * Kt + np.arange(Kt))
    assert not B.bad, B.bad[:5]
    return a


@pytest.mark.parametrize("shape", [(1, 1, 1, 1, 1), (2, 37, 150, 100, 3), (1, 3001, 100, 20, 2),
                                   (3, 5, 64, 128, 32), (1, 4, 65, 129, 16), (2, 2, 1, 1, 7),
                                   (1, 9, 70, 13, 1)])
def test_star_accesses_in_bounds(shape):
    check_star(*shape)


def test_star_grouping():
    """Point groups: at least one point per wave, more once the forward grid would exceed
    the target (the last group ragged), never more than N."""
    assert star_layout(2, 37, 150, 100, 3)["P"] == 4
    a = star_layout(1, 3001, 100, 20, 2)
    assert (a["P"], a["ngrp"]) == (4, 751)
    a = star_layout(1, 4096, 128, 128, 1)
    assert (a["P"], a["ngrp"]) == (4, 1024)
    a = star_layout(1, 9000, 128, 128, 1)
    assert (a["P"], a["ngrp"]) == (8, 1125)
    assert star_layout(1, 2, 64 * 5000, 8, 1)["P"] == 2


# ---------------------------------------------------------------------------
# log-domain matrix product
# ---------------------------------------------------------------------------

LOGMM_TILE = 128


COLMAX_CW = 32   # columns of a column-maximum workgroup of the log-domain product


def check_logmm(B, M, K, N):
    """Every global access of the log-domain product kernels (row and column maxima, the
    operand preparation, the MFMA tile kernel, the exact fix-up) per thread.  Operand
    buffers are counted in elements of one BF16 plane pair (2 B M Kp, 2 B N Kp); the FP32
    form uses the first half of each with 4-byte elements, the same bytes."""
    Kp = cdiv(K, 32) * 32
    Bf = Buffers(X=B * M * K, Y=B * K * N, Z=B * M * N, xs=B * M, ys=B * N,
                 opa=2 * B * M * Kp, opb=2 * B * N * Kp)
    t = np.arange(256)
    # operand preparation of X, rows of at most 1024 aligned floats: one read of 4
    # consecutive j per lane and 256-wide chunk, the same positions written
    if Kp <= 1024 and K % 4 == 0:
        lane = np.arange(64)
        for row in range(B * M):
            for c in range(4):
                e = 4 * (lane + 64 * c)
                for i in range(4):
                    Bf.check("X", row * K + e + i, mask=e < K)
                    Bf.check("opa", row * Kp + e + i, mask=e < Kp)
                    Bf.check("opa", B * M * Kp + row * Kp + e + i, mask=e < Kp)
            Bf.check("xs", row)
    # operand preparation of X otherwise: a wave per row (its maximum, then 8 consecutive
    # j per lane)
    for row in range(B * M):
        lane = np.arange(64)
        for jj in range(0, K, 64):
            Bf.check("X", row * K + jj + lane, mask=jj + lane < K)
        Bf.check("xs", row)
        for j0 in range(0, Kp, 8 * 64):
            jl = j0 + 8 * lane
            for s_ in range(8):
                Bf.check("X", row * K + jl + s_, mask=(jl < Kp) & (jl + s_ < K))
                Bf.check("opa", row * Kp + jl + s_, mask=jl < Kp)
                Bf.check("opa", B * M * Kp + row * Kp + jl + s_, mask=jl < Kp)
    for b in range(B):
        # column maxima: 16 waves per COLMAX_CW columns (lane: column l % CW, row group
        # 64 / CW w + l / CW), lanes past N read column 0
        CW = COLMAX_CW
        tc = np.arange(1024)
        c, g = (tc % 64) % CW, (64 // CW) * (tc // 64) + (tc % 64) // CW
        rs = 16 * (64 // CW)
        for bx in range(cdiv(N, CW)):
            col = bx * CW + c
            cc = np.where(col < N, col, 0)
            for j0 in range(0, K, rs * 8):
                for q in range(8):
                    j = j0 + g + rs * q
                    Bf.check("Y", b * K * N + j * N + cc, mask=j < K)
            colm = bx * CW + np.arange(CW)
            Bf.check("ys", b * N + colm, mask=colm < N)
        # operand preparation of Y: 64 j x 64 k tiles through LDS
        for jx in range(cdiv(Kp, 64)):
            for ky in range(cdiv(N, 64)):
                jb0, kb0 = jx * 64, ky * 64
                k = kb0 + t % 64
                Bf.check("ys", b * N + k, mask=k < N)
                for r in range(16):
                    j = jb0 + 16 * (t // 64) + r
                    Bf.check("Y", b * K * N + j * N + k, mask=(j < K) & (k < N))
                kw = kb0 + t // 4
                jc = (t % 4) * 16
                for h in range(2):
                    m = (kw < N) & (jb0 + jc + 8 * h < Kp)
                    for s_ in range(8):
                        o = (b * N + kw) * Kp + jb0 + jc + 8 * h + s_
                        Bf.check("opb", o, mask=m, block=None)
                        Bf.check("opb", B * N * Kp + o, mask=m)
        # MFMA tiles: row t / 2 of each operand tile (clamped), 16 consecutive j per slice
        for by in range(cdiv(M, LOGMM_TILE)):
            for bx in range(cdiv(N, LOGMM_TILE)):
                i0, k0 = by * LOGMM_TILE, bx * LOGMM_TILE
                r, jg = t // 2, (t % 2) * 16
                ra = (b * M + np.minimum(i0 + r, M - 1)) * Kp + jg
                rb = (b * N + np.minimum(k0 + r, N - 1)) * Kp + jg
                # slices 0 and 1 before the loop, then in step s slice s + 2 (past the
                # end the last slice again)
                ns = Kp // 32
                for jj in [0, min(32, Kp - 32)] + [min((s2 + 2) * 32, Kp - 32) for s2 in range(ns)]:
                    for s_ in range(16):
                        Bf.check("opa", ra + jj + s_, block=None)
                        Bf.check("opa", B * M * Kp + ra + jj + s_)
                        Bf.check("opb", rb + jj + s_, block=None)
                        Bf.check("opb", B * N * Kp + rb + jj + s_)
                        assert np.all((jg + s_) < 32)
                lane, w = t % 64, t // 64
                wr, wc = 64 * (w // 2), 64 * (w % 2)
                for q in range(2):
                    k = k0 + wc + 32 * q + lane % 32
                    for p in range(2):
                        for v in range(16):
                            i = i0 + wr + 32 * p + 8 * (v // 4) + 4 * (lane // 32) + v % 4
                            live = (k < N) & (i < M)
                            Bf.check("Z", (b * M + i) * N + k, mask=live)
                            Bf.check("xs", b * M + i, mask=live)
                            if p == 0 and v == 0:   # the exact recompute of an entry (rows i, columns k)
                                for j in range(K):
                                    Bf.check("X", (b * M + i) * K + j, mask=live)
                                    Bf.check("Y", b * K * N + j * N + k, mask=live)
                    Bf.check("ys", b * N + k, mask=k < N)
    assert not Bf.bad, Bf.bad[:5]


def check_logmm_f64(B, M, K, N):
    """The FP64 product kernel (8 waves per 128 x 128 tile, 16-wide slices, thread t: row
    t / 4 and 4 consecutive j of each operand tile; accumulator value v of lane l at row
    l / 16 + 4 v, column l % 16 of its 16 x 16 block).  Buffers in doubles; the row and
    column maxima and the operand preparation index like the FP32 form (one plane)."""
    Kp = cdiv(K, 32) * 32
    Bf = Buffers(X=B * M * K, Y=B * K * N, Z=B * M * N, xs=B * M, ys=B * N,
                 opa=B * M * Kp, opb=B * N * Kp)
    if Kp <= 1024 and K % 2 == 0:   # rows of X in one read: 2 j of 8 chunks per lane
        lane = np.arange(64)
        for row in range(B * M):
            for c in range(8):
                e = 2 * (lane + 64 * c)
                for i in range(2):
                    Bf.check("X", row * K + e + i, mask=e < K)
                    Bf.check("opa", row * Kp + e + i, mask=e < Kp)
            Bf.check("xs", row)
    t = np.arange(512)
    for b in range(B):
        for by in range(cdiv(M, LOGMM_TILE)):
            for bx in range(cdiv(N, LOGMM_TILE)):
                i0, k0 = by * LOGMM_TILE, bx * LOGMM_TILE
                r, jg = t // 4, (t % 4) * 4
                ra = (b * M + np.minimum(i0 + r, M - 1)) * Kp + jg
                rb = (b * N + np.minimum(k0 + r, N - 1)) * Kp + jg
                for jj in [0] + [min(j0 + 16, Kp - 16) for j0 in range(0, Kp, 16)]:
                    for s_ in range(4):
                        Bf.check("opa", ra + jj + s_, block=None)
                        Bf.check("opb", rb + jj + s_, block=None)
                        assert np.all((jg + s_) < 16)
                lane, w = t % 64, t // 64
                wr, wc = 64 * (w // 4), 32 * (w % 4)
                assert np.all(wr + 48 + 15 < LOGMM_TILE) and np.all(wc + 16 + 15 < LOGMM_TILE)
                for q in range(2):
                    k = k0 + wc + 16 * q + lane % 16
                    Bf.check("ys", b * N + k, mask=k < N)
                    for p in range(4):
                        for v in range(4):
                            i = i0 + wr + 16 * p + lane // 16 + 4 * v
                            live = (k < N) & (i < M)
                            Bf.check("Z", (b * M + i) * N + k, mask=live)
                            Bf.check("xs", b * M + i, mask=live)
                            if p == 0 and v == 0:   # the exact recompute of an entry
                                for j in range(K):
                                    Bf.check("X", (b * M + i) * K + j, mask=live)
                                    Bf.check("Y", b * K * N + j * N + k, mask=live)
    assert not Bf.bad, Bf.bad[:5]


def logmm_tile(bid, grid):
    """The product kernels' XCD-aware tile of workgroup bid = (x, y, z) in grid (nx, ny, nz)."""
    nx, ny, nz = grid
    n = nx * ny * nz
    w = bid[0] + nx * (bid[1] + ny * bid[2])
    full = n & ~7
    if w < full:
        w = (w & 7) * (full >> 3) + (w >> 3)
    return (w % nx, (w // nx) % ny, w // (nx * ny))


@pytest.mark.parametrize("grid", [(1, 1, 1), (8, 8, 8), (3, 5, 2), (9, 1, 1), (8, 8, 3), (1, 1, 7),
                                  (5, 7, 9), (1, 1, 8), (2, 9, 13)])
def test_logmm_tile_mapping_is_a_permutation(grid):
    tiles = [logmm_tile((x, y, z), grid) for z in range(grid[2]) for y in range(grid[1])
             for x in range(grid[0])]
    assert sorted(tiles) == sorted(set(tiles))
    assert set(tiles) == {(x, y, z) for x in range(grid[0]) for y in range(grid[1]) for z in range(grid[2])}
    if grid == (8, 8, 8):   # workgroup w runs on XCD w mod 8: each XCD gets one product
        per_xcd = {}
        for w, t in enumerate(tiles):
            per_xcd.setdefault(w % 8, set()).add(t[2])
        assert all(len(v) == 1 for v in per_xcd.values())


@pytest.mark.parametrize("shape", [(1, 1, 1, 1), (3, 70, 45, 130), (2, 129, 33, 257), (1, 5, 300, 7),
                                   (2, 3, 1024, 5), (1, 2, 996, 3), (1, 2, 1028, 3)])
def test_logmm_accesses_in_bounds(shape):
    check_logmm(*shape)
    check_logmm_f64(*shape)
