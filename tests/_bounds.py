"""Error bars of the GPU network's arithmetic derived from a first-order rounding-error model,
for the parity tests (test infrastructure; numpy on the oracle's FP64 values).

The oracle evaluates the network in FP64 on exactly the parameters the GPU uses (FP16 table
entries and BF16/FP16-rounded weights widened without error).  The GPU's elementary errors:

  encoding   FP32 trilinear interpolation with 32-bit fixed-point cell coordinates: a sample's
             position is off by at most N_l 2^-33 cells, which moves the eight weights by at
             most 6 N_l 2^-33 in sum; with the three products and the eight-term sum,
             |d enc| <= (6 N_l 2^-33 + 11 u32) max|table of level l| (the two features of one
             sample and level share their weights: their errors are taken as correlated).
  operands   every MFMA operand that is not a stored weight -- the input of each layer in the
             forward; d heads and each delta in the backward's chain; both factors of the
             weight gradients -- is rounded to the MLP
             precision: |d x| <= u |x| + eta, u = 2^-8 (BF16), 2^-11 (FP16), 0 (FP32), eta =
             half the smallest subnormal spacing.  A bias added from a copy of another
             precision than the oracle's: u |b|.
  sums       each dot product or batch sum of n terms accumulated in FP32: n + 1 roundings, each
             at most u32 times its partial sum, whose square is taken as at most the sum of
             the squared terms plus the square of the total.
  table      d enc = W0^T delta_0 uses the FP32 master W0 (the forward used its rounding): a
  gradient   deterministic difference (W0 - rounded W0)^T delta_0, carried exactly; the
             additions w d enc are FP32 products of weights off by up to 3 N_l 2^-33, summed in
             64-bit fixed point (each rounded to the unit 2^(e + nb - 62): the largest addition
             below 2^e, nb bits of the addition count) after FP32 merges of equal entries, and
             the element is an FP32 value.

Model (Higham and Mary, "A new approach to probabilistic rounding error analysis", SIAM J.
Sci. Comput. 2019): to first order the GPU's deviation is a linear function of these
elementary errors, which are independent, of mean zero, and uniform within their bounds
(variance bound^2 / 3).  The linearization is carried exactly -- covariance matrices through
the layers, per sample -- so the deviation of every output, activation, delta and gradient
element has a computed standard deviation sigma.  Outputs are then held to LAMBDA sigma
(a deterministic part, where there is one, added in full).  A hidden unit whose
pre-activation x has its error move it across 0 with probability p = erfc(|x| / (sigma
sqrt 2)); the other ReLU branch then costs the whole back-propagated value g, which adds
p g^2 to the variance as an independent term; in the forward, a unit that is off in the oracle
adds p times its error's variance the same way.  The loss's kinks
(the distance ReLU, the sign of the albedo L1) add their jump the same way.  Samples are
independent, so the gradients' variances add over the batch."""
from __future__ import annotations

import numpy as np

U32 = 2.0 ** -24
U_OP = {0: 0.0, 1: 2.0 ** -8, 2: 2.0 ** -11}     # NIF_PREC_FP32, _BF16, _FP16
ETA_OP = {0: 0.0, 1: 2.0 ** -134, 2: 2.0 ** -25}
EPS_DIST = 1e-4
LAMBDA = 7.0           # heads, MLP gradients, losses
LAMBDA_TABLE = 7.0     # table gradients (millions of elements)
TABLE_FLIP_FRAC = 1e-5 # table elements allowed beyond it (rare flips)
CHUNK = 128


def layers(desc, prm):
    """[(W [out][in], b [out])] of the canonical FP64 parameter vector."""
    dims = desc.layer_dims
    out, o = [], 0
    for i in range(len(dims) - 1):
        ni, no = dims[i], dims[i + 1]
        W = prm[o:o + no * ni].reshape(no, ni)
        o += no * ni
        out.append((W, prm[o:o + no]))
        o += no
    assert o == len(prm)
    return out


def _diag(C):
    return np.einsum("bii->bi", C)


def _sum_var(n, sum_sq, total):
    """Variance of the FP32 rounding of a sum of n terms: each of the n + 1 roundings is at
    most u32 times its partial sum, whose square is taken as at most sum of the squared terms
    (independent signs) plus the square of the total (terms of one sign)."""
    return (n + 1) * U32 ** 2 / 3.0 * (sum_sq + np.asarray(total) ** 2)


def gamma_raw(desc, x):
    """The raw PE values the concatenated encoding appends: value 3 s + a is sample s of
    coordinate a of the clamped point (x, sin 2^k x, cos 2^k x), Eq. (1)."""
    xc = np.clip(x, 0.0, 1.0)
    cols = [xc]
    for k in range(desc.pe_freqs):
        cols += [np.sin(2.0 ** k * xc), np.cos(2.0 ** k * xc)]
    return np.concatenate(cols, axis=1)


def encoding_interp_bound(desc, tables):
    """Bound on the interpolation error of one point's grid encoding, per element ([S][L][Fd])."""
    t = np.abs(np.asarray(tables, dtype=np.float64)).reshape(desc.table_levels // desc.levels, desc.levels, -1)
    tmax = t.max(axis=(0, 2))
    res = np.asarray(desc.res[:desc.levels], dtype=np.float64)
    per_level = (6.0 * res * 2.0 ** -33 + 11.0 * U32) * tmax
    return np.broadcast_to(per_level[None, :, None], (desc.n_samples, desc.levels, desc.feat_dim)).reshape(-1)


def forward(orc, desc, tables, prm, x0, x1, prec):
    """Oracle activations of every layer (FP64) and the covariance of the GPU's deviation.
    x0, x1: [n][3].  Returns dict: z heads [n][H], Cz [n][H][H], sz = sqrt(diag Cz); acts[k] /
    va[k] (input of layer k and the variance of its error), pre[k] / vpre[k] (pre-activation
    of layer k and its variance), enc."""
    u, eta = U_OP[prec], ETA_OP[prec]
    enc = np.concatenate([orc.encode(desc, tables, x0), orc.encode(desc, tables, x1)], axis=1)
    ib = np.tile(encoding_interp_bound(desc, tables), 2)[None, :]
    if desc.concat_encoding:                 # raw gamma values, FP32: a rounding or two
        gam = np.concatenate([gamma_raw(desc, x0), gamma_raw(desc, x1)], axis=1)
        enc = np.concatenate([enc, gam], axis=1)
        ib = np.concatenate([np.broadcast_to(ib, (1, ib.shape[1])), 2.0 * U32 * np.ones((1, gam.shape[1]))], axis=1)
    L = layers(desc, prm)
    n = enc.shape[0]
    acts = [enc]
    va = [2.0 * ib ** 2 / 3.0 + (u * enc) ** 2 / 3.0 + eta ** 2 / 3.0]
    pre, vpre = [], []
    for k, (W, b) in enumerate(L):
        z = acts[k] @ W.T + b
        pre.append(z)
        vpre.append(np.zeros_like(z))
        if k + 1 < len(L):
            acts.append(np.maximum(z, 0.0))
            va.append(np.zeros_like(z))
    H = L[-1][0].shape[0]
    Cz = np.zeros((n, H, H))
    for c0 in range(0, n, CHUNK):
        sl = slice(c0, min(n, c0 + CHUNK))
        C = None                                        # covariance of the current layer input's error
        for k, (W, b) in enumerate(L):
            a = acts[k][sl]
            acc = _sum_var(W.shape[1], a ** 2 @ (W ** 2).T + b ** 2, pre[k][sl]) + (u * b) ** 2 / 3.0
            if C is None:                               # the encoding's errors: independent (diagonal)
                Ck = np.matmul(W[None] * va[0][sl][:, None, :], W.T[None])
            else:
                Ck = np.matmul(np.matmul(W[None], C), W.T[None])
            io = np.arange(W.shape[0])
            Ck[:, io, io] += acc
            vpre[k][sl] = _diag(Ck)
            if k + 1 == len(L):
                Cz[sl] = Ck
                break
            z = pre[k][sl]
            on = z > 0.0
            C = Ck * on[:, :, None] * on[:, None, :]
            # a unit off in the oracle whose error may turn it on: at most its error, when it flips
            C[:, io, io] += np.where(on, 0.0, vpre[k][sl] * _p_flip(z, np.sqrt(vpre[k][sl])))
            an = acts[k + 1][sl]
            C[:, io, io] += (u * an) ** 2 / 3.0 + eta ** 2 / 3.0                  # operand rounding
            va[k + 1][sl] = _diag(C)
    return dict(z=pre[-1], Cz=Cz, sz=np.sqrt(_diag(Cz)), acts=acts, va=va, pre=pre, vpre=vpre, enc=enc)


def _deltas(L, fw, dz):
    """The oracle's d loss / d pre-activation of every layer (index j = layer j's output)."""
    out = [None] * len(L)
    d = dz
    for j in range(len(L) - 1, -1, -1):
        out[j] = d
        if j == 0:
            break
        d = np.where(fw["pre"][j - 1] > 0.0, d @ L[j][0], 0.0)
    return out


def backward(orc, desc, tables, prm, fw, x0, x1, dz, Cdz, prec, scale=1.0, W0_gpu=None):
    """Error model of the GPU's parameter gradients given the oracle's d heads dz [n][H] and
    the covariance Cdz [n][H][H] of the GPU's d heads around it.  `scale`: the loss scale the
    GPU's d heads carry (a power of two: exact, but it moves the FP16 underflow threshold).
    W0_gpu: the first-layer weights the GPU's table gradient uses (its FP32 masters) where they
    differ from the oracle's.  Returns dict: tables = (det, sigma) shaped like the tables,
    mlp = sigma in the canonical layout, denc = the oracle's d loss / d encoding."""
    u, eta = U_OP[prec], ETA_OP[prec] / scale
    L = layers(desc, prm)
    n = dz.shape[0]
    dch = _deltas(L, fw, dz)
    vG = [np.zeros_like(W) for W, _ in L]
    vb = [np.zeros_like(b) for _, b in L]
    vdenc = np.zeros((n, L[0][0].shape[1]))
    for c0 in range(0, n, CHUNK):
        sl = slice(c0, min(n, c0 + CHUNK))
        C = Cdz[sl].copy()                              # covariance of the stored d (FP32) error
        for j in range(len(L) - 1, -1, -1):
            W, b = L[j]
            d = dch[j][sl]
            a, sa = fw["acts"][j][sl], np.sqrt(fw["va"][j][sl])
            sd = np.sqrt(np.maximum(_diag(C), 0.0))
            ad, aa = np.abs(d), np.abs(a)
            # G_j = sum_b d a^T: (|a| sigma_d + |d| sigma_a)^2 per sample (Cauchy-Schwarz over
            # the correlation of the two factors); samples add
            vG[j] += (sd ** 2).T @ a ** 2 + 2.0 * (sd * ad).T @ (aa * sa) + (ad ** 2).T @ sa ** 2
            # BF16/FP16: the weight-gradient MFMA takes both factors rounded to that precision
            vG[j] += (((u * ad + eta) ** 2).T @ a ** 2 + (ad ** 2).T @ (u * aa + eta) ** 2) / 3.0
            vb[j] += (sd ** 2).sum(axis=0)
            io = np.arange(W.shape[0])
            Cop = C.copy()
            Cop[:, io, io] += (u * d) ** 2 / 3.0 + eta ** 2 / 3.0       # MFMA operand of the chain
            if j == 0:                                                  # d enc: FP32 operands
                Cop = C
            Cg = np.matmul(np.matmul(W.T[None], Cop), W[None])
            ii = np.arange(W.shape[1])
            g = d @ W
            Cg[:, ii, ii] += _sum_var(W.shape[0], d ** 2 @ W ** 2, g)
            if j == 0:
                vdenc[sl] = _diag(Cg)
                break
            zp = fw["pre"][j - 1][sl]
            on = zp > 0.0
            C = Cg * on[:, :, None] * on[:, None, :]
            # a flip costs the whole value, with its own error where the oracle's unit is off
            pf = _p_flip(zp, np.sqrt(fw["vpre"][j - 1][sl]))
            C[:, ii, ii] += pf * (g ** 2 + np.where(on, 0.0, _diag(Cg)))
    sig = []
    for j in range(len(L)):
        d, a = dch[j], fw["acts"][j]
        vsum = _sum_var(n, (d ** 2).T @ a ** 2, d.T @ a)             # FP32 sums over the batch
        sig.append(np.sqrt(vG[j] + vsum).reshape(-1))
        sig.append(np.sqrt(vb[j] + _sum_var(n, (d ** 2).sum(0), d.sum(0))))
    denc = dch[0] @ L[0][0]
    det_denc = dch[0] @ (W0_gpu - L[0][0]) if W0_gpu is not None else None
    tdet, tsig = _table_error(orc, desc, tables, x0, x1, denc, vdenc, det_denc)
    return dict(tables=(tdet, tsig), mlp=np.concatenate(sig), denc=denc, vdenc=vdenc)


def _table_error(orc, desc, tables, x0, x1, denc, vdenc, det_denc):
    """(deterministic part, sigma) of the table gradient's error, per table element: per sample,
    the corners that land on one entry add their amplitudes (their errors share the sample's
    d enc errors); samples and the per-addition roundings add variances."""
    Fd, Lv, S = desc.feat_dim, desc.levels, desc.n_samples
    n = denc.shape[0]
    ntab = int(np.prod(np.shape(tables)))
    PW = S * Lv * Fd                                             # grid part of one point
    res = np.asarray(desc.res[:Lv], dtype=np.float64)
    dw = 3.0 * res * 2.0 ** -33                                  # corner weight error per level
    var = np.zeros(ntab)
    det = np.zeros(ntab)
    cnt = np.zeros(ntab)
    vmax = 0.0
    rows = np.arange(n, dtype=np.int64)[:, None, None, None] * ntab
    for p, x in enumerate((x0, x1)):
        idx, w = orc.encode_corners(desc, x)                     # [n][S][L][8]
        vmax = max(vmax, float((w[..., None] * np.abs(denc[:, p * PW:(p + 1) * PW]).reshape(n, S, Lv, 1, Fd)).max()))
        for f in range(Fd):
            cnt += np.bincount((idx * Fd + f).reshape(-1), minlength=ntab)
        sd = np.sqrt(vdenc[:, p * PW:(p + 1) * PW]).reshape(n, S, Lv, Fd)
        dv = denc[:, p * PW:(p + 1) * PW].reshape(n, S, Lv, Fd)
        for f in range(Fd):
            ent = idx * Fd + f
            uk, inv = np.unique((rows + ent).reshape(-1), return_inverse=True)
            s_amp = np.bincount(inv, weights=(w * sd[:, :, :, None, f]).reshape(-1), minlength=len(uk))
            var += np.bincount(uk % ntab, weights=s_amp ** 2, minlength=ntab)
            av = np.abs(dv[:, :, :, None, f])
            e_add = (U32 * w * av) ** 2 + (dw[None, None, :, None] * av) ** 2
            var += np.bincount(ent.reshape(-1), weights=(e_add / 3.0).reshape(-1), minlength=ntab)
        if det_denc is not None:
            det += orc.encode_backward(desc, tables, x, det_denc[:, p * PW:(p + 1) * PW]).reshape(-1)
    # the gradient element itself is an FP32 value: its final rounding, and the FP32 sums that
    # merge runs of equal entries and the parts of a split slice (at most the element's
    # magnitude summed over its additions, taken from J^T |d enc|)
    gabs = (orc.encode_backward(desc, tables, x0, np.abs(denc[:, :PW])) +
            orc.encode_backward(desc, tables, x1, np.abs(denc[:, PW:2 * PW]))).reshape(-1)
    g = (orc.encode_backward(desc, tables, x0, denc[:, :PW]) +
         orc.encode_backward(desc, tables, x1, denc[:, PW:2 * PW])).reshape(-1)
    var += U32 ** 2 / 3.0 * (g ** 2 + gabs ** 2)
    # the sums run in 64-bit fixed point: each addition is rounded to the unit 2^(e + nb - 62),
    # the largest addition below 2^e (one more for the GPU's own rounding of it), nb bits of
    # the round's addition count (rounds of up to 2^18 samples)
    if vmax > 0.0:
        e = np.frexp(vmax)[1] + 1
        total = min(n, 1 << 18) * 2 * S * Lv * 8
        nb = int(np.ceil(np.log2(total + 1)))
        unit = 2.0 ** (e + nb - 62)
        var += cnt * unit ** 2 / 12.0
    return det.reshape(np.shape(tables)), np.sqrt(var).reshape(np.shape(tables))


def _sig(v):
    return 1.0 / (1.0 + np.exp(-v))


def _p_flip(x, sigma):
    """Probability that an error of standard deviation sigma moves x across 0 (a branch of
    ReLU, a sign): the variance a flip adds is its jump squared times this."""
    from scipy.special import erfc
    return erfc(np.abs(x) / (np.sqrt(2.0) * np.maximum(sigma, 1e-300)))


def _task_weights(s, fixed):
    if fixed:
        return np.ones(5)
    return np.exp(-np.asarray(s, dtype=np.float64)) * np.array([1.0, 0.5, 0.5, 0.5, 1.0])


def loss_dz_cov(desc, fw, dz_ref, hit, t, nrm, alb, s, fixed=False, x0=None, x1=None):
    """Covariance [n][H][H] of the GPU's d loss / d heads around the oracle's: the heads'
    error covariance through the loss's Hessian in the heads (first order), the kinks, and the
    FP32 evaluation of the formulas.  nrm, alb: [n][3]; x0, x1 ([n][3]) for the sigmoid
    distance head (its target is t* over the rest length)."""
    z, Cz, sz = fw["z"], fw["Cz"], fw["sz"]
    n, H = z.shape
    P = max(int(hit.sum()), 1)
    w = _task_weights(s, fixed)
    h = hit.astype(bool)
    Hs = np.zeros((n, H, H))
    kink = np.zeros((n, H))
    sg0 = _sig(z[:, 0])
    Hs[:, 0, 0] = w[0] / n * sg0 * (1.0 - sg0)
    # distance: g = 2 r / (d + eps) for d = z1 > 0, r = log(d + eps) - log(t* + eps)
    z1 = z[:, 1]
    dpos = np.maximum(z1, 0.0) + EPS_DIST
    r = np.log(dpos) - np.log(t + EPS_DIST)
    if getattr(desc, "dist_head", 0) == 1:
        # sigmoid fraction p regressed on tau = clamp(t* / l, 0, 1): g = 2 (p - tau) p (1 - p)
        lr = np.linalg.norm(x1 - x0, axis=1)
        tau = np.where(lr > 0, np.clip(t / np.where(lr > 0, lr, 1.0), 0.0, 1.0), 0.0)
        pr = _sig(z1)
        dp = pr * (1.0 - pr)
        Hs[:, 1, 1] = np.where(h, w[1] / P * 2.0 * dp * (dp + (pr - tau) * (1.0 - 2.0 * pr)), 0.0)
    else:
        Hs[:, 1, 1] = np.where(h & (z1 > 0), w[1] / P * 2.0 * (1.0 - r) / dpos ** 2, 0.0)
        top = np.maximum(z1 + LAMBDA * sz[:, 1], 0.0) + EPS_DIST
        rt = np.log(top) - np.log(t + EPS_DIST)
        jump = w[1] / P * 2.0 * np.maximum(np.abs(rt), np.abs(r)) / EPS_DIST
        kink[:, 1] = np.where(h, jump * np.sqrt(_p_flip(z1, sz[:, 1])), 0.0)
    # normal: g = -(n* - nh c) / |v|;  d g / d v = [q nh^T + c (I - nh nh^T) + nh q^T] / |v|^2
    v = z[:, 2:5]
    vl = np.linalg.norm(v, axis=1)
    nh = v / vl[:, None]
    c = np.einsum("bi,bi->b", nh, nrm)
    Pp = np.eye(3)[None] - nh[:, :, None] * nh[:, None, :]
    q = np.einsum("bij,bj->bi", Pp, nrm)
    Hn = (q[:, :, None] * nh[:, None, :] + c[:, None, None] * Pp + nh[:, :, None] * q[:, None, :]) / vl[:, None, None] ** 2
    Hs[:, 2:5, 2:5] = np.where(h[:, None, None], w[2] / P * Hn, 0.0)
    # albedo: g = sign(sig - a*) sig' / 3
    sa = _sig(z[:, 5:8])
    ds = sa * (1.0 - sa)
    ia = np.arange(5, 8)
    Hs[:, ia, ia] = np.where(h[:, None], w[3] / (3.0 * P) * np.sign(sa - alb) * ds * (1.0 - 2.0 * sa), 0.0)
    kink[:, 5:8] = np.where(h[:, None], 2.0 * w[3] / (3.0 * P) * ds * np.sqrt(_p_flip(sa - alb, ds * sz[:, 5:8])), 0.0)
    # material: softmax cross-entropy, Hessian diag(p) - p p^T (M = 1: binary)
    M = desc.n_materials
    zm = z[:, 8:8 + M]
    if M == 1:
        sm = _sig(zm[:, 0])
        Hs[:, 8, 8] = np.where(h, w[4] / P * sm * (1.0 - sm), 0.0)
    else:
        pm = np.exp(zm - zm.max(1, keepdims=True))
        pm /= pm.sum(1, keepdims=True)
        Hm = pm[:, :, None] * (np.eye(M)[None] - pm[:, None, :])
        Hs[:, 8:8 + M, 8:8 + M] = np.where(h[:, None, None], w[4] / P * Hm, 0.0)
    Cd = np.matmul(np.matmul(Hs, Cz), np.transpose(Hs, (0, 2, 1)))
    ih = np.arange(H)
    fp32 = (8.0 * U32 * np.abs(dz_ref)) ** 2
    fp32[:, 0] += (w[0] / n * 4.0 * U32) ** 2
    if getattr(desc, "dist_head", 0) != 1:
        fp32[:, 1] += np.where(h & (z1 > 0), (w[1] / P * 8.0 * U32 * (np.abs(np.log(dpos)) + np.abs(np.log(t + EPS_DIST))
                                                                       + 1.0) / dpos) ** 2, 0.0)
    Cd[:, ih, ih] += kink ** 2 + fp32 / 3.0
    return Cd


def loss_sigma(desc, fw, dz_ref, s, fixed=False):
    """Standard deviation of the GPU's five task losses around the oracle's: d L_k / d z (the
    oracle's d heads over the task weight) applied to the heads' covariance."""
    w = _task_weights(s, fixed)
    cols = [[0], [1], [2, 3, 4], [5, 6, 7], list(range(8, 8 + desc.n_materials))]
    out = np.zeros(5)
    for k, cc in enumerate(cols):
        g = np.zeros_like(dz_ref)
        g[:, cc] = dz_ref[:, cc] / w[k]
        out[k] = np.sqrt(np.einsum("bi,bij,bj->", g, fw["Cz"], g))
    return out


def check(got, ref, sigma, name, say=print, det=0.0, lam=LAMBDA, max_frac=0.0):
    """|got - ref| <= |det| + lam sigma element-wise (a fraction max_frac of the elements may
    exceed it: the rare ReLU or loss-kink flips, whose whole jump happens with probability p,
    are not Gaussian), and the norm-wise error within 2x the model's expected norm."""
    got = np.asarray(got, dtype=np.float64).reshape(-1)
    ref = np.asarray(ref, dtype=np.float64).reshape(-1)
    sigma = np.broadcast_to(np.asarray(sigma, dtype=np.float64).reshape(-1), ref.shape)
    det = np.broadcast_to(np.abs(np.asarray(det, dtype=np.float64)).reshape(-1), ref.shape)
    err = np.abs(got - ref)
    bound = det + lam * sigma
    worst = float((err / np.maximum(bound, 1e-300)).max(initial=0.0))
    nref = max(float(np.linalg.norm(ref)), 1e-300)
    nrm = float(np.linalg.norm(got - ref)) / nref
    expect = float(np.sqrt(np.sum(sigma ** 2)) + np.linalg.norm(det)) / nref
    say(f"  {name:10s} norm-wise error {nrm:.2e} (model {expect:.2e}); worst |err| / bound {worst:.3f}")
    bad = int((err > bound).sum())
    if bad:
        say(f"    {bad} of {err.size} elements beyond |det| + {lam:g} sigma (allowed {int(max_frac * err.size)})")
        for i in np.argsort(-(err / np.maximum(bound, 1e-300)))[:4]:
            say(f"    element {i}: got {got[i]:.6e} ref {ref[i]:.6e} err {err[i]:.3e} sigma {sigma[i]:.3e} det {det[i]:.3e}")
    assert bad <= max_frac * err.size, f"{name}: {bad} elements beyond |det| + {lam:g} sigma (worst ratio {worst:.3f})"
    assert nrm <= 2.0 * expect, f"{name}: norm-wise error {nrm:.2e} beyond 2x the model's {expect:.2e}"
    return worst, nrm
