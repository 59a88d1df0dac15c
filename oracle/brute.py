"""Per-pixel brute-force renderer in torch float64 (test infrastructure only).

Independent of oracle.cpp: no pair list, no sort, no tile ranges. For every
pixel it takes the set of Gaussians that are visible and whose tile-space
rectangle contains the pixel's tile (the support rule of the listing
"Implementation of XPR-3DGS": the rasterizer only ever pairs a Gaussian with
the tiles of its bounding box), orders them by (depth as float32, index), and
composites front to back with the gates of the 3DGS evaluate (power <= 0,
alpha >= alpha_thresh) and the blending of the Background section.

Decisions (gates, stop, rect, clamps) are taken on detached values, so torch
autograd yields the same piecewise derivative as the analytic oracle: this is
its independent check. Meant for tiny scenes (<= a few hundred Gaussians, <=
64x64 pixels).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import OracleConfig

_PI = math.pi


def _sh_real(deg, d):
    """Real SH (Condon-Shortley phase kept) at unit directions d [G,3]."""
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    out = [torch.full_like(x, 0.5 / math.sqrt(_PI))]
    if deg >= 1:
        k1 = math.sqrt(3 / (4 * _PI))
        out += [-k1 * y, k1 * z, -k1 * x]
    if deg >= 2:
        a, b, c = 0.5 * math.sqrt(15 / _PI), 0.25 * math.sqrt(5 / _PI), 0.25 * math.sqrt(15 / _PI)
        out += [a * x * y, -a * y * z, b * (2 * z * z - x * x - y * y), -a * x * z,
                c * (x * x - y * y)]
    if deg >= 3:
        a = 0.25 * math.sqrt(35 / (2 * _PI))
        b = 0.5 * math.sqrt(105 / _PI)
        c = 0.25 * math.sqrt(21 / (2 * _PI))
        d_ = 0.25 * math.sqrt(7 / _PI)
        e = 0.25 * math.sqrt(105 / _PI)
        out += [-a * y * (3 * x * x - y * y), b * x * y * z,
                -c * y * (4 * z * z - x * x - y * y),
                d_ * z * (2 * z * z - 3 * x * x - 3 * y * y),
                -c * x * (4 * z * z - x * x - y * y), e * z * (x * x - y * y),
                -a * x * (x * x - 3 * y * y)]
    return torch.stack(out, dim=1)  # [G, nb]


def _quat_rot(q):
    q = q / q.norm(dim=1, keepdim=True)
    w, x, y, z = q.unbind(1)
    R = torch.stack([
        1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
        2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
        2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], dim=1)
    return R.view(-1, 3, 3)


def project_torch(means, scales, quats, opac, sh, cam, cfg: OracleConfig):
    """means [G,3], scales [G,3], quats [G,4], opac [G], sh [G,K,3] (float64)."""
    Rw = torch.as_tensor(np.asarray(cam.R), dtype=torch.float64)
    tw = torch.as_tensor(np.asarray(cam.t), dtype=torch.float64)
    t = means @ Rw.T + tw
    tx, ty, tz = t.unbind(1)
    Rq = _quat_rot(quats)
    M = Rq * scales[:, None, :]
    Sigma = M @ M.transpose(1, 2)
    limx = cfg.fov_clip * cam.width / (2 * cam.fx)
    limy = cfg.fov_clip * cam.height / (2 * cam.fy)
    rx, ry = tx / tz, ty / tz
    if cfg.fov_clip > 0:
        rx = torch.clamp(rx, -limx, limx)
        ry = torch.clamp(ry, -limy, limy)
    zero = torch.zeros_like(tz)
    J = torch.stack([torch.stack([cam.fx / tz, zero, -cam.fx * rx / tz], 1),
                     torch.stack([zero, cam.fy / tz, -cam.fy * ry / tz], 1)], 1)
    T = J @ Rw
    cov = T @ Sigma @ T.transpose(1, 2)
    a = cov[:, 0, 0] + cfg.lowpass
    b = cov[:, 0, 1]
    c = cov[:, 1, 1] + cfg.lowpass
    det = a * c - b * b
    con = torch.stack([c / det, -b / det, a / det], 1)
    u = cam.fx * tx / tz + cam.cx - 0.5
    v = cam.fy * ty / tz + cam.cy - 0.5
    with torch.no_grad():
        if cfg.opacity_extents:
            # half-widths of the ellipse where o G = alpha_min
            lvl = 2 * torch.log(opac / cfg.alpha_min)
            ex = torch.where(lvl > 0, torch.sqrt(torch.clamp(lvl * a, min=0.0)), torch.zeros_like(a))
            ey = torch.where(lvl > 0, torch.sqrt(torch.clamp(lvl * c, min=0.0)), torch.zeros_like(c))
            r = torch.maximum(ex, ey)
        else:
            mid = 0.5 * (a + c)
            lam = mid + torch.sqrt(torch.clamp(mid * mid - det, min=0.0))
            r = torch.ceil(3 * torch.sqrt(lam))
            ex = ey = r
        txn = (cam.width + cfg.tile_w - 1) // cfg.tile_w
        tyn = (cam.height + cfg.tile_h - 1) // cfg.tile_h
        x0 = torch.clamp(torch.floor((u - ex) / cfg.tile_w), 0, txn)
        x1 = torch.clamp(torch.floor((u + ex) / cfg.tile_w) + 1, 0, txn)
        y0 = torch.clamp(torch.floor((v - ey) / cfg.tile_h), 0, tyn)
        y1 = torch.clamp(torch.floor((v + ey) / cfg.tile_h) + 1, 0, tyn)
        tc = (x1 - x0) * (y1 - y0)
        visible = (tz > cfg.z_near) & (det > 0) & (opac >= cfg.alpha_min) & (r > 0) & (tc > 0)
    campos = -(Rw.T @ tw)
    dvec = means - campos
    dirs = dvec / dvec.norm(dim=1, keepdim=True)
    nb = (cfg.sh_degree + 1) ** 2
    Y = _sh_real(cfg.sh_degree, dirs)
    raw = 0.5 + torch.einsum("gj,gjc->gc", Y, sh[:, :nb, :])
    colour = torch.clamp(raw, min=0.0)
    return dict(u=u, v=v, con=con, colour=colour, depth=tz, visible=visible,
                rect=torch.stack([x0, y0, x1, y1], 1).long(), opac=opac)


def render_torch(means, scales, quats, opac, sh, cam, cfg: OracleConfig):
    """Differentiable per-pixel brute force; returns image [3,H,W] float64."""
    pr = project_torch(means, scales, quats, opac, sh, cam, cfg)
    W, H = cam.width, cam.height
    G = opac.shape[0]
    ys, xs = torch.meshgrid(torch.arange(H, dtype=torch.float64),
                            torch.arange(W, dtype=torch.float64), indexing="ij")
    xs = xs.reshape(-1)
    ys = ys.reshape(-1)
    ptx = (xs // cfg.tile_w).long()
    pty = (ys // cfg.tile_h).long()
    # global front-to-back order by (depth as float32, index)
    d32 = pr["depth"].detach().to(torch.float32).numpy()
    order = np.lexsort((np.arange(G), d32))
    img = torch.zeros(3, H * W, dtype=torch.float64)
    T = torch.ones(H * W, dtype=torch.float64)
    done = torch.zeros(H * W, dtype=torch.bool)
    bg = torch.as_tensor(cfg.bg, dtype=torch.float64)
    for g in order.tolist():
        if not bool(pr["visible"][g]):
            continue
        x0, y0, x1, y1 = [int(z) for z in pr["rect"][g]]
        inside = (ptx >= x0) & (ptx < x1) & (pty >= y0) & (pty < y1)
        dx = xs - pr["u"][g]
        dy = ys - pr["v"][g]
        con = pr["con"][g]
        power = -0.5 * (con[0] * dx * dx + con[2] * dy * dy) - con[1] * dx * dy
        alpha = torch.clamp(opac[g] * torch.exp(power), max=cfg.alpha_max)
        with torch.no_grad():
            live = inside & ~done & (power <= 0) & (alpha >= cfg.alpha_min)
            Tn = T * (1 - alpha)
            stop = live & (Tn < cfg.t_min)
            done = done | stop
            blend = live & ~stop
        a = torch.where(blend, alpha, torch.zeros_like(alpha))
        img = img + pr["colour"][g][:, None] * (a * T)[None, :]
        T = T * (1 - a)
    img = img + T[None, :] * bg[:, None]
    return img.view(3, H, W), T.view(H, W)


def scene_tensors(scene, requires_grad=False):
    """float64 torch tensors [G, ...] from a synth.Scene (SoA [k][n])."""
    def t(a):
        x = torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64).clone()
        return x.requires_grad_(requires_grad)
    return (t(scene.means.T), t(scene.scales.T), t(scene.quats.T), t(scene.opacities),
            t(np.transpose(scene.sh, (2, 0, 1))))


def render(scene, cam, cfg: OracleConfig):
    with torch.no_grad():
        img, T = render_torch(*scene_tensors(scene), cam, cfg)
    return img.numpy(), T.numpy()


def render_gut(scene, cam, cfg: OracleConfig):
    """Per-pixel brute force of 3DGUT (Listing "Implementation of
    XPR-3DGUT") in torch float64: unscented-transform projection (rect,
    visibility, adjusted opacity), then for every pixel the ray response of
    every visible Gaussian whose rect contains the pixel's tile, in (float32
    depth, index) order, with the validity threshold and the gates of the
    3DGS path. No pairs, no sort, no tile ranges. Returns numpy arrays."""
    with torch.no_grad():
        img, T = render_gut_torch(*scene_tensors(scene), cam, cfg)
    return img.numpy(), T.numpy()


def render_gut_torch(means, scales, quats, opac, sh, cam, cfg: OracleConfig, keep=None):
    """render_gut on tensors, differentiable (decisions on detached values):
    returns image [3, H, W] and T_final [H, W] tensors. With a dict ``keep``
    the shader data o' [G], colour [G, 3], ro [G, 3] and M [G, 3, 3] and the
    camera position are stored in it, their gradients retained."""
    G = opac.shape[0]
    Rw = torch.as_tensor(np.asarray(cam.R), dtype=torch.float64)
    tw = torch.as_tensor(np.asarray(cam.t), dtype=torch.float64)
    Rq = _quat_rot(quats)                                    # [G, 3, 3]
    k = math.sqrt(3.0)
    # sigma points [G, 7, 3]: centre, then mu +- sqrt(3) s_j Rq[:, j]
    cols = Rq.transpose(1, 2) * scales[:, :, None]           # row j = s_j Rq[:, j]
    pts = [means]
    for j in range(3):
        pts += [means + k * cols[:, j], means - k * cols[:, j]]
    X = torch.stack(pts, 1)
    Y = X @ Rw.T + tw
    z = Y[..., 2]
    front = (z > cfg.z_near).all(1)
    P2 = torch.stack([cam.fx * Y[..., 0] / z + cam.cx, cam.fy * Y[..., 1] / z + cam.cy], -1)
    wm = torch.tensor([0.0] + [1 / 6] * 6, dtype=torch.float64)
    wc = torch.tensor([2.0] + [1 / 6] * 6, dtype=torch.float64)
    m2 = (wm[None, :, None] * P2).sum(1)
    D = P2 - m2[:, None, :]
    cxx = (wc * D[..., 0] * D[..., 0]).sum(1)
    cxy = (wc * D[..., 0] * D[..., 1]).sum(1)
    cyy = (wc * D[..., 1] * D[..., 1]).sum(1)
    det0 = cxx * cyy - cxy * cxy
    a, b, c = cxx + cfg.lowpass, cxy, cyy + cfg.lowpass
    det = a * c - b * b
    o2 = opac * torch.sqrt(torch.clamp(det0, min=0.0) / det)
    u, v = m2[:, 0] - 0.5, m2[:, 1] - 0.5
    if cfg.opacity_extents:
        lvl = 2 * torch.log(o2 / cfg.alpha_min)
        ex = torch.where(lvl > 0, torch.sqrt(torch.clamp(lvl * a, min=0.0)), torch.zeros_like(a))
        ey = torch.where(lvl > 0, torch.sqrt(torch.clamp(lvl * c, min=0.0)), torch.zeros_like(c))
        r = torch.maximum(ex, ey)
    else:
        mid = 0.5 * (a + c)
        r = torch.ceil(3 * torch.sqrt(mid + torch.sqrt(torch.clamp(mid * mid - det, min=0.0))))
        ex = ey = r
    txn = (cam.width + cfg.tile_w - 1) // cfg.tile_w
    tyn = (cam.height + cfg.tile_h - 1) // cfg.tile_h
    x0 = torch.clamp(torch.floor((u - ex) / cfg.tile_w), 0, txn)
    x1 = torch.clamp(torch.floor((u + ex) / cfg.tile_w) + 1, 0, txn)
    y0 = torch.clamp(torch.floor((v - ey) / cfg.tile_h), 0, tyn)
    y1 = torch.clamp(torch.floor((v + ey) / cfg.tile_h) + 1, 0, tyn)
    visible = front & (det > 0) & (o2 > cfg.alpha_min) & (r > 0) & ((x1 - x0) * (y1 - y0) > 0)
    # shader data: camera position and ray directions in each Gaussian's frame
    campos = -(Rw.T @ tw)
    Minv = Rq.transpose(1, 2) / scales[:, :, None]          # S^-1 R^T
    ro = (Minv @ (campos[None, :] - means)[:, :, None])[..., 0]
    dirs = (means - campos) / (means - campos).norm(dim=1, keepdim=True)
    nb = (cfg.sh_degree + 1) ** 2
    colour = torch.clamp(0.5 + torch.einsum("gj,gjc->gc", _sh_real(cfg.sh_degree, dirs),
                                            sh[:, :nb, :]), min=0.0)
    if keep is not None:
        for name, v in (("o2", o2), ("colour", colour), ("ro", ro), ("M", Minv)):
            if v.requires_grad:
                v.retain_grad()
            keep[name] = v
        keep["campos"] = campos
    W, H = cam.width, cam.height
    ys, xs = torch.meshgrid(torch.arange(H, dtype=torch.float64),
                            torch.arange(W, dtype=torch.float64), indexing="ij")
    xs, ys = xs.reshape(-1), ys.reshape(-1)
    dc = torch.stack([(xs + 0.5 - cam.cx) / cam.fx, (ys + 0.5 - cam.cy) / cam.fy,
                      torch.ones_like(xs)], 1)
    dc = dc / dc.norm(dim=1, keepdim=True)
    rd = dc @ Rw                                             # R^T dc per row
    ptx = (xs // cfg.tile_w).long()
    pty = (ys // cfg.tile_h).long()
    order = np.lexsort((np.arange(G), Y[:, 0, 2].detach().to(torch.float32).numpy()))
    img = torch.zeros(3, H * W, dtype=torch.float64)
    T = torch.ones(H * W, dtype=torch.float64)
    done = torch.zeros(H * W, dtype=torch.bool)
    for g in order.tolist():
        if not bool(visible[g]):
            continue
        inside = (ptx >= int(x0[g])) & (ptx < int(x1[g])) & (pty >= int(y0[g])) & (pty < int(y1[g]))
        rdc = rd @ Minv[g].T
        tau = -(rdc @ ro[g]) / (rdc * rdc).sum(1)
        p = ro[g][None, :] + tau[:, None] * rdc
        resp = torch.exp(-0.5 * (p * p).sum(1))
        alpha = torch.clamp(o2[g] * resp, max=cfg.alpha_max)
        with torch.no_grad():
            live = inside & ~done & (resp > 0.0113) & (alpha >= cfg.alpha_min)
            Tn = T * (1 - alpha)
            stop = live & (Tn < cfg.t_min)
            done = done | stop
            blend = live & ~stop
        a_ = torch.where(blend, alpha, torch.zeros_like(alpha))
        img = img + colour[g][:, None] * (a_ * T)[None, :]
        T = T * (1 - a_)
    img = img + T[None, :] * torch.as_tensor(cfg.bg, dtype=torch.float64)[:, None]
    return img.view(3, H, W), T.view(H, W)


def render_lin(scene, cam, cfg: OracleConfig):
    """Per-pixel brute force of LinPrim (Listing "Implementation of
    XPR-LinPrim") in torch float64: the linear map A of each octahedron
    (perspective Jacobian rows over the unit viewing direction, times the
    rotations and half-extents), its slab pairs from the rows of A^-1, the
    chord of every pixel's ray, Beer-Lambert opacity, the gates of the 3DGS
    path, in (float32 Euclidean depth, index) order over the Gaussians whose
    rect holds the pixel's tile. No pairs, no sort. Returns numpy image
    [3, H, W] and T_final [H, W]."""
    with torch.no_grad():
        img, T = render_lin_torch(*scene_tensors(scene), cam, cfg)
    return img.numpy(), T.numpy()


def render_lin_torch(means, scales, quats, opac, sh, cam, cfg: OracleConfig, keep=None):
    """render_lin on tensors, differentiable (decisions on detached values):
    returns image [3, H, W] and T_final [H, W] tensors. With a dict ``keep``
    the shader data u, v (mu_2D - 1/2) [G], sigma [G], colour [G, 3] and the
    rows of A^-1 [G, 3, 3] are stored in it, their gradients retained."""
    G = opac.shape[0]
    Rw = torch.as_tensor(np.asarray(cam.R), dtype=torch.float64)
    tw = torch.as_tensor(np.asarray(cam.t), dtype=torch.float64)
    mc = means @ Rw.T + tw
    x, y, z = mc.unbind(1)
    d = mc.norm(dim=1)
    zero = torch.zeros_like(z)
    J = torch.stack([torch.stack([cam.fx / z, zero, -cam.fx * x / (z * z)], 1),
                     torch.stack([zero, cam.fy / z, -cam.fy * y / (z * z)], 1),
                     torch.stack([x / d, y / d, z / d], 1)], 1)
    A = J @ Rw @ _quat_rot(quats) * scales[:, None, :]
    smin = scales.min(dim=1).values
    detA = torch.linalg.det(A.detach())
    ok = (z.detach() > cfg.z_near) & (smin.detach() > 0) & (detA.abs() > 0)
    Ainv = torch.linalg.inv(torch.where(ok[:, None, None], A, torch.eye(3, dtype=torch.float64)))
    u2 = cam.fx * x / z + cam.cx
    v2 = cam.fy * y / z + cam.cy
    ex = A[:, 0, :].abs().max(dim=1).values.detach()
    ey = A[:, 1, :].abs().max(dim=1).values.detach()
    o = torch.clamp(opac, 0.0, 0.999)
    sigma = -torch.log1p(-0.99 * o) / (2 * smin)
    u, v = u2 - 0.5, v2 - 0.5
    ud, vd = u.detach(), v.detach()
    txn = (cam.width + cfg.tile_w - 1) // cfg.tile_w
    tyn = (cam.height + cfg.tile_h - 1) // cfg.tile_h
    x0 = torch.clamp(torch.floor((ud - ex) / cfg.tile_w), 0, txn)
    x1 = torch.clamp(torch.floor((ud + ex) / cfg.tile_w) + 1, 0, txn)
    y0 = torch.clamp(torch.floor((vd - ey) / cfg.tile_h), 0, tyn)
    y1 = torch.clamp(torch.floor((vd + ey) / cfg.tile_h) + 1, 0, tyn)
    visible = ok & (torch.maximum(ex, ey) > 0) & ((x1 - x0) * (y1 - y0) > 0) & (d.detach() > cfg.z_near)
    campos = -(Rw.T @ tw)
    dirs = (means - campos) / (means - campos).norm(dim=1, keepdim=True)
    nb = (cfg.sh_degree + 1) ** 2
    colour = torch.clamp(0.5 + torch.einsum("gj,gjc->gc", _sh_real(cfg.sh_degree, dirs),
                                            sh[:, :nb, :]), min=0.0)
    if keep is not None:
        for name, t in (("u", u), ("v", v), ("sigma", sigma), ("colour", colour), ("c", Ainv)):
            if t.requires_grad:
                t.retain_grad()
            keep[name] = t
    W, H = cam.width, cam.height
    ys, xs = torch.meshgrid(torch.arange(H, dtype=torch.float64),
                            torch.arange(W, dtype=torch.float64), indexing="ij")
    xs, ys = xs.reshape(-1), ys.reshape(-1)
    ptx, pty = (xs // cfg.tile_w).long(), (ys // cfg.tile_h).long()
    order = np.lexsort((np.arange(G), d.detach().to(torch.float32).numpy()))
    img = torch.zeros(3, H * W, dtype=torch.float64)
    T = torch.ones(H * W, dtype=torch.float64)
    done = torch.zeros(H * W, dtype=torch.bool)
    for g in order.tolist():
        if not bool(visible[g]):
            continue
        inside = (ptx >= int(x0[g])) & (ptx < int(x1[g])) & (pty >= int(y0[g])) & (pty < int(y1[g]))
        dx, dy = xs - u[g], ys - v[g]
        c = Ainv[g]
        enter = torch.full_like(xs, -math.inf)
        exit_ = torch.full_like(xs, math.inf)
        miss = torch.zeros_like(inside)
        for e1 in (1.0, -1.0):
            for e2 in (1.0, -1.0):
                nvec = c[0] + e1 * c[1] + e2 * c[2]
                w = nvec[0] * dx + nvec[1] * dy
                if abs(float(nvec[2].detach())) >= 1e-10:
                    m, h = -w / nvec[2], 1.0 / nvec[2].abs()
                    enter = torch.maximum(enter, m - h)
                    exit_ = torch.minimum(exit_, m + h)
                else:
                    miss = miss | (w.detach().abs() > 1.0)
        chord = torch.where(miss, torch.full_like(xs, -1.0), exit_ - enter)
        # alpha of the pixels the ray misses (chord <= 0, gated out below) is
        # formed from chord 0, so that no overflowing exponential reaches
        # the gradient through the gate
        alpha = torch.clamp(-torch.expm1(-sigma[g] * torch.clamp(chord, min=0.0)),
                            max=cfg.alpha_max)
        with torch.no_grad():
            live = inside & ~done & (chord > 0) & (alpha >= cfg.alpha_min)
            Tn = T * (1 - alpha)
            stop = live & (Tn < cfg.t_min)
            done = done | stop
            blend = live & ~stop
        a_ = torch.where(blend, alpha, torch.zeros_like(alpha))
        img = img + colour[g][:, None] * (a_ * T)[None, :]
        T = T * (1 - a_)
    img = img + T[None, :] * torch.as_tensor(cfg.bg, dtype=torch.float64)[:, None]
    return img.view(3, H, W), T.view(H, W)
