"""True adjoint W^* against the approximation W^dagger in the FISTA gradient.

Sec. "The adjoint for orthogonal wavelets" deblurs an image with FISTA
(three-level Haar transform, symmetric extension, lambda = 2e-5, 2500
iterations) once with the gradient W^* R^* (A x - b) and once with W^dagger in
the place of W^*, and compares the reconstructions by their relative error
against the unblurred image and their share of nonzero coefficients; for its
biorthogonal case it adds the structural similarity (SSIM) over the
iterations. This module runs the same comparison on the library's fista_step
(the gradient map is a flag of the FISTA state) for the orthogonal Daubechies
filters and the biorthogonal CDF 9/7 pair.

The paper's test image is a resolution chart that is not available here: the
rectangle-plus-gradient generator stands in for it, blurred by the reflexive
Gaussian R and perturbed by N(0, 1e-3^2) noise. Measures, taken on the host at
checkpoints (evaluation only, outside the iteration):
  rel_err   ||W x_k - image||_2 / ||image||_2
  nonzero   share of nonzero coefficients of x_k, in percent
  ssim      mean SSIM of W x_k against the image (Wang et al. 2004: Gaussian
            window sigma 1.5 truncated to 11 taps, K1 = 0.01, K2 = 0.03,
            dynamic range 1, reflected borders)
  objective F(x_k) of eq. (1); only the true adjoint's iteration minimises it
"""
from __future__ import annotations

import argparse
import json

import numpy as np
import scipy.ndimage

from . import ops


def ssim(a: np.ndarray, b: np.ndarray, data_range: float = 1.0) -> float:
    """Mean structural similarity of two images (float64)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    c1 = (0.01 * data_range) ** 2
    c2 = (0.03 * data_range) ** 2

    def g(u):
        return scipy.ndimage.gaussian_filter(u, 1.5, truncate=5.0 / 1.5, mode="reflect")

    mu_a, mu_b = g(a), g(b)
    s_aa = g(a * a) - mu_a * mu_a
    s_bb = g(b * b) - mu_b * mu_b
    s_ab = g(a * b) - mu_a * mu_b
    m = ((2 * mu_a * mu_b + c1) * (2 * s_ab + c2)) / ((mu_a ** 2 + mu_b ** 2 + c1) *
                                                      (s_aa + s_bb + c2))
    return float(m.mean())


def make_problem(rows: int, cols: int, sigma: float, radius: int, seed: int, device):
    """(clean image on the host, b = R image + noise on the device, blur spec)."""
    import torch

    from workloads import gen_image, gen_noise, rng_for

    rng = rng_for(40, seed)
    img = gen_image(rng, rows, cols)
    noise = gen_noise(rng, (rows, cols))
    bsp = ops.BlurSpec(rows, cols, sigma=sigma, radius=radius)
    x = torch.tensor(img, dtype=torch.float32, device=device)
    b = ops.blur(bsp, x) + torch.tensor(noise, dtype=torch.float32, device=device)
    return img, b, bsp


def measures(w: ops.WaveletSpec, bsp: ops.BlurSpec, b, x, lam: float, img: np.ndarray) -> dict:
    rec = ops.wavelet_synth(w, x).double().cpu().numpy()
    xh = x.cpu().numpy()
    F = ops.objective(w, bsp, b, x, lam)[0, 2].item()
    return {"rel_err": float(np.linalg.norm(rec - img) / np.linalg.norm(img)),
            "nonzero_pct": float(100.0 * np.count_nonzero(xh) / xh.size),
            "ssim": ssim(rec, img), "objective": F}


def run(rows: int = 256, cols: int = 256, taps: int = 2, levels: int = 3, bc: str = "sym",
        sigma: float = 2.0, radius: int = 4, lam: float = 2e-5, iters: int = 2500,
        every: int = 250, seed: int = 0, device="cuda:0", family: str = "daubechies") -> dict:
    """FISTA from zero with each gradient map; measures at every `every`-th
    iteration and at the last. family="cdf97" runs the biorthogonal CDF 9/7
    pair (taps is then ignored)."""
    import torch

    w = ops.WaveletSpec(rows, cols, levels, taps=taps, bc=bc, family=family)
    img, b, bsp = make_problem(rows, cols, sigma, radius, seed, device)
    out = {"config": {"rows": rows, "cols": cols, "family": family, "taps": w.taps,
                      "levels": levels, "bc": bc,
                      "sigma": sigma, "radius": radius, "lambda": lam, "iterations": iters,
                      "seed": seed}}
    blurred = b.double().cpu().numpy()
    out["blurred"] = {"rel_err": float(np.linalg.norm(blurred - img) / np.linalg.norm(img)),
                      "ssim": ssim(blurred, img)}
    for grad in ("adjoint", "pinv"):
        st = ops.FistaState(w, bsp, b, gradient=grad)
        curve = []
        for k in range(1, iters + 1):
            ops.fista_step(st, b, lam)
            if k % every == 0 or k == iters:
                torch.cuda.synchronize()
                curve.append({"k": k, **measures(w, bsp, b, st.x, lam, img)})
        out[grad] = {**{key: curve[-1][key]
                        for key in ("rel_err", "nonzero_pct", "ssim", "objective")},
                     "curve": curve}
    return out


def main(argv=None) -> None:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--taps", type=int, default=2)
    ap.add_argument("--family", default="daubechies", choices=["daubechies", "cdf97"])
    ap.add_argument("--levels", type=int, default=3)
    ap.add_argument("--bc", default="sym")
    ap.add_argument("--sigma", type=float, default=2.0)
    ap.add_argument("--radius", type=int, default=4)
    ap.add_argument("--lam", type=float, default=2e-5)
    ap.add_argument("--iters", type=int, default=2500)
    ap.add_argument("--every", type=int, default=250)
    ap.add_argument("--seed", type=int, default=0)
    a = ap.parse_args(argv)
    res = run(a.size, a.size, a.taps, a.levels, a.bc, a.sigma, a.radius, a.lam, a.iters, a.every,
              a.seed, family=a.family)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
