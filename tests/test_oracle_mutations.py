"""Each plausible mistake planted in the oracle (on the CPU, in a private copy of
its source) must make at least one pin fail.  This checks that the pins constrain
every part of the oracle: a dropped term, a wrong sign, an off-by-one, a
transposed operand."""
import contextlib
import sys

import pytest

import oracle
from oracle import geometry, composite, sh, loss, grad, adam, binning, schedule
import tests.test_oracle_geometry as TG
import tests.test_oracle_render as TR
import tests.test_oracle_grad_loss_adam as TL
import tests.test_oracle_margins as TM

_MODS = {"geometry": geometry, "composite": composite, "sh": sh, "loss": loss, "grad": grad, "adam": adam,
         "binning": binning, "schedule": schedule}


@contextlib.contextmanager
def _mutated(modname, old, new):
    mod = _MODS[modname]
    src = open(mod.__file__).read()
    assert src.count(old) >= 1, f"mutation anchor not found: {old!r}"
    saved = dict(mod.__dict__)
    exec(compile(src.replace(old, new, 1), mod.__file__, "exec"), mod.__dict__)
    # rebind names other oracle modules imported from the mutated one
    patched = []
    for other in list(_MODS.values()) + [oracle]:
        for k, v in list(other.__dict__.items()):
            if k in saved and saved[k] is v and mod.__dict__.get(k) is not v and other is not mod:
                other.__dict__[k] = mod.__dict__[k]
                patched.append((other, k, v))
    try:
        yield
    finally:
        mod.__dict__.clear()
        mod.__dict__.update(saved)
        for other, k, v in patched:
            other.__dict__[k] = v


def _fails(tests):
    for t, args in tests:
        try:
            t(*args)
        except (AssertionError, IndexError, ValueError, RuntimeError):
            return True
    return False


MUTATIONS = [
    ("geometry", "J02 = -(fx * txc)", "J02 = (fx * txc)",
     [(TG.test_ewa_equals_fd_jacobian_route, (False,))]),
    ("geometry", "T1 = [J11 * R[1][k] + J12 * R[2][k] for k in range(3)]",
     "T1 = [J11 * R[k][1] + J12 * R[k][2] for k in range(3)]",
     [(TG.test_ewa_equals_fd_jacobian_route, (False,)), (TG.test_ewa_monte_carlo, ())]),
    ("geometry", "S11 = ((U1[0] * T1[0] + U1[1] * T1[1]) + U1[2] * T1[2]) + KAPPA",
     "S11 = ((U1[0] * T1[0] + U1[1] * T1[1]) + U1[2] * T1[2])",
     [(TG.test_isotropic_on_axis_closed_form, ())]),
    ("geometry", "b = -S01 / dets", "b = S01 / dets", [(TG.test_conic_and_extent, ())]),
    ("geometry", "xlo, xhi = np.ceil((un - rn) - 0.5)", "xlo, xhi = np.ceil((un - rn) + 0.5)",
     [(TG.test_tile_rect_brute_force, (16,))]),
    ("geometry", "txc = tzs * torch.clamp(tx / tzs, -limx, limx)", "txc = tx",
     [(TG.test_ewa_equals_fd_jacobian_route, (True,))]),
    ("geometry", "[2.0 * (x * y + w * z), 1.0", "[2.0 * (x * y - w * z), 1.0",
     [(TG.test_rotation_matches_scipy_and_is_orthonormal, ())]),
    ("geometry", "return [-((R[0][k] * t[0] + R[1][k] * t[1]) + R[2][k] * t[2]) for k in range(3)]",
     "return [-((R[k][0] * t[0] + R[k][1] * t[1]) + R[k][2] * t[2]) for k in range(3)]",
     [(TG.test_view_dependent_colour_independent_route, ())]),
    ("geometry", "raw.append(acc)", "raw.append(acc - 0.5 + 0.25)",
     [(TG.test_view_dependent_colour_independent_route, ())]),
    ("sh", "coef = norm * ((-1) ** am)", "coef = norm * (1)", [(TR.test_sh_matches_scipy_real_form, ())]),
    ("sh", "math.factorial(l - am) / math.factorial(l + am)", "math.factorial(l + am) / math.factorial(l - am)",
     [(TR.test_sh_orthonormal_by_quadrature, ())]),
    ("composite", "power = -0.5 * (a * dx * dx + c * dy * dy) - b * dx * dy",
     "power = -0.5 * (a * dx * dx + c * dy * dy) + b * dx * dy",
     [(TR.test_vectorised_equals_scalar_brute_force, (32, 3, (29, 23)))]),
    ("composite", "blended = ps & (kidx[None, :] < kstar[:, None])", "blended = ps & (kidx[None, :] <= kstar[:, None])",
     [(TR.test_blending_invariants, ()), (TR.test_vectorised_equals_scalar_brute_force, (31, 0, (32, 32)))]),
    ("composite", "Te = torch.cat([ones, Ti[:, :-1]], dim=1) if nc else Ti", "Te = Ti",
     [(TR.test_two_gaussians_depth_order, ())]),
    ("composite", "order = np.lexsort((vis, proj[\"depth_bits\"][vis]))", "order = np.lexsort((proj[\"depth_bits\"][vis], vis))",
     [(TR.test_two_gaussians_depth_order, ())]),
    ("loss", "C2 = 0.03 ** 2", "C2 = 0.02 ** 2", [(TL.test_ssim_textbook_and_constant_images, ())]),
    ("loss", "C1 = 0.01 ** 2", "C1 = 0.001 ** 2", [(TL.test_ssim_textbook_and_constant_images, ())]),
    ("loss", "sxy = blur(x * y) - mx * my", "sxy = blur(x * y)",
     [(TL.test_ssim_identity_and_l1_value, ())]),
    ("loss", "return F.conv2d(img[None], w2, padding=WIN // 2, groups=img.shape[0])[0]",
     "return F.conv2d(F.pad(img[None], (5, 5, 5, 5), mode='replicate'), w2, groups=img.shape[0])[0]",
     [(TL.test_blur_matches_scipy_gaussian_filter, ())]),
    ("grad", 'out = r["C"] + r["T_final"][None, :] * bg[:, None]', 'out = r["C"] + r["T_final"].detach()[None, :] * bg[:, None]',
     [(TL.test_param_grads_finite_differences, (41, 3, (0.3, 0.1, 0.6)))]),
    ("composite", "alpha2 = torch.clamp(o2[None, :] * torch.exp(power2), max=alpha_max)",
     "alpha2 = torch.clamp(o2[None, :].detach() * torch.exp(power2), max=alpha_max)",
     [(TL.test_param_grads_finite_differences, (42, 1, (0.0, 0.0, 0.0)))]),
    ("adam", "bc2 = 1.0 - b2 ** k", "bc2 = 1.0 - b1 ** k", [(TL.test_adam_matches_torch_fp64, ())]),
    ("binning", "    nbc = -b / c\n", "    nbc = b / c\n", [(TG.test_box_min_matches_dense_sampling, ())]),
    ("binning", "    return np.where(inside, 0.0, best)", "    return best",
     [(TG.test_box_min_matches_dense_sampling, ())]),
    ("binning", 'L = -2.0 * p["tau"]', 'L = -1.0 * p["tau"]',
     [(TG.test_ellipse_culling_keeps_every_contributing_tile, (16,))]),
    ("binning", "order = np.lexsort((gg, dp, tl))", "order = np.lexsort((dp, gg, tl))",
     [(TG.test_binning_sorted_and_ranges, ())]),
    ("adam", "return np.where(cnt > 0, s / np.maximum(cnt, 1), vs.mean())", "return np.where(cnt > 0, s, vs.mean())",
     [(TL.test_adam_view_factor_and_first_step_closed_form, ())]),
    ("schedule", "w[i] = sum(w[j] * M[j, i] for j in prev) / len(prev)", "w[i] = sum(w[j] * M[j, i] for j in prev)",
     [(TL.test_schedule_eq3_to_eq5, ())]),
    ("schedule", "t = 1.0 if trained_iters > t_a else trained_iters / t_a", "t = trained_iters / t_a",
     [(TL.test_schedule_eq6_to_eq8, ())]),
    ("schedule", "/ (len(nb) + 1)", "/ len(nb)", [(TL.test_schedule_eq6_to_eq8, ())]),
    ("schedule", "share = {i: raw[i] / (2.0 * tot) * t_i for i in top}", "share = {i: raw[i] / tot * t_i for i in top}",
     [(TL.test_schedule_eq3_to_eq5, ()), (TL.test_schedule_iteration_plan, ())]),
    ("schedule", "rest.sort(key=lambda i: (u[i], i))", "rest.sort(key=lambda i: (-u[i], i))",
     [(TL.test_schedule_iteration_plan, ())]),
    ("composite", 'out["alpha_sum"] = torch.where(blended, alpha2', 'out["alpha_sum"] = torch.where(ps, alpha2',
     [(TR.test_vectorised_equals_scalar_brute_force, (31, 0, (32, 32))),
      (TR.test_soft_count_stops_with_the_walk, ())]),
    ("loss", "var = ((g - g.mean()) ** 2).mean()", "var = (g ** 2).mean()", [(TL.test_load_balance_loss_eq9, ())]),
    ("grad", "obj = obj + (r[\"alpha_sum\"]", "obj = obj + 0.0 * (r[\"alpha_sum\"]",
     [(TL.test_param_grads_with_load_term_finite_differences, ())]),
    ("schedule", "rest = [i for i in range(n) if i not in share] or list(range(n))",
     "rest = list(range(n))", [(TL.test_schedule_iteration_plan, ())]),
    # decision margins (what the parity tests set aside)
    ("composite", "m_cut = (power - q[\"tau\"][None, :]).abs() / (q[\"tau\"][None, :].abs() + s_abs)",
     "m_cut = (power - q[\"tau\"][None, :]).abs() / (q[\"tau\"][None, :].abs())",
     [(TM.test_cap_and_sign_margins_single_splat, ())]),
    ("composite", "m_cut = (power - q[\"tau\"][None, :]).abs()", "m_cut = (power - q[\"tau\"][None, :])",
     [(TM.test_cutoff_margin_flags_every_cutoff_flip, ())]),
    ("composite", "upto = torch.arange(G)[None, :] <= stop_col[:, None]",
     "upto = torch.arange(G)[None, :] < stop_col[:, None]", [(TM.test_cutoff_margin_covers_the_stopping_splat, ())]),
    ("composite", "s_abs = 0.5 * (a.abs() * dx * dx + c.abs() * dy * dy) + (b * dx * dy).abs()",
     "s_abs = 0.5 * (a.abs() * dx * dx + c.abs() * dy * dy) + (b * dx * dy)",
     [(TM.test_cap_and_sign_margins_single_splat, ())]),
    ("composite", "m_cap = (og - alpha_max).abs() / alpha_max", "m_cap = (og - alpha_max) / alpha_max",
     [(TM.test_cap_and_sign_margins_single_splat, ())]),
    ("composite", "(t_min * sens.clamp(min=1.0))", "(t_min * 1.0)", [(TM.test_stop_margin_flags_every_stop_flip, ())]),
    ("composite", "m_T = ((T_incl - t_min).abs()", "m_T = ((T_incl - t_min)",
     [(TM.test_stop_margin_flags_every_stop_flip, ())]),
    ("composite", 'out["m_T"] = torch.where(upto_c, m_T, inf)', 'out["m_T"] = torch.where(blended, m_T, inf)',
     [(TM.test_stop_margin_flags_every_stop_flip, ())]),
    ("geometry", "o = 1.0 / (1.0 + torch.exp(-P[10]))", "o = 1.0 / (1.0 + torch.exp(P[10]))",
     [(TG.test_opacity_is_logistic, ())]),
    ("geometry", "s = [torch.exp(P[3 + i]) for i in range(3)]", "s = [torch.exp(0.5 * P[3 + i]) for i in range(3)]",
     [(TG.test_isotropic_on_axis_closed_form, ())]),
    ("geometry", "M = [[R[k][j] * s[j] for j in range(3)] for k in range(3)]",
     "M = [[R[j][k] * s[j] for j in range(3)] for k in range(3)]", [(TG.test_covariance_eigen_and_matrix_route, ())]),
    ("geometry", 'tiles_y = [(c["height"] + tile - 1) // tile for c in cams]',
     'tiles_y = [c["height"] // tile for c in cams]', [(TG.test_tile_layout_brute_force, (16,))]),
    ("sh", "acc = acc * z + cf", "acc = acc * z - cf", [(TR.test_sh_matches_scipy_real_form, ())]),
    ("adam", "g[11:14] = GROUP_SH_DC", "g[11:13] = GROUP_SH_DC", [(TL.test_adam_group_rates_follow_the_parameter_layout, ())]),
    ("adam", "g[6:10] = GROUP_ROT", "g[6:10] = GROUP_SCALE", [(TL.test_adam_group_rates_follow_the_parameter_layout, ())]),
    ("schedule", "return (lr_c[j] + sum(M[i, j] * lr_c[i] for i in nb)) / (len(nb) + 1)",
     "return (lr_c[j] + sum(lr_c[i] for i in nb)) / (len(nb) + 1)", [(TL.test_schedule_eq6_to_eq8, ())]),
    ("schedule", "raw = {i: (1.0 - math.exp(-weights[i])) for i in top}", "raw = {i: weights[i] for i in top}",
     [(TL.test_schedule_eq3_to_eq5, ())]),
    ("schedule", "for i in sorted(top, key=lambda i: (-(share[i] - base[i]), i))[:rem]:",
     "for i in sorted(top, key=lambda i: ((share[i] - base[i]), i))[:rem]:", [(TL.test_schedule_iteration_plan, ())]),
    ("loss", "val = val + w_dssim * (1.0 - ssim_map(x, y).mean())",
     "val = val + w_dssim * (1.0 - ssim_map(x, y).mean()) * 0.5", [(TL.test_ssim_textbook_and_constant_images, ())]),
    ("adam", "s = (vs[:, None] * vis).sum(0)", "s = (vs[:, None]).sum(0)",
     [(TL.test_adam_view_factor_and_first_step_closed_form, ())]),
    ("adam", "if (group_mask >> groups[r]) & 1:", "if True:", [(TL.test_adam_view_factor_and_first_step_closed_form, ())]),
    ("composite", 'order = np.lexsort((vis, proj["depth_bits"][vis]))',
     'order = np.lexsort((-vis, proj["depth_bits"][vis]))', [(TR.test_two_gaussians_depth_order, ())]),
    ("binning", "x1 = np.minimum(tx * tile + (tile - 0.5), W - 0.5)", "x1 = tx * tile + (tile - 0.5)",
     [(TG.test_ellipse_culling_box_is_the_hull_of_pixel_centres, (16,))]),
    ("binning", "y0 = ty * tile + 0.5", "y0 = ty * tile", [(TG.test_ellipse_culling_box_is_the_hull_of_pixel_centres, (16,))]),
    ("binning", 'ty = p["ty0"][rep] + local // nx', 'ty = p["ty0"][rep] + local % nx',
     [(TG.test_binning_sorted_and_ranges, ())]),
    ("geometry", "lam = 0.5 * (S00 + S11) + torch.sqrt(", "lam = 0.5 * (S00 + S11) - torch.sqrt(",
     [(TG.test_conic_and_extent, ())]),
    ("geometry", "tau = torch.clamp(-torch.log(ALPHA_MIN_INV * o), min=CUTOFF_FLOOR)", "tau = -torch.log(ALPHA_MIN_INV * o)",
     [(TG.test_cutoff_exponent, ())]),
    ("geometry", "i1 = np.nan_to_num(np.clip(xhi, -1, W - 1), nan=-1).astype(np.int64)",
     "i1 = np.nan_to_num(np.clip(xhi, -1, W), nan=-1).astype(np.int64)", [(TG.test_tile_rect_brute_force, (16,))]),
    ("geometry", "tx0, tx1, ty0, ty1 = i0 // tile, i1 // tile, j0 // tile, j1 // tile",
     "tx0, tx1, ty0, ty1 = i0 // tile, i1 // tile + 1, j0 // tile, j1 // tile",
     [(TG.test_ellipse_culling_box_is_the_hull_of_pixel_centres, (16,))]),
    ("geometry", "depth_bits = tz.detach().to(torch.float32).numpy().view(np.uint32).copy()",
     "depth_bits = tz.detach().to(torch.float64).numpy().view(np.uint64).astype(np.uint32)",
     [(TR.test_two_gaussians_depth_order, ())]),
    ("geometry", "rgb = torch.clamp(raw, min=0.0)", "rgb = raw", [(TG.test_view_dependent_colour_independent_route, ())]),
    ("geometry", "acc = SH_OFFSET + 0.0 * mx", "acc = 0.0 * mx", [(TR.test_sh_degree0_colour, ())]),
    ("geometry", "dx_, dy_, dz_ = mx - oc[0], my - oc[1], mz - oc[2]", "dx_, dy_, dz_ = mx, my, mz",
     [(TG.test_view_dependent_colour_independent_route, ())]),
    ("composite", "pxc = torch.as_tensor(np.asarray(px, np.float64) + 0.5)",
     "pxc = torch.as_tensor(np.asarray(px, np.float64))", [(TR.test_cutoffs_off_is_eq2, ())]),
    ("composite", "stop = ps & (T_incl < t_min)", "stop = ps & (T_incl <= 0.5 * t_min)", [(TR.test_blending_invariants, ())]),
    ("composite", 'out["n_eval"] = (ps & (kidx[None, :] <= kstar[:, None])).sum(1)',
     'out["n_eval"] = (ps & (kidx[None, :] < kstar[:, None])).sum(1)', [(TR.test_soft_count_stops_with_the_walk, ())]),
    ("composite", "lastk = torch.where(blended.any(1), nc - 1 - _first_true(blended.flip(1)),",
     "lastk = torch.where(blended.any(1), nc - 2 - _first_true(blended.flip(1)),",
     [(TR.test_vectorised_equals_scalar_brute_force, (31, 0, (32, 32)))]),
    ("grad", "up = torch.as_tensor(g[:, py[s:s + chunk], px[s:s + chunk]])",
     "up = torch.as_tensor(g[::-1, py[s:s + chunk], px[s:s + chunk]].copy())",
     [(TL.test_param_grads_colour_closed_form, ())]),
    ("grad", "active = np.any(g != 0, axis=0)", "active = np.all(g != 0, axis=0) & False",
     [(TL.test_param_grads_colour_closed_form, ())]),
    ("adam", "upd = (m_new / bc1[None, :]) / (np.sqrt(v_new / bc2[None, :]) + e)",
     "upd = (m_new / bc1[None, :]) / np.sqrt(v_new / bc2[None, :] + e)", [(TL.test_adam_matches_torch_fp64, ())]),
    ("adam", "m_new = b1 * m + (1.0 - b1) * g", "m_new = b1 * m + g", [(TL.test_adam_matches_torch_fp64, ())]),
    ("loss", "val = w_l1 * (x - y).abs().mean()", "val = w_l1 * (x - y).abs().sum()",
     [(TL.test_ssim_identity_and_l1_value, ())]),
]


@pytest.mark.parametrize("modname,old,new,tests", MUTATIONS, ids=[f"{m[0]}:{i}" for i, m in enumerate(MUTATIONS)])
def test_planted_mistake_is_caught(modname, old, new, tests):
    # the unmutated oracle passes the same pins
    assert not _fails(tests)
    with _mutated(modname, old, new):
        assert _fails(tests), f"planted mistake not caught: {new!r}"
