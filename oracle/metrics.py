"""PSNR as defined in Section 4 (oracle; test infrastructure).

PSNR = mean over every slice of the trailing modes (i_3, i_4, ...) of
10 log10(Max^2 / MSE over the I_1 x I_2 slice), Max = 1 for data normalized to
[0, 1].  SSIM is not implemented: its printed formula reuses one symbol for
the covariance and the standard deviation and leaves c_1, c_2 unset.
"""

import numpy as np


def psnr(truth, recon, peak=1.0):
    t = np.asarray(truth, dtype=np.float64)
    r = np.asarray(recon, dtype=np.float64)
    I1, I2 = t.shape[0], t.shape[1]
    t = t.reshape(I1 * I2, -1)
    r = r.reshape(I1 * I2, -1)
    mse = np.mean((t - r) ** 2, axis=0)
    return float(np.mean(10.0 * np.log10(peak ** 2 / mse)))
