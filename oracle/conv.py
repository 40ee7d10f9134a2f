"""FP64 reference of the grid CNN layers (test infrastructure only).

A layer is a 3x3x3 cross-correlation on the (r, e, a) grid with zero padding
along r and e and circular padding along azimuth a, plus bias; the library
step is PyTorch's CPU conv3d in float64 applied after explicit circular
padding of the azimuth axis.  Layouts follow include/tspnn.h: volumes are
channels-last [N][D0][D1][D2][C]; weights [27][Cout][Cin] with tap
t = (dr+1)*9 + (de+1)*3 + (da+1).
"""
import torch
import torch.nn.functional as F


def _to_torch_w(w):
    """[27][Cout][Cin] -> [Cout][Cin][3][3][3]."""
    w = torch.as_tensor(w, dtype=torch.float64)
    co, ci = w.shape[1], w.shape[2]
    return w.reshape(3, 3, 3, co, ci).permute(3, 4, 0, 1, 2).contiguous()


def conv(x, w, b=None):
    """x: [N][D0][D1][D2][Cin] -> [N][D0][D1][D2][Cout], float64."""
    x = torch.as_tensor(x, dtype=torch.float64).permute(0, 4, 1, 2, 3)
    x = F.pad(x, (1, 1, 0, 0, 0, 0), mode="circular")
    y = F.conv3d(x, _to_torch_w(w), None if b is None else torch.as_tensor(b, dtype=torch.float64),
                 padding=(1, 1, 0))
    return y.permute(0, 2, 3, 4, 1).contiguous()


def conv_direct(x, w, b=None):
    """The same layer by explicit loops (small inputs only)."""
    x = torch.as_tensor(x, dtype=torch.float64)
    w = torch.as_tensor(w, dtype=torch.float64)
    N, D0, D1, D2, _ = x.shape
    co = w.shape[1]
    y = torch.zeros((N, D0, D1, D2, co), dtype=torch.float64)
    for n in range(N):
        for i in range(D0):
            for j in range(D1):
                for k in range(D2):
                    acc = torch.zeros(co, dtype=torch.float64) if b is None else \
                        torch.as_tensor(b, dtype=torch.float64).clone()
                    for t in range(27):
                        dr, de, da = t // 9 - 1, (t // 3) % 3 - 1, t % 3 - 1
                        ii, jj, kk = i + dr, j + de, (k + da) % D2
                        if 0 <= ii < D0 and 0 <= jj < D1:
                            acc = acc + w[t] @ x[n, ii, jj, kk]
                    y[n, i, j, k] = acc
    return y
