"""The handle-level workspace (abft_set_workspace: calls passing dwork ==
NULL use it) and abft_report_fetch, through the C ABI, against the same
factorizations given their own workspace."""
import ctypes as C

import numpy as np
import pytest

from paper_2301_03166_amd import gen

pytestmark = pytest.mark.gpu


def test_registered_workspace_and_report_fetch():
    import torch
    from paper_2301_03166_amd import abft
    with abft.Handle() as h:
        n, nb = 700, 128
        A = gen.general(n, 8)
        f = {"iter": 1, "row": 500, "col": 400, "bit": 58}
        ref = torch.from_numpy(np.asfortranarray(A)).cuda()
        ipiv_ref, info_ref, rep_ref = h.getrf(ref, nb, faults=[f])
        opts, keep = abft.make_opts(nb, faults=[f])
        size = C.c_size_t()
        assert abft.lib().abft_workspace_size(h._h, abft.OP_GETRF, n, 0, C.byref(opts), C.byref(size)) == 0
        buf = torch.empty(size.value, dtype=torch.uint8, device="cuda")
        h.set_workspace(buf)
        dA = torch.from_numpy(np.asfortranarray(A)).cuda()
        ipiv = torch.zeros(n, dtype=torch.int32, device="cuda")
        info = torch.zeros(1, dtype=torch.int32, device="cuda")
        drep = h.new_report()
        h._sync_stream()
        rc = abft.lib().abft_getrf(h._h, n, dA.data_ptr(), n, ipiv.data_ptr(), None, 0, C.byref(opts),
                                   info.data_ptr(), drep.data_ptr())
        assert rc == 0
        rep = h.report_fetch(drep)
        assert torch.equal(dA, ref) and torch.equal(ipiv, ipiv_ref) and int(info.item()) == info_ref == 0
        assert rep.status == rep_ref.status == 1 and rep.events() == rep_ref.events() == [(1, 1, 500, 400)]
        assert h.read_report(drep).events() == rep.events()
        # unregistered: a NULL workspace is rejected again
        h.set_workspace(None)
        rc = abft.lib().abft_getrf(h._h, n, dA.data_ptr(), n, ipiv.data_ptr(), None, 0, C.byref(opts),
                                   info.data_ptr(), drep.data_ptr())
        assert rc == abft.ERR_WORKSPACE
