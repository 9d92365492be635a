"""The entry point's smoke run (one small rollout and adjoint on cuda:0,
checked against the FP64 oracle) as part of the device suite, so that a change
to the bindings that breaks it shows up with the other device tests."""
import pytest

import __graft_entry__ as entry


@pytest.mark.gpu
def test_smoke_entry_point():
    entry.smoke()
