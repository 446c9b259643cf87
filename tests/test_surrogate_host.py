"""Host-side checks of the surrogate driver (no GPU needed): the correction interval and the
training lead are validated before any device work."""
import pytest

from paper_1711_04471_amd import surrogate as S


@pytest.mark.parametrize("lead", [0, 6, 24])
def test_dataset_lead_must_be_whole_coarse_steps_within_the_spacing(lead):
    with pytest.raises(ValueError):
        S.make_dataset([1], n=64, pairs_per_run=1, every=20, lead=lead, device="cpu")


@pytest.mark.parametrize("every", [0, 3, 7])
def test_correction_interval_must_divide_the_judge_interval(every):
    with pytest.raises(ValueError):
        S.rollout(None, None, n_coarse=50, judge_every=50, correct_every=every, device="cpu")
