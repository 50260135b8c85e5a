"""Host-side checks of the tuning table (no GPU: these calls touch no device)."""
import json

import pytest

from paper_2301_08275_amd import gpe


@pytest.fixture(autouse=True)
def clean_table():
    gpe.gpe_tuning_clear()
    yield
    gpe.gpe_tuning_clear()


def desc(shape, prec="fp64"):
    return gpe.make_desc(shape, -1.0, 1.0, 0.0, prec)


def test_defaults_without_entry():
    t, found = gpe.gpe_tuning_get(desc((512, 512, 512)))
    assert not found
    assert t["width"] == [16, 8, 0] and t["xcd_remap"] == [1, 1, 0]
    assert t["pass_order"] == [2, 1, 0]
    t32, _ = gpe.gpe_tuning_get(desc((512, 512, 512), "fp32"))
    assert t32["width"] == [16, 16, 0]
    t2, _ = gpe.gpe_tuning_get(desc((128, 128)))
    assert t2["width"] == [8, 0] and t2["pass_order"] == [1, 0]


def test_radix_plan_only_where_an_alternative_exists():
    d = desc((1024, 1024, 64))
    gpe.gpe_tuning_set(d, [16, 8, 0], [1, 1, 0], [2, 1, 0], plan=[1, 0, 0])
    t, found = gpe.gpe_tuning_get(d)
    assert found and t["plan"] == [1, 0, 0]
    with pytest.raises(gpe.GpeError) as e:
        gpe.gpe_tuning_set(d, [16, 8, 0], [1, 1, 0], [2, 1, 0], plan=[0, 0, 1])  # 64 points
    assert e.value.status == gpe.GPE_EINVAL
    assert gpe.gpe_tuning_get(desc((512, 512, 512)))[0]["plan"] == [0, 0, 0]


def test_files_without_plans_load(tmp_path):
    path = tmp_path / "old.json"
    path.write_text('{"format": "gpe-tuning-1", "classes": [{"dim": 2, "n": [64, 64], '
                    '"precision": "fp64", "width": [16, 0], "xcd_remap": [0, 0], '
                    '"pass_order": [0, 1], "ms_per_step": 0.01}]}')
    gpe.gpe_tuning_load(str(path))
    t, found = gpe.gpe_tuning_get(desc((64, 64)))
    assert found and t["plan"] == [0, 0] and t["width"] == [16, 0] and t["stream"] == [0, 0]


def test_set_get_is_per_shape_class():
    d = desc((256, 256, 256))
    gpe.gpe_tuning_set(d, [8, 16, 0], [0, 1, 0], [0, 2, 1])
    t, found = gpe.gpe_tuning_get(d)
    assert found and t["width"] == [8, 16, 0] and t["pass_order"] == [0, 2, 1]
    assert t["xcd_remap"] == [0, 1, 0]
    # other precision, other shape: untouched
    assert not gpe.gpe_tuning_get(desc((256, 256, 256), "fp32"))[1]
    assert not gpe.gpe_tuning_get(desc((256, 256, 128)))[1]
    # box and g are not part of the class
    assert gpe.gpe_tuning_get(gpe.make_desc((256,) * 3, 0.0, 5.0, 3.0))[1]


@pytest.mark.parametrize("width,xcd,order", [
    ([4, 8, 0], [0, 0, 0], [2, 1, 0]),     # width not 8 or 16
    ([8, 8, 0], [2, 0, 0], [2, 1, 0]),     # xcd flag not 0/1
    ([8, 8, 0], [0, 0, 0], [2, 2, 0]),     # not a permutation
    ([8, 8, 0], [0, 0, 0], [3, 1, 0]),     # axis out of range
])
def test_invalid_entries_are_rejected(width, xcd, order):
    with pytest.raises(gpe.GpeError) as e:
        gpe.gpe_tuning_set(desc((64, 64, 64)), width, xcd, order)
    assert e.value.status == gpe.GPE_EINVAL


@pytest.mark.parametrize("bad", [[4, 0, 0], [0, -1, 0]])
def test_stream_flags_are_two_bits_per_axis(bad):
    d = desc((64, 64, 64))
    gpe.gpe_tuning_set(d, [8, 8, 0], [0, 0, 0], [2, 1, 0], stream=[3, 0, 2])
    t, found = gpe.gpe_tuning_get(d)
    assert found and t["stream"] == [3, 0, 2]
    with pytest.raises(gpe.GpeError) as e:
        gpe.gpe_tuning_set(d, [8, 8, 0], [0, 0, 0], [2, 1, 0], stream=bad)
    assert e.value.status == gpe.GPE_EINVAL


def test_save_load_round_trip(tmp_path):
    gpe.gpe_tuning_set(desc((512, 512, 512)), [16, 8, 0], [0, 1, 0], [2, 1, 0])
    gpe.gpe_tuning_set(desc((128, 256), "fp32"), [16, 0], [1, 0], [0, 1])
    gpe.gpe_tuning_set(desc((1024,) * 3, "fp32s"), [8, 16, 0], [1, 0, 0], [2, 1, 0],
                       plan=[0, 0, 1], stream=[0, 1, 1])
    path = tmp_path / "tune.json"
    gpe.gpe_tuning_save(str(path))
    data = json.loads(path.read_text())
    assert data["format"] == "gpe-tuning-1" and len(data["classes"]) == 3
    gpe.gpe_tuning_clear()
    assert not gpe.gpe_tuning_get(desc((512, 512, 512)))[1]
    gpe.gpe_tuning_load(str(path))
    t, found = gpe.gpe_tuning_get(desc((512, 512, 512)))
    assert found and t["xcd_remap"] == [0, 1, 0]
    t, found = gpe.gpe_tuning_get(desc((128, 256), "fp32"))
    assert found and t["width"] == [16, 0] and t["pass_order"] == [0, 1]
    t, found = gpe.gpe_tuning_get(desc((1024,) * 3, "fp32s"))
    assert found and t["plan"] == [0, 0, 1] and t["width"] == [8, 16, 0]
    assert t["stream"] == [0, 1, 1]


@pytest.mark.parametrize("text", [
    "",
    "{",
    '{"format": "other", "classes": []}',
    '{"format": "gpe-tuning-1", "classes": [{"dim": 3}]}',
    '{"format": "gpe-tuning-1", "classes": [{"dim": 3, "n": [512, 512, 500], "precision": "fp64",'
    ' "width": [16, 8, 0], "xcd_remap": [1, 1, 0], "pass_order": [2, 1, 0]}]}',
    '{"format": "gpe-tuning-1", "classes": [{"dim": 2, "n": [64, 64], "precision": "fp16",'
    ' "width": [8, 0], "xcd_remap": [1, 0], "pass_order": [1, 0]}]}',
    '{"format": "gpe-tuning-1", "classes": []} trailing',
])
def test_malformed_files_are_rejected_whole(tmp_path, text):
    gpe.gpe_tuning_set(desc((64, 64)), [16, 0], [0, 0], [0, 1])
    path = tmp_path / "bad.json"
    path.write_text(text)
    with pytest.raises(gpe.GpeError):
        gpe.gpe_tuning_load(str(path))
    # the table is unchanged
    t, found = gpe.gpe_tuning_get(desc((64, 64)))
    assert found and t["width"] == [16, 0]


def test_load_missing_file(tmp_path):
    with pytest.raises(gpe.GpeError):
        gpe.gpe_tuning_load(str(tmp_path / "none.json"))


def test_separable_parameters_marshal_by_name():
    """Host-side packing of the separable-potential parameters (no device)."""
    s = gpe.fill_separable(gpe.gpe_separable(), dict(w=[1.0, 2.0], lattice=[0.5, 0.0, 3.0]))
    assert list(s.w) == [1.0, 2.0, 0.0] and list(s.lattice) == [0.5, 0.0, 3.0]
    assert list(s.center) == [0.0, 0.0, 0.0] and list(s.phase) == [0.0, 0.0, 0.0]
    with pytest.raises(ValueError):
        gpe.fill_separable(gpe.gpe_separable(), dict(omega=[1.0]))


def test_rotating_passes_entry(tmp_path):
    d = desc((512, 512, 512), "fp32s")
    gpe.gpe_tuning_set(d, [16, 8, 8], [0, 1, 1], [2, 0, 1], stream=[3, 1, 0], transpose=1)
    t, found = gpe.gpe_tuning_get(d)
    # the last axis keeps its width and tile order when the passes rotate
    assert found and t["transpose"] == 1 and t["width"] == [16, 8, 8]
    assert t["xcd_remap"] == [0, 1, 1]
    path = tmp_path / "rot.json"
    gpe.gpe_tuning_save(str(path))
    assert json.loads(path.read_text())["classes"][0]["transpose"] == 1
    gpe.gpe_tuning_clear()
    gpe.gpe_tuning_load(str(path))
    assert gpe.gpe_tuning_get(d)[0] == t
    # in-place entries drop the last axis's width; entries without the key load as 0
    gpe.gpe_tuning_set(d, [16, 8, 8], [0, 1, 1], [2, 1, 0])
    t, _ = gpe.gpe_tuning_get(d)
    assert t["transpose"] == 0 and t["width"] == [16, 8, 0]
    assert gpe.gpe_tuning_get(desc((512, 512, 512)))[0]["transpose"] == 0
    for bad in [dict(d=desc((64, 64)), w=[8, 8], x=[0, 0], o=[0, 1], tr=1),
                dict(d=d, w=[16, 8, 2], x=[0, 1, 1], o=[2, 0, 1], tr=1),
                dict(d=d, w=[16, 8, 8], x=[0, 1, 1], o=[2, 0, 1], tr=2)]:
        with pytest.raises(gpe.GpeError) as e:
            gpe.gpe_tuning_set(bad["d"], bad["w"], bad["x"], bad["o"], transpose=bad["tr"])
        assert e.value.status == gpe.GPE_EINVAL


def test_two_half_tiles_need_fp32_storage_and_in_place_passes():
    for prec in ("fp32s", "fp32"):
        d = desc((512, 512, 512), prec)
        gpe.gpe_tuning_set(d, [32, 16, 0], [0, 1, 0], [2, 1, 0])
        assert gpe.gpe_tuning_get(d)[0]["width"] == [32, 16, 0]
    for d, tr in [(desc((512, 512, 512)), 0), (desc((512, 512, 512), "fp32s"), 1)]:
        with pytest.raises(gpe.GpeError) as e:
            gpe.gpe_tuning_set(d, [32, 16, 16], [0, 1, 1], [2, 0, 1], transpose=tr)
        assert e.value.status == gpe.GPE_EINVAL


def test_four_line_tiles_only_for_rotating_passes():
    d = desc((512, 512, 512))
    gpe.gpe_tuning_set(d, [4, 8, 4], [1, 1, 1], [2, 0, 1], transpose=1)
    assert gpe.gpe_tuning_get(d)[0]["width"] == [4, 8, 4]
    with pytest.raises(gpe.GpeError) as e:
        gpe.gpe_tuning_set(d, [4, 8, 0], [1, 1, 0], [2, 1, 0])
    assert e.value.status == gpe.GPE_EINVAL
