"""Tuning table persistence (hidft_tune_save / hidft_tune_load), host only."""
import pytest

native = pytest.importorskip("paper_2211_15299_amd.native")

TAG = "gfx950:sramecc+:xnack-/256"


def _write(path, text):
    path.write_text(text)
    return str(path)


def test_round_trip(tmp_path):
    native.tune_clear()
    src = _write(tmp_path / "a.txt",
                 "hidft-tune 1\n"
                 f"{TAG} 12 0 12 1 16 2 54.100\n"
                 f"{TAG} 14 1 10 0 0 0 81.700\n"
                 "\n")
    native.tune_load(src)
    out = tmp_path / "b.txt"
    native.tune_save(str(out))
    lines = out.read_text().splitlines()
    assert lines[0] == "hidft-tune 1"
    assert sorted(lines[1:]) == sorted([f"{TAG} 12 0 12 1 16 2 54.100",
                                        f"{TAG} 14 1 10 0 0 0 81.700"])
    # loading merges: an equal key is replaced, others are kept
    native.tune_load(_write(tmp_path / "c.txt", f"hidft-tune 1\n{TAG} 12 0 12 2 16 1 50.000\n"))
    native.tune_save(str(out))
    lines = out.read_text().splitlines()[1:]
    assert sorted(lines) == sorted([f"{TAG} 12 0 12 2 16 1 50.000",
                                    f"{TAG} 14 1 10 0 0 0 81.700"])
    native.tune_clear()
    native.tune_save(str(out))
    assert out.read_text() == "hidft-tune 1\n"


@pytest.mark.parametrize("text,what", [
    ("12 0 12 1 16 2 54.1\n", "header"),
    (f"hidft-tune 1\n{TAG} 12 0 12 1 8 2 54.1\n", "line 2"),       # radix 8
    (f"hidft-tune 1\n{TAG} 15 0 12 1 16 2 54.1\n", "line 2"),      # s > 14
    (f"hidft-tune 1\n{TAG} 12 3 12 1 16 2 54.1\n", "line 2"),      # precision 3
    (f"hidft-tune 1\n{TAG} 12 0 12 3 16 2 54.1\n", "line 2"),      # schedule TUNED
    (f"hidft-tune 1\n{TAG} 12 0 12 1 16\n", "line 2"),             # short line
])
def test_malformed_files_are_refused(tmp_path, text, what):
    native.tune_clear()
    native.tune_load(_write(tmp_path / "ok.txt", f"hidft-tune 1\n{TAG} 10 0 5 1 16 0 1.000\n"))
    with pytest.raises(native.HiDFTError) as ei:
        native.tune_load(_write(tmp_path / "bad.txt", text))
    assert ei.value.status_name == "HIDFT_ERR_INVALID_ARGUMENT"
    assert what in str(ei.value)
    # the table is unchanged
    out = tmp_path / "after.txt"
    native.tune_save(str(out))
    assert out.read_text().splitlines()[1:] == [f"{TAG} 10 0 5 1 16 0 1.000"]
    native.tune_clear()


def test_missing_file(tmp_path):
    with pytest.raises(native.HiDFTError) as ei:
        native.tune_load(str(tmp_path / "does_not_exist.txt"))
    assert ei.value.status_name == "HIDFT_ERR_INVALID_ARGUMENT"
    with pytest.raises(native.HiDFTError):
        native.tune_save(str(tmp_path / "no_such_dir" / "x.txt"))
