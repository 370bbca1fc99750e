"""The binding's constants and status names equal the C header's
(include/hidft.h): a value changed on one side only fails here."""
import os
import re

from paper_2211_15299_amd import native

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                      "hidft.h")


def _header_text():
    with open(HEADER) as fh:
        return fh.read()


def _value(text):
    """An integer or float literal, optionally with a u suffix, parenthesised or
    shifted (the only forms the header's #defines use)."""
    text = re.sub(r"(?<=[0-9a-fA-F])u\b", "", text.strip())
    assert re.fullmatch(r"[0-9a-fA-Fx.()<e\- ]+", text), text
    return eval(text, {"__builtins__": {}})  # noqa: S307 - checked to be a literal


def _defines():
    out = {}
    for line in _header_text().splitlines():
        m = re.match(r"#define (HIDFT_[A-Z0-9_]+)\s+(\(?[0-9][^/]*?)\s*(/\*.*)?$", line)
        if m:
            out[m.group(1)] = _value(m.group(2))
    return out


def test_defines_match_the_binding():
    d = _defines()
    expected = {
        "HIDFT_MAX_LOG2_K_DEVICE": native.MAX_LOG2_K_DEVICE,
        "HIDFT_MAX_LOG2_K_LARGE": native.MAX_LOG2_K_LARGE,
        "HIDFT_PLAN_HOST_ONLY": native.HIDFT_PLAN_HOST_ONLY,
        "HIDFT_PREC_FP32": native.PREC_FP32,
        "HIDFT_PREC_F16X2": native.PREC_F16X2,
        "HIDFT_PREC_BF16X3": native.PREC_BF16X3,
        "HIDFT_SCHED_DEFAULT": native.SCHED_DEFAULT,
        "HIDFT_SCHED_SHORT_FIRST": native.SCHED_SHORT_FIRST,
        "HIDFT_SCHED_SHORT_LAST": native.SCHED_SHORT_LAST,
        "HIDFT_SCHED_TUNED": native.SCHED_TUNED,
        "HIDFT_GROUP_ORDER_LARGEST_FIRST": native.GROUP_ORDER_LARGEST_FIRST,
        "HIDFT_GROUP_ORDER_ALTERNATE": native.GROUP_ORDER_ALTERNATE,
        "HIDFT_SAS_TWO_PASS": native.HIDFT_SAS_TWO_PASS,
        "HIDFT_SAS_WEIGHTS_ONLY": native.HIDFT_SAS_WEIGHTS_ONLY,
        "HIDFT_SAS_MAX_REL_ERR": native.SAS_MAX_REL_ERR,
        "HIDFT_SAS_SCRATCH_BYTES": native.SAS_SCRATCH_BYTES,
    }
    for name, value in expected.items():
        assert name in d, name
        assert d[name] == value, (name, d[name], value)


def test_status_names_match_the_header_enum():
    codes = {name: int(v) for name, v in
             re.findall(r"\b(HIDFT_(?:OK|ERR_[A-Z0-9_]+))\s*=\s*(\d+)", _header_text())}
    assert codes, "no status enum found"
    assert {v: k for k, v in codes.items()} == native.STATUS_NAMES
