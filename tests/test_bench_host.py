"""Host logic of bench.py: the algorithmic byte model, kernel-name mapping and the one-GPU rule."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_kernel_bytes_model():
    mib = 1 << 20
    # level-0 synthesis y = w1 x + A^T z1: read x (1024^2), read z1 (512^2), write y, 64 images
    assert bench.kernel_bytes("lp_up_2d_L16_v2_t1x32x128", 0, 64, 1024) == 4 * 64 * (2 * mib + mib // 4)
    assert bench.kernel_bytes("lp_up_2d_L16_v2_t1x32x128", 0, 64, 1024) == 603979776
    # level-1 analysis a1 = A x: read x, write a1 (512^2)
    assert bench.kernel_bytes("lp_down_2d_L16_v2_t1x16x64", 0, 64, 1024) == 4 * 64 * (mib + mib // 4)
    # a full-bank 3-D level reads and writes its block once
    assert bench.kernel_bytes("fb_down_3d_L8_v0_t2x8x16", 0, 1, 256, ndim=3) == 8 * 256 ** 3


def test_template_names():
    assert bench.template_name("lp_up_2d_L16_v2_t1x32x128") == \
        "void es::k_lp_up<2, 16, 1, 32, 128, 256, true>(es::TaskArgs, es::Filter)"
    assert bench.template_name("lp_down_s_2d_L16_v0_t1x64x256") == \
        "void es::k_lp_down_s<16, 64, 256, 256, true>(es::TaskArgs, es::Filter)"
    assert bench.template_name("fb_down_s_3d_L8_v1_t8x8x16") == \
        "void es::k_fb_down_s<8, 8, 8, 16, 256, true>(es::TaskArgs, es::Filter)"
    assert bench.template_name("lp_down_s_3d_L16_v2_t8x8x32") == \
        "void es::k_lp_down_s3<16, 8, 8, 32, 256, true>(es::TaskArgs, es::Filter)"
    assert bench.template_name("lp_up_s_3d_L4_v0_t16x16x32_scalar") == \
        "void es::k_lp_up_s3<4, 16, 16, 32, 256, false>(es::TaskArgs, es::Filter)"


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one MI355X" in r.stderr
